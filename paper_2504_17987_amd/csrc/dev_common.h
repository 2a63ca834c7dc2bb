// Device helpers shared by the libpiv kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace piv {

// Pair i is skipped when a slot mask is bound and its byte is 0.
__device__ __forceinline__ bool slot_off(const uint8_t* mask, int pair) {
  return mask != nullptr && mask[pair] == 0;
}

// Aligned 4-byte word of a row at byte offset xa (a multiple of 4, may be
// negative), with zero for bytes outside [0, rowbytes).  Reading the word is
// in bounds because row pitches are multiples of 4 and rowbytes <= pitch.
__device__ __forceinline__ uint32_t masked_word(const uint8_t* row, int rowbytes, int xa) {
  if (xa < 0 || xa >= rowbytes) return 0u;
  uint32_t w = *reinterpret_cast<const uint32_t*>(row + xa);
  int valid = rowbytes - xa;
  if (valid < 4) w &= (1u << (8 * valid)) - 1u;
  return w;
}

// Pixel value as float with zero outside the image.
template <typename T>
__device__ __forceinline__ float pixf(const uint8_t* img, int64_t pitch, int W, int H, int y, int x) {
  if ((unsigned)x >= (unsigned)W || (unsigned)y >= (unsigned)H) return 0.0f;
  return (float)reinterpret_cast<const T*>(img + (int64_t)y * pitch)[x];
}

// Bilinear sample with zero outside the image: the four corners of the
// floor cell weighted by the fractional position.
template <typename T>
__device__ __forceinline__ float bilin(const uint8_t* img, int64_t pitch, int W, int H, float x, float y) {
  float x0 = floorf(x), y0 = floorf(y);
  float fx = x - x0, fy = y - y0;
  int ix = (int)x0, iy = (int)y0;
  float p00 = pixf<T>(img, pitch, W, H, iy, ix), p01 = pixf<T>(img, pitch, W, H, iy, ix + 1);
  float p10 = pixf<T>(img, pitch, W, H, iy + 1, ix), p11 = pixf<T>(img, pitch, W, H, iy + 1, ix + 1);
  return (1.0f - fy) * ((1.0f - fx) * p00 + fx * p01) + fy * ((1.0f - fx) * p10 + fx * p11);
}

// Rank selection among the first k of N values (static indexing only):
// the value whose rank interval holds `idx` (0-based, ascending).
template <int N, typename V>
__device__ __forceinline__ V select_rank(const V (&v)[N], int k, int idx) {
  V out = v[0];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    if (i < k) {
      int lt = 0, le = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        if (j < k) {
          lt += v[j] < v[i];
          le += v[j] <= v[i];
        }
      }
      if (lt <= idx && idx < le) out = v[i];
    }
  }
  return out;
}

// Median of the first k (>= 1) values; even k: mean of the two middle ones.
template <int N>
__device__ __forceinline__ float median_f(const float (&v)[N], int k) {
  if (k & 1) return select_rank<N, float>(v, k, k >> 1);
  return 0.5f * (select_rank<N, float>(v, k, (k >> 1) - 1) + select_rank<N, float>(v, k, k >> 1));
}

// Lower median of the first k (>= 1) integers.
template <int N>
__device__ __forceinline__ int median_low_i(const int (&v)[N], int k) {
  return select_rank<N, int>(v, k, (k - 1) >> 1);
}

}  // namespace piv
