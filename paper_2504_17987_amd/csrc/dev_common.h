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
// negative or past the row), with zero for bytes outside [0, rowbytes).  The
// read is clamped into the row and always issued, so that a run of such
// reads is not serialised behind branches; it is in bounds because row
// pitches are multiples of 4 and rowbytes <= pitch.
__device__ __forceinline__ uint32_t masked_word(const uint8_t* row, int rowbytes, int xa) {
  const int xc = min(max(xa, 0), (rowbytes - 1) & ~3);
  const uint32_t w = *reinterpret_cast<const uint32_t*>(row + xc);
  const int valid = rowbytes - xa;
  const uint32_t part = (1u << (8 * (valid & 3))) - 1u;
  const uint32_t keep = (xa < 0 || valid <= 0) ? 0u : (valid >= 4 ? 0xffffffffu : part);
  return w & keep;
}

// Workgroups are dealt round-robin to the 8 XCDs, each with its own L2.
// xcd_order() renumbers them so that each XCD takes one contiguous run of
// the linear grid order (x fastest, then y, then z): neighbouring tiles,
// which read the same cache lines, then meet in the same L2.
struct WgIdx {
  int x, y, z;
};
__device__ __forceinline__ WgIdx xcd_order() {
  const int gx = gridDim.x, gy = gridDim.y;
  const int n = gx * gy * gridDim.z;
  int p = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
  const int full = n & ~7;
  if (p < full) p = (p & 7) * (full >> 3) + (p >> 3);
  WgIdx w;
  w.x = p % gx;
  p /= gx;
  w.y = p % gy;
  w.z = p / gy;
  return w;
}

// Whole-wave reductions by DPP (all 64 lanes active), returned wave-uniform:
// pairs and quads by quad permutes, rows of 16 by the half-row and row
// mirrors, then row 15 -> row 1, row 31 -> rows 2 and 3; lane 63 ends
// with the reduction of every lane.  For min and max a lane whose row is
// masked keeps its own value (harmless: the operations are idempotent); for
// the sum it takes 0.
#define PIV_DPP_I(v, ctrl, rmask, old) __builtin_amdgcn_update_dpp((old), (v), (ctrl), (rmask), 0xF, false)
#define PIV_WAVE_REDUCE_F(x, OP)                                                        \
  do {                                                                                 \
    int xi_ = __float_as_int(x);                                                       \
    x = OP(x, __int_as_float(PIV_DPP_I(xi_, 0xB1, 0xF, xi_)));                         \
    xi_ = __float_as_int(x);                                                           \
    x = OP(x, __int_as_float(PIV_DPP_I(xi_, 0x4E, 0xF, xi_)));                         \
    xi_ = __float_as_int(x);                                                           \
    x = OP(x, __int_as_float(PIV_DPP_I(xi_, 0x141, 0xF, xi_)));                        \
    xi_ = __float_as_int(x);                                                           \
    x = OP(x, __int_as_float(PIV_DPP_I(xi_, 0x140, 0xF, xi_)));                        \
    xi_ = __float_as_int(x);                                                           \
    x = OP(x, __int_as_float(PIV_DPP_I(xi_, 0x142, 0xA, xi_)));                        \
    xi_ = __float_as_int(x);                                                           \
    x = OP(x, __int_as_float(PIV_DPP_I(xi_, 0x143, 0xC, xi_)));                        \
    x = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63));              \
  } while (0)

__device__ __forceinline__ float wave_min(float x) {
  PIV_WAVE_REDUCE_F(x, fminf);
  return x;
}
__device__ __forceinline__ float wave_max(float x) {
  PIV_WAVE_REDUCE_F(x, fmaxf);
  return x;
}
// Two 16-bit unsigned fields per word, each reduced to its own maximum
// (v_pk_max_u16: a per-field max, not a 32-bit one).
typedef unsigned short piv_u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pk_max_u16(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(piv_u16x2, a),
                                                                __builtin_bit_cast(piv_u16x2, b)));
}
__device__ __forceinline__ uint32_t wave_max_pk16(uint32_t x) {
  int xi = (int)x;
  x = pk_max_u16(x, (uint32_t)PIV_DPP_I(xi, 0xB1, 0xF, xi));
  xi = (int)x;
  x = pk_max_u16(x, (uint32_t)PIV_DPP_I(xi, 0x4E, 0xF, xi));
  xi = (int)x;
  x = pk_max_u16(x, (uint32_t)PIV_DPP_I(xi, 0x141, 0xF, xi));
  xi = (int)x;
  x = pk_max_u16(x, (uint32_t)PIV_DPP_I(xi, 0x140, 0xF, xi));
  xi = (int)x;
  x = pk_max_u16(x, (uint32_t)PIV_DPP_I(xi, 0x142, 0xA, xi));
  xi = (int)x;
  x = pk_max_u16(x, (uint32_t)PIV_DPP_I(xi, 0x143, 0xC, xi));
  return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}
__device__ __forceinline__ int wave_sum(int x) {
  x += PIV_DPP_I(x, 0xB1, 0xF, 0);
  x += PIV_DPP_I(x, 0x4E, 0xF, 0);
  x += PIV_DPP_I(x, 0x141, 0xF, 0);
  x += PIV_DPP_I(x, 0x140, 0xF, 0);
  x += PIV_DPP_I(x, 0x142, 0xA, 0);
  x += PIV_DPP_I(x, 0x143, 0xC, 0);
  return __builtin_amdgcn_readlane(x, 63);
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

// Compare-exchange on static indices.
template <typename V>
__device__ __forceinline__ void cswap(V& a, V& b) {
  V lo = a < b ? a : b, hi = a < b ? b : a;
  a = lo;
  b = hi;
}
// Minimum and maximum of finite floats: IEEE minimum/maximum, one
// instruction each, with no quieting of the operands first.
__device__ __forceinline__ float fmin_fin(float a, float b) { return __builtin_elementwise_minimum(a, b); }
__device__ __forceinline__ float fmax_fin(float a, float b) { return __builtin_elementwise_maximum(a, b); }

// floats (finite here) by minimum/maximum
template <>
__device__ __forceinline__ void cswap<float>(float& a, float& b) {
  const float lo = fmin_fin(a, b), hi = fmax_fin(a, b);
  a = lo;
  b = hi;
}

// Sort the first 8 of N >= 8 values ascending (Batcher's odd-even merge
// network, 19 exchanges).
template <int N, typename V>
__device__ __forceinline__ void sort8(V (&v)[N]) {
  static_assert(N >= 8, "needs 8 values");
  cswap(v[0], v[1]); cswap(v[2], v[3]); cswap(v[4], v[5]); cswap(v[6], v[7]);
  cswap(v[0], v[2]); cswap(v[1], v[3]); cswap(v[4], v[6]); cswap(v[5], v[7]);
  cswap(v[1], v[2]); cswap(v[5], v[6]);
  cswap(v[0], v[4]); cswap(v[1], v[5]); cswap(v[2], v[6]); cswap(v[3], v[7]);
  cswap(v[2], v[4]); cswap(v[3], v[5]);
  cswap(v[1], v[2]); cswap(v[3], v[4]); cswap(v[5], v[6]);
}

// Sort 9 values ascending: sort the first 8, then insert the ninth.
template <typename V>
__device__ __forceinline__ void sort9(V (&v)[9]) {
  sort8<9, V>(v);
#pragma unroll
  for (int i = 7; i >= 0; --i) cswap(v[i], v[i + 1]);
}

// Element idx of an array, as a sum of masked elements: written with bit
// operations so that it stays a register computation (a select chain is
// turned back into an indexed load from memory by the optimiser).
__device__ __forceinline__ uint32_t as_u(float x) { return __float_as_uint(x); }
__device__ __forceinline__ uint32_t as_u(int x) { return (uint32_t)x; }
__device__ __forceinline__ float from_u(uint32_t x, float) { return __uint_as_float(x); }
__device__ __forceinline__ int from_u(uint32_t x, int) { return (int)x; }

template <int N, typename V>
__device__ __forceinline__ V pick(const V (&v)[N], int idx) {
  uint32_t out = 0u;
#pragma unroll
  for (int i = 0; i < N; ++i) out |= as_u(v[i]) & (0u - (uint32_t)(idx == i));
  return from_u(out, V());
}

// Sentinels for unused slots: they sort above every real value, so the k
// real values of a slot array are the first k after sorting.  (Slots stay
// at static positions: compacting valid values to the front would need a
// dynamic index.)
constexpr float kSlotF = 3.0e38f;
constexpr int kSlotI = 0x7fffffff;

// Median of the k (>= 1) real values among 8 slots; even k: mean of the
// two middle values.
__device__ __forceinline__ float median8_f(float (&v)[8], int k) {
  sort8<8, float>(v);
  if (k == 8) return 0.5f * (v[3] + v[4]);   // every slot real (the usual case)
  if (k & 1) return pick<8>(v, k >> 1);
  return 0.5f * (pick<8>(v, (k >> 1) - 1) + pick<8>(v, k >> 1));
}

__device__ __forceinline__ int med3i(int a, int b, int c) { return max(min(a, b), min(max(a, b), c)); }

// Median of nine values: order each group of three (slots 0-2, 3-5, 6-8);
// the median is the median of the largest group minimum, the median of the
// group medians and the smallest group maximum.  A min/max network, so by
// the 0-1 principle it is exact for any input, ties included.
__device__ __forceinline__ int median9_groups(const int (&v)[9]) {
  int lo[3], md[3], hi[3];
#pragma unroll
  for (int g = 0; g < 3; ++g) {
    const int a = v[3 * g], b = v[3 * g + 1], c = v[3 * g + 2];
    lo[g] = min(min(a, b), c);
    md[g] = med3i(a, b, c);
    hi[g] = max(max(a, b), c);
  }
  return med3i(max(max(lo[0], lo[1]), lo[2]), med3i(md[0], md[1], md[2]), min(min(hi[0], hi[1]), hi[2]));
}

// Lower median of the k (>= 1) real values among 9 slots.
__device__ __forceinline__ int median9_low_i(int (&v)[9], int k) {
  if (k == 9) return median9_groups(v);   // every slot real (the usual case)
  sort9(v);
  return pick<9>(v, (k - 1) >> 1);
}

}  // namespace piv
