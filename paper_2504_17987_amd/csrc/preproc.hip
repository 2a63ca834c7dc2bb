// Pre-processing of the frames (Sec. 2: a high-pass filter removes the
// static background, then contrast-limited adaptive histogram equalisation
// brightens the image; Sec. 3.1 uses both to match the intensities of
// stitched images).  Integer arithmetic throughout, so the results are
// exact.  Both passes stream the frames once (reads and writes coalesced by
// rows); the tile halos of the high-pass come from L2.
#include "dev_common.h"
#include "piv_internal.h"

namespace piv {
namespace {

// ---------------------------------------------------------------------------
// High-pass: out = max(0, I - floor(sum / count)) over the image part of the
// (2r+1)^2 box around each pixel.  A workgroup owns HT rows x HW columns of
// output: it stages the tile with an r-pixel halo in LDS, forms the
// horizontal box sums of every staged row (a running sum per 16-column
// segment), then the vertical sums down each output column (a running sum
// per 8-row segment).  The pixel count of the clipped box is a product of
// two clipped spans.
// ---------------------------------------------------------------------------
constexpr int HW = 64, HT = 32, kMaxR = 16;
constexpr int RWmax = HW + 2 * kMaxR, RHmax = HT + 2 * kMaxR;

template <typename T>
__global__ __launch_bounds__(256) void k_highpass(const uint8_t* __restrict__ in, uint8_t* __restrict__ out,
                                                  int64_t pitch, int64_t stride, int W, int H, int r,
                                                  const uint8_t* mask) {
  __shared__ uint32_t reg[RHmax][RWmax];   // staged pixels (0 outside the image)
  __shared__ uint32_t hs[RHmax][HW];       // horizontal box sums of the output columns
  const int pair = blockIdx.z;
  if (slot_off(mask, pair)) return;
  const int t = threadIdx.x;
  const int x0 = blockIdx.x * HW, y0 = blockIdx.y * HT;
  const int RW = HW + 2 * r, RH = HT + 2 * r;
  const uint8_t* src = in + (int64_t)pair * stride;
  for (int i = t; i < RW * RH; i += 256) {
    const int ry = i / RW, rx = i - (i / RW) * RW;
    const int y = y0 - r + ry, x = x0 - r + rx;
    uint32_t v = 0u;
    if ((unsigned)y < (unsigned)H && (unsigned)x < (unsigned)W)
      v = reinterpret_cast<const T*>(src + (int64_t)y * pitch)[x];
    reg[ry][rx] = v;
  }
  __syncthreads();
  // horizontal sums: (row, 16-column segment) per thread
  for (int i = t; i < RH * (HW / 16); i += 256) {
    const int ry = i / (HW / 16), c0 = (i - ry * (HW / 16)) * 16;
    uint32_t s = 0u;
    for (int u = 0; u <= 2 * r; ++u) s += reg[ry][c0 + u];
    hs[ry][c0] = s;
#pragma unroll
    for (int c = 1; c < 16; ++c) {
      s += reg[ry][c0 + c + 2 * r] - reg[ry][c0 + c - 1];
      hs[ry][c0 + c] = s;
    }
  }
  __syncthreads();
  // vertical sums: (column, 8-row segment) per thread; consecutive threads
  // take consecutive columns, so the writes of a row coalesce
  const int col = t & (HW - 1), seg = t >> 6;   // 4 segments of 8 rows
  const int x = x0 + col;
  if (x >= W) return;
  const int cx = min(x + r, W - 1) - max(x - r, 0) + 1;
  uint8_t* dst = out + (int64_t)pair * stride;
  const int r0 = seg * 8;
  uint32_t s = 0u;
  for (int v = 0; v <= 2 * r; ++v) s += hs[r0 + v][col];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (k) s += hs[r0 + k + 2 * r][col] - hs[r0 + k - 1][col];
    const int y = y0 + r0 + k;
    if (y >= H) break;
    const int cy = min(y + r, H - 1) - max(y - r, 0) + 1;
    const uint32_t m = s / (uint32_t)(cx * cy);
    const uint32_t I = reg[r0 + k + r][col + r];
    reinterpret_cast<T*>(dst + (int64_t)y * pitch)[x] = (T)(I > m ? I - m : 0u);
  }
}

// ---------------------------------------------------------------------------
// CLAHE, pass 1: one workgroup per tile.  Histogram in LDS (integer atomics,
// so the order of the adds does not matter), clip at
// max(1, floor(clip * npix / nbins)) (the same double arithmetic as the
// host), the clipped excess spread evenly (excess / nbins to every bin, one
// more to the first `rest` bins at a stride of max(nbins / rest, 1)), then a
// prefix sum and lut[b] = (cdf * maxval + npix / 2) / npix.
// ---------------------------------------------------------------------------
constexpr int kLutT = 256;

__device__ __forceinline__ int tile_edge(int j, int L, int n) { return (int)(((int64_t)j * L) / n); }

template <typename T>
__global__ __launch_bounds__(kLutT) void k_clahe_lut(const uint8_t* __restrict__ in, int64_t pitch, int64_t stride,
                                                     int W, int H, int tx, int ty, int nbins, int shift, int maxval,
                                                     double clip_factor, uint16_t* lut, const uint8_t* mask) {
  __shared__ uint32_t hist[4096];
  __shared__ uint32_t part[kLutT];
  const int pair = blockIdx.z;
  if (slot_off(mask, pair)) return;
  const int t = threadIdx.x;
  const int i = blockIdx.x, j = blockIdx.y;
  const int xa = tile_edge(i, W, tx), xb = tile_edge(i + 1, W, tx);
  const int ya = tile_edge(j, H, ty), yb = tile_edge(j + 1, H, ty);
  const int tw = xb - xa, th = yb - ya;
  const int64_t npix = (int64_t)tw * th;
  for (int b = t; b < nbins; b += kLutT) hist[b] = 0u;
  __syncthreads();
  const uint8_t* src = in + (int64_t)pair * stride;
  for (int p = t; p < tw * th; p += kLutT) {
    const int y = ya + p / tw, x = xa + (p - (p / tw) * tw);
    const uint32_t v = reinterpret_cast<const T*>(src + (int64_t)y * pitch)[x];
    atomicAdd(&hist[v >> shift], 1u);
  }
  __syncthreads();
  // (a limit at or above npix clips nothing)
  const double cd = floor(clip_factor * (double)npix / (double)nbins);
  const uint32_t clip = cd < 1.0 ? 1u : cd >= (double)npix ? (uint32_t)npix : (uint32_t)cd;
  uint32_t ex = 0u;
  for (int b = t; b < nbins; b += kLutT) {
    const uint32_t h = hist[b];
    if (h > clip) {
      ex += h - clip;
      hist[b] = clip;
    }
  }
  part[t] = ex;
  __syncthreads();
  for (int o = kLutT / 2; o > 0; o >>= 1) {
    if (t < o) part[t] += part[t + o];
    __syncthreads();
  }
  const uint32_t excess = part[0];
  __syncthreads();
  const uint32_t each = excess / (uint32_t)nbins, rest = excess - each * (uint32_t)nbins;
  const uint32_t sstep = rest ? max((uint32_t)nbins / rest, 1u) : 1u;
  // contiguous chunk of bins per thread for the prefix sum
  const int per = nbins / kLutT > 0 ? nbins / kLutT : 1;
  const int b0 = t * per;
  uint32_t local = 0u;
  for (int b = b0; b < b0 + per && b < nbins; ++b) {
    const uint32_t extra = (rest && (uint32_t)b % sstep == 0u && (uint32_t)b / sstep < rest) ? 1u : 0u;
    const uint32_t h = hist[b] + each + extra;
    hist[b] = h;
    local += h;
  }
  part[t] = local;
  __syncthreads();
  // inclusive scan of the per-thread totals (Hillis-Steele)
  for (int o = 1; o < kLutT; o <<= 1) {
    const uint32_t add = t >= o ? part[t - o] : 0u;
    __syncthreads();
    part[t] += add;
    __syncthreads();
  }
  uint64_t cdf = t ? part[t - 1] : 0u;
  uint16_t* L = lut + (((int64_t)pair * ty + j) * tx + i) * nbins;
  for (int b = b0; b < b0 + per && b < nbins; ++b) {
    cdf += hist[b];
    L[b] = (uint16_t)((cdf * (uint64_t)maxval + (uint64_t)(npix / 2)) / (uint64_t)npix);
  }
}

// CLAHE, pass 2: every pixel blends the mappings of the (up to) four tiles
// whose centres surround it.  In doubled coordinates (centres may be
// half-integers) the tile holding x is k = ceil((x+1) tx / W) - 1 and the
// centre at or left of 2x is k or k - 1; before the first centre or after
// the last a single tile is used.  Four pixels of a row per thread.
struct Axis {
  int a, b;
  int64_t w, d;
};
__device__ __forceinline__ Axis clahe_axis(int x, int L, int n) {
  const int X = 2 * x;
  const int k = (int)((((int64_t)x + 1) * n + L - 1) / L) - 1;
  const int ck = tile_edge(k, L, n) + tile_edge(k + 1, L, n) - 1;
  const int a = ck <= X ? k : k - 1;
  Axis r;
  if (a < 0 || a >= n - 1) {
    r.a = r.b = a < 0 ? 0 : n - 1;
    r.w = 0;
    r.d = 1;
  } else {
    const int ca = tile_edge(a, L, n) + tile_edge(a + 1, L, n) - 1;
    const int cb = tile_edge(a + 1, L, n) + tile_edge(a + 2, L, n) - 1;
    r.a = a;
    r.b = a + 1;
    r.w = X - ca;
    r.d = cb - ca;
  }
  return r;
}

template <typename T>
__global__ __launch_bounds__(256) void k_clahe_map(const uint8_t* in, uint8_t* out, int64_t pitch, int64_t stride,
                                                   int W, int H, int tx, int ty, int nbins, int shift,
                                                   const uint16_t* __restrict__ lut, const uint8_t* mask) {
  const int pair = blockIdx.z;
  if (slot_off(mask, pair)) return;
  const int y = blockIdx.y;
  const int x0 = (blockIdx.x * 256 + threadIdx.x) * 4;
  if (x0 >= W) return;
  const Axis ay = clahe_axis(y, H, ty);
  const uint16_t* Lp = lut + (int64_t)pair * ty * tx * nbins;
  const T* row = reinterpret_cast<const T*>(in + (int64_t)pair * stride + (int64_t)y * pitch);
  T* orow = reinterpret_cast<T*>(out + (int64_t)pair * stride + (int64_t)y * pitch);
  T v[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) v[e] = x0 + e < W ? row[x0 + e] : (T)0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int x = x0 + e;
    if (x >= W) break;
    const Axis ax = clahe_axis(x, W, tx);
    const int b = (int)v[e] >> shift;
    const int64_t l00 = Lp[((int64_t)ay.a * tx + ax.a) * nbins + b];
    const int64_t l01 = Lp[((int64_t)ay.a * tx + ax.b) * nbins + b];
    const int64_t l10 = Lp[((int64_t)ay.b * tx + ax.a) * nbins + b];
    const int64_t l11 = Lp[((int64_t)ay.b * tx + ax.b) * nbins + b];
    const int64_t num = (ay.d - ay.w) * ((ax.d - ax.w) * l00 + ax.w * l01) + ay.w * ((ax.d - ax.w) * l10 + ax.w * l11);
    const int64_t den = ax.d * ay.d;
    orow[x] = (T)((num + den / 2) / den);
  }
}

}  // namespace

int clahe_bins(const Plan& P) {
  const int bits = P.p.dtype == PIV_U8 ? 8 : P.p.bit_depth;
  return 1 << (bits < 12 ? bits : 12);
}

hipError_t launch_highpass(const Plan& P, const void* in, void* out, int64_t pitch, int n, int r, hipStream_t s) {
  dim3 grid((P.p.width + HW - 1) / HW, (P.p.height + HT - 1) / HT, n);
  const int64_t stride = pitch * P.p.height;
  if (P.es == 1)
    hipLaunchKernelGGL(k_highpass<uint8_t>, grid, dim3(256), 0, s, (const uint8_t*)in, (uint8_t*)out, pitch, stride,
                       P.p.width, P.p.height, r, P.slot_mask);
  else
    hipLaunchKernelGGL(k_highpass<uint16_t>, grid, dim3(256), 0, s, (const uint8_t*)in, (uint8_t*)out, pitch,
                       stride, P.p.width, P.p.height, r, P.slot_mask);
  return hipGetLastError();
}

hipError_t launch_clahe(const Plan& P, const void* in, void* out, int64_t pitch, int n, int tx, int ty,
                        double clip_factor, uint16_t* lut, hipStream_t s) {
  const int bits = P.p.dtype == PIV_U8 ? 8 : P.p.bit_depth;
  const int nbins = clahe_bins(P), shift = bits - (bits < 12 ? bits : 12), maxval = (1 << bits) - 1;
  const int64_t stride = pitch * P.p.height;
  dim3 g1(tx, ty, n);
  dim3 g2((P.p.width + 1023) / 1024, P.p.height, n);
  if (P.es == 1) {
    hipLaunchKernelGGL(k_clahe_lut<uint8_t>, g1, dim3(kLutT), 0, s, (const uint8_t*)in, pitch, stride, P.p.width,
                       P.p.height, tx, ty, nbins, shift, maxval, clip_factor, lut, P.slot_mask);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(k_clahe_map<uint8_t>, g2, dim3(256), 0, s, (const uint8_t*)in, (uint8_t*)out, pitch, stride,
                       P.p.width, P.p.height, tx, ty, nbins, shift, (const uint16_t*)lut, P.slot_mask);
  } else {
    hipLaunchKernelGGL(k_clahe_lut<uint16_t>, g1, dim3(kLutT), 0, s, (const uint8_t*)in, pitch, stride, P.p.width,
                       P.p.height, tx, ty, nbins, shift, maxval, clip_factor, lut, P.slot_mask);
    if (hipError_t e = hipGetLastError()) return e;
    hipLaunchKernelGGL(k_clahe_map<uint16_t>, g2, dim3(256), 0, s, (const uint8_t*)in, (uint8_t*)out, pitch, stride,
                       P.p.width, P.p.height, tx, ty, nbins, shift, (const uint16_t*)lut, P.slot_mask);
  }
  return hipGetLastError();
}

}  // namespace piv
