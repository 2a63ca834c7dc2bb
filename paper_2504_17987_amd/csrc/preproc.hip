// Pre-processing of the frames (Sec. 2: a high-pass filter removes the
// static background, then contrast-limited adaptive histogram equalisation
// brightens the image; Sec. 3.1 uses both to match the intensities of
// stitched images).  Integer arithmetic throughout, so the results are
// exact.  Both passes stream the frames once (reads and writes coalesced by
// rows); the tile halos of the high-pass come from L2.
#include <algorithm>

#include "dev_common.h"
#include "piv_internal.h"

namespace piv {
namespace {

// ---------------------------------------------------------------------------
// High-pass: out = max(0, I - floor(sum / count)) over the image part of the
// (2r+1)^2 box around each pixel.  One wave owns a strip of columns and a
// band of rows and walks down it: lane L holds the vertical box sums of the
// PX pixels of one aligned word (PX = 4 for u8, 2 for u16), updated per row
// by the row entering and the row leaving the box (each a coalesced word
// read; the leaving row comes from cache); the wave's sums go through LDS,
// where each lane adds the 2r+1 columns around its pixels.  The strip's
// first and last h = ceil(r / PX) lanes only supply sums, so strips overlap
// by 2h words.  The pixel count of the clipped box is a product of two
// clipped spans; the quotient comes from a float reciprocal, corrected to
// the exact floor.
// ---------------------------------------------------------------------------
constexpr int HBAND = 64;

// floor(s / c) for quotients below 2^16 (s < 2^27, 1 <= c < 2^11): the
// float estimate is then within one of the quotient, and integer
// corrections make it exact
__device__ __forceinline__ uint32_t udiv_small(uint32_t s, uint32_t c) {
  int q = (int)((float)s * __builtin_amdgcn_rcpf((float)c));
  int r = (int)s - q * (int)c;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    q += r < 0 ? -1 : (r >= (int)c ? 1 : 0);
    r = (int)s - q * (int)c;
  }
  return (uint32_t)q;
}

// floor(s / d) for the whole box, d = (2R+1)^2, s < 2^27: the product with
// M = ceil(2^(32+k) / d), k = ceil(log2 d) - 1 (so that M < 2^32), keeps
// its error s (M d - 2^(32+k)) / d below 2^(32+k) / d > 2^31 > s, hence exact
template <int D>
struct BoxDiv {
  static constexpr int K = []() { int k = 0; while ((1 << (k + 1)) < D) ++k; return k; }();
  static constexpr uint32_t M = (uint32_t)((((uint64_t)1 << (32 + K)) + D - 1) / D);
  static_assert((1ull << K) < (unsigned long long)D && (((uint64_t)1 << (32 + K)) / D) > (1u << 27), "magic range");
};

template <typename T, int R>
__global__ __launch_bounds__(64) void k_highpass(const uint8_t* __restrict__ in, uint8_t* __restrict__ out,
                                                 int64_t pitch, int64_t stride, int W, int H,
                                                 const uint8_t* mask) {
  constexpr int ES = (int)sizeof(T), PX = 4 / ES;   // pixels per word
  constexpr int r = R;
  using Div = BoxDiv<(2 * R + 1) * (2 * R + 1)>;
  __shared__ uint32_t vbuf[2][64 * PX + 1];          // the wave's vertical sums of a row (two rows alternate)
  const int pair = blockIdx.z;
  if (slot_off(mask, pair)) return;
  const int L = threadIdx.x;
  constexpr int h = (r + PX - 1) / PX, nout = 64 - 2 * h;
  const int word = blockIdx.x * nout + L - h;        // this lane's word column (may lie off the image)
  const int xa = 4 * word;                           // its byte offset in a row
  const int rowbytes = W * ES;
  const uint8_t* src = in + (int64_t)pair * stride;
  // the lane's word in a row, zero where it leaves the image (the column
  // clamp and byte mask are the lane's own, the row's test is uniform)
  const int xc = min(max(xa, 0), (rowbytes - 1) & ~3);
  const int valid = rowbytes - xa;
  const uint32_t keep = (xa < 0 || valid <= 0) ? 0u : (valid >= 4 ? 0xffffffffu : (1u << (8 * (valid & 3))) - 1u);
  auto row_word = [&](int y) -> uint32_t {
    const uint32_t ok = (unsigned)y < (unsigned)H ? keep : 0u;
    return *reinterpret_cast<const uint32_t*>(src + (int64_t)min(max(y, 0), H - 1) * pitch + xc) & ok;
  };
  auto px = [&](uint32_t w, int e) -> uint32_t { return ES == 1 ? (w >> (8 * e)) & 0xffu : (w >> (16 * e)) & 0xffffu; };
  const bool outl = L >= h && L < 64 - h;            // lanes whose pixels are written
  const int x0 = word * PX;                          // first pixel column of the lane
  uint32_t cx[PX];
  bool fx = true;
#pragma unroll
  for (int e = 0; e < PX; ++e) {
    cx[e] = (uint32_t)(min(x0 + e + r, W - 1) - max(x0 + e - r, 0) + 1);
    fx = fx && cx[e] == 2 * r + 1;
  }
  // (every written pixel of the strip has its box's full width)
  const bool full_x = __all(fx || !(L >= h && L < 64 - h));
  const int ys = blockIdx.y * HBAND, ye = min(ys + HBAND, H);
  uint32_t V[PX];
#pragma unroll
  for (int e = 0; e < PX; ++e) V[e] = 0u;
  for (int dy = -r; dy <= r; ++dy) {
    const uint32_t w = row_word(ys + dy);
#pragma unroll
    for (int e = 0; e < PX; ++e) V[e] += px(w, e);
  }
  uint8_t* dst = out + (int64_t)pair * stride;
  // rows in groups of G: the words of the next group (entering, leaving and
  // centre rows) are requested while this group is worked
  constexpr int G = 4;
  uint32_t ci[G], co[G], cc[G], ni[G], no[G], nc[G];
  auto fetch = [&](int yg, uint32_t* wi, uint32_t* wo, uint32_t* wc) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
      wi[g] = row_word(yg + g + r);
      wo[g] = row_word(yg + g - r - 1);
      wc[g] = row_word(yg + g);
    }
  };
  fetch(ys, ci, co, cc);
  for (int yg = ys; yg < ye; yg += G) {
    if (yg + G < ye) fetch(yg + G, ni, no, nc);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int y = yg + g;
      if (y >= ye) break;
      if (y > ys) {
#pragma unroll
        for (int e = 0; e < PX; ++e) V[e] += px(ci[g], e) - px(co[g], e);
      }
      const uint32_t wc = cc[g];
      // (rows alternate between two buffers: a row's buffer is written again
      // two rows later, after the next row's barrier, when every lane has
      // finished reading it)
      uint32_t* vb = vbuf[(y - ys) & 1];
#pragma unroll
      for (int e = 0; e < PX; ++e) vb[L * PX + e] = V[e];
      __syncthreads();
      if (outl) {
        // box sums of the lane's pixels: the first by 2r+1 columns, then slid
        const int c0 = L * PX;
        uint32_t hsum = 0u;
#pragma unroll
        for (int i = -r; i <= r; ++i) hsum += vb[c0 + i];
        const uint32_t cy = (uint32_t)(min(y + r, H - 1) - max(y - r, 0) + 1);
        uint32_t hs[PX];
#pragma unroll
        for (int e = 0; e < PX; ++e) {
          if (e) hsum += vb[c0 + e + r] - vb[c0 + e - 1 - r];
          hs[e] = hsum;
        }
        uint32_t m[PX];
        if (cy == 2 * r + 1 && full_x) {
          // the whole box inside the image (the usual case, taken by the
          // whole wave): the constant divisor's product
#pragma unroll
          for (int e = 0; e < PX; ++e) m[e] = __umulhi(hs[e], Div::M) >> Div::K;
        } else {
#pragma unroll
          for (int e = 0; e < PX; ++e) m[e] = udiv_small(hs[e], cx[e] * cy);
        }
        uint32_t o[PX];
#pragma unroll
        for (int e = 0; e < PX; ++e) {
          const uint32_t I = px(wc, e);
          o[e] = I > m[e] ? I - m[e] : 0u;
        }
        T* orow = reinterpret_cast<T*>(dst + (int64_t)y * pitch);
        if (x0 >= 0 && x0 + PX <= W) {
          if constexpr (ES == 1) *reinterpret_cast<uint32_t*>(orow + x0) = o[0] | (o[1] << 8) | (o[2] << 16) | (o[3] << 24);
          else *reinterpret_cast<uint32_t*>(orow + x0) = o[0] | (o[1] << 16);
        } else {
#pragma unroll
          for (int e = 0; e < PX; ++e)
            if (x0 + e >= 0 && x0 + e < W) orow[x0 + e] = (T)o[e];
        }
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      ci[g] = ni[g];
      co[g] = no[g];
      cc[g] = nc[g];
    }
  }
}

// ---------------------------------------------------------------------------
// CLAHE, pass 1: one workgroup per tile.  Histogram in LDS with integer
// atomics (the order of the adds does not matter): 8 copies for u8 (2 for
// u16) spread the atomics of a wave over different addresses, and zeros (the
// bulk of a particle image's background) are counted in registers and added
// once.  Then the clip at max(1, floor(clip * npix / nbins)) (the same
// double arithmetic as the host), the clipped excess spread evenly
// (excess / nbins to every bin, one more to the first `rest` bins at a
// stride of max(nbins / rest, 1)), a prefix sum and
// lut[b] = (cdf * maxval + npix / 2) / npix.
// ---------------------------------------------------------------------------
constexpr int kLutT = 256;

// (j L < 2^31: frames are at most 32767 px and grids 64 tiles)
__device__ __forceinline__ int tile_edge(int j, int L, int n) { return (j * L) / n; }

template <typename T>
__global__ __launch_bounds__(kLutT) void k_clahe_lut(const uint8_t* __restrict__ in, int64_t pitch, int64_t stride,
                                                     int W, int H, int tx, int ty, int nbins, int shift, int maxval,
                                                     double clip_factor, uint16_t* lut, const uint8_t* mask) {
  constexpr int ES = (int)sizeof(T), PW = 4 / ES;
  constexpr int NH = ES == 1 ? 8 : 2;               // histogram copies
  constexpr int HB = ES == 1 ? 256 : 4096;
  __shared__ uint32_t hist[NH * HB];
  __shared__ uint32_t part[kLutT];
  const int pair = blockIdx.z;
  if (slot_off(mask, pair)) return;
  const int t = threadIdx.x;
  const int i = blockIdx.x, j = blockIdx.y;
  const int xa = tile_edge(i, W, tx), xb = tile_edge(i + 1, W, tx);
  const int ya = tile_edge(j, H, ty), yb = tile_edge(j + 1, H, ty);
  const int tw = xb - xa, th = yb - ya;
  const int64_t npix = (int64_t)tw * th;
  for (int b = t; b < NH * nbins; b += kLutT) hist[b] = 0u;
  __syncthreads();
  uint32_t* hc = hist + (t / (kLutT / NH)) * nbins;   // this thread's copy
  const uint8_t* src = in + (int64_t)pair * stride;
  const int rowbytes = W * ES;
  const int w0 = (xa * ES) >> 2, nw = ((xb * ES + 3) >> 2) - w0;
  uint32_t zeros = 0u;
  for (int p = t; p < th * nw; p += kLutT) {
    const int ry = p / nw, k = p - (p / nw) * nw;
    const uint32_t wd = masked_word(src + (int64_t)(ya + ry) * pitch, rowbytes, 4 * (w0 + k));
#pragma unroll
    for (int e = 0; e < PW; ++e) {
      const int x = (4 * (w0 + k)) / ES + e;
      if (x >= xa && x < xb) {
        const uint32_t v = ES == 1 ? (wd >> (8 * e)) & 0xffu : (wd >> (16 * e)) & 0xffffu;
        if (v == 0u) ++zeros;
        else atomicAdd(&hc[v >> shift], 1u);
      }
    }
  }
  part[t] = zeros;
  __syncthreads();
  for (int o = kLutT / 2; o > 0; o >>= 1) {
    if (t < o) part[t] += part[t + o];
    __syncthreads();
  }
  const uint32_t nzero = part[0];
  __syncthreads();
  // merge the copies into copy 0 (bin 0 takes the zeros)
  for (int b = t; b < nbins; b += kLutT) {
    uint32_t h = b == 0 ? nzero : 0u;
#pragma unroll
    for (int c = 0; c < NH; ++c) h += hist[c * nbins + b];
    hist[b] = h;
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
// the last a single tile is used.
struct Axis {
  int a, b;
  int w, d;
};
__device__ __forceinline__ Axis clahe_axis(int x, int L, int n) {
  const int X = 2 * x;
  const int k = ((x + 1) * n + L - 1) / L - 1;
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

// A workgroup covers MQ columns (four per thread) and MR rows.  The column
// blend data (tile pair and weights) is tabulated once per workgroup in LDS;
// when the mappings the block touches fit (u8), they are staged in LDS too,
// otherwise they are read from memory (L1/L2).  Every thread reads its four
// pixels, then writes them, so the pass may run in place.
constexpr int MQ = 1024, MR = 16;

// floor((num + den / 2) / den) for 0 <= num < 2^52, 1 <= den < 2^32: the
// double quotient is within one of the result, then an integer correction
// makes it exact (cheaper than a 64-bit integer division)
__device__ __forceinline__ int64_t round_div(int64_t num, int64_t den) {
  const int64_t n2 = num + den / 2;
  int64_t q = (int64_t)((double)n2 / (double)den);
  int64_t r = n2 - q * den;
  q += r < 0 ? -1 : (r >= den ? 1 : 0);
  return q;
}
constexpr int kStageWords = 6144;   // LDS words for staged mappings (24 KB)

template <typename T, bool kStaged, bool kNarrow>
__global__ __launch_bounds__(256) void k_clahe_map(const uint8_t* in, uint8_t* out, int64_t pitch, int64_t stride,
                                                   int W, int H, int tx, int ty, int nbins, int shift,
                                                   const uint16_t* __restrict__ lut, const uint8_t* mask) {
  constexpr int ES = (int)sizeof(T);
  __shared__ uint32_t s_ax[MQ];          // per column: a | b << 8 | w << 16 (w < 2^16, d in s_ad)
  __shared__ uint16_t s_ad[MQ];
  __shared__ Axis s_ay[MR];
  __shared__ uint32_t s_lut[kStaged ? kStageWords : 1];
  const int pair = blockIdx.z;
  if (slot_off(mask, pair)) return;
  const int t = threadIdx.x;
  const int x0 = blockIdx.x * MQ, y0 = blockIdx.y * MR;
  const int nq = min(MQ, W - x0);
  for (int c = t; c < nq; c += 256) {
    const Axis a = clahe_axis(x0 + c, W, tx);
    s_ax[c] = (uint32_t)a.a | ((uint32_t)a.b << 8) | ((uint32_t)a.w << 16);
    s_ad[c] = (uint16_t)a.d;
  }
  if (t < MR && y0 + t < H) s_ay[t] = clahe_axis(y0 + t, H, ty);
  const uint16_t* Lp = lut + (int64_t)pair * ty * tx * nbins;
  // tiles the block can touch: columns of its first and last pixel, rows of
  // its first and last row
  const Axis axl = clahe_axis(x0, W, tx), axr = clahe_axis(x0 + nq - 1, W, tx);
  const int yl = min(y0 + MR, H) - 1;
  const Axis ayt = clahe_axis(y0, H, ty), ayb = clahe_axis(yl, H, ty);
  const int i0 = axl.a, i1 = axr.b, j0 = ayt.a, j1 = ayb.b;
  const int ni = i1 - i0 + 1;
  if constexpr (kStaged) {
    const int words = (j1 - j0 + 1) * ni * nbins / 2;
    for (int k = t; k < words; k += 256) {
      const int e = 2 * k;
      const int tile = e / nbins, b = e - tile * nbins;
      const int jj = j0 + tile / ni, ii = i0 + tile - (tile / ni) * ni;
      s_lut[k] = *reinterpret_cast<const uint32_t*>(Lp + ((int64_t)jj * tx + ii) * nbins + b);
    }
  }
  __syncthreads();
  const uint16_t* sl = reinterpret_cast<const uint16_t*>(s_lut);
  // a mapping entry at (row part, column part, bin): the staged copy or the
  // global one, with the parts of the offset formed once per row and column
  auto L = [&](int rpart, int cpart, int b) -> int {
    if constexpr (kStaged) return sl[rpart + cpart + b];
    else return Lp[(int64_t)rpart + cpart + b];
  };
  auto rpart_of = [&](int jj) { return kStaged ? (jj - j0) * ni * nbins : jj * tx * nbins; };
  auto cpart_of = [&](int ii) { return kStaged ? (ii - i0) * nbins : ii * nbins; };
  const int c0 = 4 * t;
  if (c0 >= nq) return;
  const int xq = x0 + c0;
  const bool full = c0 + 4 <= nq;
  // this thread's four columns: tiles, weights and mapping offsets (the
  // same on every row)
  int ca[4], cb[4], cwx[4], cdx[4], kdx[4];
  float rdx[4];   // 1 / dx (the quotient's estimate is corrected exactly below)
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int c = min(c0 + e, nq - 1);
    const uint32_t ax = s_ax[c];
    ca[e] = cpart_of((int)(ax & 0xff));
    cb[e] = cpart_of((int)((ax >> 8) & 0xff));
    cwx[e] = (int)(ax >> 16);
    cdx[e] = s_ad[c];
    rdx[e] = __builtin_amdgcn_rcpf((float)cdx[e]);
    kdx[e] = (cdx[e] & (cdx[e] - 1)) == 0 ? __builtin_ctz((unsigned)cdx[e]) : -1;   // log2 dx, or -1
  }
  for (int k = 0; k < MR; ++k) {
    const int y = y0 + k;
    if (y >= H) break;
    const Axis ay = s_ay[k];
    const int ra = rpart_of(ay.a), rb = rpart_of(ay.b);
    const float rdy = __builtin_amdgcn_rcpf((float)ay.d);
    const int kdy = (ay.d & (ay.d - 1)) == 0 ? __builtin_ctz((unsigned)ay.d) : -1;
    const T* row = reinterpret_cast<const T*>(in + (int64_t)pair * stride + (int64_t)y * pitch);
    T* orow = reinterpret_cast<T*>(out + (int64_t)pair * stride + (int64_t)y * pitch);
    uint32_t v[4];
    if (full) {
      if constexpr (ES == 1) {
        const uint32_t wd = *reinterpret_cast<const uint32_t*>(row + xq);
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = (wd >> (8 * e)) & 0xffu;
      } else {
        const uint32_t w0 = *reinterpret_cast<const uint32_t*>(row + xq);
        const uint32_t w1 = *reinterpret_cast<const uint32_t*>(row + xq + 2);
        v[0] = w0 & 0xffffu; v[1] = w0 >> 16; v[2] = w1 & 0xffffu; v[3] = w1 >> 16;
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) v[e] = c0 + e < nq ? (uint32_t)row[xq + e] : 0u;
    }
    uint32_t o[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int wx = cwx[e], dx = cdx[e];
      const int b = (int)(v[e] >> shift);
      if constexpr (kNarrow) {
        // every numerator and denominator below 2^24 (checked on the host):
        // float estimate of the rounded quotient, then an exact correction
        const int l00 = L(ra, ca[e], b), l01 = L(ra, cb[e], b), l10 = L(rb, ca[e], b), l11 = L(rb, cb[e], b);
        const int num = (ay.d - ay.w) * ((dx - wx) * l00 + wx * l01) + ay.w * ((dx - wx) * l10 + wx * l11);
        const int den = dx * ay.d;
        const int n2 = num + den / 2;
        int q;
        if (kdx[e] >= 0 && kdy >= 0) {
          // a power-of-two denominator (tile spans of 2^k px): the floor by a shift
          q = n2 >> (kdx[e] + kdy);
        } else {
          // (the rounded quotient is below 2^16, so the estimate from the two
          // reciprocals is within one of it)
          q = (int)((float)n2 * rdx[e] * rdy);
          const int rr = n2 - q * den;
          q += rr < 0 ? -1 : (rr >= den ? 1 : 0);
        }
        o[e] = (uint32_t)q;
      } else {
        const int64_t l00 = L(ra, ca[e], b), l01 = L(ra, cb[e], b), l10 = L(rb, ca[e], b), l11 = L(rb, cb[e], b);
        const int64_t num = (int64_t)(ay.d - ay.w) * ((dx - wx) * l00 + wx * l01) +
                            (int64_t)ay.w * ((dx - wx) * l10 + wx * l11);
        const int64_t den = (int64_t)dx * ay.d;
        o[e] = (uint32_t)round_div(num, den);
      }
    }
    if (full) {
      if constexpr (ES == 1) {
        *reinterpret_cast<uint32_t*>(orow + xq) = o[0] | (o[1] << 8) | (o[2] << 16) | (o[3] << 24);
      } else {
        *reinterpret_cast<uint32_t*>(orow + xq) = o[0] | (o[1] << 16);
        *reinterpret_cast<uint32_t*>(orow + xq + 2) = o[2] | (o[3] << 16);
      }
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (c0 + e < nq) orow[xq + e] = (T)o[e];
    }
  }
}

}  // namespace

int clahe_bins(const Plan& P) {
  const int bits = P.p.dtype == PIV_U8 ? 8 : P.p.bit_depth;
  return 1 << (bits < 12 ? bits : 12);
}

hipError_t launch_highpass(const Plan& P, const void* in, void* out, int64_t pitch, int n, int r, hipStream_t s) {
  const int px = P.es == 1 ? 4 : 2;
  const int nout = 64 - 2 * ((r + px - 1) / px);       // words written per strip
  const int words = (P.p.width + px - 1) / px;
  dim3 grid((words + nout - 1) / nout, (P.p.height + HBAND - 1) / HBAND, n);
  const int64_t stride = pitch * P.p.height;
  const uint8_t* i8 = (const uint8_t*)in;
  uint8_t* o8 = (uint8_t*)out;
  switch (r) {
#define PIV_HP(R_)                                                                                               \
  case R_:                                                                                                     \
    if (P.es == 1)                                                                                             \
      hipLaunchKernelGGL((k_highpass<uint8_t, R_>), grid, dim3(64), 0, s, i8, o8, pitch, stride, P.p.width,   \
                         P.p.height, P.slot_mask);                                                              \
    else                                                                                                       \
      hipLaunchKernelGGL((k_highpass<uint16_t, R_>), grid, dim3(64), 0, s, i8, o8, pitch, stride, P.p.width,  \
                         P.p.height, P.slot_mask);                                                              \
    break;
    PIV_HP(1) PIV_HP(2) PIV_HP(3) PIV_HP(4) PIV_HP(5) PIV_HP(6) PIV_HP(7) PIV_HP(8)
    PIV_HP(9) PIV_HP(10) PIV_HP(11) PIV_HP(12) PIV_HP(13) PIV_HP(14) PIV_HP(15) PIV_HP(16)
#undef PIV_HP
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// The staged map kernel holds the mappings of every tile a block can touch:
// at most (columns of MQ pixels' tiles + 2) x (rows of MR rows' tiles + 2).
static bool clahe_stage_fits(const Plan& P, int tx, int ty, int nbins) {
  const int tw = P.p.width / tx, th = P.p.height / ty;   // smallest tile sizes
  if (tw < 1 || th < 1) return false;
  const int ncol = MQ / tw + 3, nrow = MR / th + 3;
  return (int64_t)ncol * nrow * nbins / 2 <= kStageWords;
}

hipError_t launch_clahe(const Plan& P, const void* in, void* out, int64_t pitch, int n, int tx, int ty,
                        double clip_factor, uint16_t* lut, hipStream_t s) {
  const int bits = P.p.dtype == PIV_U8 ? 8 : P.p.bit_depth;
  const int nbins = clahe_bins(P), shift = bits - (bits < 12 ? bits : 12), maxval = (1 << bits) - 1;
  const int64_t stride = pitch * P.p.height;
  dim3 g1(tx, ty, n);
  dim3 g2((P.p.width + MQ - 1) / MQ, (P.p.height + MR - 1) / MR, n);
  const bool staged = clahe_stage_fits(P, tx, ty, nbins);
  // the blend denominator per axis is a centre distance in doubled
  // coordinates, e(a+2) - e(a); the 32-bit path needs
  // maxval dx dy + dx dy / 2 < 2^24 for the largest ones
  auto dmax = [](int L, int n) {
    int64_t m = 1;
    for (int a = 0; a + 2 <= n; ++a) m = std::max<int64_t>(m, (int64_t)(a + 2) * L / n - (int64_t)a * L / n);
    return m;
  };
  const int64_t dd = dmax(P.p.width, tx) * dmax(P.p.height, ty);
  const bool narrow = (int64_t)maxval * dd + dd / 2 < (int64_t(1) << 24);
#define PIV_MAP(T_, ST_, NA_)                                                                              \
  hipLaunchKernelGGL((k_clahe_map<T_, ST_, NA_>), g2, dim3(256), 0, s, (const uint8_t*)in, (uint8_t*)out, pitch, \
                     stride, P.p.width, P.p.height, tx, ty, nbins, shift, (const uint16_t*)lut, P.slot_mask)
#define PIV_CLAHE(T_)                                                                                           \
  hipLaunchKernelGGL(k_clahe_lut<T_>, g1, dim3(kLutT), 0, s, (const uint8_t*)in, pitch, stride, P.p.width,        \
                     P.p.height, tx, ty, nbins, shift, maxval, clip_factor, lut, P.slot_mask);                  \
  if (hipError_t e = hipGetLastError()) return e;                                                              \
  if (staged && narrow) PIV_MAP(T_, true, true);                                                                \
  else if (staged) PIV_MAP(T_, true, false);                                                                    \
  else if (narrow) PIV_MAP(T_, false, true);                                                                    \
  else PIV_MAP(T_, false, false)
  if (P.es == 1) {
    PIV_CLAHE(uint8_t);
  } else {
    PIV_CLAHE(uint16_t);
  }
#undef PIV_CLAHE
#undef PIV_MAP
  return hipGetLastError();
}

}  // namespace piv
