// Correction kernels (Sec. 2 of the paper): deform the pair by the
// interpolated predictor, correlate every window with the deformed frame B
// over the search shifts (Pearson coefficient), pick the best shift and fit
// a 3-point Gaussian per axis.
//
// Two implementations of the same definition:
//  * k_correct_generic -- one workgroup per window; any window/step/radius.
//  * k_correct_tiled   -- the fast path for 50%-overlap windows (win = 2 step):
//    a workgroup owns a TW x TH tile of windows; the deformed B' tile and the
//    A tile live in LDS; each thread correlates one step x step cell with a
//    band of SYG shift rows, so every pixel-shift product is formed once and
//    shared by the four windows that contain the cell; window sums are then
//    assembled from cell sums.
//
// Numerics (FP32): all sums are taken about a per-tile integer offset K
// (the rounded mean intensity of the tile), which leaves the coefficient
// unchanged and keeps E[x^2] - E[x]^2 well conditioned.  A window counts as
// flat when its variance is below 1e-6 of its second moment about K (an
// exact zero cannot be certified in FP32); a flat window has coefficient 0.
#include "dev_common.h"
#include "piv_internal.h"

namespace piv {
namespace {

constexpr float kFlatRel = 1e-6f;

struct CorrArgs {
  const uint8_t* A;
  const uint8_t* B;
  int64_t pitch, stride;   // bytes per row / per pair
  int W, H, nx, ny;
  int win, step, R;        // R: searched radius (1 in fixed-centre mode)
  int central;             // deform both frames by -u/2, +u/2
  int fixed;               // fixed-centre 5-point stencil
  const float* pred;       // [n][2][ny][nx] or null
  float* disp;
  int64_t dstride;         // floats per pair of disp
  float* peak;             // nullable
  uint8_t* flags;
  const uint8_t* mask;
};

// tie key: smaller is preferred among equal coefficients (|sx|+|sy|, sy, sx)
constexpr int kKeyNone = 0x7fffffff;   // a shift that takes no part in the peak search
__device__ __forceinline__ int tie_key(int sy, int sx) {
  return ((abs(sx) + abs(sy)) << 12) | ((sy + 32) << 6) | (sx + 32);
}

__device__ __forceinline__ bool better(float r1, int k1, float r2, int k2) {
  return r1 > r2 || (r1 == r2 && k1 < k2);
}

// 3-point Gaussian offset on coefficients floored at 1e-3; nocurv when the
// log-parabola does not open downward.
__device__ __forceinline__ float gauss3(float cm, float c0, float cp, bool& nocurv) {
  float lm = logf(fmaxf(cm, 1e-3f)), l0 = logf(fmaxf(c0, 1e-3f)), lp = logf(fmaxf(cp, 1e-3f));
  float den = 2.0f * (lm - 2.0f * l0 + lp);
  nocurv = !(den < 0.0f);
  return nocurv ? 0.0f : (lm - lp) / den;
}

// displacement at pixel (x, y) from a node field read through `node(c, a, b)`
// (clamped to the hull of node centres), bilinear.
template <typename NodeFn>
__device__ __forceinline__ void interp_u(float x, float y, int nx, int ny, int step, NodeFn node,
                                         float& u, float& v) {
  const float c = 0.5f * (float)(step - 1);
  float tx = (x - c) / (float)step, ty = (y - c) / (float)step;
  tx = fminf(fmaxf(tx, 0.0f), (float)(nx - 1));
  ty = fminf(fmaxf(ty, 0.0f), (float)(ny - 1));
  int bx = min((int)tx, max(nx - 2, 0)), by = min((int)ty, max(ny - 2, 0));
  float fx = tx - (float)bx, fy = ty - (float)by;
  int bx1 = nx > 1 ? bx + 1 : bx, by1 = ny > 1 ? by + 1 : by;
  u = (1.0f - fy) * ((1.0f - fx) * node(0, by, bx) + fx * node(0, by, bx1)) +
      fy * ((1.0f - fx) * node(0, by1, bx) + fx * node(0, by1, bx1));
  v = (1.0f - fy) * ((1.0f - fx) * node(1, by, bx) + fx * node(1, by, bx1)) +
      fy * ((1.0f - fx) * node(1, by1, bx) + fx * node(1, by1, bx1));
}

// The correction is relative to the deformation applied to the window, so
// it is added to the window mean of the interpolated predictor.  Bilinear
// interpolation with clamping is separable, so the mean is a product of
// per-axis node weights: for 50%-overlap windows (win = 2 step, step even)
// these are (1/4, 1/2, 1/4) inside, (3/4, 1/4) on the first node and
// (1/4, 3/4) on the last.
__device__ __forceinline__ void half_overlap_weights(int b, int n, float& wm, float& w0, float& wp) {
  if (n == 1) { wm = 0.0f; w0 = 1.0f; wp = 0.0f; }
  else if (b == 0) { wm = 0.0f; w0 = 0.75f; wp = 0.25f; }
  else if (b == n - 1) { wm = 0.25f; w0 = 0.75f; wp = 0.0f; }
  else { wm = 0.25f; w0 = 0.5f; wp = 0.25f; }
}

template <typename NodeFn>
__device__ __forceinline__ void window_mean_half_overlap(int a, int b, int nx, int ny, NodeFn node,
                                                         float& pu, float& pv) {
  float wy[3], wx[3];
  half_overlap_weights(a, ny, wy[0], wy[1], wy[2]);
  half_overlap_weights(b, nx, wx[0], wx[1], wx[2]);
  pu = pv = 0.0f;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      float w = wy[i] * wx[j];
      if (w != 0.0f) {
        pu += w * node(0, a + i - 1, b + j - 1);
        pv += w * node(1, a + i - 1, b + j - 1);
      }
    }
}

// Four consecutive pixels of row y from pixel x on (zero outside the image),
// with aligned word loads realigned by alignbyte.
template <typename T, bool kAligned = false>
__device__ __forceinline__ void load4(const uint8_t* img, int64_t pitch, int H, int rowbytes, int y, int x,
                                      float (&v)[4]) {
  // rows outside the image read row 0 or H-1 and are zeroed afterwards
  const uint32_t rowok = (unsigned)y < (unsigned)H ? 0xffffffffu : 0u;
  const uint8_t* row = img + (int64_t)min(max(y, 0), H - 1) * pitch;
  if constexpr (sizeof(T) == 1 && kAligned) {
    const uint32_t w = masked_word(row, rowbytes, x) & rowok;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (float)((w >> (8 * k)) & 0xffu);
  } else if constexpr (sizeof(T) == 2 && kAligned) {
    const uint32_t lo = masked_word(row, rowbytes, 2 * x) & rowok, hi = masked_word(row, rowbytes, 2 * x + 4) & rowok;
    v[0] = (float)(lo & 0xffffu);
    v[1] = (float)(lo >> 16);
    v[2] = (float)(hi & 0xffffu);
    v[3] = (float)(hi >> 16);
  } else if constexpr (sizeof(T) == 1) {
    const int xb = x, xa = xb & ~3, sh = xb & 3;
    uint32_t w = __builtin_amdgcn_alignbyte(masked_word(row, rowbytes, xa + 4), masked_word(row, rowbytes, xa), sh);
    w &= rowok;
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = (float)((w >> (8 * k)) & 0xffu);
  } else if constexpr (sizeof(T) == 2) {
    const int xb = 2 * x, xa = xb & ~3, sh = xb & 3;
    uint32_t w0 = masked_word(row, rowbytes, xa), w1 = masked_word(row, rowbytes, xa + 4),
             w2 = masked_word(row, rowbytes, xa + 8);
    uint32_t lo = __builtin_amdgcn_alignbyte(w1, w0, sh) & rowok, hi = __builtin_amdgcn_alignbyte(w2, w1, sh) & rowok;
    v[0] = (float)(lo & 0xffffu);
    v[1] = (float)(lo >> 16);
    v[2] = (float)(hi & 0xffffu);
    v[3] = (float)(hi >> 16);
  } else {
    if (y < 0 || y >= H) {
      v[0] = v[1] = v[2] = v[3] = 0.0f;
      return;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) v[k] = pixf<T>(img, pitch, rowbytes / 4, H, y, x + k);
  }
}

// Fit and compose one vector from its coefficient lookup rho(sy, sx).
template <typename RhoFn>
__device__ __forceinline__ void finish_vector(const CorrArgs& g, int pair, int a, int b, int sy, int sx,
                                              bool flat, float pu, float pv, RhoFn rho) {
  const int R = g.R;
  uint8_t fl = flat ? PIV_F_FLAT : 0;
  float c0 = rho(sy, sx);
  float ex = 0.0f, ey = 0.0f;
  bool nc;
  if (!g.fixed && (sx == -R || sx == R)) fl |= PIV_F_BORDER;
  else {
    ex = gauss3(rho(sy, sx - 1), c0, rho(sy, sx + 1), nc);
    if (nc) fl |= PIV_F_NOCURV;
  }
  if (!g.fixed && (sy == -R || sy == R)) fl |= PIV_F_BORDER;
  else {
    ey = gauss3(rho(sy - 1, sx), c0, rho(sy + 1, sx), nc);
    if (nc) fl |= PIV_F_NOCURV;
  }
  if (g.fixed) {
    ex = fminf(fmaxf(ex, -1.0f), 1.0f);
    ey = fminf(fmaxf(ey, -1.0f), 1.0f);
  }
  const int np = g.nx * g.ny, i = a * g.nx + b;
  float* D = g.disp + (int64_t)pair * g.dstride;
  D[i] = pu + (float)sx + ex;
  D[np + i] = pv + (float)sy + ey;
  if (g.peak) g.peak[(int64_t)pair * np + i] = c0;
  g.flags[(int64_t)pair * np + i] = fl;
}

// ---------------------------------------------------------------------------
// Generic: one workgroup per window.  The window and its B' box are staged
// in LDS; a thread takes one shift and one of H parts of the window's rows
// (H = as many parts as fit the workgroup, so that a window with many shifts
// still gives every SIMD several waves), the parts' sums meet in LDS in a
// fixed order, and a thread per shift forms the coefficient.
// ---------------------------------------------------------------------------
constexpr int kGenT = 1024;

template <typename T>
__global__ __launch_bounds__(kGenT) void k_correct_generic(CorrArgs g) {
  extern __shared__ float s_mem[];
  __shared__ float s_red[kGenT], s_red2[kGenT];
  __shared__ int s_key[kGenT];
  __shared__ float s_K;
  const int pair = blockIdx.z;
  if (slot_off(g.mask, pair)) return;
  const int a = blockIdx.y, b = blockIdx.x, t = threadIdx.x;
  const int win = g.win, R = g.R, S = 2 * R + 1, BWd = win + 2 * R, S2 = S * S;
  const int H = max(1, min(win, kGenT / S2));   // row parts per shift
  float* sA = s_mem;                 // [win][win]
  float* sB = sA + win * win;        // [BWd][BWd]
  float* sRho = sB + BWd * BWd;      // [S][S]
  float* sPart = sRho + S2;          // [3][H][S2]: P, S, Q of each shift's row parts
  const uint8_t* Ai = g.A + (int64_t)pair * g.stride;
  const uint8_t* Bi = g.B + (int64_t)pair * g.stride;
  const float* Pn = g.pred ? g.pred + (int64_t)pair * 2 * g.nx * g.ny : nullptr;
  const int np = g.nx * g.ny;
  auto node = [&](int c, int y, int x) { return Pn[c * np + y * g.nx + x]; };
  const int h = (win - g.step) / 2, oy = a * g.step - h, ox = b * g.step - h;
  const float sgnA = -0.5f, sgnB = g.central ? 0.5f : 1.0f;
  // fixed-order tree over the workgroup (every thread returns the total)
  auto tree2 = [&](float x, float y, float& sx_, float& sy_) {
    s_red[t] = x;
    s_red2[t] = y;
    __syncthreads();
    for (int o = kGenT / 2; o > 0; o >>= 1) {
      if (t < o) {
        s_red[t] += s_red[t + o];
        s_red2[t] += s_red2[t + o];
      }
      __syncthreads();
    }
    sx_ = s_red[0];
    sy_ = s_red2[0];
    __syncthreads();
  };

  float part = 0.0f;
  for (int idx = t; idx < win * win; idx += kGenT) {
    int y = oy + idx / win, x = ox + idx % win;
    float v;
    if (g.central && Pn) {
      float u, w;
      interp_u((float)x, (float)y, g.nx, g.ny, g.step, node, u, w);
      v = bilin<T>(Ai, g.pitch, g.W, g.H, x + sgnA * u, y + sgnA * w);
    } else {
      v = pixf<T>(Ai, g.pitch, g.W, g.H, y, x);
    }
    sA[idx] = v;
    part += v;
  }
  {
    float tot, unused;
    tree2(part, 0.0f, tot, unused);
    if (t == 0) s_K = rintf(tot / (float)(win * win));
    __syncthreads();
  }
  const float K = s_K;
  for (int idx = t; idx < win * win; idx += kGenT) sA[idx] -= K;
  for (int idx = t; idx < BWd * BWd; idx += kGenT) {
    int y = oy - R + idx / BWd, x = ox - R + idx % BWd;
    float v;
    if (Pn) {
      float u, w;
      interp_u((float)x, (float)y, g.nx, g.ny, g.step, node, u, w);
      v = bilin<T>(Bi, g.pitch, g.W, g.H, x + sgnB * u, y + sgnB * w);
    } else {
      v = pixf<T>(Bi, g.pitch, g.W, g.H, y, x);
    }
    sB[idx] = v - K;
  }
  __syncthreads();
  // A statistics (of A - K)
  float sa, saa;
  {
    float p1 = 0.0f, p2 = 0.0f;
    for (int idx = t; idx < win * win; idx += kGenT) {
      const float v = sA[idx];
      p1 += v;
      p2 += v * v;
    }
    tree2(p1, p2, sa, saa);
  }
  const float n = (float)(win * win);
  const float mA = sa / n;
  const float varA = saa - sa * mA;
  const bool flatA = !(varA > kFlatRel * saa);

  // shift s, row part hp: rows [hp win / H, (hp + 1) win / H) of the window
  for (int item = t; item < S2 * H; item += kGenT) {
    const int hp = item / S2, sidx = item - hp * S2;
    const int sy = sidx / S - R, sx = sidx % S - R;
    float P = 0.0f, Sb = 0.0f, Q = 0.0f;
    if (!g.fixed || sx == 0 || sy == 0) {
      const int r0 = hp * win / H, r1 = (hp + 1) * win / H;
      for (int i = r0; i < r1; ++i) {
        const float* arow = sA + i * win;
        const float* brow = sB + (i + sy + R) * BWd + sx + R;
        // eight pixels' reads in flight together
        int j = 0;
        for (; j + 8 <= win; j += 8) {
          float av[8], bv[8];
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            av[u] = arow[j + u];
            bv[u] = brow[j + u];
          }
#pragma unroll
          for (int u = 0; u < 8; ++u) {
            P += av[u] * bv[u];
            Sb += bv[u];
            Q += bv[u] * bv[u];
          }
        }
        for (; j < win; ++j) {
          const float bv = brow[j];
          P += arow[j] * bv;
          Sb += bv;
          Q += bv * bv;
        }
      }
    }
    sPart[(0 * H + hp) * S2 + sidx] = P;
    sPart[(1 * H + hp) * S2 + sidx] = Sb;
    sPart[(2 * H + hp) * S2 + sidx] = Q;
  }
  __syncthreads();

  float best = -2.0f;
  int bkey = 1 << 30, nflat = 0;
  for (int sidx = t; sidx < S2; sidx += kGenT) {
    const int sy = sidx / S - R, sx = sidx % S - R;
    float r = 0.0f;
    const bool used = !g.fixed || sx == 0 || sy == 0;
    if (used) {
      float P = 0.0f, Sb = 0.0f, Q = 0.0f;
      for (int hp = 0; hp < H; ++hp) {
        P += sPart[(0 * H + hp) * S2 + sidx];
        Sb += sPart[(1 * H + hp) * S2 + sidx];
        Q += sPart[(2 * H + hp) * S2 + sidx];
      }
      float num = P - mA * Sb;
      float varB = Q - Sb * Sb / n;
      bool flat = flatA || !(varB > kFlatRel * Q);
      r = flat ? 0.0f : num * rsqrtf(varA * varB);
      nflat += flat;
      int key = tie_key(sy, sx);
      if (!g.fixed && better(r, key, best, bkey)) {
        best = r;
        bkey = key;
      }
    }
    sRho[sidx] = r;
  }
  s_red[t] = best;
  s_key[t] = bkey;
  __syncthreads();
  for (int o = kGenT / 2; o > 0; o >>= 1) {
    if (t < o && better(s_red[t + o], s_key[t + o], s_red[t], s_key[t])) {
      s_red[t] = s_red[t + o];
      s_key[t] = s_key[t + o];
    }
    __syncthreads();
  }
  // count flat shifts
  __shared__ int s_nflat;
  if (t == 0) s_nflat = 0;
  __syncthreads();
  if (nflat) atomicAdd(&s_nflat, nflat);
  __syncthreads();
  if (t == 0) {
    int sy = 0, sx = 0;
    if (!g.fixed) {
      int k = s_key[0];
      sx = (k & 63) - 32;
      sy = ((k >> 6) & 63) - 32;
    }
    // window mean of the interpolated predictor: per-axis node weights
    float pu = 0.0f, pv = 0.0f;
    if (Pn) {
      float* wx = sA;                     // A tile is no longer needed
      float* wy = sA + (win / g.step + 3);
      const float c = 0.5f * (float)(g.step - 1);
      int bxl, byl;
      {
        float tx = fminf(fmaxf(((float)ox - c) / g.step, 0.0f), (float)(g.nx - 1));
        float ty = fminf(fmaxf(((float)oy - c) / g.step, 0.0f), (float)(g.ny - 1));
        bxl = min((int)tx, max(g.nx - 2, 0));
        byl = min((int)ty, max(g.ny - 2, 0));
      }
      const int nw = win / g.step + 3;
      for (int q = 0; q < 2 * nw; ++q) sA[q] = 0.0f;
      for (int j = 0; j < win; ++j) {
        float tx = fminf(fmaxf(((float)(ox + j) - c) / g.step, 0.0f), (float)(g.nx - 1));
        int bx = min((int)tx, max(g.nx - 2, 0));
        float fx = tx - (float)bx;
        wx[bx - bxl] += 1.0f - fx;
        wx[(g.nx > 1 ? bx + 1 : bx) - bxl] += fx;
        float ty = fminf(fmaxf(((float)(oy + j) - c) / g.step, 0.0f), (float)(g.ny - 1));
        int by = min((int)ty, max(g.ny - 2, 0));
        float fy = ty - (float)by;
        wy[by - byl] += 1.0f - fy;
        wy[(g.ny > 1 ? by + 1 : by) - byl] += fy;
      }
      for (int i = 0; i < nw; ++i)
        for (int j = 0; j < nw; ++j) {
          float w = wy[i] * wx[j];
          if (w != 0.0f) {
            pu += w * node(0, byl + i, bxl + j);
            pv += w * node(1, byl + i, bxl + j);
          }
        }
      const float inv = 1.0f / ((float)win * (float)win);
      pu *= inv;
      pv *= inv;
    }
    const int nev = g.fixed ? 5 : S * S;
    auto rho = [&](int y, int x) { return sRho[(y + R) * S + x + R]; };
    finish_vector(g, pair, a, b, sy, sx, s_nflat == nev, pu, pv, rho);
  }
}

// ---------------------------------------------------------------------------
// Tiled, cell-shared (win = 2 step).
// ---------------------------------------------------------------------------
template <int STEP, int R, int SYG, int TW, int TH>
struct TileCfg {
  static constexpr int CW = TW + 1, CH = TH + 1, NC = CW * CH;
  static constexpr int NSY = 2 * R + 1, NS = NSY * NSY, NG = NSY / SYG;
  static constexpr int AW = CW * STEP, AH = CH * STEP;
  static constexpr int BW = AW + 2 * R, BH = AH + 2 * R;
  static constexpr int AP = AW + 4;   // LDS row pitches (floats)
  static constexpr int BP = (BW + 3) / 4 * 4 + 4;
  static constexpr int NNX = BW / STEP + 4, NNY = BH / STEP + 3;
  static constexpr int IN_FLOATS = AH * AP + BH * BP;
  // one shift band (SYG rows of NSY shifts) is split over the window's four
  // threads, PER shifts each, stored SLOTW apart (16-byte aligned chunks)
  static constexpr int NBS = SYG * NSY;
  static constexpr int PER = (NBS + 3) / 4;
  static constexpr int SLOTW = (PER + 3) / 4 * 4;
  static constexpr int BANDP = 4 * SLOTW;
  static constexpr int CSTR = BANDP + 4;                  // cell stride (spreads LDS banks)
  static constexpr int WSTR = NG * BANDP + 4;             // window stride of the coefficients
  static constexpr int XBUF = 3 * NC * CSTR;              // P, S, Q of one band, all cells
  static constexpr int RES_FLOATS = 2 * XBUF;             // two band buffers
  // room for the raw source tile of B behind the A and B' tiles: what the
  // result arrays leave free, else what fits a 71 KiB union (two
  // workgroups per CU with the small arrays), at least 16 KiB
  static constexpr int UNION_CAP = 71 * 1024 / 4;
  static constexpr int RAW_FIT = UNION_CAP - IN_FLOATS > 4096 ? UNION_CAP - IN_FLOATS : 4096;
  static constexpr int RAW_WORDS = RES_FLOATS - IN_FLOATS > RAW_FIT ? RES_FLOATS - IN_FLOATS : RAW_FIT;
  static constexpr int UNION = IN_FLOATS + RAW_WORDS > RES_FLOATS ? IN_FLOATS + RAW_WORDS : RES_FLOATS;
  static constexpr int NWIN = TW * TH;
  static_assert(NSY % SYG == 0, "shift rows must split evenly");
  static_assert(NWIN * WSTR <= XBUF, "window coefficients fit one band buffer");
  static_assert(STEP % 2 == 0, "50% overlap needs an even step");
  static_assert(STEP >= 4, "a group of four pixels spans at most two node columns");
};

template <typename T, int STEP, int R, int SYG, int TW, int TH, int NT>
__global__ __launch_bounds__(NT) void k_correct_tiled(CorrArgs g) {
  using C = TileCfg<STEP, R, SYG, TW, TH>;
  // workers: whole cell rows per wave (lane = row-in-wave * CW + column),
  // so that a cell's right-hand neighbour is the next lane of its wave
  constexpr int RPW = 64 / C::CW;
  static_assert((NT / 64) * RPW >= C::NG * C::CH, "one thread per (cell, shift band)");
  static_assert(4 * C::NWIN <= NT, "four threads per window");
  __shared__ __align__(16) float s_u[C::UNION];
  __shared__ float s_node[2][C::NNY][C::NNX];
  __shared__ float s_wsum[C::NWIN], s_wsq[C::NWIN];
  __shared__ float s_red[NT / 64];
  __shared__ float s_rng[NT / 64][5];
  __shared__ int s_rb[C::BH], s_cb[C::BW];
  __shared__ float s_rf[C::BH], s_cf[C::BW];
  __shared__ int s_tkey[C::NG * 4 * C::PER];   // tie key of (band, thread, shift), or kKeyNone

  const WgIdx wg = xcd_order();
  const int pair = wg.z;
  if (slot_off(g.mask, pair)) return;
  const int t = threadIdx.x;
  const int a0 = wg.y * TH, b0 = wg.x * TW;
  constexpr int h = STEP / 2;
  const int y0 = a0 * STEP - h, x0 = b0 * STEP - h;      // A tile origin
  const int yb = y0 - R, xb = x0 - R;                    // B' tile origin
  const uint8_t* Ai = g.A + (int64_t)pair * g.stride;
  const uint8_t* Bi = g.B + (int64_t)pair * g.stride;
  const int np = g.nx * g.ny;
  const float* Pn = g.pred ? g.pred + (int64_t)pair * 2 * np : nullptr;
  float* sA = s_u;                   // [AH][AP]
  float* sB = s_u + C::AH * C::AP;   // [BH][BP]

  constexpr int AQ = C::AW / 4;
  constexpr int NA = (C::AH * AQ + NT - 1) / NT;
  // plain A tile: when the tile origin is 4-byte aligned (STEP/2 pixels
  // are), its words are read here, all in flight together ahead of the node
  // cache, and unpacked after the first barrier
  constexpr bool kAlignedA = ((STEP / 2) * (int)sizeof(T)) % 4 == 0;
  constexpr int NWA = kAlignedA ? (int)sizeof(T) : 1;
  const bool plainA = !(g.central && Pn);
  uint32_t aw[NA][NWA], ak[NA][NWA];   // raw words and their keep masks
  if (kAlignedA && plainA) {
    const int rowbytes = g.W * (int)sizeof(T);
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int idx0 = t + i * NT;
      const bool in = idx0 < C::AH * AQ;
      const int idx = in ? idx0 : 0;
      const int r = idx / AQ, q = 4 * (idx - (idx / AQ) * AQ);
      const int y = y0 + r;
      const uint32_t ok = (in && (unsigned)y < (unsigned)g.H) ? 0xffffffffu : 0u;
      const uint8_t* row = Ai + (int64_t)min(max(y, 0), g.H - 1) * g.pitch;
#pragma unroll
      for (int k = 0; k < NWA; ++k) {
        // masked_word, with the mask applied after the first barrier so that
        // nothing waits for these reads before the node cache is requested
        const int xa = (x0 + q) * (int)sizeof(T) + 4 * k;
        aw[i][k] = *reinterpret_cast<const uint32_t*>(row + min(max(xa, 0), (rowbytes - 1) & ~3));
        const int valid = rowbytes - xa;
        const uint32_t part = (1u << (8 * (valid & 3))) - 1u;
        ak[i][k] = ((xa < 0 || valid <= 0) ? 0u : (valid >= 4 ? 0xffffffffu : part)) & ok;
      }
    }
  }

  // tie keys of the shifts each window thread will see, per band
  for (int i = t; i < C::NG * 4 * C::PER; i += NT) {
    const int bnd = i / (4 * C::PER), o = i - bnd * 4 * C::PER;   // o = thread * PER + shift
    int key = kKeyNone;
    if (o < C::NBS) {
      const int sy = bnd * SYG + o / C::NSY - R, sx = o % C::NSY - R;
      if (!g.fixed || sx == 0 || sy == 0) key = tie_key(sy, sx);
    }
    s_tkey[i] = key;
  }
  // node cache covering the B' tile, and the range of the predictor over it
  // (every interpolated displacement is a convex combination of cached nodes)
  const float cen = 0.5f * (float)(STEP - 1);
  const int nlo_y = max(0, (int)floorf(((float)yb - cen) / STEP));
  const int nlo_x = max(0, (int)floorf(((float)xb - cen) / STEP));
  float umin = 0.0f, umax = 0.0f, vmin = 0.0f, vmax = 0.0f, bad = 0.0f;
  if (Pn) {
    umin = vmin = 3.0e38f;
    umax = vmax = -3.0e38f;
    for (int idx = t; idx < C::NNY * C::NNX; idx += NT) {
      int r = idx / C::NNX, q = idx % C::NNX;
      int ny_ = min(nlo_y + r, g.ny - 1), nx_ = min(nlo_x + q, g.nx - 1);
      float u = Pn[ny_ * g.nx + nx_], v = Pn[np + ny_ * g.nx + nx_];
      s_node[0][r][q] = u;
      s_node[1][r][q] = v;
      umin = fminf(umin, u);
      umax = fmaxf(umax, u);
      vmin = fminf(vmin, v);
      vmax = fmaxf(vmax, v);
      if (!(fabsf(u) < 1.0e6f && fabsf(v) < 1.0e6f)) bad = 1.0f;   // also NaN
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      bad = fmaxf(bad, __shfl_xor(bad, o));
      umin = fminf(umin, __shfl_xor(umin, o));
      umax = fmaxf(umax, __shfl_xor(umax, o));
      vmin = fminf(vmin, __shfl_xor(vmin, o));
      vmax = fmaxf(vmax, __shfl_xor(vmax, o));
    }
    if ((t & 63) == 0) {
      s_rng[t >> 6][0] = umin;
      s_rng[t >> 6][1] = umax;
      s_rng[t >> 6][2] = vmin;
      s_rng[t >> 6][3] = vmax;
      s_rng[t >> 6][4] = bad;
    }
  }
  // per-row / per-column interpolation tables of the B' tile (the A tile is
  // the same grid shifted by R): base node (cache index) and fraction, the
  // same arithmetic as interp_u
  for (int i = t; i < C::BH + C::BW; i += NT) {
    const bool row = i < C::BH;
    const int p = row ? yb + i : xb + (i - C::BH);
    const int n = row ? g.ny : g.nx;
    float tt = fminf(fmaxf(((float)p - cen) / (float)STEP, 0.0f), (float)(n - 1));
    int bb = min((int)tt, max(n - 2, 0));
    float ff = tt - (float)bb;
    if (row) { s_rb[i] = bb - nlo_y; s_rf[i] = ff; }
    else { s_cb[i - C::BH] = bb - nlo_x; s_cf[i - C::BH] = ff; }
  }
  __syncthreads();
  if (Pn) {
    umin = s_rng[0][0]; umax = s_rng[0][1]; vmin = s_rng[0][2]; vmax = s_rng[0][3]; bad = s_rng[0][4];
#pragma unroll
    for (int i = 1; i < NT / 64; ++i) {
      bad = fmaxf(bad, s_rng[i][4]);
      umin = fminf(umin, s_rng[i][0]);
      umax = fmaxf(umax, s_rng[i][1]);
      vmin = fminf(vmin, s_rng[i][2]);
      vmax = fmaxf(vmax, s_rng[i][3]);
    }
  }
  auto node = [&](int c, int y, int x) { return s_node[c][y - nlo_y][x - nlo_x]; };
  auto interp_tab = [&](int r, int q, float& u, float& v) {
    const int rb = s_rb[r], cb = s_cb[q];
    const float fy = s_rf[r], fx = s_cf[q];
    u = (1.0f - fy) * ((1.0f - fx) * s_node[0][rb][cb] + fx * s_node[0][rb][cb + 1]) +
        fy * ((1.0f - fx) * s_node[0][rb + 1][cb] + fx * s_node[0][rb + 1][cb + 1]);
    v = (1.0f - fy) * ((1.0f - fx) * s_node[1][rb][cb] + fx * s_node[1][rb][cb + 1]) +
        fy * ((1.0f - fx) * s_node[1][rb + 1][cb] + fx * s_node[1][rb + 1][cb + 1]);
  };

  // A tile in groups of four pixels (deformed by -u/2 in central mode), held
  // in registers until the tile offset K is known
  float av[NA][4];
#pragma unroll
  for (int i = 0; i < NA; ++i) av[i][0] = av[i][1] = av[i][2] = av[i][3] = 0.0f;
  float part = 0.0f;
  if (plainA) {
    if constexpr (kAlignedA) {
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const uint32_t w0 = aw[i][0] & ak[i][0], w1 = aw[i][NWA - 1] & ak[i][NWA - 1];
        if constexpr (sizeof(T) == 1) {
#pragma unroll
          for (int e = 0; e < 4; ++e) av[i][e] = (float)((w0 >> (8 * e)) & 0xffu);
        } else {
          av[i][0] = (float)(w0 & 0xffffu);
          av[i][1] = (float)(w0 >> 16);
          av[i][2] = (float)(w1 & 0xffffu);
          av[i][3] = (float)(w1 >> 16);
        }
      }
    } else {
      const int rowbytes = g.W * (int)sizeof(T);
#pragma unroll
      for (int i = 0; i < NA; ++i) {
        const int idx0 = t + i * NT;
        const bool in = idx0 < C::AH * AQ;
        const int idx = in ? idx0 : 0;
        const int r = idx / AQ, q = 4 * (idx - (idx / AQ) * AQ);
        float v[4];
        load4<T>(Ai, g.pitch, g.H, rowbytes, y0 + r, x0 + q, v);
#pragma unroll
        for (int e = 0; e < 4; ++e) av[i][e] = in ? v[e] : 0.0f;
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int idx = t + i * NT;
      if (idx < C::AH * AQ) {
        const int r = idx / AQ, q = 4 * (idx - (idx / AQ) * AQ);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float u, w;
          interp_tab(r + R, q + e + R, u, w);
          av[i][e] = bilin<T>(Ai, g.pitch, g.W, g.H, (x0 + q + e) - 0.5f * u, (y0 + r) - 0.5f * w);
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < NA; ++i) part += (av[i][0] + av[i][1]) + (av[i][2] + av[i][3]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o);
  if ((t & 63) == 0) s_red[t >> 6] = part;

  // raw source tile of B for the deformation, when its bounding box fits
  const float sgnB = g.central ? 0.5f : 1.0f;
  const int ix0 = (int)floorf((float)xb + sgnB * umin) - 1;
  const int ix1 = (int)floorf((float)(xb + C::BW - 1) + sgnB * umax) + 2;
  const int iy0 = (int)floorf((float)yb + sgnB * vmin) - 1;
  const int iy1 = (int)floorf((float)(yb + C::BH - 1) + sgnB * vmax) + 2;
  const int xw0 = (ix0 * (int)sizeof(T)) >> 2;
  const int nwords = ((ix1 * (int)sizeof(T) + (int)sizeof(T) - 1) >> 2) - xw0 + 1;
  const int nrows = iy1 - iy0 + 1;
  // (a displacement range that is not finite or wider than a window takes
  // the unstaged path, whose reads are checked one by one)
  const bool sane = bad == 0.0f && (umax - umin) < 64.0f && (vmax - vmin) < 64.0f;
  const bool staged = sane && nwords <= NT && nwords * nrows <= C::RAW_WORDS;
  uint32_t* sraw = reinterpret_cast<uint32_t*>(s_u + C::IN_FLOATS);
  if (staged) {
    // thread -> (word column, first row); rows advance by rstep, U reads in
    // flight per thread
    const int rowbytes = g.W * (int)sizeof(T);
    const int rstep = NT / nwords;
    const int r0 = t / nwords, w = t - r0 * nwords;
    constexpr int U = 8;
    if (r0 < rstep) {
      for (int rb = r0; rb < nrows; rb += U * rstep) {
        uint32_t val[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int y = iy0 + rb + u * rstep;
          const uint32_t ok = (unsigned)y < (unsigned)g.H ? 0xffffffffu : 0u;
          val[u] = masked_word(Bi + (int64_t)min(max(y, 0), g.H - 1) * g.pitch, rowbytes, 4 * (xw0 + w)) & ok;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (rb + u * rstep < nrows) sraw[(rb + u * rstep) * nwords + w] = val[u];
      }
    }
  }
  __syncthreads();
  // the tile offset K (every thread sums the per-wave partials itself)
  float ksum = 0.0f;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) ksum += s_red[i];
  const float K = rintf(ksum / (float)(C::AH * C::AW));
#pragma unroll
  for (int i = 0; i < NA; ++i) {
    const int idx = t + i * NT;
    if (idx < C::AH * AQ) {
      const int r = idx / AQ, q = 4 * (idx - (idx / AQ) * AQ);
      *reinterpret_cast<float4*>(sA + r * C::AP + q) =
          make_float4(av[i][0] - K, av[i][1] - K, av[i][2] - K, av[i][3] - K);
    }
  }
  // deformed B' tile
  if (staged) {
    // groups of four pixels of one row: the node row and its fraction are
    // shared, and the group spans at most two node columns (STEP > 4), so
    // the displacement is interpolated vertically at three node columns and
    // then horizontally per pixel.  The deformed coordinates stay inside the
    // raw box by its construction (a convex combination of cached nodes plus
    // a one-pixel margin); the clamps only keep the padding columns of a
    // ragged last group inside it.
    constexpr int BQ = (C::BW + 3) / 4;
    constexpr int RPI = NT / BQ;              // rows per pass
    // groups never straddle a node-column boundary when the tile origin and
    // the boundaries agree modulo 4
    constexpr bool kUniformCols = (STEP + R) % 4 == 0;
    const uint8_t* rawb = reinterpret_cast<const uint8_t*>(sraw);
    const int rowb = 4 * nwords, xoff = 4 * xw0;
    constexpr int ES = (int)sizeof(T);
    auto rawv = [&](const uint8_t* p) -> float { return (float)*reinterpret_cast<const T*>(p); };
    const int r_t = t / BQ, q = 4 * (t - (t / BQ) * BQ);
    const float fxlo = (float)ix0, fxhi = (float)(ix1 - 1), fylo = (float)iy0, fyhi = (float)(iy1 - 1);
    const int rbase = iy0 * rowb + xoff;
    const bool lane_on = t < RPI * BQ;
    const float xq = (float)(xb + q);
    for (int r = r_t; lane_on && r < C::BH; r += RPI) {
      float uu[4] = {0.0f, 0.0f, 0.0f, 0.0f}, vv[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      if (Pn) {
        const int rb = s_rb[r];
        const float fy = s_rf[r];
        const int cb0 = s_cb[q];
        if constexpr (kUniformCols) {
          const float u0 = s_node[0][rb][cb0] + fy * (s_node[0][rb + 1][cb0] - s_node[0][rb][cb0]);
          const float u1 = s_node[0][rb][cb0 + 1] + fy * (s_node[0][rb + 1][cb0 + 1] - s_node[0][rb][cb0 + 1]);
          const float v0 = s_node[1][rb][cb0] + fy * (s_node[1][rb + 1][cb0] - s_node[1][rb][cb0]);
          const float v1 = s_node[1][rb][cb0 + 1] + fy * (s_node[1][rb + 1][cb0 + 1] - s_node[1][rb][cb0 + 1]);
          const float du = u1 - u0, dv = v1 - v0;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float fx = s_cf[min(q + e, C::BW - 1)];
            uu[e] = u0 + fx * du;
            vv[e] = v0 + fx * dv;
          }
        } else {
          float Vu[3], Vv[3];
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            Vu[j] = s_node[0][rb][cb0 + j] + fy * (s_node[0][rb + 1][cb0 + j] - s_node[0][rb][cb0 + j]);
            Vv[j] = s_node[1][rb][cb0 + j] + fy * (s_node[1][rb + 1][cb0 + j] - s_node[1][rb][cb0 + j]);
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const int qq = min(q + e, C::BW - 1);
            const bool nxt = s_cb[qq] != cb0;
            const float fx = s_cf[qq];
            const float ul = nxt ? Vu[1] : Vu[0], ur = nxt ? Vu[2] : Vu[1];
            const float vl = nxt ? Vv[1] : Vv[0], vr = nxt ? Vv[2] : Vv[1];
            uu[e] = ul + fx * (ur - ul);
            vv[e] = vl + fx * (vr - vl);
          }
        }
      }
      const float yr = (float)(yb + r);
      float out[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float qx = (xq + (float)e) + sgnB * uu[e], qy = yr + sgnB * vv[e];
        const float fx0 = floorf(qx), fy0 = floorf(qy);
        const float fx = qx - fx0, fy = qy - fy0;
        const int ix = (int)__builtin_amdgcn_fmed3f(fx0, fxlo, fxhi);
        const int iy = (int)__builtin_amdgcn_fmed3f(fy0, fylo, fyhi);
        const uint8_t* p0 = rawb + (iy * rowb + ix * ES) - rbase;
        const float p00 = rawv(p0), p01 = rawv(p0 + ES), p10 = rawv(p0 + rowb), p11 = rawv(p0 + rowb + ES);
        const float top = p00 + fx * (p01 - p00), bot = p10 + fx * (p11 - p10);
        out[e] = (top + fy * (bot - top)) - K;
      }
      *reinterpret_cast<float4*>(sB + r * C::BP + q) = make_float4(out[0], out[1], out[2], out[3]);
    }
  } else {
    for (int idx = t; idx < C::BH * C::BW; idx += NT) {
      int r = idx / C::BW, q = idx % C::BW;
      int y = yb + r, x = xb + q;
      float v;
      if (Pn) {
        float u, w;
        interp_tab(r, q, u, w);
        v = bilin<T>(Bi, g.pitch, g.W, g.H, x + sgnB * u, y + sgnB * w);
      } else {
        v = pixf<T>(Bi, g.pitch, g.W, g.H, y, x);
      }
      sB[r * C::BP + q] = v - K;
    }
  }
  __syncthreads();
  // A window statistics: four threads per window, four rows... of 2 STEP each
  if (t < 4 * C::NWIN) {
    int w = t >> 2, p = t & 3;
    int wi = w / TW, wj = w % TW;
    float s = 0.0f, ss = 0.0f;
    for (int r = p; r < 2 * STEP; r += 4) {
      const float* row = sA + (wi * STEP + r) * C::AP + wj * STEP;
#pragma unroll
      for (int q = 0; q < 2 * STEP; ++q) {
        float v = row[q];
        s += v;
        ss += v * v;
      }
    }
    s += __shfl_xor(s, 1);
    ss += __shfl_xor(ss, 1);
    s += __shfl_xor(s, 2);
    ss += __shfl_xor(ss, 2);
    if (p == 0) {
      s_wsum[w] = s;
      s_wsq[w] = ss;
    }
  }

  // ---- per cell and shift band: P = sum (A-K)(B'-K), S = sum (B'-K), Q = sum (B'-K)^2
  constexpr int BRW = STEP + 2 * R;   // B' columns one cell row needs
  float Pacc[SYG][C::NSY];
  float Sacc[SYG][C::NSY], Qacc[SYG][C::NSY];
  const int lrow = (t & 63) / C::CW;
  const int cj = (t & 63) - lrow * C::CW;
  const int grow = (t >> 6) * RPW + lrow;                // over (band, cell row)
  const bool worker = lrow < RPW && grow < C::NG * C::CH;
  const int grp = grow / C::CH, ci = grow - grp * C::CH;
  const int cell = ci * C::CW + cj;
  if (worker) {
#pragma unroll
    for (int k = 0; k < SYG; ++k)
#pragma unroll
      for (int j = 0; j < C::NSY; ++j) Pacc[k][j] = 0.0f;
    float cs[BRW], cq[BRW];
#pragma unroll
    for (int x = 0; x < BRW; ++x) cs[x] = cq[x] = 0.0f;
    const float* abase = sA + (ci * STEP) * C::AP + cj * STEP;
    const float* bbase = sB + (ci * STEP + grp * SYG) * C::BP + cj * STEP;
    float br[SYG][BRW];
    // rows of the band for py = 0
#pragma unroll
    for (int k = 0; k < SYG; ++k)
#pragma unroll
      for (int x = 0; x < BRW; ++x) br[k][x] = bbase[k * C::BP + x];
#pragma unroll
    for (int py = 0; py < STEP; ++py) {
      float ar[STEP];
#pragma unroll
      for (int x = 0; x < STEP; ++x) ar[x] = abase[py * C::AP + x];
#pragma unroll
      for (int x = 0; x < BRW; ++x) {
        cs[x] += br[0][x];
        cq[x] += br[0][x] * br[0][x];
      }
#pragma unroll
      for (int k = 0; k < SYG; ++k)
#pragma unroll
        for (int j = 0; j < C::NSY; ++j) {
          float s = Pacc[k][j];
#pragma unroll
          for (int x = 0; x < STEP; ++x) s += ar[x] * br[k][x + j];
          Pacc[k][j] = s;
        }
      if (py + 1 < STEP) {
        // slide the band one row down
#pragma unroll
        for (int k = 0; k + 1 < SYG; ++k)
#pragma unroll
          for (int x = 0; x < BRW; ++x) br[k][x] = br[k + 1][x];
#pragma unroll
        for (int x = 0; x < BRW; ++x) br[SYG - 1][x] = bbase[(py + SYG) * C::BP + x];
      }
    }
    // column sums for the band's first row -> window-free cell box sums
#pragma unroll
    for (int k = 0; k < SYG; ++k) {
      if (k > 0) {
        const float* rin = bbase + (STEP + k - 1) * C::BP;
        const float* rout = bbase + (k - 1) * C::BP;
#pragma unroll
        for (int x = 0; x < BRW; ++x) {
          float vi = rin[x], vo = rout[x];
          cs[x] += vi - vo;
          cq[x] += vi * vi - vo * vo;
        }
      }
      float s = 0.0f, q = 0.0f;
#pragma unroll
      for (int x = 0; x < STEP; ++x) {
        s += cs[x];
        q += cq[x];
      }
      Sacc[k][0] = s;
      Qacc[k][0] = q;
#pragma unroll
      for (int j = 1; j < C::NSY; ++j) {
        s += cs[j + STEP - 1] - cs[j - 1];
        q += cq[j + STEP - 1] - cq[j - 1];
        Sacc[k][j] = s;
        Qacc[k][j] = q;
      }
    }
  }
  __syncthreads();   // everyone is done with the A and B' tiles
  // ---- windows, one shift band at a time.  Band b (shift rows
  // [b SYG, (b+1) SYG)) of every cell goes to LDS buffer X[b & 1] as three
  // arrays [cell][CSTR]; the window's four threads take PER consecutive
  // shifts each, stored at p*SLOTW so that every thread reads aligned
  // 16-byte chunks.  While band b is read, band b+1 is written to the other
  // buffer.
  constexpr int PER = C::PER, SLOTW = C::SLOTW, BANDP = C::BANDP, NB = C::NBS;
  constexpr int XB = C::XBUF, CSTR = C::CSTR, WSTR = C::WSTR;
  const int w = t >> 2, p = t & 3;
  const bool wact = t < 4 * C::NWIN;
  const int wi = w / TW, wj = w - (w / TW) * TW;
  const int c00 = wi * C::CW + wj, c10 = c00 + C::CW;
  // a cell plus its right-hand neighbour (the next lane: wave_shl:1 DPP);
  // the sum is garbage only in the last column, which no window uses
  auto hpair = [](float x) {
    return x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130, 0xF, 0xF, false));
  };
  auto write_band = [&](float* X) {
    // slot o of the band (row o / NSY, column o % NSY) sits at
    // (o / PER) * SLOTW + o % PER; what is stored is the sum over the cell
    // and its right-hand neighbour
#pragma unroll
    for (int v4 = 0; v4 < BANDP / 4; ++v4) {
      float p4[4], s4[4], q4[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int pos = 4 * v4 + e, th = pos / SLOTW, i = pos % SLOTW;
        const int o = th * PER + i;
        const bool real = i < PER && o < NB;
        const int k = real ? o / C::NSY : 0, j = real ? o % C::NSY : 0;
        p4[e] = real ? hpair(Pacc[k][j]) : 0.0f;
        s4[e] = real ? hpair(Sacc[k][j]) : 0.0f;
        q4[e] = real ? hpair(Qacc[k][j]) : 1.0f;
      }
      reinterpret_cast<float4*>(X + cell * CSTR)[v4] = make_float4(p4[0], p4[1], p4[2], p4[3]);
      reinterpret_cast<float4*>(X + XB / 3 + cell * CSTR)[v4] = make_float4(s4[0], s4[1], s4[2], s4[3]);
      reinterpret_cast<float4*>(X + 2 * (XB / 3) + cell * CSTR)[v4] = make_float4(q4[0], q4[1], q4[2], q4[3]);
    }
  };
  float* const X0 = s_u;
  float* const X1 = s_u + XB;
  if (worker && grp == 0) write_band(X0);
  __syncthreads();

  float rho[C::NG][PER];
  float best = -2.0f;
  int bkey = 1 << 30, nflat = 0;
  const float n = (float)(4 * STEP * STEP);
  float mA = 0.0f, varA = 0.0f;
  bool flatA = true;
  if (wact) {
    const float sa = s_wsum[w], saa = s_wsq[w];
    mA = sa / n;
    varA = saa - sa * mA;
    flatA = !(varA > kFlatRel * saa);
  }
#pragma unroll
  for (int bnd = 0; bnd < C::NG; ++bnd) {
    const float* X = (bnd & 1) ? X1 : X0;
    if (bnd + 1 < C::NG && worker && grp == bnd + 1) write_band((bnd & 1) ? X0 : X1);
#pragma unroll
    for (int i = 0; i < PER; ++i) rho[bnd][i] = 0.0f;
    if (wact) {
      float Pv[SLOTW], Sv[SLOTW], Qv[SLOTW];
#pragma unroll
      for (int v4 = 0; v4 < SLOTW / 4; ++v4) {
        auto ld = [&](int arr, int c) {
          return reinterpret_cast<const float4*>(X + arr * (XB / 3) + c * CSTR + p * SLOTW)[v4];
        };
        // stored values already hold (cell + right neighbour): the window
        // is its top pair plus its bottom pair
        const float4 P0 = ld(0, c00), P2 = ld(0, c10);
        const float4 S0 = ld(1, c00), S2 = ld(1, c10);
        const float4 Q0 = ld(2, c00), Q2 = ld(2, c10);
        Pv[4 * v4 + 0] = P0.x + P2.x;
        Pv[4 * v4 + 1] = P0.y + P2.y;
        Pv[4 * v4 + 2] = P0.z + P2.z;
        Pv[4 * v4 + 3] = P0.w + P2.w;
        Sv[4 * v4 + 0] = S0.x + S2.x;
        Sv[4 * v4 + 1] = S0.y + S2.y;
        Sv[4 * v4 + 2] = S0.z + S2.z;
        Sv[4 * v4 + 3] = S0.w + S2.w;
        Qv[4 * v4 + 0] = Q0.x + Q2.x;
        Qv[4 * v4 + 1] = Q0.y + Q2.y;
        Qv[4 * v4 + 2] = Q0.z + Q2.z;
        Qv[4 * v4 + 3] = Q0.w + Q2.w;
      }
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int key = s_tkey[(bnd * 4 + p) * PER + i];   // kKeyNone: not a used shift
        float num = Pv[i] - mA * Sv[i];
        float varB = Qv[i] - Sv[i] * Sv[i] / n;
        bool flat = flatA || !(varB > kFlatRel * Qv[i]);
        float r = flat ? 0.0f : num * rsqrtf(varA * varB);
        if (key != kKeyNone) {
          nflat += flat;
          if (!g.fixed && better(r, key, best, bkey)) {
            best = r;
            bkey = key;
          }
        }
        rho[bnd][i] = r;
      }
    }
    __syncthreads();
  }
  // reduce over the window's four lanes
#pragma unroll
  for (int o = 1; o <= 2; o <<= 1) {
    float ob = __shfl_xor(best, o);
    int ok = __shfl_xor(bkey, o);
    nflat += __shfl_xor(nflat, o);
    if (better(ob, ok, best, bkey)) {
      best = ob;
      bkey = ok;
    }
  }
  // coefficients of the window for the fit, in the buffer no round reads
  // any more: [window][band][thread][SLOTW], windows WSTR apart
  float* const rhoW = (C::NG & 1) ? X1 : X0;
  if (wact) {
#pragma unroll
    for (int bnd = 0; bnd < C::NG; ++bnd) {
      float* d = rhoW + w * WSTR + bnd * BANDP + p * SLOTW;
#pragma unroll
      for (int i = 0; i < PER; ++i) d[i] = rho[bnd][i];
    }
  }
  __syncthreads();
  if (wact && p == 0) {
    const int a = a0 + wi, b = b0 + wj;
    if (a < g.ny && b < g.nx) {
      int sy = 0, sx = 0;
      if (!g.fixed) {
        sx = (bkey & 63) - 32;
        sy = ((bkey >> 6) & 63) - 32;
      }
      const float* rr = rhoW + w * WSTR;
      auto rhof = [&](int y, int x) {
        const int yi = y + R, bnd = yi / SYG;
        const int o = (yi - bnd * SYG) * C::NSY + x + R;
        return rr[bnd * BANDP + (o / PER) * SLOTW + o % PER];
      };
      float pu = 0.0f, pv = 0.0f;
      if (Pn) window_mean_half_overlap(a, b, g.nx, g.ny, node, pu, pv);
      finish_vector(g, pair, a, b, sy, sx, nflat == (g.fixed ? 5 : C::NS), pu, pv, rhof);
    }
  }
}

// ---------------------------------------------------------------------------
// Band per wave (win = 2 step, frames deformed by the whole predictor): a
// workgroup owns TW x TH windows whose (TW+1)(TH+1) <= 64 cells map one to a
// lane, and wave g correlates every cell with shift band g (SYG rows of
// shifts).  Window sums are pair sums of lanes, the right-hand cell by DPP
// and the cell below by a lane permute, so that after the products the only
// LDS traffic is one coefficient per window and shift.  The A cell stays in
// registers as packed pixels.  Small LDS and register footprints give four
// workgroups per compute unit.
// ---------------------------------------------------------------------------
template <int STEP, int R, int SYG, int TW, int TH>
struct BandCfg {
  static constexpr int CW = TW + 1, CH = TH + 1, NC = CW * CH;
  static constexpr int NSY = 2 * R + 1, NS = NSY * NSY, NG = NSY / SYG;
  static constexpr int AW = CW * STEP, AH = CH * STEP;
  static constexpr int BW = AW + 2 * R, BH = AH + 2 * R;
  static constexpr int BP = (BW + 3) / 4 * 4 + 4;   // B' row pitch (floats)
  static constexpr int NNX = BW / STEP + 4, NNY = BH / STEP + 3;
  static constexpr int NWIN = TW * TH;
  // union after the B' tile: raw source box + interpolation tables while the
  // tile is deformed, then coefficients [window][shift] and the per-band
  // peaks [band][window] (value, key << 1 | all shifts flat)
  static constexpr int BW4 = (BW + 3) / 4 * 4;            // B' columns written (whole groups)
  static constexpr int TAB_WORDS = 2 * (BH + BW4);
  static constexpr int RES_WORDS = NWIN * NS + 2 * NG * NWIN;
  // raw source box of B (words): at step 8 a 3888-word box; at step 12 room
  // for a predictor range of 16 px across the tile (u16 rows)
  static constexpr int RAW_WORDS = STEP == 8 ? 3888 : ((BW + 19) * 2 / 4 + 2) * (BH + 19);
  static constexpr int UNION = RAW_WORDS + TAB_WORDS > RES_WORDS ? RAW_WORDS + TAB_WORDS : RES_WORDS;
  static_assert(NC <= 64, "a cell per lane");
  static_assert(NSY % SYG == 0, "shift rows must split evenly");
  static_assert(STEP % 2 == 0 && STEP > 4, "50% overlap; a group of four pixels spans two node columns");
};

template <typename T, int STEP, int R, int SYG, int TW, int TH>
__global__ __launch_bounds__(64 * ((2 * R + 1) / SYG)) __attribute__((amdgpu_waves_per_eu(STEP == 8 ? 3 : 2)))
void k_correct_bands(CorrArgs g) {
  using C = BandCfg<STEP, R, SYG, TW, TH>;
  constexpr int NT = 64 * C::NG;
  constexpr int ES = (int)sizeof(T);
  constexpr int NWR = STEP * ES / 4;   // words per cell row
  static_assert(((STEP / 2) * ES) % 4 == 0 && (STEP * ES) % 4 == 0, "cell rows are whole aligned words");
  __shared__ __align__(16) float sB[C::BH * C::BP];
  __shared__ __align__(16) float s_un[C::UNION];
  __shared__ float s_node[2][C::NNY][C::NNX];
  __shared__ float s_asum[2][ES == 1 ? 1 : C::NG][64];   // u16 cell sums, per wave

  const WgIdx wg = xcd_order();
  const int pair = wg.z;
  if (slot_off(g.mask, pair)) return;
  const int t = threadIdx.x, lane = t & 63;
  const int band = __builtin_amdgcn_readfirstlane(t >> 6);
  const int a0 = wg.y * TH, b0 = wg.x * TW;
  const int y0 = a0 * STEP - STEP / 2, x0 = b0 * STEP - STEP / 2;   // A tile origin
  const int yb = y0 - R, xb = x0 - R;                              // B' tile origin
  const uint8_t* Ai = g.A + (int64_t)pair * g.stride;
  const uint8_t* Bi = g.B + (int64_t)pair * g.stride;
  const int np = g.nx * g.ny;
  const float* Pn = g.pred ? g.pred + (int64_t)pair * 2 * np : nullptr;
  const bool cell_ok = lane < C::NC;
  const int ci = cell_ok ? lane / C::CW : 0, cj = cell_ok ? lane - (lane / C::CW) * C::CW : 0;

  // predictor nodes covering the B' tile: every wave reads all of them and
  // takes their range itself (no barrier before the raw box is requested)
  const float cen = 0.5f * (float)(STEP - 1);
  const int nlo_y = max(0, (int)floorf(((float)yb - cen) / STEP));
  const int nlo_x = max(0, (int)floorf(((float)xb - cen) / STEP));
  constexpr int NNODE = C::NNY * C::NNX, NL = (NNODE + 63) / 64;
  float nu[NL], nv[NL];
  if (Pn) {
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int idx = min(lane + 64 * i, NNODE - 1);
      const int r = idx / C::NNX, q = idx - (idx / C::NNX) * C::NNX;
      const int o = __umul24(min(nlo_y + r, g.ny - 1), g.nx) + min(nlo_x + q, g.nx - 1);
      nu[i] = Pn[(unsigned)o];
      nv[i] = Pn[(unsigned)(np + o)];
    }
  }
  // the A cell of this lane as packed pixels (zero outside the image)
  // a frame whose bytes fit 31 bits (pitch below 2^24) is addressed by 32-bit
  // offsets from its base, with 24-bit products
  const bool off32 = g.pitch < (1 << 24) && g.pitch * (int64_t)g.H <= 0x7fffffff;
  const unsigned pitch32 = (unsigned)g.pitch;
  uint32_t aw[STEP][NWR];
  {
    const int rowbytes = g.W * ES;
    const int xa0 = (x0 + cj * STEP) * ES;
    if (off32 && y0 >= 0 && y0 + C::AH <= g.H && x0 >= 0 && (x0 + C::AW) * ES <= rowbytes) {
      // the whole A tile lies inside the image
      const uint32_t ok = cell_ok ? 0xffffffffu : 0u;
      const unsigned o0 = __umul24((unsigned)(y0 + ci * STEP), pitch32) + (unsigned)xa0;
#pragma unroll
      for (int py = 0; py < STEP; ++py)
#pragma unroll
        for (int k = 0; k < NWR; ++k)
          aw[py][k] = *reinterpret_cast<const uint32_t*>(Ai + (size_t)(o0 + py * pitch32 + 4 * k)) & ok;
    } else {
#pragma unroll
      for (int py = 0; py < STEP; ++py) {
        const int y = y0 + ci * STEP + py;
        const uint32_t ok = (cell_ok && (unsigned)y < (unsigned)g.H) ? 0xffffffffu : 0u;
        const uint8_t* row = Ai + (int64_t)min(max(y, 0), g.H - 1) * g.pitch;
#pragma unroll
        for (int k = 0; k < NWR; ++k) aw[py][k] = masked_word(row, rowbytes, xa0 + 4 * k) & ok;
      }
    }
  }
  // range of the nodes as integer floors: the raw box only needs floor(u)
  // and floor(v) (the tile origin is an integer).  A node that is not finite
  // or not below 100 px marks the tile (range 255), which sends it to the
  // checked path.
  int flu = 0, fhu = 0, flv = 0, fhv = 0;
  if (Pn) {
    float lu = nu[0], hu = nu[0], lv = nv[0], hv = nv[0];
    bool ok = true;
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      lu = fminf(lu, nu[i]);
      hu = fmaxf(hu, nu[i]);
      lv = fminf(lv, nv[i]);
      hv = fmaxf(hv, nv[i]);
      ok = ok && fabsf(nu[i]) < 100.0f && fabsf(nv[i]) < 100.0f;   // false for NaN
    }
    // encoded so that a max serves every bound: 127 - floor(lo) and
    // floor(hi) + 128, two 16-bit fields per word, each reduced on its own
    const uint32_t el_u = ok ? 127 - (int)floorf(lu) : 255, eh_u = ok ? (int)floorf(hu) + 128 : 255;
    const uint32_t el_v = ok ? 127 - (int)floorf(lv) : 255, eh_v = ok ? (int)floorf(hv) + 128 : 255;
    const uint32_t ru = wave_max_pk16((el_u << 16) | eh_u), rv = wave_max_pk16((el_v << 16) | eh_v);
    flu = 127 - (int)(ru >> 16);
    fhu = (int)(ru & 0xffffu) - 128;
    flv = 127 - (int)(rv >> 16);
    fhv = (int)(rv & 0xffffu) - 128;
    if (band == 0) {
#pragma unroll
      for (int i = 0; i < NL; ++i) {
        const int idx = lane + 64 * i;
        if (idx < NNODE) {
          const int r = idx / C::NNX, q = idx - (idx / C::NNX) * C::NNX;
          s_node[0][r][q] = nu[i];
          s_node[1][r][q] = nv[i];
        }
      }
    }
  }

  // raw source box of B for the deformation, when it fits
  const int ix0 = xb + flu - 1;
  const int ix1 = xb + C::BW - 1 + fhu + 2;
  const int iy0 = yb + flv - 1;
  const int iy1 = yb + C::BH - 1 + fhv + 2;
  const int xw0 = (ix0 * ES) >> 2;
  const int nwords = ((ix1 * ES + ES - 1) >> 2) - xw0 + 1;
  const int nrows = iy1 - iy0 + 1;
  // (a displacement range that is marked or wider than a window takes the
  // unstaged path, whose reads are checked one by one)
  const bool sane = fhu - flu < 64 && fhv - flv < 64;
  const bool staged = sane && nwords <= NT && nwords * nrows <= C::RAW_WORDS;
  uint32_t* sraw = reinterpret_cast<uint32_t*>(s_un);
  int* s_rb = reinterpret_cast<int*>(s_un + C::RAW_WORDS);   // per B' row: base node, fraction
  float* s_rf = s_un + C::RAW_WORDS + C::BH;
  int* s_cb = reinterpret_cast<int*>(s_un + C::RAW_WORDS + 2 * C::BH);   // per B' column
  float* s_cf = s_un + C::RAW_WORDS + 2 * C::BH + C::BW4;
  if (staged) {
    // thread -> (word column, first row); U reads in flight per thread
    const int rowbytes = g.W * ES;
    const int rstep = NT / nwords;
    const int r0 = t / nwords, w = t - r0 * nwords;
    // reads in flight per thread: enough for the whole box in one round
    // (about 9 rows per thread at step 8 u8, 33 at step 12 u16)
    constexpr int U = STEP == 8 ? 12 : 36;
    const bool inside = off32 && iy0 >= 0 && iy0 + nrows <= g.H && xw0 >= 0 && 4 * (xw0 + nwords) <= rowbytes;
    if (r0 < rstep) {
      // slots past the box take its last row again (the same word is
      // written twice with the same value), so the stores need no branch
      for (int rb = r0; rb < nrows; rb += U * rstep) {
        uint32_t val[U];
        if (inside) {
          const unsigned col = 4u * (unsigned)(xw0 + w);
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const unsigned y = (unsigned)(iy0 + min(rb + u * rstep, nrows - 1));
            val[u] = *reinterpret_cast<const uint32_t*>(Bi + (size_t)(__umul24(y, pitch32) + col));
          }
        } else {
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int y = iy0 + min(rb + u * rstep, nrows - 1);
            const uint32_t ok = (unsigned)y < (unsigned)g.H ? 0xffffffffu : 0u;
            val[u] = masked_word(Bi + (int64_t)min(max(y, 0), g.H - 1) * g.pitch, rowbytes, 4 * (xw0 + w)) & ok;
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) sraw[min(rb + u * rstep, nrows - 1) * nwords + w] = val[u];
      }
    }
  }
  // interpolation tables of the B' tile (the same arithmetic as interp_u)
  // (columns past BW pad the last group: written to B', never correlated)
  for (int i = t; i < C::BH + C::BW4; i += NT) {
    const bool row = i < C::BH;
    const int p = row ? yb + i : xb + (i - C::BH);
    const int n = row ? g.ny : g.nx;
    float tt = fminf(fmaxf(((float)p - cen) / (float)STEP, 0.0f), (float)(n - 1));
    int bb = min((int)tt, max(n - 2, 0));
    float ff = tt - (float)bb;
    if (row) { s_rb[i] = bb - nlo_y; s_rf[i] = ff; }
    else { s_cb[i - C::BH] = bb - nlo_x; s_cf[i - C::BH] = ff; }
  }
  // the tile offset K: the rounded mean of the A tile (every wave holds all
  // of its cells and reduces them in the same order)
  int isum = 0;
#pragma unroll
  for (int py = 0; py < STEP; ++py)
#pragma unroll
    for (int k = 0; k < NWR; ++k) {
      if constexpr (ES == 1) isum = (int)__builtin_amdgcn_sad_u8(aw[py][k], 0u, (uint32_t)isum);
      else isum = (int)__builtin_amdgcn_sad_u16(aw[py][k], 0u, (uint32_t)isum);
    }
  isum = wave_sum(isum);
  const float K = (float)((isum + C::AH * C::AW / 2) / (C::AH * C::AW));   // (isum >= 0)
  // u16: the cell's sums of (A-K) and (A-K)^2 in FP32, rows dealt to the
  // waves (row py to wave py mod NG); the partial sums meet in LDS
  if constexpr (ES != 1) {
    float s1 = 0.0f, s2 = 0.0f;
#pragma unroll
    for (int py = 0; py < STEP; ++py) {
      if (py % C::NG != band) continue;
#pragma unroll
      for (int x = 0; x < STEP; ++x) {
        const uint32_t wd = aw[py][(x * ES) >> 2];
        const float d = (float)((wd >> (16 * (x & 1))) & 0xffffu) - K;
        s1 += d;
        s2 += d * d;
      }
    }
    s_asum[0][band][lane] = s1;
    s_asum[1][band][lane] = s2;
  }
  __syncthreads();

  // deformed B' tile, in groups of four pixels of one row
  if (staged) {
    constexpr int BQ = (C::BW + 3) / 4;
    constexpr bool kUniformCols = (STEP + R) % 4 == 0;
    const uint8_t* rawb = reinterpret_cast<const uint8_t*>(sraw);
    const int rowb = 4 * nwords, xoff = 4 * xw0;
    auto rawv = [&](const uint8_t* p) -> float { return (float)*reinterpret_cast<const T*>(p); };
    // coordinates relative to the box: every real pixel lands at >= 1 (the
    // box has a one-pixel margin), so truncation is the floor; the clamps
    // only keep the padding columns of a ragged last group inside the box
    const int ixhi = ix1 - 1 - ix0, iyhi = iy1 - 1 - iy0;
    const int xadd = ix0 * ES - xoff;   // byte offset of box column 0 in a staged row
    const uint8_t* rawx = rawb + xadd;  // (folded into the base: one multiply-add per pixel)
    // one group of four pixels; two groups per pass, so that one group's
    // LDS round trips overlap the other's arithmetic
    auto group = [&](int idx) __attribute__((always_inline)) {
      const int r = idx / BQ, q = 4 * (idx - (idx / BQ) * BQ);
      float uu[4] = {0.0f, 0.0f, 0.0f, 0.0f}, vv[4] = {0.0f, 0.0f, 0.0f, 0.0f};
      if (Pn) {
        const int rb = s_rb[r];
        const float fy = s_rf[r];
        const int cb0 = s_cb[q];
        if constexpr (kUniformCols) {
          const float u0 = s_node[0][rb][cb0] + fy * (s_node[0][rb + 1][cb0] - s_node[0][rb][cb0]);
          const float u1 = s_node[0][rb][cb0 + 1] + fy * (s_node[0][rb + 1][cb0 + 1] - s_node[0][rb][cb0 + 1]);
          const float v0 = s_node[1][rb][cb0] + fy * (s_node[1][rb + 1][cb0] - s_node[1][rb][cb0]);
          const float v1 = s_node[1][rb][cb0 + 1] + fy * (s_node[1][rb + 1][cb0 + 1] - s_node[1][rb][cb0 + 1]);
          const float du = u1 - u0, dv = v1 - v0;
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const float fx = s_cf[q + e];
            uu[e] = u0 + fx * du;
            vv[e] = v0 + fx * dv;
          }
        } else {
          float Vu[3], Vv[3];
#pragma unroll
          for (int j = 0; j < 3; ++j) {
            Vu[j] = s_node[0][rb][cb0 + j] + fy * (s_node[0][rb + 1][cb0 + j] - s_node[0][rb][cb0 + j]);
            Vv[j] = s_node[1][rb][cb0 + j] + fy * (s_node[1][rb + 1][cb0 + j] - s_node[1][rb][cb0 + j]);
          }
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            const bool nxt = s_cb[q + e] != cb0;
            const float fx = s_cf[q + e];
            const float ul = nxt ? Vu[1] : Vu[0], ur = nxt ? Vu[2] : Vu[1];
            const float vl = nxt ? Vv[1] : Vv[0], vr = nxt ? Vv[2] : Vv[1];
            uu[e] = ul + fx * (ur - ul);
            vv[e] = vl + fx * (vr - vl);
          }
        }
      }
      const float yr = (float)(yb + r - iy0), xq = (float)(xb + q - ix0);
      float out[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const float qx = (xq + (float)e) + uu[e], qy = yr + vv[e];
        const float fx = __builtin_amdgcn_fractf(qx), fy = __builtin_amdgcn_fractf(qy);
        // Without padding columns the box bounds every coordinate: qx lies in
        // [q + e + 1 - floor(lo) + lo, q + e + 1 - floor(lo) + hi] up to the
        // interpolation's rounding, so floor(qx) is in [0, ixhi] (and its
        // right-hand neighbour in the box), likewise in y; with padding
        // columns the clamps keep their reads inside the box.  (As unsigned,
        // a negative index would clamp to the top as well.)
        unsigned ix = (unsigned)(int)qx, iy = (unsigned)(int)qy;
        if constexpr (C::BW4 != C::BW) {
          ix = min(ix, (unsigned)ixhi);
          iy = min(iy, (unsigned)iyhi);
        }
        const uint8_t* p0 = rawx + (__umul24(iy, (unsigned)rowb) + ix * ES);
        const float p00 = rawv(p0), p01 = rawv(p0 + ES), p10 = rawv(p0 + rowb), p11 = rawv(p0 + rowb + ES);
        const float top = p00 + fx * (p01 - p00), bot = p10 + fx * (p11 - p10);
        out[e] = (top + fy * (bot - top)) - K;
      }
      *reinterpret_cast<float4*>(sB + r * C::BP + q) = make_float4(out[0], out[1], out[2], out[3]);
    };
    constexpr int NGR = C::BH * BQ;
    int idx = t;
    for (; idx + NT < NGR; idx += 2 * NT) {
      group(idx);
      group(idx + NT);
    }
    if (idx < NGR) group(idx);
  } else {
    for (int idx = t; idx < C::BH * C::BW; idx += NT) {
      const int r = idx / C::BW, q = idx - (idx / C::BW) * C::BW;
      const int y = yb + r, x = xb + q;
      float v;
      if (Pn) {
        const int rb = s_rb[r], cb = s_cb[q];
        const float fy = s_rf[r], fx = s_cf[q];
        const float u = (1.0f - fy) * ((1.0f - fx) * s_node[0][rb][cb] + fx * s_node[0][rb][cb + 1]) +
                        fy * ((1.0f - fx) * s_node[0][rb + 1][cb] + fx * s_node[0][rb + 1][cb + 1]);
        const float w = (1.0f - fy) * ((1.0f - fx) * s_node[1][rb][cb] + fx * s_node[1][rb][cb + 1]) +
                        fy * ((1.0f - fx) * s_node[1][rb + 1][cb] + fx * s_node[1][rb + 1][cb + 1]);
        v = bilin<T>(Bi, g.pitch, g.W, g.H, x + u, y + w);
      } else {
        v = pixf<T>(Bi, g.pitch, g.W, g.H, y, x);
      }
      sB[r * C::BP + q] = v - K;
    }
  }
  __syncthreads();

  // ---- this lane's cell against the wave's shift band: P = sum A (B'-K),
  // S = sum (B'-K), Q = sum (B'-K)^2, and the cell's own sum (A-K), (A-K)^2
  // (the covariance sum (A-K)(B'-K) - mean(A-K) S equals P - mean(A) S)
  constexpr int BRW = STEP + 2 * R;   // B' columns one cell row needs
  float Pacc[SYG][C::NSY], Sacc[SYG][C::NSY], Qacc[SYG][C::NSY];
  float sa = 0.0f, saa = 0.0f;
  if constexpr (ES == 1) {
    // the cell's sums of (A-K) and (A-K)^2 from exact integer sums of A, A^2
    uint32_t s1 = 0u, s2 = 0u;
#pragma unroll
    for (int py = 0; py < STEP; ++py)
#pragma unroll
      for (int k = 0; k < NWR; ++k) {
        s1 = __builtin_amdgcn_sad_u8(aw[py][k], 0u, s1);
        s2 = __builtin_amdgcn_udot4(aw[py][k], aw[py][k], s2, false);
      }
    const int Ki = (int)K;
    sa = (float)((int)s1 - STEP * STEP * Ki);
    saa = (float)((int)s2 - 2 * Ki * (int)s1 + STEP * STEP * Ki * Ki);
  } else {
#pragma unroll
    for (int q = 0; q < C::NG; ++q) {
      sa += s_asum[0][q][lane];
      saa += s_asum[1][q][lane];
    }
  }
  // (with large cells the S/Q column sums take a second pass over the band's
  // rows, after the products, so that their registers and the A cell's are
  // never live together)
  constexpr bool kSplitSQ = STEP > 8;
  const float* bbase = sB + (ci * STEP + band * SYG) * C::BP + cj * STEP;
  float cs[BRW], cq[BRW];
  {
#pragma unroll
    for (int k = 0; k < SYG; ++k)
#pragma unroll
      for (int j = 0; j < C::NSY; ++j) Pacc[k][j] = 0.0f;
    if constexpr (!kSplitSQ) {
#pragma unroll
      for (int x = 0; x < BRW; ++x) cs[x] = cq[x] = 0.0f;
    }
    // stream the B' rows of the band once each; B' row rb meets A row
    // rb - k for shift row k, so the last SYG A rows are kept (converted)
    float ar[SYG][STEP];
#pragma unroll
    for (int rb = 0; rb < STEP + SYG - 1; ++rb) {
      float brow[BRW];
#pragma unroll
      for (int x = 0; x < BRW; ++x) brow[x] = bbase[rb * C::BP + x];
      if (rb < STEP) {
        float* an = ar[rb % SYG];
#pragma unroll
        for (int x = 0; x < STEP; ++x) {
          const uint32_t wd = aw[rb][(x * ES) >> 2];
          const uint32_t px = ES == 1 ? (wd >> (8 * (x & 3))) & 0xffu : (wd >> (16 * (x & 1))) & 0xffffu;
          an[x] = (float)px;   // raw A: the offset K enters through the mean below
        }
        if constexpr (!kSplitSQ) {
#pragma unroll
          for (int x = 0; x < BRW; ++x) {
            cs[x] += brow[x];
            cq[x] += brow[x] * brow[x];
          }
        }
      }
#pragma unroll
      for (int k = 0; k < SYG; ++k) {
        const int py = rb - k;
        if (py >= 0 && py < STEP) {
          const float* ap = ar[py % SYG];
#pragma unroll
          for (int j = 0; j < C::NSY; ++j) {
            float s = Pacc[k][j];
#pragma unroll
            for (int x = 0; x < STEP; ++x) s += ap[x] * brow[x + j];
            Pacc[k][j] = s;
          }
        }
      }
    }
  }
  if constexpr (kSplitSQ) {
    // column sums of the band's first STEP rows
#pragma unroll
    for (int x = 0; x < BRW; ++x) cs[x] = cq[x] = 0.0f;
#pragma unroll
    for (int rb = 0; rb < STEP; ++rb) {
#pragma unroll
      for (int x = 0; x < BRW; ++x) {
        const float b = bbase[rb * C::BP + x];
        cs[x] += b;
        cq[x] += b * b;
      }
    }
  }
  {
    // column sums of the band's first row, slid down for the other rows;
    // box sums over STEP columns for every shift column
#pragma unroll
    for (int k = 0; k < SYG; ++k) {
      if (k > 0) {
        const float* rin = bbase + (STEP + k - 1) * C::BP;
        const float* rout = bbase + (k - 1) * C::BP;
#pragma unroll
        for (int x = 0; x < BRW; ++x) {
          const float vi = rin[x], vo = rout[x];
          cs[x] += vi - vo;
          cq[x] += vi * vi - vo * vo;
        }
      }
      float s = 0.0f, q = 0.0f;
#pragma unroll
      for (int x = 0; x < STEP; ++x) {
        s += cs[x];
        q += cq[x];
      }
      Sacc[k][0] = s;
      Qacc[k][0] = q;
#pragma unroll
      for (int j = 1; j < C::NSY; ++j) {
        s += cs[j + STEP - 1] - cs[j - 1];
        q += cq[j + STEP - 1] - cq[j - 1];
        Sacc[k][j] = s;
        Qacc[k][j] = q;
      }
    }
  }
  // ---- window sums: (cell + right-hand neighbour) by DPP wave_shl:1, then
  // + the same pair one cell row down (lane + CW) by a lane permute.  Only
  // lanes of a window's top-left cell keep meaningful sums.
  auto quad = [&](float x) {
    const float h = x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130, 0xF, 0xF, false));
    return h + __int_as_float(__builtin_amdgcn_ds_bpermute((lane + C::CW) << 2, __float_as_int(h)));
  };
  sa = quad(sa);
  saa = quad(saa);
#pragma unroll
  for (int k = 0; k < SYG; ++k)
#pragma unroll
    for (int j = 0; j < C::NSY; ++j) {
      Pacc[k][j] = quad(Pacc[k][j]);
      Sacc[k][j] = quad(Sacc[k][j]);
      Qacc[k][j] = quad(Qacc[k][j]);
    }
  // ---- Pearson coefficient per shift, the band's peak by the tie key
  const bool wact = cell_ok && ci < TH && cj < TW;
  const int w = ci * TW + cj;
  float* const rhoW = s_un;                      // [window][shift]
  float* const s_best = s_un + C::NWIN * C::NS;  // [band][window]
  int* const s_pk = reinterpret_cast<int*>(s_best + C::NG * C::NWIN);
  {
    constexpr float kInvN = 1.0f / (float)(4 * STEP * STEP);
    const float mA = sa * kInvN;
    const float varA = saa - sa * mA;
    const float meanA = K + mA;
    const bool flatA = !(varA > kFlatRel * saa);
    // coefficients first (no control flow), then the band's peak
    float rv[SYG][C::NSY];
    bool allflat = true;   // every used shift of the band is flat
#pragma unroll
    for (int k = 0; k < SYG; ++k)
#pragma unroll
      for (int j = 0; j < C::NSY; ++j) {
        const int sy = band * SYG + k - R, sx = j - R;
        const float num = Pacc[k][j] - meanA * Sacc[k][j];
        const float varB = Qacc[k][j] - Sacc[k][j] * Sacc[k][j] * kInvN;
        const bool flat = flatA || !(varB > kFlatRel * Qacc[k][j]);
        // (varA varB > 0 unless flat; the flat value replaces the quotient)
        const float r = num * __builtin_amdgcn_rsqf(varA * varB);
        rv[k][j] = flat ? 0.0f : r;
        const bool used = !g.fixed || sx == 0 || sy == 0;
        if (used) allflat = allflat && flat;
      }
    // the band's peak: the largest coefficient, then the smallest tie key
    // among the shifts that reach it
    float best = -2.0f;
    int bkey = 1 << 20;
    if (!g.fixed) {
#pragma unroll
      for (int k = 0; k < SYG; ++k)
#pragma unroll
        for (int j = 0; j < C::NSY; ++j) best = fmaxf(best, rv[k][j]);
#pragma unroll
      for (int k = 0; k < SYG; ++k)
#pragma unroll
        for (int j = 0; j < C::NSY; ++j)
          bkey = rv[k][j] == best ? min(bkey, tie_key(band * SYG + k - R, j - R)) : bkey;
    }
    if (wact) {
      float* d = rhoW + w * C::NS + band * SYG * C::NSY;
#pragma unroll
      for (int k = 0; k < SYG; ++k)
#pragma unroll
        for (int j = 0; j < C::NSY; ++j) d[k * C::NSY + j] = rv[k][j];
      s_best[band * C::NWIN + w] = best;
      s_pk[band * C::NWIN + w] = (bkey << 1) | (allflat ? 1 : 0);
    }
  }
  __syncthreads();
  // ---- peak over the bands, fit, composition with the predictor's window mean
  // (with large cells, whose kernel has two workgroups per CU and is bound
  // by latency, the windows are dealt to the waves so that the fits of a
  // tile run side by side; with small cells, where VALU issue bounds the
  // kernel, one wave fits them all and the others end)
  constexpr int WPW = STEP > 8 ? (C::NWIN + C::NG - 1) / C::NG : C::NWIN;   // windows per wave
  const int wt = band * WPW + lane;
  if (lane < WPW && wt < C::NWIN) {
    const int wi = wt / TW, wj = wt - (wt / TW) * TW;
    const int a = a0 + wi, b = b0 + wj;
    if (a < g.ny && b < g.nx) {
      float best = -2.0f;
      int bkey = 1 << 20;
      bool allflat = true;
#pragma unroll
      for (int q = 0; q < C::NG; ++q) {
        const float bq = s_best[q * C::NWIN + wt];
        const int pk = s_pk[q * C::NWIN + wt];
        allflat = allflat && (pk & 1);
        if (better(bq, pk >> 1, best, bkey)) {
          best = bq;
          bkey = pk >> 1;
        }
      }
      int sy = 0, sx = 0;
      if (!g.fixed) {
        sx = (bkey & 63) - 32;
        sy = ((bkey >> 6) & 63) - 32;
      }
      const float* rr = rhoW + wt * C::NS;
      auto rhof = [&](int y, int x) { return rr[(y + R) * C::NSY + x + R]; };
      auto node = [&](int c, int y, int x) { return s_node[c][y - nlo_y][x - nlo_x]; };
      float pu = 0.0f, pv = 0.0f;
      if (Pn) window_mean_half_overlap(a, b, g.nx, g.ny, node, pu, pv);
      finish_vector(g, pair, a, b, sy, sx, allflat, pu, pv, rhof);
    }
  }
}

template <typename T, int STEP, int R, int SYG, int TW, int TH, int NT>
hipError_t launch_tiled(const CorrArgs& g, int n, hipStream_t s) {
  dim3 grid((g.nx + TW - 1) / TW, (g.ny + TH - 1) / TH, n);
  hipLaunchKernelGGL((k_correct_tiled<T, STEP, R, SYG, TW, TH, NT>), grid, dim3(NT), 0, s, g);
  return hipGetLastError();
}

template <typename T, int STEP, int R, int SYG, int TW, int TH>
hipError_t launch_bands(const CorrArgs& g, int n, hipStream_t s) {
  dim3 grid((g.nx + TW - 1) / TW, (g.ny + TH - 1) / TH, n);
  hipLaunchKernelGGL((k_correct_bands<T, STEP, R, SYG, TW, TH>), grid, dim3(64 * ((2 * R + 1) / SYG)), 0, s, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_tiled_t(const CorrArgs& g, int n, hipStream_t s) {
  if (!g.central && g.step == 8 && g.R == 4) return launch_bands<T, 8, 4, 3, 8, 6>(g, n, s);
  if (!g.central && g.step == 8 && g.R == 1) return launch_bands<T, 8, 1, 1, 8, 6>(g, n, s);
  if constexpr (sizeof(T) == 2) {   // (u8 cells of 12 px are not whole words at half a cell)
    if (!g.central && g.step == 12 && g.R == 4) return launch_bands<T, 12, 4, 3, 8, 6>(g, n, s);
  }
  if (g.step == 8 && g.R == 4) return launch_tiled<T, 8, 4, 3, 8, 8, 256>(g, n, s);
  if (g.step == 8 && g.R == 1) return launch_tiled<T, 8, 1, 1, 8, 8, 256>(g, n, s);
  if (g.step == 12 && g.R == 4) return launch_tiled<T, 12, 4, 3, 5, 5, 128>(g, n, s);
  if (g.step == 12 && g.R == 1) return launch_tiled<T, 12, 1, 1, 5, 5, 128>(g, n, s);
  return hipErrorInvalidValue;
}

}  // namespace

int correct_impl(const Plan& P) {
  const int R = P.p.peak == PIV_PEAK_FIXED_CENTER ? 1 : P.p.radius;
  if (P.p.dtype == PIV_F32) return 0;
  if (P.p.win != 2 * P.p.step) return 0;
  if ((P.p.step == 8 || P.p.step == 12) && (R == 4 || R == 1)) return 1;
  return 0;
}

hipError_t launch_correct(const Plan& P, const void* A, const void* B, int64_t pitch, int n,
                          const float* pred, float* disp, float* peak, uint8_t* flags, hipStream_t s,
                          int64_t disp_stride) {
  CorrArgs g;
  g.A = (const uint8_t*)A;
  g.B = (const uint8_t*)B;
  g.pitch = pitch;
  g.stride = pitch * P.p.height;
  g.W = P.p.width;
  g.H = P.p.height;
  g.nx = P.nx;
  g.ny = P.ny;
  g.win = P.p.win;
  g.step = P.p.step;
  g.fixed = P.p.peak == PIV_PEAK_FIXED_CENTER;
  g.R = g.fixed ? 1 : P.p.radius;
  g.central = P.p.warp == PIV_WARP_CENTRAL;
  g.pred = pred;
  g.disp = disp;
  g.dstride = disp_stride ? disp_stride : 2 * (int64_t)P.nx * P.ny;
  g.peak = peak;
  g.flags = flags;
  g.mask = P.slot_mask;
  if (correct_impl(P) == 1) {
    return P.p.dtype == PIV_U8 ? launch_tiled_t<uint8_t>(g, n, s) : launch_tiled_t<uint16_t>(g, n, s);
  }
  const int BWd = g.win + 2 * g.R, S = 2 * g.R + 1, S2 = S * S;
  const int H = std::max(1, std::min(g.win, kGenT / S2));   // (as in the kernel)
  size_t lds = sizeof(float) * ((size_t)g.win * g.win + (size_t)BWd * BWd + (size_t)S2 + 3 * (size_t)H * S2);
  dim3 grid(P.nx, P.ny, n);
  switch (P.p.dtype) {
    case PIV_U8: hipLaunchKernelGGL(k_correct_generic<uint8_t>, grid, dim3(kGenT), lds, s, g); break;
    case PIV_U16: hipLaunchKernelGGL(k_correct_generic<uint16_t>, grid, dim3(kGenT), lds, s, g); break;
    default: hipLaunchKernelGGL(k_correct_generic<float>, grid, dim3(kGenT), lds, s, g); break;
  }
  return hipGetLastError();
}

}  // namespace piv
