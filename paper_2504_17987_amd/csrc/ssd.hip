// Differentiable windowed SSD of the deformation (an addition of this
// library, not in the paper): forward loss per window and its adjoint with
// respect to the node displacement field, with the Gauss-Newton diagonal.
//
// The tiled forms (win = 2 step) cache the nodes of a tile in LDS; the
// backward forms each pixel's terms 2 m r dB'/du and 2 m (dB'/du)^2 once per
// tile, splits them into left/right node-column partials per pixel row and
// lets every node sum its partials over its rows.  The general forms gather
// per node with per-pixel weights.  No atomics anywhere, so the results are
// bitwise reproducible.
#include <type_traits>

#include "dev_common.h"
#include "piv_internal.h"

namespace piv {
namespace {

struct SsdArgs {
  const float* A;
  const float* B;
  const float* U;
  int W, H, nx, ny, win, step;
  float* loss;
  const float* g;       // NULL: every window's upstream gradient is 1
  float* gU;
  float* D;
  int64_t lstride;      // floats per pair of loss
  int64_t gstride;      // floats per pair of gU and D
  const uint8_t* mask;
  // (tiled adjoint, nullable) per node tile: [tile][2] = the tile's sum of
  // the GN diagonal (both components) and of the window losses (each pixel
  // counted by the tile owning its base node), pair stride pstride floats
  float* part;
  int64_t pstride;
};

__device__ __forceinline__ float ldA(const float* I, int W, int H, int y, int x) {
  return ((unsigned)x < (unsigned)W && (unsigned)y < (unsigned)H) ? I[(int64_t)y * W + x] : 0.0f;
}

// clamped bilinear node coordinates of a pixel: base node and fractions
__device__ __forceinline__ void node_coord(float p, int n, int step, int& b, float& f) {
  const float c = 0.5f * (float)(step - 1);
  float t = fminf(fmaxf((p - c) / (float)step, 0.0f), (float)(n - 1));
  b = min((int)t, max(n - 2, 0));
  f = t - (float)b;
}

__device__ __forceinline__ void disp_at(const float* U, int nx, int ny, int step, int x, int y, float& u,
                                        float& v) {
  int bx, by;
  float fx, fy;
  node_coord((float)x, nx, step, bx, fx);
  node_coord((float)y, ny, step, by, fy);
  int bx1 = nx > 1 ? bx + 1 : bx, by1 = ny > 1 ? by + 1 : by;
  const int np = nx * ny;
  const float* P = U;
  u = (1.0f - fy) * ((1.0f - fx) * P[by * nx + bx] + fx * P[by * nx + bx1]) +
      fy * ((1.0f - fx) * P[by1 * nx + bx] + fx * P[by1 * nx + bx1]);
  P = U + np;
  v = (1.0f - fy) * ((1.0f - fx) * P[by * nx + bx] + fx * P[by * nx + bx1]) +
      fy * ((1.0f - fx) * P[by1 * nx + bx] + fx * P[by1 * nx + bx1]);
}

// weight of node index `b` in the clamped interpolation of coordinate p
__device__ __forceinline__ float node_weight(float p, int n, int step, int b) {
  int bb;
  float f;
  node_coord(p, n, step, bb, f);
  float w = 0.0f;
  if (b == bb) w += 1.0f - f;
  if (b == (n > 1 ? bb + 1 : bb)) w += f;
  return w;
}

// residual r = B(p+u) - A(p) and the floor-cell gradient of the sample
__device__ __forceinline__ void residual(const SsdArgs& a, const float* A, const float* B, const float* U,
                                         int x, int y, float& r, float& gx, float& gy) {
  float u, v;
  disp_at(U, a.nx, a.ny, a.step, x, y, u, v);
  float qx = (float)x + u, qy = (float)y + v;
  float x0 = floorf(qx), y0 = floorf(qy);
  float fx = qx - x0, fy = qy - y0;
  int ix = (int)x0, iy = (int)y0;
  float p00 = ldA(B, a.W, a.H, iy, ix), p01 = ldA(B, a.W, a.H, iy, ix + 1);
  float p10 = ldA(B, a.W, a.H, iy + 1, ix), p11 = ldA(B, a.W, a.H, iy + 1, ix + 1);
  float bs = (1.0f - fy) * ((1.0f - fx) * p00 + fx * p01) + fy * ((1.0f - fx) * p10 + fx * p11);
  r = bs - ldA(A, a.W, a.H, y, x);
  gx = (1.0f - fy) * (p01 - p00) + fy * (p11 - p10);
  gy = (1.0f - fx) * (p10 - p00) + fx * (p11 - p01);
}

__device__ __forceinline__ int fdiv(int p, int q) { return p >= 0 ? p / q : -((-p + q - 1) / q); }

// Forward: a workgroup owns a TN x TN tile of windows; squared residuals of
// the tile's pixel region go to LDS, then every window sums its block.
__global__ __launch_bounds__(256) void k_ssd_forward(SsdArgs a, int TN) {
  extern __shared__ float s_r2[];
  const int pair = blockIdx.z;
  if (slot_off(a.mask, pair)) return;
  const int t = threadIdx.x;
  const int np = a.nx * a.ny;
  const int64_t img = (int64_t)a.W * a.H;
  const float* A = a.A + pair * img;
  const float* B = a.B + pair * img;
  const float* U = a.U + (int64_t)pair * 2 * np;
  const int h = (a.win - a.step) / 2;
  const int ta = blockIdx.y * TN, tb = blockIdx.x * TN;
  const int RW = (TN - 1) * a.step + a.win;
  const int y0 = ta * a.step - h, x0 = tb * a.step - h;
  for (int idx = t; idx < RW * RW; idx += 256) {
    int y = y0 + idx / RW, x = x0 + idx % RW;
    float r, gx, gy;
    residual(a, A, B, U, x, y, r, gx, gy);
    s_r2[idx] = r * r;
  }
  __syncthreads();
  // one window per 4 threads (TN*TN <= 64)
  const int w = t >> 2, p = t & 3;
  const int wi = w / TN, wj = w % TN;
  float s = 0.0f;
  if (w < TN * TN) {
    for (int i = p; i < a.win; i += 4) {
      const float* row = s_r2 + (wi * a.step + i) * RW + wj * a.step;
      for (int j = 0; j < a.win; ++j) s += row[j];
    }
  }
  s += __shfl_xor(s, 1);
  s += __shfl_xor(s, 2);
  if (w < TN * TN && p == 0) {
    int aa = ta + wi, bb = tb + wj;
    if (aa < a.ny && bb < a.nx) a.loss[(int64_t)pair * a.lstride + aa * a.nx + bb] = s;
  }
}

// Backward: a workgroup owns a TN x TN tile of nodes.  Pass 1 writes per
// pixel of the tile's support region: 2 m r gx, 2 m r gy, 2 m gx^2, 2 m gy^2
// (m = sum of upstream gradients of the windows holding the pixel).  Pass 2:
// 16 threads per node gather weight * term over the node's support rows,
// then reduce over their 16 lanes.
__global__ __launch_bounds__(256) void k_ssd_backward(SsdArgs a, int TN) {
  extern __shared__ float s_t[];
  const int pair = blockIdx.z;
  if (slot_off(a.mask, pair)) return;
  const int t = threadIdx.x;
  const int np = a.nx * a.ny;
  const int64_t img = (int64_t)a.W * a.H;
  const float* A = a.A + pair * img;
  const float* B = a.B + pair * img;
  const float* U = a.U + (int64_t)pair * 2 * np;
  const float* G = a.g ? a.g + (int64_t)pair * np : nullptr;
  const int h = (a.win - a.step) / 2;
  const int ta = blockIdx.y * TN, tb = blockIdx.x * TN;
  // pixel support of the tile's nodes (clamped interpolation extends the
  // edge nodes' support to the outermost window pixel)
  const int lo_all = -h, hi_x = a.nx * a.step + h - 1, hi_y = a.ny * a.step + h - 1;
  int ylo = ta == 0 ? lo_all : (ta - 1) * a.step + a.step / 2;   // > centre of node ta-1
  int xlo = tb == 0 ? lo_all : (tb - 1) * a.step + a.step / 2;
  int tae = min(ta + TN, a.ny) - 1, tbe = min(tb + TN, a.nx) - 1;
  int yhi = tae == a.ny - 1 ? hi_y : (tae + 1) * a.step + (a.step - 1) / 2;  // < centre of node tae+1
  int xhi = tbe == a.nx - 1 ? hi_x : (tbe + 1) * a.step + (a.step - 1) / 2;
  const int RH = yhi - ylo + 1, RW = xhi - xlo + 1;
  float* T0 = s_t;
  float* T1 = T0 + RH * RW;
  float* T2 = T1 + RH * RW;
  float* T3 = T2 + RH * RW;
  for (int idx = t; idx < RH * RW; idx += 256) {
    int y = ylo + idx / RW, x = xlo + idx % RW;
    // m(p): windows whose block holds the pixel, i.e. the a with
    // a step - h <= y <= a step - h + win - 1 (ceiling for the lower bound)
    int a0 = max(fdiv(y + h - a.win + a.step, a.step), 0), a1 = min(fdiv(y + h, a.step), a.ny - 1);
    int b0 = max(fdiv(x + h - a.win + a.step, a.step), 0), b1 = min(fdiv(x + h, a.step), a.nx - 1);
    float m = 0.0f;
    for (int i = a0; i <= a1; ++i)
      for (int j = b0; j <= b1; ++j) m += G ? G[i * a.nx + j] : 1.0f;
    float r = 0.0f, gx = 0.0f, gy = 0.0f;
    if (m != 0.0f) residual(a, A, B, U, x, y, r, gx, gy);
    T0[idx] = 2.0f * m * r * gx;
    T1[idx] = 2.0f * m * r * gy;
    T2[idx] = 2.0f * m * gx * gx;
    T3[idx] = 2.0f * m * gy * gy;
  }
  __syncthreads();
  const int nd = t >> 4, lane = t & 15;
  const int na = ta + nd / TN, nb = tb + nd % TN;
  float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f;
  const bool act = nd < TN * TN && na < a.ny && nb < a.nx;
  if (act) {
    // node support rows/cols, intersected with the region
    int sy0 = na == 0 ? lo_all : (na - 1) * a.step + a.step / 2;
    int sy1 = na == a.ny - 1 ? hi_y : (na + 1) * a.step + (a.step - 1) / 2;
    int sx0 = nb == 0 ? lo_all : (nb - 1) * a.step + a.step / 2;
    int sx1 = nb == a.nx - 1 ? hi_x : (nb + 1) * a.step + (a.step - 1) / 2;
    for (int y = sy0 + lane; y <= sy1; y += 16) {
      float wy = node_weight((float)y, a.ny, a.step, na);
      if (wy == 0.0f) continue;
      const int ro = (y - ylo) * RW - xlo;
      for (int x = sx0; x <= sx1; ++x) {
        float wx = node_weight((float)x, a.nx, a.step, nb);
        float w = wx * wy;
        s0 += w * T0[ro + x];
        s1 += w * T1[ro + x];
        s2 += w * w * T2[ro + x];
        s3 += w * w * T3[ro + x];
      }
    }
  }
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) {
    s0 += __shfl_xor(s0, o);
    s1 += __shfl_xor(s1, o);
    s2 += __shfl_xor(s2, o);
    s3 += __shfl_xor(s3, o);
  }
  if (act && lane == 0) {
    const int i = na * a.nx + nb;
    float* gU = a.gU + (int64_t)pair * a.gstride;
    gU[i] = s0;
    gU[np + i] = s1;
    if (a.D) {
      float* D = a.D + (int64_t)pair * a.gstride;
      D[i] = s2;
      D[np + i] = s3;
    }
  }
}

// ---------------------------------------------------------------------------
// Tiled forms for win = 2 step (the plans' geometry).  A workgroup owns a
// TN x TN tile (of windows forward, of nodes backward).  The nodes covering
// the tile's pixel region are cached in LDS with per-row / per-column
// interpolation tables; samples of A and B are read from global memory (L1
// serves the bilinear neighbours), which keeps LDS small and occupancy high
// enough to hide the read latency.
// ---------------------------------------------------------------------------
template <int STEP, int TN>
struct SsdTile {
  static constexpr int H2 = STEP / 2;                 // (win - step) / 2
  static constexpr int RW = (TN + 1) * STEP;          // max region side (px)
  static constexpr int NNC = RW / STEP + 3;           // cached node rows / columns
  static constexpr int NG = RW / STEP + 2;            // cached window rows / columns
};

// The cached nodes and tables of a region [ylo, ylo+RH) x [xlo, xlo+RW_).
template <int STEP, int TN>
struct SsdShared {
  using C = SsdTile<STEP, TN>;
  float node[2][C::NNC][C::NNC];
  int rb[C::RW], cb[C::RW];       // base node (cache index)
  float rf[C::RW], cf[C::RW];     // fraction towards base + 1
};

// Loads the node cache and the interpolation tables of the region rows and
// columns (base node as a cache index, fraction towards base + 1).
// Returns (the same in every thread) whether the tile is interior: every
// pixel of the region lies in the frames and so does every bilinear sample
// with its right and lower neighbours, with a pixel to spare.  The samples
// of region pixel x lie at x + u with u between the cached nodes' extremes
// (the interpolation stays within them), so the nodes decide; a NaN node
// makes the tile not interior.
template <int STEP, int TN>
__device__ __forceinline__ bool ssd_prepare(const SsdArgs& a, const float* U, int ylo, int xlo, int RH, int RWc,
                                            SsdShared<STEP, TN>& sh, int& nly, int& nlx) {
  using C = SsdTile<STEP, TN>;
  const int t = threadIdx.x;
  const float cen = 0.5f * (float)(STEP - 1);
  nly = max(0, (int)floorf(((float)ylo - cen) / STEP));
  nlx = max(0, (int)floorf(((float)xlo - cen) / STEP));
  const int np = a.nx * a.ny;
  const int xhi = xlo + RWc - 1, yhi = ylo + RH - 1;
  bool inside = xlo >= 0 && ylo >= 0 && xhi <= a.W - 1 && yhi <= a.H - 1;
  for (int i = t; i < C::NNC * C::NNC; i += 256) {
    const int r = i / C::NNC, q = i - (i / C::NNC) * C::NNC;
    const int ny_ = min(nly + r, a.ny - 1), nx_ = min(nlx + q, a.nx - 1);
    const float u = U[ny_ * a.nx + nx_], v = U[np + ny_ * a.nx + nx_];
    sh.node[0][r][q] = u;
    sh.node[1][r][q] = v;
    inside = inside && (float)xlo + u >= 1.0f && (float)xhi + u <= (float)(a.W - 3) && (float)ylo + v >= 1.0f &&
             (float)yhi + v <= (float)(a.H - 3);
  }
  for (int i = t; i < RH + RWc; i += 256) {
    const bool row = i < RH;
    const int pp = row ? ylo + i : xlo + (i - RH);
    const int n = row ? a.ny : a.nx;
    int bb;
    float ff;
    node_coord((float)pp, n, STEP, bb, ff);
    if (row) { sh.rb[i] = bb - nly; sh.rf[i] = ff; }
    else { sh.cb[i - RH] = bb - nlx; sh.cf[i - RH] = ff; }
  }
  return __syncthreads_and(inside ? 1 : 0) != 0;
}

// bilinear sample bs = B(x + u, y + v) at the pixel (x, y), given as floats
// xf, yf, and its floor-cell gradient: with top/bottom the row
// interpolations of the cell, bs = top + ey (bottom - top), dbs/dy =
// bottom - top and dbs/dx the row differences interpolated in y.  kInside:
// the tile is interior (every read in the frames), so the reads need no
// bounds tests and take 32-bit byte offsets from the frame base (a frame
// holds fewer than 2^30 pixels).
template <bool kInside>
__device__ __forceinline__ void ssd_sample(const SsdArgs& a, const float* B, float xf, float yf, float u, float v,
                                           float& bs, float& gx, float& gy) {
  const float qx = xf + u, qy = yf + v;
  const float x0 = floorf(qx), y0 = floorf(qy);
  const float ex = qx - x0, ey = qy - y0;
  const int ix = (int)x0, iy = (int)y0;
  float p00, p01, p10, p11;
  if constexpr (kInside) {
    const char* Bb = reinterpret_cast<const char*>(B);
    const uint32_t o = 4u * (uint32_t)(iy * a.W + ix), ow = 4u * (uint32_t)a.W;
    p00 = *reinterpret_cast<const float*>(Bb + o);
    p01 = *reinterpret_cast<const float*>(Bb + o + 4u);
    p10 = *reinterpret_cast<const float*>(Bb + (o + ow));
    p11 = *reinterpret_cast<const float*>(Bb + (o + ow) + 4u);
  } else {
    p00 = ldA(B, a.W, a.H, iy, ix);
    p01 = ldA(B, a.W, a.H, iy, ix + 1);
    p10 = ldA(B, a.W, a.H, iy + 1, ix);
    p11 = ldA(B, a.W, a.H, iy + 1, ix + 1);
  }
  const float d0 = p01 - p00, d1 = p11 - p10;
  const float top = p00 + ex * d0, bot = p10 + ex * d1;
  gy = bot - top;
  bs = top + ey * gy;
  gx = d0 + ey * (d1 - d0);
}

// A at the pixel (x, y) (zero outside the frame)
template <bool kInside>
__device__ __forceinline__ float ssd_a(const SsdArgs& a, const float* A, int x, int y) {
  if constexpr (kInside)
    return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(A) + 4u * (uint32_t)(y * a.W + x));
  else
    return ldA(A, a.W, a.H, y, x);
}

// residual r = B'(p) - A(p) and the sample's gradient at the pixel (x, y)
// for a given displacement (u, v) of that pixel
template <bool kInside>
__device__ __forceinline__ void ssd_residual_uv(const SsdArgs& a, const float* A, const float* B, int x, int y,
                                                float xf, float yf, float u, float v, float& r, float& gx,
                                                float& gy) {
  float bs;
  ssd_sample<kInside>(a, B, xf, yf, u, v, bs, gx, gy);
  r = bs - ssd_a<kInside>(a, A, x, y);
}

// the same at region pixel (i, j), its displacement interpolated from the
// cached nodes
template <bool kInside, int STEP, int TN>
__device__ __forceinline__ void ssd_residual(const SsdArgs& a, const float* A, const float* B,
                                             const SsdShared<STEP, TN>& sh, int ylo, int xlo, int i, int j,
                                             float& r, float& gx, float& gy) {
  const int rb = sh.rb[i], cb = sh.cb[j];
  const float fy = sh.rf[i], fx = sh.cf[j];
  const float u = (1.0f - fy) * ((1.0f - fx) * sh.node[0][rb][cb] + fx * sh.node[0][rb][cb + 1]) +
                  fy * ((1.0f - fx) * sh.node[0][rb + 1][cb] + fx * sh.node[0][rb + 1][cb + 1]);
  const float v = (1.0f - fy) * ((1.0f - fx) * sh.node[1][rb][cb] + fx * sh.node[1][rb][cb + 1]) +
                  fy * ((1.0f - fx) * sh.node[1][rb + 1][cb] + fx * sh.node[1][rb + 1][cb + 1]);
  ssd_residual_uv<kInside>(a, A, B, xlo + j, ylo + i, (float)(xlo + j), (float)(ylo + i), u, v, r, gx, gy);
}

// Forward, TN x TN windows per workgroup: squared residuals of the tile's
// pixel region in LDS, then 4 threads per window sum its block.
template <int STEP, int TN>
__global__ __launch_bounds__(256) void k_ssd_forward_t(SsdArgs a) {
  using C = SsdTile<STEP, TN>;
  constexpr int WIN = 2 * STEP, RWF = (TN - 1) * STEP + WIN;
  static_assert(RWF <= C::RW, "forward region");
  __shared__ SsdShared<STEP, TN> sh;
  __shared__ float s_r2[RWF * RWF];
  const WgIdx wg = xcd_order();
  const int pair = wg.z;
  if (slot_off(a.mask, pair)) return;
  const int t = threadIdx.x;
  const int np = a.nx * a.ny;
  const int64_t img = (int64_t)a.W * a.H;
  const float* A = a.A + pair * img;
  const float* B = a.B + pair * img;
  const float* U = a.U + (int64_t)pair * 2 * np;
  const int ta = wg.y * TN, tb = wg.x * TN;
  const int ylo = ta * STEP - C::H2, xlo = tb * STEP - C::H2;
  int nly, nlx;
  const bool interior = ssd_prepare<STEP, TN>(a, U, ylo, xlo, RWF, RWF, sh, nly, nlx);
  auto squares = [&](auto inside) {
    constexpr bool kIn = decltype(inside)::value;
    for (int idx = t; idx < RWF * RWF; idx += 256) {
      const int i = idx / RWF, j = idx - (idx / RWF) * RWF;
      float r, gx, gy;
      ssd_residual<kIn, STEP, TN>(a, A, B, sh, ylo, xlo, i, j, r, gx, gy);
      s_r2[idx] = r * r;
    }
  };
  if (interior) squares(std::true_type{});
  else squares(std::false_type{});
  __syncthreads();
  const int w = t >> 2, p = t & 3;
  const int wi = w / TN, wj = w - (w / TN) * TN;
  float s = 0.0f;
  if (w < TN * TN) {
    for (int i = p; i < WIN; i += 4) {
      const float* row = s_r2 + (wi * STEP + i) * RWF + wj * STEP;
#pragma unroll
      for (int j = 0; j < WIN; ++j) s += row[j];
    }
  }
  s += __shfl_xor(s, 1);
  s += __shfl_xor(s, 2);
  if (w < TN * TN && p == 0) {
    const int aa = ta + wi, bb = tb + wj;
    if (aa < a.ny && bb < a.nx) a.loss[(int64_t)pair * a.lstride + aa * a.nx + bb] = s;
  }
}

// Sum over a 256-thread workgroup in a fixed order (every thread gets it).
__device__ __forceinline__ float tile_sum(float x, float* red) {
  const int t = threadIdx.x;
  __syncthreads();
  red[t] = x;
  __syncthreads();
#pragma unroll
  for (int o = 128; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  return red[0];
}

// Backward, TN x TN nodes per workgroup.  Every pixel of the nodes' support
// region contributes to the two node columns and two node rows of its
// bilinear cell (weights 1-f and f, squared for the diagonal), so the
// adjoint separates: pass 1 sums each (pixel row, STEP-pixel chunk) into
// left/right column partials of the four terms 2 m r gx, 2 m r gy,
// 2 m gx^2, 2 m gy^2; pass 2 sums a node's partials over its rows with the
// row weights.  Chunks of STEP pixels starting at the region edge share one
// base node column (the region starts on a cell boundary), and m (the sum
// of the upstream gradients of the windows holding the pixel) is constant
// along a chunk.
template <int STEP, int TN, bool kPart>
__global__ __launch_bounds__(256) void k_ssd_backward_t(SsdArgs a) {
  using C = SsdTile<STEP, TN>;
  constexpr int NCH = C::RW / STEP;                    // chunks per region row
  static_assert(STEP % 4 == 0, "chunks of whole groups of four pixels");
  __shared__ SsdShared<STEP, TN> sh;
  __shared__ float s_part[C::RW][NCH][8];              // [row][chunk][term*2 + side]
  __shared__ float s_g[C::NG][C::NG];                  // upstream window gradients
  __shared__ int s_chb[NCH];                           // base node column of a chunk
  __shared__ int s_rfirst[C::NNC], s_rlast[C::NNC];    // region rows based on each cached node row
  __shared__ float s_red[256];                         // fixed-order tile sums
  __shared__ uint8_t s_ownr[C::RW], s_ownc[C::RW];     // region rows / columns whose nearest node is the tile's
  __shared__ float4 s_cw[C::RW];                       // per region column: wr (the fraction), wl, wr^2, wl^2
  const WgIdx wg = xcd_order();
  const int pair = wg.z;
  if (slot_off(a.mask, pair)) return;
  const int t = threadIdx.x;
  const int np = a.nx * a.ny;
  const int64_t img = (int64_t)a.W * a.H;
  const float* A = a.A + pair * img;
  const float* B = a.B + pair * img;
  const float* U = a.U + (int64_t)pair * 2 * np;
  const float* G = a.g ? a.g + (int64_t)pair * np : nullptr;
  const int ta = wg.y * TN, tb = wg.x * TN;
  constexpr int h = C::H2;
  const int lo_all = -h, hi_x = a.nx * STEP + h - 1, hi_y = a.ny * STEP + h - 1;
  const int ylo = ta == 0 ? lo_all : (ta - 1) * STEP + STEP / 2;
  const int xlo = tb == 0 ? lo_all : (tb - 1) * STEP + STEP / 2;
  const int tae = min(ta + TN, a.ny) - 1, tbe = min(tb + TN, a.nx) - 1;
  const int yhi = tae == a.ny - 1 ? hi_y : (tae + 1) * STEP + (STEP - 1) / 2;
  const int xhi = tbe == a.nx - 1 ? hi_x : (tbe + 1) * STEP + (STEP - 1) / 2;
  const int RH = yhi - ylo + 1, RWc = xhi - xlo + 1;
  // upstream gradients of the windows that can hold a region pixel:
  // window rows i with i STEP - h <= y <= i STEP - h + 2 STEP - 1
  const int gi0 = max((ylo + h) / STEP - 1, 0), gj0 = max((xlo + h) / STEP - 1, 0);
  for (int i = t; i < C::NG * C::NG; i += 256) {
    const int r = i / C::NG, q = i - (i / C::NG) * C::NG;
    const int gi = gi0 + r, gj = gj0 + q;
    s_g[r][q] = (gi < a.ny && gj < a.nx) ? (G ? G[gi * a.nx + gj] : 1.0f) : 0.0f;
  }
  int nly, nlx;
  if (t < C::NNC) s_rfirst[t] = s_rlast[t] = -1;
  const bool interior = ssd_prepare<STEP, TN>(a, U, ylo, xlo, RH, RWc, sh, nly, nlx);   // (ends with a barrier)
  if (t < NCH) s_chb[t] = t * STEP < RWc ? sh.cb[t * STEP] : -100;
  for (int i = t; i < RH; i += 256) {
    const int rb = sh.rb[i];
    if (i == 0 || sh.rb[i - 1] != rb) s_rfirst[rb] = i;
    if (i == RH - 1 || sh.rb[i + 1] != rb) s_rlast[rb] = i;
  }
  // column weights towards the left and right node columns (one node
  // column: all on the left)
  for (int j = t; j < RWc; j += 256) {
    const float f = sh.cf[j];
    const float wr = a.nx > 1 ? f : 0.0f, wl = a.nx > 1 ? 1.0f - f : 1.0f;
    s_cw[j] = make_float4(wr, wl, wr * wr, wl * wl);
  }
  // (the loss: a pixel counts at the tile holding its nearest node, whose
  // support region holds it)
  for (int i = t; kPart && i < RH + RWc; i += 256) {
    const bool row = i < RH;
    const int p = row ? ylo + i : xlo + (i - RH);
    const int n = row ? a.ny : a.nx, lo = row ? ta : tb;
    const int nn = min(max(fdiv(2 * p + 1, 2 * STEP), 0), n - 1);
    const uint8_t o = nn >= lo && nn < lo + TN;
    if (row) s_ownr[i] = o;
    else s_ownc[i - RH] = o;
  }
  __syncthreads();
  const int nchunks = (RWc + STEP - 1) / STEP;
  // chunks start 16-byte aligned in A (frame base, row length and the
  // region's first column multiples of four floats)
  const bool a16 = (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (a.W & 3) == 0 && (xlo & 3) == 0;
  float lsum = 0.0f;   // this thread's share of the tile's loss (owned items)
  for (int item = t; item < RH * nchunks; item += 256) {
    const int i = item / nchunks, c = item - (item / nchunks) * nchunks;
    const int y = ylo + i;
    // windows holding row y: rows a0..a1; columns from the chunk
    const int a0 = max(fdiv(y + h - STEP, STEP), 0), a1 = min(fdiv(y + h, STEP), a.ny - 1);
    const int x0c = xlo + c * STEP;
    const int b0 = max(fdiv(x0c + h - STEP, STEP), 0), b1 = min(fdiv(x0c + h, STEP), a.nx - 1);
    float m = 0.0f;
    for (int ii = a0; ii <= a1; ++ii)
      for (int jj = b0; jj <= b1; ++jj) m += s_g[ii - gi0][jj - gj0];
    float acc[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) acc[k] = 0.0f;
    const bool own = kPart && s_ownr[i];
    float lacc = 0.0f;   // the loss terms r^2 of the chunk's pixels this tile counts
    if (m != 0.0f) {
      // the chunk's pixels share their node row and node columns (it starts
      // on a cell boundary), so the node field is interpolated down the
      // two node columns once and across per pixel
      const int rb = sh.rb[i], cbase = s_chb[c];
      const float fy = sh.rf[i];
      const float uL = sh.node[0][rb][cbase] + fy * (sh.node[0][rb + 1][cbase] - sh.node[0][rb][cbase]);
      const float uR = sh.node[0][rb][cbase + 1] + fy * (sh.node[0][rb + 1][cbase + 1] - sh.node[0][rb][cbase + 1]);
      const float vL = sh.node[1][rb][cbase] + fy * (sh.node[1][rb + 1][cbase] - sh.node[1][rb][cbase]);
      const float vR = sh.node[1][rb][cbase + 1] + fy * (sh.node[1][rb + 1][cbase + 1] - sh.node[1][rb][cbase + 1]);
      // the pixels' terms without the chunk's common factor 2 m, which
      // scales the sums once below; a whole chunk (every one when the
      // region width is a multiple of STEP) runs without per-pixel tests,
      // so its pixels' reads can be in flight together
      const float xf0 = (float)x0c, yf = (float)y;
      auto pixels = [&](auto inside) {
        constexpr bool kIn = decltype(inside)::value;
        auto px = [&](int e, float av) __attribute__((always_inline)) {
          const int j = c * STEP + e;
          const float4 w = s_cw[j];
          float bs, gx, gy;
          ssd_sample<kIn>(a, B, xf0 + (float)e, yf, uL + w.x * (uR - uL), vL + w.x * (vR - vL), bs, gx, gy);
          const float r = bs - av;
          const float t0 = r * gx, t1 = r * gy, t2 = gx * gx, t3 = gy * gy;
          acc[0] += w.y * t0; acc[1] += w.x * t0;
          acc[2] += w.y * t1; acc[3] += w.x * t1;
          acc[4] += w.w * t2; acc[5] += w.z * t2;
          acc[6] += w.w * t3; acc[7] += w.z * t3;
          if constexpr (kPart) lacc += s_ownc[j] ? r * r : 0.0f;
        };
        if (kIn && a16 && (c + 1) * STEP <= RWc) {
          // A's pixels of the chunk four at a time (16-byte aligned)
          const float4* a4 = reinterpret_cast<const float4*>(reinterpret_cast<const char*>(A) +
                                                             4u * (uint32_t)(y * a.W + x0c));
#pragma unroll 1
          for (int e4 = 0; e4 < STEP; e4 += 4) {
            const float4 av = a4[e4 / 4];
            px(e4, av.x);
            px(e4 + 1, av.y);
            px(e4 + 2, av.z);
            px(e4 + 3, av.w);
          }
        } else if ((c + 1) * STEP <= RWc) {
#pragma unroll 1
          for (int e4 = 0; e4 < STEP; e4 += 4) {
#pragma unroll
            for (int e = 0; e < 4; ++e) px(e4 + e, ssd_a<kIn>(a, A, x0c + e4 + e, y));
          }
        } else {
          for (int e = 0; e < STEP && c * STEP + e < RWc; ++e) px(e, ssd_a<kIn>(a, A, x0c + e, y));
        }
      };
      if (interior) pixels(std::true_type{});
      else pixels(std::false_type{});
    }
    if (kPart && own) lsum += m * lacc;
    const float m2 = 2.0f * m;
#pragma unroll
    for (int k = 0; k < 8; ++k) s_part[i][c][k] = m2 * acc[k];
  }
  __syncthreads();
  // pass 2: thread = (node, term); a node collects the left partials of the
  // chunks based on its column and the right partials of the chunks based
  // on the column before, weighted by its row weight
  const int nd = t >> 2, term = t & 3;
  const int na = ta + nd / TN, nb = tb + nd % TN;
  float dsum = 0.0f;   // this thread's GN diagonal value (terms 2, 3)
  if (nd < TN * TN && na < a.ny && nb < a.nx) {
    const int cbn = nb - nlx;                          // node column in cache indices
    const int rbn = na - nly;
    const bool sq = term >= 2;
    // base rows and chunk bases do not decrease along the region: the rows
    // and chunks that touch the node are contiguous runs (rows: those based
    // on the node's row and, with more than one node row, on the row before)
    int rf = RH, rl = -1, cf0 = nchunks, cl = -1;
    if (rbn >= 0 && rbn < C::NNC && s_rfirst[rbn] >= 0) { rf = s_rfirst[rbn]; rl = s_rlast[rbn]; }
    if (a.ny > 1 && rbn >= 1 && rbn - 1 < C::NNC && s_rfirst[rbn - 1] >= 0) {
      rf = min(rf, s_rfirst[rbn - 1]);
      rl = max(rl, s_rlast[rbn - 1]);
    }
    // the chunks based on the node's column (their left partials) and on
    // the column before (their right partials), found once: one or two each
    // (two where the region's edge chunks are clamped to the end cells;
    // three when the grid is two nodes wide and every chunk has base 0); a
    // missing one reads chunk 0 with weight 0
    int lc[3] = {0, 0, 0}, rc[3] = {0, 0, 0};
    float lw[3] = {0.0f, 0.0f, 0.0f}, rw[3] = {0.0f, 0.0f, 0.0f};
    int nl = 0, nr = 0;
    for (int c = 0; c < nchunks; ++c) {
      const int base = s_chb[c];
      if (base == cbn && nl < 3) { lc[nl] = c; lw[nl] = 1.0f; ++nl; }
      if (a.nx > 1 && base + 1 == cbn && nr < 3) { rc[nr] = c; rw[nr] = 1.0f; ++nr; }
    }
    (void)cf0;
    (void)cl;
    float s = 0.0f;
    for (int i = rf; i <= rl; ++i) {
      const int rb = sh.rb[i];
      const float f = sh.rf[i];
      float wy = 0.0f;
      if (rb == rbn) wy += a.ny > 1 ? 1.0f - f : 1.0f;
      if (a.ny > 1 && rb + 1 == rbn) wy += f;
      float rowsum = 0.0f;
#pragma unroll
      for (int q = 0; q < 3; ++q)
        rowsum += lw[q] * s_part[i][lc[q]][2 * term] + rw[q] * s_part[i][rc[q]][2 * term + 1];
      s += (sq ? wy * wy : wy) * rowsum;
    }
    const int idx = na * a.nx + nb;
    if (term < 2) {
      a.gU[(int64_t)pair * a.gstride + term * np + idx] = s;
    } else {
      if (a.D) a.D[(int64_t)pair * a.gstride + (term - 2) * np + idx] = s;
      dsum = s;
    }
  }
  if constexpr (kPart) {
    // fixed-order sums over the workgroup (bitwise reproducible)
    const float ls = tile_sum(lsum, s_red);
    const float ds = tile_sum(dsum, s_red);
    if (t == 0) {
      float* o = a.part + (int64_t)pair * a.pstride + 2 * (wg.y * ((a.nx + TN - 1) / TN) + wg.x);
      o[0] = ds;
      o[1] = ls;
    }
  }
}

SsdArgs make_args(const Plan& P, const float* A, const float* B, const float* U) {
  SsdArgs a;
  a.A = A;
  a.B = B;
  a.U = U;
  a.W = P.p.width;
  a.H = P.p.height;
  a.nx = P.nx;
  a.ny = P.ny;
  a.win = P.p.win;
  a.step = P.p.step;
  a.loss = nullptr;
  a.g = nullptr;
  a.gU = nullptr;
  a.D = nullptr;
  a.lstride = (int64_t)P.nx * P.ny;
  a.gstride = 2 * (int64_t)P.nx * P.ny;
  a.mask = P.slot_mask;
  a.part = nullptr;
  a.pstride = 0;
  return a;
}

// Refinement update, one workgroup per pair: the total window loss into the
// history, and U <- U - tau gU / (D + lambda) with lambda = lam_rel mean(D).
// Sums run in a fixed order (per-thread strided partials, then a fixed
// tree), so results are bitwise reproducible.  A node component whose
// D + lambda is not positive is left unchanged.
constexpr int kUpdT = 256;

__device__ __forceinline__ float block_sum(float x, float* red) {
  const int t = threadIdx.x;
  red[t] = x;
  __syncthreads();
#pragma unroll
  for (int o = kUpdT / 2; o > 0; o >>= 1) {
    if (t < o) red[t] += red[t + o];
    __syncthreads();
  }
  const float r = red[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(kUpdT) void k_ssd_update(float* U, const float* gU, const float* D,
                                                      const float* loss, int64_t wstride, int np, float tau,
                                                      float lam_rel, float* hist, int hstride, int k,
                                                      int update, const uint8_t* mask) {
  __shared__ float red[kUpdT];
  const int pair = blockIdx.x;
  if (slot_off(mask, pair)) return;
  const int t = threadIdx.x;
  if (hist) {
    const float* L = loss + (int64_t)pair * wstride;
    float s = 0.0f;
    for (int i = t; i < np; i += kUpdT) s += L[i];
    s = block_sum(s, red);
    if (t == 0) hist[(int64_t)pair * hstride + k] = s;
  }
  if (!update) return;
  const float* G = gU + (int64_t)pair * wstride;
  const float* Dp = D + (int64_t)pair * wstride;
  float* Up = U + (int64_t)pair * 2 * np;
  float s = 0.0f;
  for (int i = t; i < 2 * np; i += kUpdT) s += Dp[i];
  s = block_sum(s, red);
  const float lam = lam_rel * (s / (float)(2 * np));
  for (int i = t; i < 2 * np; i += kUpdT) {
    const float den = Dp[i] + lam;
    if (den > 0.0f) Up[i] -= tau * G[i] / den;
  }
}

// Refinement update from the adjoint's tile sums: every workgroup adds the
// pair's tile sums in the same fixed order (so all agree on lambda and the
// loss), the first writes the loss into the history, and each updates its
// share of U.
__global__ __launch_bounds__(kUpdT) void k_ssd_update_tiles(float* U, const float* gU, const float* D,
                                                            const float* part, int64_t wstride, int np, int ntiles,
                                                            float tau, float lam_rel, float* hist, int hstride,
                                                            int k, const uint8_t* mask) {
  __shared__ float red[kUpdT];
  const int pair = blockIdx.y;
  if (slot_off(mask, pair)) return;
  const int t = threadIdx.x;
  const float* pp = part + (int64_t)pair * wstride;
  float ds = 0.0f, ls = 0.0f;
  for (int i = t; i < ntiles; i += kUpdT) {
    ds += pp[2 * i];
    ls += pp[2 * i + 1];
  }
  ds = block_sum(ds, red);
  ls = block_sum(ls, red);
  if (hist && blockIdx.x == 0 && t == 0) hist[(int64_t)pair * hstride + k] = ls;
  const float lam = lam_rel * (ds / (float)(2 * np));
  const float* G = gU + (int64_t)pair * wstride;
  const float* Dp = D + (int64_t)pair * wstride;
  float* Up = U + (int64_t)pair * 2 * np;
  for (int i = blockIdx.x * kUpdT + t; i < 2 * np; i += gridDim.x * kUpdT) {
    const float den = Dp[i] + lam;
    if (den > 0.0f) Up[i] -= tau * G[i] / den;
  }
}

}  // namespace

hipError_t launch_ssd_forward(const Plan& P, const float* A, const float* B, const float* U, int n,
                              float* loss, hipStream_t s) {
  SsdArgs a = make_args(P, A, B, U);
  a.loss = loss;
  if (!loss) {   // the workspace's window losses
    a.loss = reinterpret_cast<float*>(P.ws + P.off_loss);
    a.lstride = (int64_t)(P.per_pair / sizeof(float));
  }
  // tile: at most 8 x 8 windows with a pixel region of at most 96 x 96
  if (a.step == 8 && a.win == 16) {
    dim3 grid((a.nx + 7) / 8, (a.ny + 7) / 8, n);
    hipLaunchKernelGGL((k_ssd_forward_t<8, 8>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  int TN = max(1, min(8, (96 - a.win) / a.step + 1));
  int RW = (TN - 1) * a.step + a.win;
  size_t lds = sizeof(float) * (size_t)RW * RW;
  dim3 grid((a.nx + TN - 1) / TN, (a.ny + TN - 1) / TN, n);
  hipLaunchKernelGGL(k_ssd_forward, grid, dim3(256), lds, s, a, TN);
  return hipGetLastError();
}

hipError_t launch_ssd_backward(const Plan& P, const float* A, const float* B, const float* U,
                               const float* g, int n, float* gU, float* D, hipStream_t s) {
  SsdArgs a = make_args(P, A, B, U);
  a.g = g;
  a.gU = gU;
  a.D = D;
  if (!gU) {   // the workspace's gradient and diagonal
    a.gU = reinterpret_cast<float*>(P.ws + P.off_gu);
    a.D = reinterpret_cast<float*>(P.ws + P.off_dd);
    a.gstride = (int64_t)(P.per_pair / sizeof(float));
  }
  if (a.step == 8 && a.win == 16) {
    dim3 grid((a.nx + 7) / 8, (a.ny + 7) / 8, n);
    hipLaunchKernelGGL((k_ssd_backward_t<8, 8, false>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
  }
  // 16 threads per node -> 16 nodes per workgroup; support region of a
  // 4 x 4 node tile spans (TN+1) step + h px plus edge extension
  const int TN = 4;
  const int h = (a.win - a.step) / 2;
  int RWmax = (TN + 1) * a.step + 2 * h + 2;
  size_t lds = sizeof(float) * 4 * (size_t)RWmax * RWmax;
  if (lds > 65536) return hipErrorInvalidValue;
  dim3 grid((a.nx + TN - 1) / TN, (a.ny + TN - 1) / TN, n);
  hipLaunchKernelGGL(k_ssd_backward, grid, dim3(256), lds, s, a, TN);
  return hipGetLastError();
}

bool ssd_tiled(const Plan& P) { return P.p.step == 8 && P.p.win == 16; }

hipError_t launch_ssd_refine_step(const Plan& P, const float* A, const float* B, float* U, int n, float tau,
                                  float lam_rel, float* hist, int hstride, int k, hipStream_t s) {
  SsdArgs a = make_args(P, A, B, U);
  a.gU = reinterpret_cast<float*>(P.ws + P.off_gu);
  a.D = reinterpret_cast<float*>(P.ws + P.off_dd);
  a.gstride = (int64_t)(P.per_pair / sizeof(float));
  a.part = reinterpret_cast<float*>(P.ws + P.off_part);
  a.pstride = a.gstride;
  dim3 grid((a.nx + 7) / 8, (a.ny + 7) / 8, n);
  hipLaunchKernelGGL((k_ssd_backward_t<8, 8, true>), grid, dim3(256), 0, s, a);
  if (hipError_t e = hipGetLastError()) return e;
  const int np = P.nx * P.ny;
  const int ntiles = (int)(grid.x * grid.y);
  dim3 gu((unsigned)max(1, min(64, (2 * np + 4 * kUpdT - 1) / (4 * kUpdT))), n);
  hipLaunchKernelGGL(k_ssd_update_tiles, gu, dim3(kUpdT), 0, s, U, a.gU, a.D, a.part, a.gstride, np, ntiles, tau,
                     lam_rel, hist, hstride, k, P.slot_mask);
  return hipGetLastError();
}

hipError_t launch_ssd_update(const Plan& P, float* U, int n, float tau, float lam_rel, float* hist, int hstride,
                             int k, int update, hipStream_t s) {
  const int64_t ws_f = (int64_t)(P.per_pair / sizeof(float));
  hipLaunchKernelGGL(k_ssd_update, dim3(n), dim3(kUpdT), 0, s, U,
                     reinterpret_cast<const float*>(P.ws + P.off_gu), reinterpret_cast<const float*>(P.ws + P.off_dd),
                     reinterpret_cast<const float*>(P.ws + P.off_loss), ws_f, P.nx * P.ny, tau, lam_rel, hist,
                     hstride, k, update, P.slot_mask);
  return hipGetLastError();
}

}  // namespace piv
