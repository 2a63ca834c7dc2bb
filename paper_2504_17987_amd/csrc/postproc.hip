// Validation (universal outlier detection with median replacement, Sec. 2
// and Sec. 3 of the paper) and vorticity on the vector grid.
#include "dev_common.h"
#include "piv_internal.h"

namespace piv {
namespace {

constexpr uint8_t kInvalid = PIV_F_FLAT | PIV_F_BORDER;

// Universal outlier detection and replacement, one workgroup per tile of
// TW x TH vectors.  Detection: FLAT/BORDER vectors are outliers and never
// neighbours; per component r0 = |u0 - med| / (med|u_j - med| + eps) over the
// usable 3x3 neighbours (centre excluded); outlier when the larger component
// value exceeds the threshold; no usable neighbour: kept.  Replacement:
// outliers take the component medians of their non-outlier neighbours from
// the detection-pass field; none -> kept, UNRESOLVED.
//
// The workgroup stages the field on its tile and two rings around it in LDS
// (one coalesced pass over global memory), detects on the tile and the first
// ring (the replacement of a tile vector needs the outcome of its
// neighbours), and writes the validated tile to a field other than its
// source, so that no workgroup reads what another one writes.
constexpr int TW = 64, TH = 16;             // tile; one thread per vector
constexpr int NT = TW * TH;
constexpr int E1W = TW + 2, E1H = TH + 2;   // detection region: tile + 1 ring
constexpr int E2W = TW + 4, E2H = TH + 4;   // staged field: tile + 2 rings

struct UodTile {
  float u[E2H][E2W], v[E2H][E2W];
  uint8_t ok[E2H][E2W];    // in the grid and not FLAT/BORDER
  uint8_t out[E1H][E1W];   // 1: outlier or outside the grid (never a usable neighbour)
  int n_out;               // outliers of the tile (the caller zeroes it before its barrier)
  uint16_t list[NT];       // their tile positions, in no particular order
};

__device__ __forceinline__ int clampi(int v, int hi) { return min(max(v, 0), hi); }

// One component of the detection test on a vector whose 8 neighbour slots
// hold k usable values (the rest the sentinel): med = their median, the
// residual median med|u_j - med|, and r0 = |x - med| / (residual median +
// eps) > thr, tested as |x - med| > thr (residual median + eps).
__device__ __forceinline__ bool uod_component_out(float (&s)[8], int k, float x, float thr, float eps) {
  sort8<8, float>(s);
  float um, rm;
  if (k == 8) {
    um = 0.5f * (s[3] + s[4]);
    // the residuals of the sorted values form two ascending runs, below the
    // median (a1..a4) and above it (b1..b4); their 4th and 5th smallest are
    // the least over the splits i + j = 4 (5) of max(a_i, b_j)
    const float a1 = um - s[3], a2 = um - s[2], a3 = um - s[1], a4 = um - s[0];
    const float b1 = s[4] - um, b2 = s[5] - um, b3 = s[6] - um, b4 = s[7] - um;
    const float r4 = fmin_fin(fmin_fin(fmin_fin(b4, a4), fmax_fin(a1, b3)),
                              fmin_fin(fmax_fin(a2, b2), fmax_fin(a3, b1)));
    const float r5 = fmin_fin(fmin_fin(fmax_fin(a1, b4), fmax_fin(a2, b3)),
                              fmin_fin(fmax_fin(a3, b2), fmax_fin(a4, b1)));
    rm = 0.5f * (r4 + r5);
  } else {
    um = (k & 1) ? pick<8>(s, k >> 1) : 0.5f * (pick<8>(s, (k >> 1) - 1) + pick<8>(s, k >> 1));
    float res[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) res[q] = fabsf(s[q] - um);
    rm = median8_f(res, k);
  }
  return fabsf(x - um) > thr * (rm + eps);
}

// Detection and replacement on a staged tile (the caller has filled u, v, ok
// and passed a barrier).  dst: the pair's output field [2][ny][nx]; fl: the
// pair's flags (nullable).
__device__ __forceinline__ void uod_tile(UodTile& T, int x0, int y0, int nx, int ny, float thr,
                                         float eps, float* dst, uint8_t* fl) {
  const int t = threadIdx.x;
  for (int idx = t; idx < E1H * E1W; idx += NT) {
    const int r = idx / E1W, c = idx - r * E1W;
    const int y = y0 - 1 + r, x = x0 - 1 + c;
    uint8_t o = 1;
    if (y >= 0 && x >= 0 && y < ny && x < nx && T.ok[r + 1][c + 1]) {
      // neighbours in static slots; unusable ones hold a sentinel that sorts last
      float v[2][8];
      int k = 0, slot = 0;
#pragma unroll
      for (int di = 0; di < 3; ++di)
#pragma unroll
        for (int dj = 0; dj < 3; ++dj) {
          if (di == 1 && dj == 1) continue;
          const bool ok = T.ok[r + di][c + dj];
          v[0][slot] = ok ? T.u[r + di][c + dj] : kSlotF;
          v[1][slot] = ok ? T.v[r + di][c + dj] : kSlotF;
          k += ok;
          ++slot;
        }
      if (k > 0)
        o = (int)uod_component_out(v[0], k, T.u[r + 1][c + 1], thr, eps) |
            (int)uod_component_out(v[1], k, T.v[r + 1][c + 1], thr, eps);   // both, no branch
      else
        o = 0;
    }
    T.out[r][c] = o;
    // outliers of the tile itself are replaced below, by consecutive threads
    if (o && r >= 1 && r <= TH && c >= 1 && c <= TW && y < ny && x < nx)
      T.list[atomicAdd(&T.n_out, 1)] = (uint16_t)((r - 1) * TW + c - 1);
  }
  __syncthreads();
  const int np = nx * ny;
  {
    const int ty = t / TW, tx = t - ty * TW, y = y0 + ty, x = x0 + tx;
    if (y < ny && x < nx && !T.out[ty + 1][tx + 1]) {
      dst[y * nx + x] = T.u[ty + 2][tx + 2];
      dst[np + y * nx + x] = T.v[ty + 2][tx + 2];
    }
  }
  const int n_out = T.n_out;
  for (int j = t; j < n_out; j += NT) {
    const int p = T.list[j], ty = p / TW, tx = p - ty * TW, i = (y0 + ty) * nx + x0 + tx;
    float vu[8], vv[8];
    int k = 0, slot = 0;
#pragma unroll
    for (int di = 0; di < 3; ++di)
#pragma unroll
      for (int dj = 0; dj < 3; ++dj) {
        if (di == 1 && dj == 1) continue;
        const bool ok = !T.out[ty + di][tx + dj];
        vu[slot] = ok ? T.u[ty + 1 + di][tx + 1 + dj] : kSlotF;
        vv[slot] = ok ? T.v[ty + 1 + di][tx + 1 + dj] : kSlotF;
        k += ok;
        ++slot;
      }
    float ru = T.u[ty + 2][tx + 2], rv = T.v[ty + 2][tx + 2];
    uint8_t f = PIV_F_OUTLIER;
    if (k == 0) {
      f |= PIV_F_UNRESOLVED;
    } else {
      ru = median8_f(vu, k);
      rv = median8_f(vv, k);
      f |= PIV_F_REPLACED;
    }
    if (fl) fl[i] |= f;
    dst[i] = ru;
    dst[np + i] = rv;
  }
}

// Validation of src (pair stride sstride floats) into dst ([n][2][ny][nx]).
// flags: in FLAT/BORDER, out + OUTLIER/REPLACED/UNRESOLVED.  Other workgroups
// read a flag byte this one updates only for its FLAT/BORDER bits, which the
// update leaves as they are.
template <bool HAS_FL>
__global__ __launch_bounds__(NT) void k_uod(const float* src, int64_t sstride, float* dst,
                                             uint8_t* flags, int nx, int ny, float thr, float eps,
                                             const uint8_t* smask) {
  __shared__ UodTile T;
  const int pair = blockIdx.z;
  if (slot_off(smask, pair)) return;
  const int x0 = blockIdx.x * TW, y0 = blockIdx.y * TH, t = threadIdx.x;
  const int np = nx * ny;
  const float* S = src + (int64_t)pair * sstride;
  uint8_t* FL = HAS_FL ? flags + (int64_t)pair * np : nullptr;
  // every load first (clamped, always valid addresses), then the LDS stores
  constexpr int NE = E2H * E2W, NP = (NE + NT - 1) / NT;
  float lu[NP], lv[NP];
  uint8_t lf[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const int idx = t + NT * q, r = idx / E2W, c = idx - r * E2W;
    const int o = clampi(y0 - 2 + r, ny - 1) * nx + clampi(x0 - 2 + c, nx - 1);
    lu[q] = S[o];
    lv[q] = S[np + o];
    lf[q] = HAS_FL ? FL[o] : 0;
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const int idx = t + NT * q, r = idx / E2W, c = idx - r * E2W;
    if (idx < NE) {
      const int y = y0 - 2 + r, x = x0 - 2 + c;
      T.u[r][c] = lu[q];
      T.v[r][c] = lv[q];
      T.ok[r][c] = y >= 0 && x >= 0 && y < ny && x < nx && !(lf[q] & kInvalid);
    }
  }
  if (t == 0) T.n_out = 0;
  __syncthreads();
  uod_tile(T, x0, y0, nx, ny, thr, eps, dst + (int64_t)pair * 2 * np, FL);
}

// Final level-0 predictor field -> validated float predictor: the 3x3 median
// (when enabled) on the tile and two rings, from the int32 field staged with
// three rings, then detection and replacement as above (no flags).
__global__ __launch_bounds__(NT) void k_pred_uod(const int32_t* d, int64_t dstride, int nx, int ny,
                                                  int median, float thr, float eps, float* pred,
                                                  const uint8_t* smask) {
  constexpr int E3W = TW + 6, E3H = TH + 6, NE = E3H * E3W, NP = (NE + NT - 1) / NT;
  __shared__ int sd[2][E3H][E3W];
  __shared__ UodTile T;
  const int pair = blockIdx.z;
  if (slot_off(smask, pair)) return;
  const int x0 = blockIdx.x * TW, y0 = blockIdx.y * TH, t = threadIdx.x;
  const int np = nx * ny;
  const int32_t* D = d + (int64_t)pair * dstride;
  int lu[NP], lv[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const int idx = t + NT * q, r = idx / E3W, c = idx - r * E3W;
    const int o = clampi(y0 - 3 + r, ny - 1) * nx + clampi(x0 - 3 + c, nx - 1);
    lu[q] = D[o];
    lv[q] = D[np + o];
  }
#pragma unroll
  for (int q = 0; q < NP; ++q) {
    const int idx = t + NT * q, r = idx / E3W, c = idx - r * E3W;
    if (idx < NE) {
      const int y = y0 - 3 + r, x = x0 - 3 + c;
      const bool in = y >= 0 && x >= 0 && y < ny && x < nx;
      sd[0][r][c] = in ? lu[q] : kSlotI;
      sd[1][r][c] = in ? lv[q] : kSlotI;
    }
  }
  if (t == 0) T.n_out = 0;
  __syncthreads();
  for (int idx = t; idx < E2H * E2W; idx += NT) {
    const int r = idx / E2W, c = idx - r * E2W;
    const int y = y0 - 2 + r, x = x0 - 2 + c;
    const bool in = y >= 0 && x >= 0 && y < ny && x < nx;
    int val[2] = {sd[0][r + 1][c + 1], sd[1][r + 1][c + 1]};
    if (in && median) {
      // in-grid count of the 3x3; out-of-grid slots hold the sentinel
      const int k = (3 - (y == 0) - (y == ny - 1)) * (3 - (x == 0) - (x == nx - 1));
#pragma unroll
      for (int comp = 0; comp < 2; ++comp) {
        int v[9];
#pragma unroll
        for (int di = 0; di < 3; ++di)
#pragma unroll
          for (int dj = 0; dj < 3; ++dj) v[di * 3 + dj] = sd[comp][r + di][c + dj];
        val[comp] = median9_low_i(v, k);
      }
    }
    T.u[r][c] = (float)val[0];
    T.v[r][c] = (float)val[1];
    T.ok[r][c] = in;
  }
  __syncthreads();
  uod_tile(T, x0, y0, nx, ny, thr, eps, pred + (int64_t)pair * 2 * np, nullptr);
}

__device__ __forceinline__ float dline(const float* f, int n, int stride, int i, float h) {
  if (n == 1) return 0.0f;
  if (n == 2) return (f[stride] - f[0]) / h;
  if (i == 0) return (-3.0f * f[0] + 4.0f * f[stride] - f[2 * stride]) / (2.0f * h);
  if (i == n - 1) return (3.0f * f[i * stride] - 4.0f * f[(i - 1) * stride] + f[(i - 2) * stride]) / (2.0f * h);
  return (f[(i + 1) * stride] - f[(i - 1) * stride]) / (2.0f * h);
}

__global__ __launch_bounds__(256) void k_vorticity(const float* disp, float* omega, int nx, int ny,
                                                   float h, const uint8_t* smask) {
  const int pair = blockIdx.y;
  if (slot_off(smask, pair)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int np = nx * ny;
  if (i >= np) return;
  const int a = i / nx, b = i - a * nx;
  const float* U = disp + (int64_t)pair * 2 * np;
  const float* V = U + np;
  float dvdx = dline(V + a * nx, nx, 1, b, h);
  float dudy = dline(U + b, ny, nx, a, h);
  omega[(int64_t)pair * np + i] = dvdx - dudy;
}

// Exponential smoothing in time (Sec. 2: constants alpha1 on the validated
// predictor, alpha2 on the validated final field).  One thread per field
// element walks the batch in order, so that pairs of one state slot (frames
// of one stream) chain: slot k >= 0 continues, s_k <- alpha x + (1 - alpha)
// s_k; slot -1 - k starts, s_k <- x; the field takes s_k.  Slots outside
// [0, nstate) leave their pair untouched.
__global__ __launch_bounds__(256) void k_smooth(float* field, float* state, const int32_t* slot, int nstate,
                                                float alpha, int n, int np2, const uint8_t* smask) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= np2) return;
  const float beta = 1.0f - alpha;
  for (int i = 0; i < n; ++i) {
    if (slot_off(smask, i)) continue;
    int k = slot[i];
    const bool first = k < 0;
    if (first) k = -1 - k;
    if (k >= nstate) continue;
    float* st = state + (int64_t)k * np2 + j;
    float* f = field + (int64_t)i * np2 + j;
    const float x = *f;
    const float y = first ? x : alpha * x + beta * *st;
    *st = y;
    *f = y;
  }
}

}  // namespace

hipError_t launch_smooth(const Plan& P, float* field, float* state, const int32_t* slot, int nstate, float alpha,
                         int n, hipStream_t s) {
  const int np2 = 2 * P.nx * P.ny;
  hipLaunchKernelGGL(k_smooth, dim3((np2 + 255) / 256), dim3(256), 0, s, field, state, slot, nstate, alpha, n, np2,
                     P.slot_mask);
  return hipGetLastError();
}

hipError_t launch_uod(const Plan& P, const float* src, int64_t sstride, float* dst, uint8_t* flags,
                      int n, hipStream_t s) {
  dim3 grid((P.nx + TW - 1) / TW, (P.ny + TH - 1) / TH, n);
  if (flags)
    hipLaunchKernelGGL(k_uod<true>, grid, dim3(NT), 0, s, src, sstride, dst, flags, P.nx, P.ny,
                       P.p.uod_threshold, P.p.uod_epsilon, P.slot_mask);
  else
    hipLaunchKernelGGL(k_uod<false>, grid, dim3(NT), 0, s, src, sstride, dst, flags, P.nx, P.ny,
                       P.p.uod_threshold, P.p.uod_epsilon, P.slot_mask);
  return hipGetLastError();
}

hipError_t launch_validate(const Plan& P, float* field, uint8_t* flags, int n, hipStream_t s) {
  // in place: the detection-pass field goes to the workspace first
  const size_t bytes = sizeof(float) * 2 * (size_t)P.nx * P.ny;
  if (hipError_t e = hipMemcpy2DAsync(P.ws + P.off_raw, P.per_pair, field, bytes, bytes, n,
                                      hipMemcpyDeviceToDevice, s))
    return e;
  return launch_uod(P, reinterpret_cast<const float*>(P.ws + P.off_raw),
                    (int64_t)(P.per_pair / sizeof(float)), field, flags, n, s);
}

hipError_t launch_pred_validate(const Plan& P, int n, float* pred, hipStream_t s) {
  const Level& v = P.lv[0];
  dim3 grid((v.nx + TW - 1) / TW, (v.ny + TH - 1) / TH, n);
  hipLaunchKernelGGL(k_pred_uod, grid, dim3(NT), 0, s, reinterpret_cast<const int32_t*>(P.ws + v.off_d),
                     (int64_t)(P.per_pair / sizeof(int32_t)), v.nx, v.ny, P.p.median,
                     P.p.uod_threshold, P.p.uod_epsilon, pred, P.slot_mask);
  return hipGetLastError();
}

hipError_t launch_vorticity(const Plan& P, const float* disp, float* omega, int n, hipStream_t s) {
  const int np = P.nx * P.ny;
  dim3 grid((np + 255) / 256, n);
  hipLaunchKernelGGL(k_vorticity, grid, dim3(256), 0, s, disp, omega, P.nx, P.ny, (float)P.p.step,
                     P.slot_mask);
  return hipGetLastError();
}

}  // namespace piv
