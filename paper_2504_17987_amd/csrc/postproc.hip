// Validation (universal outlier detection with median replacement, Sec. 2
// and Sec. 3 of the paper) and vorticity on the vector grid.
#include "dev_common.h"
#include "piv_internal.h"

namespace piv {
namespace {

constexpr uint8_t kInvalid = PIV_F_FLAT | PIV_F_BORDER;

// Detection: mask[i] = 1 for an outlier.  FLAT/BORDER vectors are outliers
// and never neighbours.  Per component r0 = |u0 - med| / (med|u_j - med| + eps)
// over the valid 3x3 neighbours (centre excluded); outlier when the larger
// component value exceeds the threshold.  No valid neighbour: kept.
__global__ __launch_bounds__(256) void k_uod_detect(const float* field, const uint8_t* flags, int nx,
                                                    int ny, float thr, float eps, uint8_t* ws,
                                                    int64_t ws_stride, int64_t off_mask,
                                                    const uint8_t* smask) {
  const int pair = blockIdx.y;
  if (slot_off(smask, pair)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int np = nx * ny;
  if (i >= np) return;
  const int a = i / nx, b = i - a * nx;
  const float* F = field + (int64_t)pair * 2 * np;
  const uint8_t* FL = flags ? flags + (int64_t)pair * np : nullptr;
  uint8_t* mask = ws + (int64_t)pair * ws_stride + off_mask;
  if (FL && (FL[i] & kInvalid)) {
    mask[i] = 1;
    return;
  }
  // neighbours in static slots; unusable ones hold a sentinel that sorts last
  float v[2][8];
  int k = 0, slot = 0;
#pragma unroll
  for (int di = -1; di <= 1; ++di)
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
      if (di == 0 && dj == 0) continue;
      int y = a + di, x = b + dj;
      bool ok = y >= 0 && x >= 0 && y < ny && x < nx;
      if (ok && FL) ok = !(FL[y * nx + x] & kInvalid);
      v[0][slot] = ok ? F[y * nx + x] : kSlotF;
      v[1][slot] = ok ? F[np + y * nx + x] : kSlotF;
      k += ok;
      ++slot;
    }
  uint8_t out = 0;
  if (k > 0) {
    float worst = 0.0f;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      float vals[8], res[8];
#pragma unroll
      for (int s = 0; s < 8; ++s) vals[s] = v[c][s];
#pragma unroll
      for (int s = 0; s < 8; ++s) res[s] = v[c][s];
      float um = median8_f(vals, k);
#pragma unroll
      for (int s = 0; s < 8; ++s) res[s] = fabsf(res[s] - um);
      float rm = median8_f(res, k);
      float r0 = fabsf(F[c * np + i] - um) / (rm + eps);
      worst = fmaxf(worst, r0);
    }
    out = worst > thr;
  }
  mask[i] = out;
}

// Replacement from the detection-pass field: outliers take the component
// medians of their non-outlier neighbours; none -> kept, UNRESOLVED.
// Non-outlier values are never written, so the in-place update reads only
// values of the detection pass.
__global__ __launch_bounds__(256) void k_uod_replace(float* field, uint8_t* flags, int nx, int ny,
                                                     const uint8_t* ws, int64_t ws_stride,
                                                     int64_t off_mask, const uint8_t* smask) {
  const int pair = blockIdx.y;
  if (slot_off(smask, pair)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int np = nx * ny;
  if (i >= np) return;
  const int a = i / nx, b = i - a * nx;
  float* F = field + (int64_t)pair * 2 * np;
  uint8_t* FL = flags ? flags + (int64_t)pair * np : nullptr;
  const uint8_t* mask = ws + (int64_t)pair * ws_stride + off_mask;
  if (!mask[i]) return;
  float v[2][8];
  int k = 0, slot = 0;
#pragma unroll
  for (int di = -1; di <= 1; ++di)
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj) {
      if (di == 0 && dj == 0) continue;
      int y = a + di, x = b + dj;
      bool ok = y >= 0 && x >= 0 && y < ny && x < nx && !mask[y * nx + x];
      v[0][slot] = ok ? F[y * nx + x] : kSlotF;
      v[1][slot] = ok ? F[np + y * nx + x] : kSlotF;
      k += ok;
      ++slot;
    }
  uint8_t fl = PIV_F_OUTLIER;
  if (k == 0) {
    fl |= PIV_F_UNRESOLVED;
  } else {
    float vu[8], vv[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      vu[s] = v[0][s];
      vv[s] = v[1][s];
    }
    F[i] = median8_f(vu, k);
    F[np + i] = median8_f(vv, k);
    fl |= PIV_F_REPLACED;
  }
  if (FL) FL[i] |= fl;
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

}  // namespace

hipError_t launch_validate(const Plan& P, float* field, uint8_t* flags, int n, hipStream_t s) {
  const int np = P.nx * P.ny;
  dim3 grid((np + 255) / 256, n);
  hipLaunchKernelGGL(k_uod_detect, grid, dim3(256), 0, s, field, flags, P.nx, P.ny, P.p.uod_threshold,
                     P.p.uod_epsilon, P.ws, (int64_t)P.per_pair, (int64_t)P.off_mask, P.slot_mask);
  if (hipError_t e = hipGetLastError()) return e;
  hipLaunchKernelGGL(k_uod_replace, grid, dim3(256), 0, s, field, flags, P.nx, P.ny, P.ws,
                     (int64_t)P.per_pair, (int64_t)P.off_mask, P.slot_mask);
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
