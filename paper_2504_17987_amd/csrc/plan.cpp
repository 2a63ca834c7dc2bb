// Host side of libpiv: parameter validation, plan and workspace layout,
// entry points of the C ABI (declared in include/piv.h).
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "piv_internal.h"

using piv::Plan;

namespace {

thread_local char g_err[512] = "";

piv_status fail(piv_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return s;
}

piv_status dev(hipError_t e, const char* what) {
  if (e == hipSuccess) return PIV_OK;
  return fail(PIV_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

const Plan* cplan(piv_plan_t p) { return reinterpret_cast<const Plan*>(p); }
Plan* mplan(piv_plan_t p) { return reinterpret_cast<Plan*>(p); }

piv_status check_images(const Plan& P, const void* A, const void* B, int64_t pitch, int32_t n) {
  if (!A || !B) return fail(PIV_EINVAL, "image pointers must not be NULL");
  if (n < 0 || n > P.p.max_batch) return fail(PIV_EINVAL, "n=%d outside [0, max_batch=%d]", n, P.p.max_batch);
  if (pitch < (int64_t)P.p.width * P.es) return fail(PIV_EINVAL, "pitch_bytes %lld < width*elem", (long long)pitch);
  if (pitch % 4) return fail(PIV_EINVAL, "pitch_bytes must be a multiple of 4");
  if (((uintptr_t)A | (uintptr_t)B) & 3) return fail(PIV_EINVAL, "image pointers must be 4-byte aligned");
  return PIV_OK;
}

piv_status need_ws(const Plan& P, int32_t n) {
  if (!P.ws) return fail(PIV_ENOWORKSPACE, "no workspace bound");
  if (n > P.ws_pairs) return fail(PIV_ENOWORKSPACE, "workspace holds %d pairs, n=%d", P.ws_pairs, n);
  return PIV_OK;
}

}  // namespace

extern "C" {

void piv_params_default(piv_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->width = 1024;
  p->height = 1024;
  p->max_batch = 1;
  p->dtype = PIV_U8;
  p->bit_depth = 8;
  p->win = 16;
  p->step = 8;
  p->radius = 4;
  p->levels = 3;
  p->block = 0;
  p->radius_coarse = 6;
  p->radius_fine = 2;
  p->median = 1;
  p->warp = PIV_WARP_B;
  p->peak = PIV_PEAK_ARGMAX;
  p->uod_threshold = 2.0f;
  p->uod_epsilon = 0.1f;
  p->sgm = 0;
  p->sgm_p1 = 2;
  p->sgm_p2 = 16;
}

piv_status piv_plan(const piv_params* pp, piv_plan_t* out) {
  if (!out) return fail(PIV_EINVAL, "out is NULL");
  *out = nullptr;
  if (!pp) return fail(PIV_EINVAL, "params is NULL");
  const piv_params& p = *pp;
  if (p.width <= 0 || p.height <= 0) return fail(PIV_EINVAL, "image size must be positive");
  if (p.max_batch <= 0 || p.max_batch > 16384) return fail(PIV_EINVAL, "max_batch outside [1, 16384]");
  int es = p.dtype == PIV_U8 ? 1 : p.dtype == PIV_U16 ? 2 : p.dtype == PIV_F32 ? 4 : 0;
  if (!es) return fail(PIV_EINVAL, "unknown dtype %d", (int)p.dtype);
  if (p.dtype == PIV_U16 && p.bit_depth != 12 && p.bit_depth != 16)
    return fail(PIV_EINVAL, "U16 bit_depth must be 12 or 16");
  if (p.step <= 0 || p.win <= 0) return fail(PIV_EINVAL, "win and step must be positive");
  if (p.win < p.step) return fail(PIV_EINVAL, "win (%d) < step (%d)", p.win, p.step);
  if ((p.win - p.step) % 2) return fail(PIV_EINVAL, "win - step must be even");
  if (p.win > 64) return fail(PIV_EINVAL, "win > 64");
  if (p.width % p.step || p.height % p.step)
    return fail(PIV_EINVAL, "width and height must be multiples of step");
  if (p.radius < 1 || p.radius > 16) return fail(PIV_EINVAL, "radius outside [1, 16]");
  if (p.levels < 1 || p.levels > piv::kMaxLevels) return fail(PIV_EINVAL, "levels outside [1, 6]");
  if (p.warp != PIV_WARP_B && p.warp != PIV_WARP_CENTRAL) return fail(PIV_EINVAL, "bad warp mode");
  if (p.peak != PIV_PEAK_ARGMAX && p.peak != PIV_PEAK_FIXED_CENTER) return fail(PIV_EINVAL, "bad peak mode");
  if (!(p.uod_threshold > 0) || !(p.uod_epsilon >= 0)) return fail(PIV_EINVAL, "bad UOD parameters");
  int block = p.block ? p.block : p.win;
  if (block < p.step || (block - p.step) % 2) return fail(PIV_EINVAL, "block must be >= step with block - step even");
  if (block > 64) return fail(PIV_EINVAL, "block > 64");
  if (p.radius_coarse < 0 || p.radius_coarse > 16 || p.radius_fine < 0 || p.radius_fine > 16)
    return fail(PIV_EINVAL, "predictor radii outside [0, 16]");
  // largest predictor displacement: Rc 2^(L-1) + Rf (2^(L-1) - 1); keys hold |d| <= 127
  long reach = (long)p.radius_coarse * (1L << (p.levels - 1)) + (long)p.radius_fine * ((1L << (p.levels - 1)) - 1);
  if (reach > 127) return fail(PIV_EINVAL, "predictor reach %ld px exceeds 127", reach);
  if (p.sgm != 0 && p.sgm != 1) return fail(PIV_EINVAL, "sgm must be 0 or 1");
  if (p.sgm && (p.sgm_p1 < 0 || p.sgm_p1 > 255 || p.sgm_p2 < 0 || p.sgm_p2 > 255))
    return fail(PIV_EINVAL, "sgm penalties outside [0, 255]");
  if (p.sgm && p.radius_coarse < 1) return fail(PIV_EINVAL, "semi-global matching needs radius_coarse >= 1");
  if (p.sgm && p.dtype == PIV_F32) return fail(PIV_EUNSUPPORTED, "the predictor takes U8/U16 frames");
  if (p.dtype == PIV_F32 && p.levels > 1)
    return fail(PIV_EUNSUPPORTED, "the integer predictor takes U8/U16 frames (F32 is for the SSD path)");
  if ((block * es) % 4) return fail(PIV_EUNSUPPORTED, "block*bytes_per_pixel must be a multiple of 4");
  if (p.dtype != PIV_F32 && !piv::sad_supported(block * es / 4))
    return fail(PIV_EUNSUPPORTED, "predictor block of %d bytes per row is not built", block * es);

  Plan* P = new (std::nothrow) Plan();
  if (!P) return fail(PIV_EINVAL, "out of host memory");
  P->p = p;
  P->es = es;
  P->block = block;
  P->L = p.levels;
  P->nx = p.width / p.step;
  P->ny = p.height / p.step;
  size_t off = 0;
  for (int l = 0; l < P->L; ++l) {
    piv::Level& v = P->lv[l];
    if (l == 0) {
      v.W = p.width; v.H = p.height; v.nx = P->nx; v.ny = P->ny;
    } else {
      const piv::Level& u = P->lv[l - 1];
      v.W = (u.W + 1) / 2; v.H = (u.H + 1) / 2;
      v.nx = (u.nx + 1) / 2; v.ny = (u.ny + 1) / 2;
    }
    v.R = l == P->L - 1 ? p.radius_coarse : p.radius_fine;
  }
  // search reach per level: |cand_l| <= 2 maxd_{l+1}, maxd_l = R_l + |cand_l|
  int maxd = 0;
  for (int l = P->L - 1; l >= 0; --l) {
    piv::Level& v = P->lv[l];
    int cand = l == P->L - 1 ? 0 : 2 * maxd;
    maxd = cand + v.R;
    // node grid may overhang the image by < step; block offset (block-step)/2;
    // word-granular loads read up to 8 bytes past the search span
    int m = p.step + (block - p.step) / 2 + cand + v.R + 8;
    v.margin = (m + 15) & ~15;   // 16 px: every level's core starts 16-byte aligned
    v.pitch = (int)((size_t)((v.W + 2 * v.margin) * es + 63) & ~size_t(63));
    v.rows = v.H + 2 * v.margin;
  }
  for (int l = 0; l < P->L; ++l) {
    piv::Level& v = P->lv[l];
    if (p.dtype == PIV_F32) { v.off_a = v.off_b = 0; continue; }   // no predictor on F32 plans
    v.off_a = off; off = align256(off + (size_t)v.pitch * v.rows);
    v.off_b = off; off = align256(off + (size_t)v.pitch * v.rows);
  }
  for (int l = 0; l < P->L; ++l) {
    piv::Level& v = P->lv[l];
    v.off_d = off;
    off = align256(off + sizeof(int32_t) * 2 * (size_t)v.nx * v.ny);
  }
  P->off_raw = off;
  off = align256(off + sizeof(float) * 2 * (size_t)P->nx * P->ny);
  if (p.sgm) {
    const piv::Level& c = P->lv[P->L - 1];
    const size_t cells = (size_t)c.nx * c.ny * (size_t)(2 * c.R + 1) * (2 * c.R + 1);
    P->off_sgm_c = off;
    off = align256(off + sizeof(uint32_t) * cells);
    P->off_sgm_s = off;
    off = align256(off + sizeof(uint32_t) * cells);
  }
  if (p.dtype == PIV_F32) {
    const size_t np = (size_t)P->nx * P->ny;
    P->off_gu = off;
    off = align256(off + sizeof(float) * 2 * np);
    P->off_dd = off;
    off = align256(off + sizeof(float) * 2 * np);
    P->off_loss = off;
    off = align256(off + sizeof(float) * np);
    P->off_part = off;   // per node tile of 8 x 8: two floats
    off = align256(off + sizeof(float) * 2 * (size_t)((P->nx + 7) / 8) * ((P->ny + 7) / 8));
  }
  P->per_pair = off;
  *out = reinterpret_cast<piv_plan_t>(P);
  g_err[0] = 0;
  return PIV_OK;
}

piv_status piv_plan_grid(piv_plan_t plan, int32_t* nx, int32_t* ny) {
  if (!plan) return fail(PIV_EINVAL, "plan is NULL");
  if (nx) *nx = cplan(plan)->nx;
  if (ny) *ny = cplan(plan)->ny;
  return PIV_OK;
}

size_t piv_plan_workspace_bytes(piv_plan_t plan, int32_t batch) {
  if (!plan || batch < 0) return 0;
  return cplan(plan)->per_pair * (size_t)batch;
}

piv_status piv_plan_bind_workspace(piv_plan_t plan, void* d_ws, size_t bytes, hipStream_t stream) {
  if (!plan) return fail(PIV_EINVAL, "plan is NULL");
  Plan* P = mplan(plan);
  if (d_ws && ((uintptr_t)d_ws & 255)) return fail(PIV_EINVAL, "workspace must be 256-byte aligned");
  const size_t cap = d_ws ? bytes / P->per_pair : 0;
  if (d_ws && cap == 0)
    return fail(PIV_ENOWORKSPACE, "workspace of %zu bytes holds no pair (need %zu)", bytes, P->per_pair);
  // calls never pass more than max_batch pairs
  const int pairs = (int)(cap < (size_t)P->p.max_batch ? cap : (size_t)P->p.max_batch);
  if (d_ws) {
    // the pyramid margins are zeroed here, once, so that every later call
    // only reads the plan (and may be captured into a graph)
    if (piv_status s = dev(piv::launch_clear_margins(*P, static_cast<uint8_t*>(d_ws), pairs, stream),
                           "clear_margins"))
      return s;
  }
  P->ws = static_cast<uint8_t*>(d_ws);
  P->ws_bytes = d_ws ? bytes : 0;
  P->ws_pairs = pairs;
  return PIV_OK;
}

piv_status piv_plan_bind_slot_mask(piv_plan_t plan, const uint8_t* d_mask) {
  if (!plan) return fail(PIV_EINVAL, "plan is NULL");
  mplan(plan)->slot_mask = d_mask;
  return PIV_OK;
}

void piv_plan_destroy(piv_plan_t plan) { delete mplan(plan); }

piv_status piv_predict(piv_plan_t plan, const void* A, const void* B, int64_t pitch, int32_t n,
                       float* pred, hipStream_t stream) {
  if (!plan) return fail(PIV_EINVAL, "plan is NULL");
  const Plan& P = *cplan(plan);
  if (piv_status s = check_images(P, A, B, pitch, n)) return s;
  if (!pred) return fail(PIV_EINVAL, "pred must not be NULL");
  if (P.p.dtype == PIV_F32) return fail(PIV_EUNSUPPORTED, "the predictor takes U8/U16 frames");
  if (piv_status s = need_ws(P, n)) return s;
  if (n == 0) return PIV_OK;
  if (piv_status s = dev(piv::launch_pyramid(P, A, B, pitch, n, stream), "pyramid")) return s;
  for (int l = P.L - 1; l >= 0; --l)
    if (piv_status s = dev(piv::launch_sad_level(P, l, A, B, pitch, n, stream), "sad_search")) return s;
  return dev(piv::launch_pred_out(P, n, pred, stream), "pred_out");
}

piv_status piv_correct(piv_plan_t plan, const void* A, const void* B, int64_t pitch, int32_t n,
                       const float* pred, float* disp, float* peak, uint8_t* flags,
                       hipStream_t stream) {
  if (!plan) return fail(PIV_EINVAL, "plan is NULL");
  const Plan& P = *cplan(plan);
  if (piv_status s = check_images(P, A, B, pitch, n)) return s;
  if (!disp || !flags) return fail(PIV_EINVAL, "disp and flags must not be NULL");
  if (n == 0) return PIV_OK;
  return dev(piv::launch_correct(P, A, B, pitch, n, pred, disp, peak, flags, stream), "correct");
}

piv_status piv_validate(piv_plan_t plan, float* field, uint8_t* flags, int32_t n, hipStream_t stream) {
  if (!plan) return fail(PIV_EINVAL, "plan is NULL");
  const Plan& P = *cplan(plan);
  if (!field) return fail(PIV_EINVAL, "field must not be NULL");
  if (n < 0 || n > P.p.max_batch) return fail(PIV_EINVAL, "n=%d outside [0, max_batch]", n);
  if (piv_status s = need_ws(P, n)) return s;
  if (n == 0) return PIV_OK;
  return dev(piv::launch_validate(P, field, flags, n, stream), "validate");
}

piv_status piv_vorticity(piv_plan_t plan, const float* disp, float* omega, int32_t n, hipStream_t stream) {
  if (!plan) return fail(PIV_EINVAL, "plan is NULL");
  const Plan& P = *cplan(plan);
  if (!disp || !omega) return fail(PIV_EINVAL, "disp and omega must not be NULL");
  if (n < 0 || n > P.p.max_batch) return fail(PIV_EINVAL, "n=%d outside [0, max_batch]", n);
  if (n == 0) return PIV_OK;
  return dev(piv::launch_vorticity(P, disp, omega, n, stream), "vorticity");
}

namespace {

// The steps of piv_run (and of piv_run_temporal with smoothing states): the
// predictor's output step and its validation are one kernel, and the
// correction writes the detection-pass field to the workspace, from which
// validation writes disp.
struct Temporal {
  const int32_t* slot;
  int32_t nstate;
  float* state_pred;
  float* state_disp;
  float alpha1, alpha2;
};

piv_status run_path(const Plan& P, const void* A, const void* B, int64_t pitch, int32_t n, float* pred,
                    float* disp, float* peak, uint8_t* flags, float* omega, const Temporal* tm,
                    hipStream_t stream) {
  if (piv_status s = dev(piv::launch_pyramid(P, A, B, pitch, n, stream), "pyramid")) return s;
  for (int l = P.L - 1; l >= 0; --l)
    if (piv_status s = dev(piv::launch_sad_level(P, l, A, B, pitch, n, stream), "sad_search")) return s;
  if (piv_status s = dev(piv::launch_pred_validate(P, n, pred, stream), "pred_validate")) return s;
  if (tm && tm->state_pred)
    if (piv_status s = dev(piv::launch_smooth(P, pred, tm->state_pred, tm->slot, tm->nstate, tm->alpha1, n,
                                              stream), "smooth_pred"))
      return s;
  float* raw = reinterpret_cast<float*>(P.ws + P.off_raw);
  const int64_t rstride = (int64_t)(P.per_pair / sizeof(float));
  if (piv_status s = dev(piv::launch_correct(P, A, B, pitch, n, pred, raw, peak, flags, stream, rstride),
                         "correct"))
    return s;
  if (piv_status s = dev(piv::launch_uod(P, raw, rstride, disp, flags, n, stream), "validate")) return s;
  if (tm && tm->state_disp)
    if (piv_status s = dev(piv::launch_smooth(P, disp, tm->state_disp, tm->slot, tm->nstate, tm->alpha2, n,
                                              stream), "smooth_disp"))
      return s;
  return dev(piv::launch_vorticity(P, disp, omega, n, stream), "vorticity");
}

piv_status check_run(const Plan& P, const void* A, const void* B, int64_t pitch, int32_t n, float* pred,
                     float* disp, uint8_t* flags, float* omega) {
  if (piv_status s = check_images(P, A, B, pitch, n)) return s;
  if (!pred || !disp || !flags || !omega) return fail(PIV_EINVAL, "pred, disp, flags, omega must not be NULL");
  if (P.p.dtype == PIV_F32) return fail(PIV_EUNSUPPORTED, "the predictor takes U8/U16 frames");
  return need_ws(P, n);
}

piv_status check_alpha(float a, const char* name) {
  if (!(a > 0.0f && a <= 1.0f)) return fail(PIV_EINVAL, "%s=%g outside (0, 1]", name, (double)a);
  return PIV_OK;
}

}  // namespace

extern "C++" {
namespace piv {

piv_status check_on_workspace(const Plan& P, size_t ws_bytes, const void* A, const void* B, int64_t pitch,
                              int32_t n, float* pred, float* disp, uint8_t* flags, float* omega) {
  if (piv_status s = check_images(P, A, B, pitch, n)) return s;
  if (!pred || !disp || !flags || !omega) return fail(PIV_EINVAL, "pred, disp, flags, omega must not be NULL");
  if (P.p.dtype == PIV_F32) return fail(PIV_EUNSUPPORTED, "the predictor takes U8/U16 frames");
  if ((size_t)n * P.per_pair > ws_bytes)
    return fail(PIV_ENOWORKSPACE, "%d pairs need %zu bytes of workspace, the scratch holds %zu", n,
                (size_t)n * P.per_pair, ws_bytes);
  return PIV_OK;
}

piv_status run_on_workspace(const Plan& P, uint8_t* ws, size_t ws_bytes, const void* A, const void* B,
                            int64_t pitch, int32_t n, float* pred, float* disp, float* peak, uint8_t* flags,
                            float* omega, hipStream_t stream) {
  if (piv_status s = check_on_workspace(P, ws_bytes, A, B, pitch, n, pred, disp, flags, omega)) return s;
  if (n == 0) return PIV_OK;
  Plan Q = P;   // host copy: the same geometry on the given workspace
  Q.ws = ws;
  Q.ws_bytes = ws_bytes;
  Q.ws_pairs = n;
  // the memory holds whatever the previous call left: zero the margins first
  if (piv_status s = dev(launch_clear_margins(Q, ws, n, stream), "clear_margins")) return s;
  return run_path(Q, A, B, pitch, n, pred, disp, peak, flags, omega, nullptr, stream);
}

piv_status set_error(piv_status s, const char* msg) { return fail(s, "%s", msg); }

}  // namespace piv
}  // extern "C++"

piv_status piv_run(piv_plan_t plan, const void* A, const void* B, int64_t pitch, int32_t n,
                   float* pred, float* disp, float* peak, uint8_t* flags, float* omega,
                   hipStream_t stream) {
  if (!plan) return fail(PIV_EINVAL, "plan is NULL");
  const Plan& P = *cplan(plan);
  if (piv_status s = check_run(P, A, B, pitch, n, pred, disp, flags, omega)) return s;
  if (n == 0) return PIV_OK;
  return run_path(P, A, B, pitch, n, pred, disp, peak, flags, omega, nullptr, stream);
}

piv_status piv_smooth(piv_plan_t plan, float* field, float* state, const int32_t* slot, int32_t nstate,
                      float alpha, int32_t n, hipStream_t stream) {
  if (!plan) return fail(PIV_EINVAL, "plan is NULL");
  const Plan& P = *cplan(plan);
  if (!field || !state || !slot) return fail(PIV_EINVAL, "field, state and slot must not be NULL");
  if (n < 0 || n > P.p.max_batch) return fail(PIV_EINVAL, "n=%d outside [0, max_batch]", n);
  if (nstate <= 0) return fail(PIV_EINVAL, "nstate must be positive");
  if (piv_status s = check_alpha(alpha, "alpha")) return s;
  if (n == 0) return PIV_OK;
  return dev(piv::launch_smooth(P, field, state, slot, nstate, alpha, n, stream), "smooth");
}

piv_status piv_run_temporal(piv_plan_t plan, const void* A, const void* B, int64_t pitch, int32_t n,
                            const int32_t* slot, int32_t nstate, float* state_pred, float* state_disp,
                            float alpha1, float alpha2, float* pred, float* disp, float* peak,
                            uint8_t* flags, float* omega, hipStream_t stream) {
  if (!plan) return fail(PIV_EINVAL, "plan is NULL");
  const Plan& P = *cplan(plan);
  if (piv_status s = check_run(P, A, B, pitch, n, pred, disp, flags, omega)) return s;
  if (!slot) return fail(PIV_EINVAL, "slot must not be NULL");
  if (nstate <= 0) return fail(PIV_EINVAL, "nstate must be positive");
  if (state_pred)
    if (piv_status s = check_alpha(alpha1, "alpha1")) return s;
  if (state_disp)
    if (piv_status s = check_alpha(alpha2, "alpha2")) return s;
  if (n == 0) return PIV_OK;
  const Temporal tm{slot, nstate, state_pred, state_disp, alpha1, alpha2};
  return run_path(P, A, B, pitch, n, pred, disp, peak, flags, omega, &tm, stream);
}

piv_status piv_highpass(piv_plan_t plan, const void* in, void* out, int64_t pitch, int32_t n, int32_t radius,
                        hipStream_t stream) {
  if (!plan) return fail(PIV_EINVAL, "plan is NULL");
  const Plan& P = *cplan(plan);
  if (P.p.dtype == PIV_F32) return fail(PIV_EUNSUPPORTED, "pre-processing takes U8/U16 frames");
  if (piv_status s = check_images(P, in, out, pitch, n)) return s;
  if (in == out) return fail(PIV_EINVAL, "the high-pass cannot run in place (in == out)");
  if (radius < 1 || radius > 16) return fail(PIV_EINVAL, "radius %d outside [1, 16]", radius);
  if (n == 0) return PIV_OK;
  return dev(piv::launch_highpass(P, in, out, pitch, n, radius, stream), "highpass");
}

size_t piv_clahe_lut_bytes(piv_plan_t plan, int32_t n, int32_t tiles_x, int32_t tiles_y) {
  if (!plan || n < 0 || tiles_x <= 0 || tiles_y <= 0) return 0;
  const Plan& P = *cplan(plan);
  if (P.p.dtype == PIV_F32) return 0;
  return sizeof(uint16_t) * (size_t)n * tiles_x * tiles_y * piv::clahe_bins(P);
}

piv_status piv_clahe(piv_plan_t plan, const void* in, void* out, int64_t pitch, int32_t n, int32_t tiles_x,
                     int32_t tiles_y, double clip_factor, void* lut, size_t lut_bytes, hipStream_t stream) {
  if (!plan) return fail(PIV_EINVAL, "plan is NULL");
  const Plan& P = *cplan(plan);
  if (P.p.dtype == PIV_F32) return fail(PIV_EUNSUPPORTED, "pre-processing takes U8/U16 frames");
  if (piv_status s = check_images(P, in, out, pitch, n)) return s;
  if (tiles_x < 1 || tiles_y < 1 || tiles_x > 64 || tiles_y > 64 || tiles_x > P.p.width || tiles_y > P.p.height)
    return fail(PIV_EINVAL, "tiles %d x %d outside [1, min(64, size)]", tiles_x, tiles_y);
  if (!(clip_factor > 0.0) || !(clip_factor < 1e300)) return fail(PIV_EINVAL, "clip_factor must be positive and finite");
  if (!lut) return fail(PIV_EINVAL, "lut must not be NULL");
  if ((uintptr_t)lut & 3) return fail(PIV_EINVAL, "lut must be 4-byte aligned");
  if (lut_bytes < piv_clahe_lut_bytes(plan, n, tiles_x, tiles_y))
    return fail(PIV_EINVAL, "lut holds %zu bytes, needs %zu", lut_bytes, piv_clahe_lut_bytes(plan, n, tiles_x, tiles_y));
  if (P.p.width > 32767 || P.p.height > 32767)
    return fail(PIV_EUNSUPPORTED, "CLAHE takes frames of at most 32767 x 32767 pixels");
  if (n == 0) return PIV_OK;
  return dev(piv::launch_clahe(P, in, out, pitch, n, tiles_x, tiles_y, clip_factor, static_cast<uint16_t*>(lut),
                               stream),
             "clahe");
}

piv_status piv_ssd_forward(piv_plan_t plan, const float* A, const float* B, const float* U, int32_t n,
                           float* loss, hipStream_t stream) {
  if (!plan) return fail(PIV_EINVAL, "plan is NULL");
  const Plan& P = *cplan(plan);
  if (P.p.dtype != PIV_F32) return fail(PIV_EINVAL, "SSD needs a PIV_F32 plan");
  if (!A || !B || !U || !loss) return fail(PIV_EINVAL, "NULL pointer");
  if (n < 0 || n > P.p.max_batch) return fail(PIV_EINVAL, "n=%d outside [0, max_batch]", n);
  if (n == 0) return PIV_OK;
  return dev(piv::launch_ssd_forward(P, A, B, U, n, loss, stream), "ssd_forward");
}

piv_status piv_ssd_backward(piv_plan_t plan, const float* A, const float* B, const float* U,
                            const float* g, int32_t n, float* gU, float* D, hipStream_t stream) {
  if (!plan) return fail(PIV_EINVAL, "plan is NULL");
  const Plan& P = *cplan(plan);
  if (P.p.dtype != PIV_F32) return fail(PIV_EINVAL, "SSD needs a PIV_F32 plan");
  if (!A || !B || !U || !g || !gU) return fail(PIV_EINVAL, "NULL pointer");
  if (n < 0 || n > P.p.max_batch) return fail(PIV_EINVAL, "n=%d outside [0, max_batch]", n);
  if (n == 0) return PIV_OK;
  return dev(piv::launch_ssd_backward(P, A, B, U, g, n, gU, D, stream), "ssd_backward");
}

piv_status piv_ssd_refine(piv_plan_t plan, const float* A, const float* B, float* U, int32_t n,
                          int32_t steps, float tau, float lam_rel, float* hist, hipStream_t stream) {
  if (!plan) return fail(PIV_EINVAL, "plan is NULL");
  const Plan& P = *cplan(plan);
  if (P.p.dtype != PIV_F32) return fail(PIV_EINVAL, "SSD needs a PIV_F32 plan");
  if (!A || !B || !U) return fail(PIV_EINVAL, "NULL pointer");
  if (n < 0 || n > P.p.max_batch) return fail(PIV_EINVAL, "n=%d outside [0, max_batch]", n);
  if (steps < 0 || steps > 10000) return fail(PIV_EINVAL, "steps=%d outside [0, 10000]", steps);
  if (!(tau > 0.0f) || !(tau <= 16.0f)) return fail(PIV_EINVAL, "tau=%g outside (0, 16]", (double)tau);
  if (!(lam_rel >= 0.0f) || !(lam_rel <= 1e6f)) return fail(PIV_EINVAL, "lam_rel=%g outside [0, 1e6]", (double)lam_rel);
  if (piv_status s = need_ws(P, n)) return s;
  if (n == 0) return PIV_OK;
  if (piv::ssd_tiled(P)) {
    // per step: the adjoint (gradient, GN diagonal and, per tile, the sums of
    // the diagonal and of the loss before the step), then the update; the
    // loss after the last step by the forward
    for (int k = 0; k < steps; ++k)
      if (piv_status s = dev(piv::launch_ssd_refine_step(P, A, B, U, n, tau, lam_rel, hist, steps + 1, k, stream),
                             "ssd_refine_step"))
        return s;
    if (hist) {
      if (piv_status s = dev(piv::launch_ssd_forward(P, A, B, U, n, nullptr, stream), "ssd_forward")) return s;
      if (piv_status s = dev(piv::launch_ssd_update(P, U, n, tau, lam_rel, hist, steps + 1, steps, 0, stream),
                             "ssd_update"))
        return s;
    }
    return PIV_OK;
  }
  // per step: window losses (for the history), gradient and Gauss-Newton
  // diagonal of the total loss into the workspace, then the update
  for (int k = 0; k <= steps; ++k) {
    const bool upd = k < steps;
    if (hist)
      if (piv_status s = dev(piv::launch_ssd_forward(P, A, B, U, n, nullptr, stream), "ssd_forward")) return s;
    if (upd)
      if (piv_status s = dev(piv::launch_ssd_backward(P, A, B, U, nullptr, n, nullptr, nullptr, stream),
                             "ssd_backward"))
        return s;
    if (hist || upd)
      if (piv_status s = dev(piv::launch_ssd_update(P, U, n, tau, lam_rel, hist, steps + 1, k, upd ? 1 : 0,
                                                    stream), "ssd_update"))
        return s;
  }
  return PIV_OK;
}

const char* piv_status_string(piv_status s) {
  switch (s) {
    case PIV_OK: return "PIV_OK";
    case PIV_EINVAL: return "PIV_EINVAL";
    case PIV_EUNSUPPORTED: return "PIV_EUNSUPPORTED";
    case PIV_ENOWORKSPACE: return "PIV_ENOWORKSPACE";
    case PIV_EDEVICE: return "PIV_EDEVICE";
  }
  return "PIV_UNKNOWN";
}

const char* piv_last_error(void) { return g_err; }

// Diagnostics (declared at the end of include/piv.h): which correlation
// kernel a plan selects (0 = generic per-window, 1 = cell-shared tiled).
int piv_debug_correct_impl(piv_plan_t plan) { return plan ? piv::correct_impl(*cplan(plan)) : -1; }

// Geometry of pyramid level l, for host-side checks of the kernels' read
// extents.  out: W, H, margin, pitch, rows, R,
// nx, ny, es, step, block.  Returns 0, or -1 for a bad level.
int piv_debug_level(piv_plan_t plan, int32_t l, int32_t* out) {
  if (!plan || !out) return -1;
  const Plan& P = *cplan(plan);
  if (l < 0 || l >= P.L) return -1;
  const piv::Level& v = P.lv[l];
  int32_t vals[11] = {v.W, v.H, v.margin, v.pitch, v.rows, v.R, v.nx, v.ny, P.es, P.p.step, P.block};
  for (int i = 0; i < 11; ++i) out[i] = vals[i];
  return 0;
}

}  // extern "C"
