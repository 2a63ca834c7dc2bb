/*
 * piv.h -- C ABI of the MI355X (gfx950) PIV hot path.
 *
 * The library turns particle-image pairs into dense, validated displacement
 * fields with vorticity, following the processing pipeline of "RapidPIV:
 * Full Flow-Field kHz PIV for Real-Time Display and Control" (Bollt,
 * Foxman, Gharib), Sec. 2: a coarse predictor of the displacement field,
 * deformation of the pair by that predictor, correlation with a Gaussian
 * sub-pixel fit about the best shift, universal outlier detection with
 * median replacement (Sec. 3: threshold 2, regulariser 0.1 px), and the
 * vorticity that the paper displays and compares (Sec. 4).  The paper's
 * predictor is a fixed-function optical-flow engine; here it is a
 * coarse-to-fine integer block-matching search written for the GPU's
 * compute units.
 *
 * Conventions shared by every entry point:
 *  - Every image/field pointer is a DEVICE pointer owned by the caller.
 *    Pointers marked "host" are host memory.
 *  - Images are [n][height][pitch_bytes] with separate A (first exposure)
 *    and B (second exposure) pointers; pitch_bytes is a multiple of 4 and
 *    both base pointers are 4-byte aligned.  Intensity outside the image is 0.
 *  - Pixel (row i, col j) has its centre at x = j, y = i.  The vector grid
 *    has nx = width/step by ny = height/step nodes; node (a, b) sits at
 *    (b*step + (step-1)/2, a*step + (step-1)/2) and its win x win window
 *    starts at b*step - (win-step)/2.
 *  - Fields are float32 [n][2][ny][nx] (u plane, then v plane), in pixels
 *    per frame pair, displacement from A to B.  Per-vector flags are
 *    uint8 [n][ny][nx]; scalar per-vector outputs float32 [n][ny][nx].
 *  - Every call only enqueues kernels on `stream` and returns: it never
 *    allocates, never synchronises, never reads device memory on the host,
 *    so it may be captured into a HIP graph.  Argument errors are detected
 *    on the host before any launch (no partial work).  Faults inside a
 *    kernel surface at the caller's next synchronisation.
 *  - A plan is immutable after workspace binding (the binding call itself
 *    prepares the workspace on the stream it is given); use one plan (and
 *    one workspace) per concurrently used stream.
 */
#ifndef PIV_H
#define PIV_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct piv_plan_s* piv_plan_t;

typedef enum {
  PIV_OK = 0,
  PIV_EINVAL = 1,          /* bad argument, shape or parameter              */
  PIV_EUNSUPPORTED = 2,    /* valid for the method, not built in this library */
  PIV_ENOWORKSPACE = 3,    /* workspace missing or too small for n            */
  PIV_EDEVICE = 4          /* a HIP launch or query failed                    */
} piv_status;

typedef enum { PIV_U8 = 1, PIV_U16 = 2, PIV_F32 = 3 } piv_dtype;

/* Deformation of the pair by the predictor (Sec. 2).  PIV_WARP_B deforms
 * frame B only: B'(p) = B(p + u(p)).  PIV_WARP_CENTRAL deforms both frames
 * symmetrically: A'(p) = A(p - u(p)/2), B'(p) = B(p + u(p)/2). */
typedef enum { PIV_WARP_B = 0, PIV_WARP_CENTRAL = 1 } piv_warp;

/* Peak selection (Sec. 2, Sec. 4.3).  PIV_PEAK_ARGMAX searches every shift
 * in [-radius, radius]^2; PIV_PEAK_FIXED_CENTER uses the paper's a-priori
 * 5-point stencil centred at zero shift. */
typedef enum { PIV_PEAK_ARGMAX = 0, PIV_PEAK_FIXED_CENTER = 1 } piv_peak;

typedef struct {
  int32_t width, height;   /* image size in pixels                                   */
  int32_t max_batch;       /* largest n any call will pass                           */
  piv_dtype dtype;         /* element type of A and B                                */
  int32_t bit_depth;       /* meaningful bits of U16 data (12 or 16); ignored else   */
  int32_t win;             /* correlation window (px); 2*step for 50% overlap        */
  int32_t step;            /* node spacing (px)                                      */
  int32_t radius;          /* correction search radius r: shifts in [-r, r]^2        */
  int32_t levels;          /* predictor pyramid levels (1 = no pyramid)              */
  int32_t block;           /* predictor block size (0 = win)                         */
  int32_t radius_coarse;   /* predictor search radius on the coarsest level          */
  int32_t radius_fine;     /* predictor search radius on every finer level           */
  int32_t median;          /* 3x3 median of the predictor after every level (0/1)    */
  piv_warp warp;
  piv_peak peak;
  float uod_threshold;     /* normalised-median threshold (Sec. 3: 2)                */
  float uod_epsilon;       /* normalised-median regulariser in px (Sec. 3: 0.1)      */
  int32_t sgm;             /* 1: the coarsest level by semi-global matching (0: off) */
  int32_t sgm_p1;          /* its penalty for a 1 px change between path neighbours, */
  int32_t sgm_p2;          /*   and for a larger one, per block pixel (0..255)       */
} piv_params;

/* Per-vector flag bits. */
enum {
  PIV_F_FLAT = 1,        /* correlation denominator zero at every shift (blank window) */
  PIV_F_BORDER = 2,      /* best shift on the edge of the search: no sub-pixel fit     */
  PIV_F_NOCURV = 4,      /* log-coefficients not concave on an axis: no fit on it      */
  PIV_F_OUTLIER = 8,     /* rejected by validation                                     */
  PIV_F_REPLACED = 16,   /* replaced by the median of non-outlier neighbours           */
  PIV_F_UNRESOLVED = 32  /* outlier without a non-outlier neighbour: value kept        */
};

/* Fill *p (host) with the paper's processing parameters for 1 MP u8 pairs:
 * 16 x 16 windows at 50% step-over, UOD threshold 2 and regulariser 0.1 px
 * (Sec. 3.1), +-4 px correction search, a 3-level predictor with radii 6/2. */
void piv_params_default(piv_params* p);

/* Validate *p (host) and create a plan.  Host-only: no device work.
 * Errors: PIV_EINVAL for shapes/parameters the method cannot take
 * (width/height not multiples of step, win < step, (win-step) odd,
 * win > 64, radius outside [1, 16], levels outside [1, 6], bad dtype ...),
 * PIV_EUNSUPPORTED for combinations the kernels are not built for.
 * On error *out is NULL and piv_last_error() tells why. */
piv_status piv_plan(const piv_params* p, piv_plan_t* out);

/* Vector grid size of the plan (host outputs). */
piv_status piv_plan_grid(piv_plan_t plan, int32_t* nx, int32_t* ny);

/* Bytes of device workspace needed for `batch` pairs: predictor pyramids,
 * per-level integer fields and one float field [2][ny][nx] (the input of
 * validation); PIV_F32 plans also hold the refinement's gradient, diagonal
 * and window losses.  Exact, so that callers can admit work against an HBM
 * budget. */
size_t piv_plan_workspace_bytes(piv_plan_t plan, int32_t batch);

/* Bind caller-owned device workspace (e.g. a torch tensor) to the plan,
 * 256-byte aligned.  The plan remembers how many pairs it can hold (at most
 * max_batch); later calls with a larger n fail with PIV_ENOWORKSPACE.  The
 * memory must outlive its use.  Binding enqueues, on `stream`, the zeroing
 * of the pyramid margins of every pair the workspace holds; later calls
 * (on any stream ordered after it) rely on them, so the caller must not
 * write to bound workspace.  Binding again (the same pointer included)
 * repeats the zeroing.  d_ws NULL unbinds (no device work).
 * Errors: PIV_EINVAL (misaligned), PIV_ENOWORKSPACE (holds no pair),
 * PIV_EDEVICE (the launch failed; the previous binding is kept). */
piv_status piv_plan_bind_workspace(piv_plan_t plan, void* d_ws, size_t bytes, hipStream_t stream);

/* Optional device slot mask uint8 [max_batch]: when bound, every kernel of
 * every call skips pair i whose mask byte is 0 (its outputs are left
 * untouched).  Lets a graph captured for max_batch pairs run a partial
 * batch.  NULL unbinds. */
piv_status piv_plan_bind_slot_mask(piv_plan_t plan, const uint8_t* d_mask);

void piv_plan_destroy(piv_plan_t plan);

/* Predictor (Sec. 2: the coarse displacement estimate that the correlation
 * then corrects, there from a fixed-function optical-flow engine; here
 * block matching on the compute units): coarse-to-fine integer SAD block
 * matching.  For each level l
 * (coarsest first) and node, the block of `block` x `block` level-l pixels
 * at the node is compared with frame B moved by every integer d in
 * cand + [-R, R]^2 (R = radius_coarse on the coarsest level around 0,
 * radius_fine below, around twice the parent node's result); the d with the
 * least (SAD, |dx|+|dy|, dy, dx) wins.  Pyramid levels are 2x2 box means
 * floor((sum+2)/4).  With params.sgm the coarsest level is searched by
 * semi-global matching instead (the family of methods of the paper's
 * optical-flow engine): the block SAD of every candidate d in
 * [-radius_coarse, radius_coarse]^2 at every node, aggregated along four
 * paths over the node grid (left to right, right to left, top to bottom,
 * bottom to top), L(p,d) = C(p,d) + min(L(q,d), min over the 8 candidates
 * adjacent to d of L(q,d') + P1, min L(q,.) + P2) - min L(q,.) with q the
 * previous node on the path (L = C at a path's first node), P1 = sgm_p1 *
 * block^2, P2 = sgm_p2 * block^2; the least (sum of the four, |dx|+|dy|,
 * dy, dx) wins.  pred: [n][2][ny][nx] float32 holding integers.
 * Needs a bound workspace. */
piv_status piv_predict(piv_plan_t plan, const void* A, const void* B, int64_t pitch_bytes,
                       int32_t n, float* pred, hipStream_t stream);

/* Correction (Sec. 2): deform the pair by the bilinearly interpolated
 * predictor (NULL = zero), compute the Pearson correlation coefficient of
 * each window with the deformed B window moved by every shift s in
 * [-r, r]^2 (or the 5-point stencil), take the best shift (largest
 * coefficient; ties to smaller |sx|+|sy|, then smaller sy, then smaller sx)
 * and a 3-point Gaussian fit per axis on coefficients floored at 1e-3.
 * disp = pred(node) + s* + fit.  peak (nullable) = coefficient at s*.
 * flags: FLAT / BORDER / NOCURV.  Needs no workspace. */
piv_status piv_correct(piv_plan_t plan, const void* A, const void* B, int64_t pitch_bytes,
                       int32_t n, const float* pred, float* disp, float* peak, uint8_t* flags,
                       hipStream_t stream);

/* Universal outlier detection (Sec. 2, Sec. 3) in place on field [n][2][ny][nx].
 * Vectors whose input flags hold FLAT or BORDER are outliers and never
 * neighbours.  Per component r0 = |u0 - med(u_j)| / (med|u_j - med(u_j)| + eps)
 * over the valid 3x3 neighbours; outlier if the larger r0 exceeds the
 * threshold.  Outliers take the component medians of their non-outlier
 * neighbours from the detection-pass field (UNRESOLVED if none).  flags
 * (nullable) in/out gain OUTLIER / REPLACED / UNRESOLVED.  Needs a bound
 * workspace. */
piv_status piv_validate(piv_plan_t plan, float* field, uint8_t* flags, int32_t n, hipStream_t stream);

/* Vorticity (Sec. 1 and Sec. 4: the field the paper displays and compares;
 * its scheme is not given) omega = dv/dx - du/dy (1/frame) on the node grid, spacing step:
 * central differences inside, second-order one-sided on the edges.
 * disp [n][2][ny][nx] -> omega [n][ny][nx]. */
piv_status piv_vorticity(piv_plan_t plan, const float* disp, float* omega, int32_t n,
                         hipStream_t stream);

/* The whole plain path in one call: predict, validate the predictor,
 * correct, validate, vorticity, with the same results as those calls made
 * one by one.  pred (scratch for the predictor, also an output), disp, flags
 * and omega are required; peak is nullable.  Needs a bound workspace.  With
 * a level-0 search radius <= 2 (u8, or u16 with 12-24 px blocks), level 0 of
 * the predictor (here and in piv_predict) reads A and B in place (only a 32 px frame along the edges
 * is copied). */
piv_status piv_run(piv_plan_t plan, const void* A, const void* B, int64_t pitch_bytes, int32_t n,
                   float* pred, float* disp, float* peak, uint8_t* flags, float* omega,
                   hipStream_t stream);

/* Size of the device array piv_run_noalloc works in, per GPU. */
#define PIV_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* piv_run for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same steps and
 * results as piv_run, with the workspace taken from a fixed device array of
 * the library (PIV_NOALLOC_SCRATCH_BYTES on every GPU it runs on, held from
 * library load to process end) instead of the plan's bound workspace, which
 * may be absent.  The call allocates nothing; the caller passes inputs and
 * outputs as for piv_run.  Each call first zeroes the array's pyramid
 * margins for its n pairs (the array keeps whatever the previous call on
 * that GPU left).  All calls on one GPU share its array: calls that overlap
 * on one GPU (other streams, other threads) race.  Errors as piv_run, and
 * PIV_ENOWORKSPACE, before any device work, when n pairs need more than
 * PIV_NOALLOC_SCRATCH_BYTES (piv_plan_workspace_bytes(plan, n)). */
piv_status piv_run_noalloc(piv_plan_t plan, const void* A, const void* B, int64_t pitch_bytes, int32_t n,
                           float* pred, float* disp, float* peak, uint8_t* flags, float* omega,
                           hipStream_t stream);

/* Exponential smoothing in time (Sec. 2; alpha1 = alpha2 = 0.5 in both
 * experiments of Sec. 3), in place on field [n][2][ny][nx] with per-stream
 * state [nstate][2][ny][nx] (device, caller-owned).  Pairs are taken in
 * batch order; pair i uses state slot slot[i] (device int32 [n]):
 *   slot[i] = k >= 0:      s_k <- alpha * field_i + (1 - alpha) * s_k
 *   slot[i] = -1 - k:      s_k <- field_i (the first frame of a stream)
 * and field_i <- s_k.  Pairs sharing a slot (consecutive frames of one
 * stream in one batch) chain in batch order.  A slot outside [0, nstate)
 * leaves its pair and every state untouched.  alpha in (0, 1]; 1 = off.
 * Errors: PIV_EINVAL (NULL pointers, nstate <= 0, alpha out of range). */
piv_status piv_smooth(piv_plan_t plan, float* field, float* state, const int32_t* slot, int32_t nstate,
                      float alpha, int32_t n, hipStream_t stream);

/* The paper's whole pipeline with temporal smoothing (Sec. 2): predict,
 * validate the predictor, smooth it with alpha1 and state_pred, correct
 * about the smoothed predictor, validate, smooth the final field with
 * alpha2 and state_disp, vorticity of the smoothed field.  slot and nstate
 * as in piv_smooth (one slot table for both states).  state_pred or
 * state_disp NULL skips that smoothing (its alpha is then ignored); with
 * both NULL the results equal piv_run's.  The states make results depend
 * on each stream's history, unlike piv_run's.  Needs a bound workspace. */
piv_status piv_run_temporal(piv_plan_t plan, const void* A, const void* B, int64_t pitch_bytes,
                            int32_t n, const int32_t* slot, int32_t nstate, float* state_pred,
                            float* state_disp, float alpha1, float alpha2, float* pred, float* disp,
                            float* peak, uint8_t* flags, float* omega, hipStream_t stream);

/* Pre-processing (Sec. 2: every frame is high-pass filtered to remove the
 * static background, then contrast-enhanced by CLAHE, before the predictor
 * and the correlation; Sec. 3.1 uses both to match the intensities of
 * stitched images).  The paper does not specify the filters; these are
 * exact integer readings.  Frames as for piv_run (the plan's size, dtype
 * U8 or U16 and bit_depth); out has the same layout and pitch as in.
 *
 * piv_highpass: out = max(0, in - floor(mean of in over the image part of
 * the (2 radius + 1)^2 box around each pixel)), radius in [1, 16].  out
 * must not alias in.  Errors: PIV_EINVAL (arguments), PIV_EUNSUPPORTED
 * (F32 plan). */
piv_status piv_highpass(piv_plan_t plan, const void* in, void* out, int64_t pitch_bytes, int32_t n,
                        int32_t radius, hipStream_t stream);

/* Device bytes of the CLAHE mappings for n pairs on a tiles_x x tiles_y
 * grid: n * tiles_x * tiles_y * nbins uint16, nbins = 2^min(bits, 12)
 * (256 for U8, 4096 for U16).  0 for bad arguments. */
size_t piv_clahe_lut_bytes(piv_plan_t plan, int32_t n, int32_t tiles_x, int32_t tiles_y);

/* Contrast-limited adaptive histogram equalisation.  Tile j of a row spans
 * [floor(j W / tiles_x), floor((j+1) W / tiles_x)) (likewise in y).  Per
 * tile: histogram of value >> (bits - log2 nbins); every bin clipped at
 * max(1, floor(clip_factor * npix / nbins)) (double arithmetic), the
 * clipped excess spread evenly (excess / nbins to every bin, then one more
 * to the first excess % nbins bins taken at a stride of
 * max(nbins / (excess % nbins), 1) from bin 0); mapping
 * lut[b] = (cdf(b) * maxval + npix / 2) / npix, maxval = 2^bits - 1.
 * Every pixel blends the mappings of the up to four tiles whose centres
 * surround it (bilinear weights in doubled coordinates, clamped at the
 * outer centres, rounded half up in integers).  lut: caller-owned device
 * scratch of at least piv_clahe_lut_bytes (4-byte aligned), left holding
 * the mappings.  out may equal in.  tiles in [1, min(64, size)]; frames
 * up to 32767 x 32767 (PIV_EUNSUPPORTED beyond). */
piv_status piv_clahe(piv_plan_t plan, const void* in, void* out, int64_t pitch_bytes, int32_t n,
                     int32_t tiles_x, int32_t tiles_y, double clip_factor, void* lut, size_t lut_bytes,
                     hipStream_t stream);

/* Windowed SSD of the deformation (an addition, not in the paper): for
 * float32 frames A, B [n][height][width] (pitch = width) and a node field
 * U [n][2][ny][nx], loss[n][ny][nx] = sum over each window of
 * (B(p + u(p)) - A(p))^2 with u the clamped bilinear interpolation of U.
 * The plan's dtype must be PIV_F32. */
piv_status piv_ssd_forward(piv_plan_t plan, const float* A, const float* B, const float* U,
                           int32_t n, float* loss, hipStream_t stream);

/* Adjoint of piv_ssd_forward: g_U = d(sum g_loss * loss)/dU (derivative of
 * the bilinear sample taken on its floor cell), and the Gauss-Newton
 * diagonal gn_diag = sum_p 2 m(p) (dB'/du)^2 w_n(p)^2 with m(p) the sum of
 * g_loss over the windows holding p (nullable).  Deterministic: every node
 * gathers its own terms, no atomics. */
piv_status piv_ssd_backward(piv_plan_t plan, const float* A, const float* B, const float* U,
                            const float* g_loss, int32_t n, float* g_U, float* gn_diag,
                            hipStream_t stream);

/* Gradient refinement by the windowed SSD (an addition, compared with the
 * paper's Gaussian fit): `steps` diagonally preconditioned gradient steps
 * on the total loss L = sum of every window's SSD, in place on U
 * [n][2][ny][nx]:
 *   U <- U - tau * dL/dU / (D + lambda),  lambda = lam_rel * mean(D),
 * D the Gauss-Newton diagonal (as in piv_ssd_backward with g_loss = 1) and
 * mean(D) over both components of each pair's grid; a node component whose
 * D + lambda is not positive is left unchanged.  hist (nullable, device
 * float [n][steps + 1]) receives the total loss before each step and after
 * the last.  Everything runs on the device (no host synchronisation); the
 * gradient, diagonal and losses live in the plan's workspace, so a bound
 * workspace is needed (PIV_F32 plan).  tau in (0, 16], lam_rel in
 * [0, 1e6], steps in [0, 10000]. */
piv_status piv_ssd_refine(piv_plan_t plan, const float* A, const float* B, float* U, int32_t n,
                          int32_t steps, float tau, float lam_rel, float* hist, hipStream_t stream);

const char* piv_status_string(piv_status s);

/* Detail of the last failure on the calling thread (never NULL). */
const char* piv_last_error(void);

/* Diagnostics for tests and benchmarks (no device work).
 * piv_debug_correct_impl: which correlation kernel the plan selects
 * (0 generic per window, 1 cell-shared tiled or band), -1 for NULL.
 * piv_debug_level: geometry of pyramid level l into out[11] (host):
 * W, H, margin, pitch, rows, R, nx, ny, bytes per pixel, step, block;
 * returns 0, or -1 for a bad plan, pointer or level. */
int piv_debug_correct_impl(piv_plan_t plan);
int piv_debug_level(piv_plan_t plan, int32_t l, int32_t* out);

#ifdef __cplusplus
}
#endif

#endif /* PIV_H */
