// Internal plan layout and kernel launchers of libpiv (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/piv.h"

namespace piv {

constexpr int kMaxLevels = 6;

// Every pyramid level (level 0 included, as a copy of the input) lives in
// the workspace with a zero margin of `margin` pixels on all four sides,
// wide enough for the level's whole search reach, so that the SAD kernels
// read without bounds checks.
struct Level {
  int W, H;           // level image size (px)
  int margin;         // zero border (px); a multiple of 4
  int pitch;          // bytes per padded row (multiple of 64)
  int rows;           // padded rows: H + 2 margin
  int R;              // search radius on this level
  int nx, ny;         // level node grid
  size_t off_a, off_b;  // per-pair offset of the padded images (row 0 of the margin)
  size_t off_d;         // per-pair offset of the level's int32 [2][ny][nx] field
  size_t origin() const { return (size_t)margin * pitch; }  // + margin * es for the column
};

struct Plan {
  piv_params p;
  int es;             // bytes per pixel (1, 2, 4)
  int nx, ny;         // level-0 grid
  int block;          // predictor block (resolved)
  int L;
  Level lv[kMaxLevels];
  size_t off_raw;     // per-pair offset of a float [2][ny][nx] field: the detection-pass
                      // input of validation
  // F32 plans only: per-pair offsets of the refinement's gradient and
  // Gauss-Newton diagonal ([2][ny][nx] each) and window losses ([ny][nx])
  size_t off_gu = 0, off_dd = 0, off_loss = 0, off_part = 0;
  // with semi-global matching: per-pair offsets of the coarsest level's cost
  // volume and aggregated cost (uint32 [node][candidate] each)
  size_t off_sgm_c = 0, off_sgm_s = 0;
  size_t per_pair;    // workspace bytes per pair
  uint8_t* ws = nullptr;
  size_t ws_bytes = 0;
  int ws_pairs = 0;   // pairs the bound workspace can hold
  const uint8_t* slot_mask = nullptr;
};

// Image view of one frame batch.
struct Img {
  const uint8_t* base;  // pair 0, row 0
  int64_t pitch;        // bytes per row
  int64_t stride;       // bytes per pair
};

// ---- launchers (return hipError_t of the launch) ----
// zero every pyramid margin of `pairs` pairs of the workspace at ws (laid out
// as the plan's); the pyramid copy kernels write the image cores only
hipError_t launch_clear_margins(const Plan& P, uint8_t* ws, int pairs, hipStream_t s);
hipError_t launch_pyramid(const Plan& P, const void* A, const void* B, int64_t pitch, int n,
                          hipStream_t s);
hipError_t launch_sad_level(const Plan& P, int l, const void* A, const void* B, int64_t pitch,
                            int n, hipStream_t s);
hipError_t launch_pred_out(const Plan& P, int n, float* pred, hipStream_t s);
// the coarsest level by semi-global matching into its level field (sgm.hip)
hipError_t launch_sgm_level(const Plan& P, int n, hipStream_t s);
hipError_t launch_sad_cost_cells(const Plan& P, uint32_t* C, int64_t cstride, int n, hipStream_t s);
// disp_stride: floats per pair of disp (0: 2 nx ny)
hipError_t launch_correct(const Plan& P, const void* A, const void* B, int64_t pitch, int n,
                          const float* pred, float* disp, float* peak, uint8_t* flags,
                          hipStream_t s, int64_t disp_stride = 0);
hipError_t launch_validate(const Plan& P, float* field, uint8_t* flags, int n, hipStream_t s);
// validation from src (pair stride in floats) into dst [n][2][ny][nx]; src != dst
hipError_t launch_uod(const Plan& P, const float* src, int64_t sstride, float* dst, uint8_t* flags,
                      int n, hipStream_t s);
// level-0 predictor field (through the median) -> validated float predictor
hipError_t launch_pred_validate(const Plan& P, int n, float* pred, hipStream_t s);
hipError_t launch_vorticity(const Plan& P, const float* disp, float* omega, int n, hipStream_t s);
hipError_t launch_ssd_forward(const Plan& P, const float* A, const float* B, const float* U, int n,
                              float* loss, hipStream_t s);
// g NULL: every window's upstream gradient is 1
hipError_t launch_ssd_backward(const Plan& P, const float* A, const float* B, const float* U,
                               const float* g, int n, float* gU, float* D, hipStream_t s);
// one refinement update per pair from the workspace's gradient, diagonal and
// losses: hist[pair * hstride + k] = total loss (if hist), and, when update
// is set, U -= tau gU / (D + lam_rel mean(D))
// refinement step for the tiled geometry (win = 2 step = 16): the adjoint
// with per-tile sums of the GN diagonal and the loss, then the update
bool ssd_tiled(const Plan& P);
hipError_t launch_ssd_refine_step(const Plan& P, const float* A, const float* B, float* U, int n, float tau,
                                  float lam_rel, float* hist, int hstride, int k, hipStream_t s);
hipError_t launch_ssd_update(const Plan& P, float* U, int n, float tau, float lam_rel, float* hist,
                             int hstride, int k, int update, hipStream_t s);
// exponential smoothing in time: see piv_smooth in include/piv.h
hipError_t launch_smooth(const Plan& P, float* field, float* state, const int32_t* slot, int nstate,
                         float alpha, int n, hipStream_t s);

// pre-processing: high-pass background removal and CLAHE (preproc.hip);
// lut holds n * ty * tx * clahe_bins(P) uint16 entries
hipError_t launch_highpass(const Plan& P, const void* in, void* out, int64_t pitch, int n, int r, hipStream_t s);
hipError_t launch_clahe(const Plan& P, const void* in, void* out, int64_t pitch, int n, int tx, int ty,
                        double clip_factor, uint16_t* lut, hipStream_t s);
int clahe_bins(const Plan& P);

// Block widths (in 4-byte words) the SAD kernel is built for.
bool sad_supported(int block_words);

// Which correlation kernel a plan uses (exposed for tests and the bench).
int correct_impl(const Plan& P);

// piv_run's host checks for a workspace of ws_bytes (no device work), and
// piv_run's checks and steps on the workspace `ws` of ws_bytes (instead of
// the plan's bound one), whose margins are zeroed first (plan.cpp).
piv_status check_on_workspace(const Plan& P, size_t ws_bytes, const void* A, const void* B, int64_t pitch,
                              int32_t n, float* pred, float* disp, uint8_t* flags, float* omega);
piv_status run_on_workspace(const Plan& P, uint8_t* ws, size_t ws_bytes, const void* A, const void* B,
                            int64_t pitch, int32_t n, float* pred, float* disp, float* peak, uint8_t* flags,
                            float* omega, hipStream_t stream);
// records msg as the calling thread's last error and returns s
piv_status set_error(piv_status s, const char* msg);

}  // namespace piv
