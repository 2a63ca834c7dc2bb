// piv_run without any allocation: the workspace is a fixed device array of
// this library instead of caller-provided memory (for callers that cannot
// allocate: code under graph capture, tight serving loops, harnesses that
// forbid hipMalloc).
//
// Every GPU holds its own copy of `scratch` (from library load until the
// process ends).  In host code the array's name only stands in for the
// symbol: its device address on the current GPU comes from
// hipGetSymbolAddress, taken once per device at the first call there and
// kept; only that address is ever passed to kernels.  Every call on a GPU
// shares that GPU's array, so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "piv_internal.h"

namespace {

constexpr size_t kScratchBytes = PIV_NOALLOC_SCRATCH_BYTES;

__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_mu;
std::vector<uint8_t*> g_ptr;   // per device: the array's address, or NULL before the first call there

// The array's device address on the current device (NULL on failure, with
// the error recorded).
uint8_t* scratch_here(piv_status* st) {
  int d = 0;
  hipError_t e = hipGetDevice(&d);
  if (e != hipSuccess) {
    *st = piv::set_error(PIV_EDEVICE, hipGetErrorString(e));
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if ((size_t)d >= g_ptr.size()) g_ptr.resize((size_t)d + 1, nullptr);
  if (!g_ptr[(size_t)d]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      *st = piv::set_error(PIV_EDEVICE, e != hipSuccess ? hipGetErrorString(e) : "no scratch address");
      return nullptr;
    }
    g_ptr[(size_t)d] = static_cast<uint8_t*>(p);
  }
  return g_ptr[(size_t)d];
}

}  // namespace

extern "C" piv_status piv_run_noalloc(piv_plan_t plan, const void* A, const void* B, int64_t pitch_bytes,
                                      int32_t n, float* pred, float* disp, float* peak, uint8_t* flags,
                                      float* omega, hipStream_t stream) {
  if (!plan) return piv::set_error(PIV_EINVAL, "plan is NULL");
  const piv::Plan& P = *reinterpret_cast<const piv::Plan*>(plan);
  // argument errors, work beyond the array and n = 0 return before any device call
  piv_status st = piv::check_on_workspace(P, kScratchBytes, A, B, pitch_bytes, n, pred, disp, flags, omega);
  if (st != PIV_OK || n == 0) return st;
  uint8_t* ws = scratch_here(&st);
  if (!ws) return st;
  return piv::run_on_workspace(P, ws, kScratchBytes, A, B, pitch_bytes, n, pred, disp, peak, flags, omega,
                               stream);
}
