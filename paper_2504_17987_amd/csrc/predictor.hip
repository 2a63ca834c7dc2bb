// Predictor kernels: 2x2 pyramid, per-level integer SAD block search with
// a packed-key argmin, and the final 3x3 median to the float field.
//
// The predictor stands where the paper (Sec. 2) uses a fixed-function
// optical-flow engine: a coarse, integer-accurate displacement estimate
// that the correlation stage then corrects.
#include "dev_common.h"
#include "piv_internal.h"

namespace piv {
namespace {

// ---------------------------------------------------------------------------
// Pyramid: out(y,x) = floor((in(2y,2x) + in(2y,2x+1) + in(2y+1,2x) + in(2y+1,2x+1) + 2) / 4),
// zero outside the input.  One thread writes 4 consecutive output pixels of
// one frame; the grid covers the output pitch so that the pad columns are
// written (as zeros).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_pyr_down(const uint8_t* __restrict__ srcA,
                                                  const uint8_t* __restrict__ srcB, int64_t spitch,
                                                  int64_t sstride, int sW, int sH, uint8_t* dst,
                                                  int64_t dA, int64_t dB, int dpitch, int64_t dstride,
                                                  int dH, const uint8_t* mask) {
  const int pair = blockIdx.z >> 1, frame = blockIdx.z & 1;
  if (slot_off(mask, pair)) return;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  const int x0 = (blockIdx.x * blockDim.x + threadIdx.x) * 4;
  const int dcols = dpitch / (int)sizeof(T);
  if (y >= dH || x0 >= dcols) return;
  const uint8_t* src = (frame ? srcB : srcA) + (int64_t)pair * sstride;
  T* out = reinterpret_cast<T*>(dst + (int64_t)pair * dstride + (frame ? dB : dA) + (int64_t)y * dpitch);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int x = x0 + i;
    if (x >= dcols) break;
    uint32_t s = 0;
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
#pragma unroll
      for (int dx = 0; dx < 2; ++dx) {
        int sy = 2 * y + dy, sx = 2 * x + dx;
        if (sy < sH && sx < sW) s += reinterpret_cast<const T*>(src + (int64_t)sy * spitch)[sx];
      }
    out[x] = (T)((s + 2u) >> 2);
  }
}

// ---------------------------------------------------------------------------
// SAD block search on one level.
//
// Lanes: a group of G = 2R+1 lanes per node, lane k owning the column of
// candidates dx = cand_x - R + k; NPW = 256/G nodes of one node row per
// workgroup.  The node's A block is staged in LDS as packed words; every
// lane streams the rows of frame B its column needs (aligned 4-byte loads,
// realigned once per row with alignbyte), and accumulates, for each of its
// G candidates dy, v_sad_u8 / v_sad_u16 over the row pairs.  The winner
// minimises the packed key (SAD, |dx|+|dy|, dy, dx) -- a plain u64 min, so
// the result does not depend on the reduction order.
// ---------------------------------------------------------------------------
struct SadArgs {
  const uint8_t* A;   // level image base (pair 0)
  const uint8_t* B;
  int64_t pitch, stride;
  int W, H;           // level image size (px)
  int nx, ny;         // level grid
  int step, block, R;
  const int32_t* parent;  // parent level field [.][2][pny][pnx] or null (coarsest)
  int64_t pstride;        // int32 elements per pair of the parent field
  int pnx, pny;
  int median;
  int32_t* out;           // this level's field
  int64_t ostride;        // int32 elements per pair
  const uint8_t* mask;
  int npw;                // nodes per workgroup
};

template <int ES>
__device__ __forceinline__ uint32_t sad_word(uint32_t a, uint32_t b, uint32_t c) {
  if constexpr (ES == 1) return __builtin_amdgcn_sad_u8(a, b, c);
  else return __builtin_amdgcn_sad_u16(a, b, c);
}

__device__ __forceinline__ int parent_value(const SadArgs& g, const int32_t* par, int comp, int pa,
                                            int pb) {
  const int32_t* P = par + (int64_t)comp * g.pnx * g.pny;
  if (!g.median) return P[pa * g.pnx + pb];
  int v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  int k = 0;
#pragma unroll
  for (int i = -1; i <= 1; ++i)
#pragma unroll
    for (int j = -1; j <= 1; ++j) {
      int y = pa + i, x = pb + j;
      bool in = y >= 0 && x >= 0 && y < g.pny && x < g.pnx;
      int val = in ? P[y * g.pnx + x] : 0;
      // pack the in-bounds values to the front (static indices)
#pragma unroll
      for (int s = 0; s < 9; ++s)
        if (in && s == k) v[s] = val;
      k += in;
    }
  return median_low_i<9>(v, k);
}

template <int ES, int NW, int KMAX>
__global__ __launch_bounds__(256) void k_sad(SadArgs g) {
  extern __shared__ uint32_t s_ablk[];        // [NPW][block][NW]
  __shared__ unsigned long long s_key[256];

  const int pair = blockIdx.z;
  if (slot_off(g.mask, pair)) return;
  const int G = 2 * g.R + 1;
  const int npw = g.npw;
  const int t = threadIdx.x;
  const int j = t / G, k = t - j * G;
  const int a = blockIdx.y;
  const int b0 = blockIdx.x * npw;
  const int b = b0 + j;
  const bool active = j < npw && b < g.nx;
  const int off = (g.step - g.block) / 2;
  const int oy = a * g.step + off;
  const int rowbytes = g.W * ES;
  const uint8_t* Ab = g.A + (int64_t)pair * g.stride;
  const uint8_t* Bb = g.B + (int64_t)pair * g.stride;

  // stage the A blocks of this workgroup's nodes (unaligned spans -> words)
  const int nblk = min(npw, g.nx - b0);
  const int words = g.block * NW;
  for (int idx = t; idx < nblk * words; idx += 256) {
    int jj = idx / words, r = (idx / NW) % g.block, w = idx % NW;
    int y = oy + r;
    uint32_t val = 0;
    if (y >= 0 && y < g.H) {
      const uint8_t* row = Ab + (int64_t)y * g.pitch;
      int xb = ((b0 + jj) * g.step + off) * ES + 4 * w;
      int xa = xb & ~3, sh = xb & 3;
      uint32_t lo = masked_word(row, rowbytes, xa);
      uint32_t hi = sh ? masked_word(row, rowbytes, xa + 4) : 0u;
      val = sh ? __builtin_amdgcn_alignbyte(hi, lo, sh) : lo;
    }
    s_ablk[idx] = val;
  }

  // candidate centre: twice the (median-filtered) parent result
  int cx = 0, cy = 0;
  if (g.parent && active) {
    const int32_t* par = g.parent + (int64_t)pair * g.pstride;
    int pa = min(a >> 1, g.pny - 1), pb = min(b >> 1, g.pnx - 1);
    cx = 2 * parent_value(g, par, 0, pa, pb);
    cy = 2 * parent_value(g, par, 1, pa, pb);
  }
  __syncthreads();

  unsigned long long best = ~0ull;
  if (active) {
    const int dx = cx - g.R + k;
    const int xb = (b * g.step + off + dx) * ES;
    const int xa = xb & ~3, sh = xb & 3;
    const int by0 = oy + cy - g.R;
    uint32_t acc[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) acc[q] = 0u;
    const uint32_t* ablk = s_ablk + j * words;
    const int nrows = g.block + 2 * g.R;
    for (int rb = 0; rb < nrows; ++rb) {
      const int y = by0 + rb;
      uint32_t bw[NW];
      if (y >= 0 && y < g.H) {
        const uint8_t* row = Bb + (int64_t)y * g.pitch;
        uint32_t w[NW + 1];
#pragma unroll
        for (int i = 0; i <= NW; ++i) w[i] = masked_word(row, rowbytes, xa + 4 * i);
#pragma unroll
        for (int i = 0; i < NW; ++i) bw[i] = sh ? __builtin_amdgcn_alignbyte(w[i + 1], w[i], sh) : w[i];
      } else {
#pragma unroll
        for (int i = 0; i < NW; ++i) bw[i] = 0u;
      }
#pragma unroll
      for (int q = 0; q < KMAX; ++q) {
        const int ar = rb - q;
        if (q < G && ar >= 0 && ar < g.block) {
          const uint32_t* arow = ablk + ar * NW;
          uint32_t s = acc[q];
#pragma unroll
          for (int i = 0; i < NW; ++i) s = sad_word<ES>(arow[i], bw[i], s);
          acc[q] = s;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < KMAX; ++q) {
      if (q < G) {
        const int dy = cy - g.R + q;
        const unsigned l1 = (unsigned)(abs(dx) + abs(dy));
        unsigned long long key = ((unsigned long long)acc[q] << 25) | ((unsigned long long)l1 << 16) |
                                 ((unsigned long long)(dy + 128) << 8) | (unsigned long long)(dx + 128);
        best = key < best ? key : best;
      }
    }
  }
  s_key[t] = best;
  __syncthreads();
  if (active && k == 0) {
    unsigned long long m = s_key[t];
    for (int q = 1; q < G; ++q) m = s_key[t + q] < m ? s_key[t + q] : m;
    int32_t* out = g.out + (int64_t)pair * g.ostride;
    out[a * g.nx + b] = (int)(m & 0xff) - 128;
    out[g.nx * g.ny + a * g.nx + b] = (int)((m >> 8) & 0xff) - 128;
  }
}

// final level-0 field -> float predictor, through the 3x3 median when enabled
__global__ __launch_bounds__(256) void k_pred_out(const int32_t* d, int64_t dstride, int nx, int ny,
                                                  int median, float* pred, const uint8_t* mask) {
  const int pair = blockIdx.y;
  if (slot_off(mask, pair)) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nx * ny) return;
  const int a = i / nx, b = i - a * nx;
  const int32_t* D = d + (int64_t)pair * dstride;
  float* out = pred + (int64_t)pair * 2 * nx * ny;
  for (int c = 0; c < 2; ++c) {
    const int32_t* P = D + c * nx * ny;
    int val;
    if (!median) {
      val = P[i];
    } else {
      int v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
      int k = 0;
#pragma unroll
      for (int di = -1; di <= 1; ++di)
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj) {
          int y = a + di, x = b + dj;
          bool in = y >= 0 && x >= 0 && y < ny && x < nx;
          int w = in ? P[y * nx + x] : 0;
#pragma unroll
          for (int s = 0; s < 9; ++s)
            if (in && s == k) v[s] = w;
          k += in;
        }
      val = median_low_i<9>(v, k);
    }
    out[c * nx * ny + i] = (float)val;
  }
}

template <int ES, int NW>
hipError_t sad_dispatch_k(int G, dim3 grid, size_t lds, hipStream_t s, const SadArgs& g) {
  if (G <= 5) hipLaunchKernelGGL((k_sad<ES, NW, 5>), grid, dim3(256), lds, s, g);
  else if (G <= 9) hipLaunchKernelGGL((k_sad<ES, NW, 9>), grid, dim3(256), lds, s, g);
  else if (G <= 13) hipLaunchKernelGGL((k_sad<ES, NW, 13>), grid, dim3(256), lds, s, g);
  else if (G <= 17) hipLaunchKernelGGL((k_sad<ES, NW, 17>), grid, dim3(256), lds, s, g);
  else hipLaunchKernelGGL((k_sad<ES, NW, 33>), grid, dim3(256), lds, s, g);
  return hipGetLastError();
}

template <int ES>
hipError_t sad_dispatch(int NW, int G, dim3 grid, size_t lds, hipStream_t s, const SadArgs& g) {
  switch (NW) {
    case 1: return sad_dispatch_k<ES, 1>(G, grid, lds, s, g);
    case 2: return sad_dispatch_k<ES, 2>(G, grid, lds, s, g);
    case 3: return sad_dispatch_k<ES, 3>(G, grid, lds, s, g);
    case 4: return sad_dispatch_k<ES, 4>(G, grid, lds, s, g);
    case 5: return sad_dispatch_k<ES, 5>(G, grid, lds, s, g);
    case 6: return sad_dispatch_k<ES, 6>(G, grid, lds, s, g);
    case 7: return sad_dispatch_k<ES, 7>(G, grid, lds, s, g);
    case 8: return sad_dispatch_k<ES, 8>(G, grid, lds, s, g);
    case 10: return sad_dispatch_k<ES, 10>(G, grid, lds, s, g);
    case 12: return sad_dispatch_k<ES, 12>(G, grid, lds, s, g);
    case 14: return sad_dispatch_k<ES, 14>(G, grid, lds, s, g);
    case 16: return sad_dispatch_k<ES, 16>(G, grid, lds, s, g);
    default: break;
  }
  return hipErrorInvalidValue;
}

}  // namespace

bool sad_supported(int block_words) {
  return (block_words >= 1 && block_words <= 8) || block_words == 10 || block_words == 12 ||
         block_words == 14 || block_words == 16;
}

hipError_t launch_pyramid(const Plan& P, const void* A, const void* B, int64_t pitch, int n,
                          hipStream_t s) {
  for (int l = 1; l < P.L; ++l) {
    const Level& u = P.lv[l - 1];
    const Level& v = P.lv[l];
    const uint8_t* sA = l == 1 ? (const uint8_t*)A : P.ws + u.off_a;
    const uint8_t* sB = l == 1 ? (const uint8_t*)B : P.ws + u.off_b;
    int64_t sp = l == 1 ? pitch : u.pitch;
    int64_t ss = l == 1 ? pitch * P.p.height : (int64_t)P.per_pair;
    int dcols = v.pitch / P.es;
    dim3 blk(64, 4);
    dim3 grid(((dcols + 3) / 4 + 63) / 64, (v.H + 3) / 4, 2 * n);
    if (P.es == 1)
      hipLaunchKernelGGL(k_pyr_down<uint8_t>, grid, blk, 0, s, sA, sB, sp, ss, u.W, u.H, P.ws,
                         (int64_t)v.off_a, (int64_t)v.off_b, v.pitch, (int64_t)P.per_pair, v.H, P.slot_mask);
    else
      hipLaunchKernelGGL(k_pyr_down<uint16_t>, grid, blk, 0, s, sA, sB, sp, ss, u.W, u.H, P.ws,
                         (int64_t)v.off_a, (int64_t)v.off_b, v.pitch, (int64_t)P.per_pair, v.H, P.slot_mask);
    if (hipError_t e = hipGetLastError()) return e;
  }
  return hipSuccess;
}

hipError_t launch_sad_level(const Plan& P, int l, const void* A, const void* B, int64_t pitch, int n,
                            hipStream_t s) {
  const Level& v = P.lv[l];
  SadArgs g;
  g.A = l == 0 ? (const uint8_t*)A : P.ws + v.off_a;
  g.B = l == 0 ? (const uint8_t*)B : P.ws + v.off_b;
  g.pitch = l == 0 ? pitch : v.pitch;
  g.stride = l == 0 ? pitch * P.p.height : (int64_t)P.per_pair;
  g.W = v.W;
  g.H = v.H;
  g.nx = v.nx;
  g.ny = v.ny;
  g.step = P.p.step;
  g.block = P.block;
  g.R = l == P.L - 1 ? P.p.radius_coarse : P.p.radius_fine;
  if (l == P.L - 1) {
    g.parent = nullptr;
    g.pstride = 0;
    g.pnx = g.pny = 0;
  } else {
    const Level& u = P.lv[l + 1];
    g.parent = reinterpret_cast<const int32_t*>(P.ws + u.off_d);
    g.pstride = (int64_t)(P.per_pair / sizeof(int32_t));
    g.pnx = u.nx;
    g.pny = u.ny;
  }
  g.median = P.p.median;
  g.out = reinterpret_cast<int32_t*>(P.ws + v.off_d);
  g.ostride = (int64_t)(P.per_pair / sizeof(int32_t));
  g.mask = P.slot_mask;
  const int G = 2 * g.R + 1;
  const int NW = P.block * P.es / 4;
  // nodes per workgroup: G lanes each, A blocks within 64 KiB of LDS
  const int npw = min(256 / G, 65536 / (P.block * NW * 4));
  g.npw = npw;
  dim3 grid((v.nx + npw - 1) / npw, v.ny, n);
  size_t lds = sizeof(uint32_t) * (size_t)npw * P.block * NW;
  return P.es == 1 ? sad_dispatch<1>(NW, G, grid, lds, s, g) : sad_dispatch<2>(NW, G, grid, lds, s, g);
}

hipError_t launch_pred_out(const Plan& P, int n, float* pred, hipStream_t s) {
  const Level& v = P.lv[0];
  dim3 grid((v.nx * v.ny + 255) / 256, n);
  hipLaunchKernelGGL(k_pred_out, grid, dim3(256), 0, s, reinterpret_cast<const int32_t*>(P.ws + v.off_d),
                     (int64_t)(P.per_pair / sizeof(int32_t)), v.nx, v.ny, P.p.median, pred, P.slot_mask);
  return hipGetLastError();
}

}  // namespace piv
