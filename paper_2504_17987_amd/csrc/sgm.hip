// Semi-global matching on the predictor's coarsest level (the family of
// methods the paper's optical-flow engine implements, Sec. 2): the block-SAD
// cost of every candidate displacement at every node, aggregated along four
// paths over the node grid (left to right, right to left, top to bottom,
// bottom to top) with penalty P1 for a one-pixel change of either component
// between path neighbours and P2 for any larger change, then the winner by
// the key (cost, |dx|+|dy|, dy, dx).  Integer arithmetic throughout, so the
// result is exact.  The level field it writes is read by the finer levels'
// block matching exactly as a block-matched coarsest level is.
#include "dev_common.h"
#include "piv_internal.h"

namespace piv {
namespace {

struct SgmArgs {
  const uint8_t* A;   // padded coarsest level, pair 0, at the core origin (0, 0)
  const uint8_t* B;
  int64_t pitch, stride;   // bytes per padded row; bytes per pair of the workspace
  int nx, ny, step, block, R, nd;
  uint32_t* C;        // cost volume [pair][node][nd] (pair stride cstride)
  uint32_t* S;        // aggregated cost, same layout
  int64_t cstride;    // uint32 elements per pair
  uint32_t P1, P2;
  int32_t* out;       // level field [pair][2][ny][nx] (pair stride ostride int32)
  int64_t ostride;
  const uint8_t* mask;
};

// 4 bytes at an arbitrary byte address (two aligned words and a byte
// realignment; the level's margin keeps the second word inside the row)
__device__ __forceinline__ uint32_t ld_u32(const uint8_t* p) {
  const uintptr_t a = reinterpret_cast<uintptr_t>(p);
  const uint32_t* w = reinterpret_cast<const uint32_t*>(a & ~uintptr_t(3));
  return __builtin_amdgcn_alignbyte(w[1], w[0], (uint32_t)(a & 3));
}

// Cost volume: one thread per (node, candidate); SAD of the block of A at
// the node with B moved by the candidate, four pixels per v_sad.
template <int ES>
__global__ __launch_bounds__(256) void k_sgm_cost(SgmArgs g) {
  const int pair = blockIdx.z;
  if (slot_off(g.mask, pair)) return;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t total = (int64_t)g.nx * g.ny * g.nd;
  if (i >= total) return;
  const int node = (int)(i / g.nd), k = (int)(i - (int64_t)node * g.nd);
  const int n1 = 2 * g.R + 1;
  const int dy = k / n1 - g.R, dx = k - (k / n1) * n1 - g.R;
  const int a = node / g.nx, b = node - (node / g.nx) * g.nx;
  const int off = (g.step - g.block) / 2;
  const int oy = a * g.step + off, ox = b * g.step + off;
  const uint8_t* Ab = g.A + (int64_t)pair * g.stride + (int64_t)oy * g.pitch + (int64_t)ox * ES;
  const uint8_t* Bb = g.B + (int64_t)pair * g.stride + (int64_t)(oy + dy) * g.pitch + (int64_t)(ox + dx) * ES;
  const int nw = g.block * ES / 4;
  uint32_t s = 0u;
  for (int r = 0; r < g.block; ++r) {
    const uint8_t* ar = Ab + (int64_t)r * g.pitch;
    const uint8_t* br = Bb + (int64_t)r * g.pitch;
    for (int w = 0; w < nw; ++w) {
      const uint32_t x = ld_u32(ar + 4 * w), y = ld_u32(br + 4 * w);
      s = ES == 1 ? __builtin_amdgcn_sad_u8(x, y, s) : __builtin_amdgcn_sad_u16(x, y, s);
    }
  }
  g.C[(int64_t)pair * g.cstride + i] = s;
}

constexpr int kAggT = 256;

// Minimum over the workgroup (every thread gets it)
__device__ __forceinline__ uint32_t block_min(uint32_t v, uint32_t* red) {
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, (uint32_t)__shfl_xor((int)v, o));
  if (lane == 0) red[w] = v;
  __syncthreads();
  uint32_t m = red[0];
#pragma unroll
  for (int q = 1; q < kAggT / 64; ++q) m = min(m, red[q]);
  __syncthreads();
  return m;
}

// One path direction over one line of nodes.  Candidates are spread over
// the workgroup's threads (kPer per thread); the previous node's path costs
// live in LDS.  With `write` the path's costs are stored into S (the first
// of the four passes), otherwise added to it.
template <int kPer>
__device__ void sgm_path(const SgmArgs& g, const uint32_t* C, uint32_t* S, int len, int64_t nstride, bool reverse,
                         bool write, uint32_t* prev, uint32_t* red) {
  const int t = threadIdx.x;
  const int n1 = 2 * g.R + 1;
  uint32_t cur[kPer];
  for (int s = 0; s < len; ++s) {
    const int pos = reverse ? len - 1 - s : s;
    const uint32_t* c = C + pos * nstride;
    uint32_t* sp = S + pos * nstride;
    if (s == 0) {
#pragma unroll
      for (int e = 0; e < kPer; ++e) {
        const int k = t + e * kAggT;
        cur[e] = k < g.nd ? c[k] : 0xffffffffu;
      }
    } else {
      uint32_t lmin = 0xffffffffu;
#pragma unroll
      for (int e = 0; e < kPer; ++e) {
        const int k = t + e * kAggT;
        if (k < g.nd) lmin = min(lmin, prev[k]);
      }
      const uint32_t m = block_min(lmin, red);
#pragma unroll
      for (int e = 0; e < kPer; ++e) {
        const int k = t + e * kAggT;
        if (k < g.nd) {
          const int ky = k / n1, kx = k - (k / n1) * n1;
          uint32_t nb = 0xffffffffu;
#pragma unroll
          for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
            for (int ox = -1; ox <= 1; ++ox) {
              if (!oy && !ox) continue;
              const int y2 = ky + oy, x2 = kx + ox;
              if (y2 >= 0 && x2 >= 0 && y2 < n1 && x2 < n1) nb = min(nb, prev[y2 * n1 + x2]);
            }
          const uint32_t best = min(min(prev[k], nb == 0xffffffffu ? nb : nb + g.P1), m + g.P2);
          cur[e] = c[k] + best - m;
        }
      }
    }
    __syncthreads();   // every thread has read prev
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int k = t + e * kAggT;
      if (k < g.nd) {
        prev[k] = cur[e];
        sp[k] = write ? cur[e] : sp[k] + cur[e];
      }
    }
    __syncthreads();
  }
}

// dir 0: one workgroup per node row, left to right then right to left;
// dir 1: one workgroup per node column, top to bottom then bottom to top.
template <int kPer>
__global__ __launch_bounds__(kAggT) void k_sgm_aggregate(SgmArgs g, int dir) {
  __shared__ uint32_t prev[kPer * kAggT];
  __shared__ uint32_t red[kAggT / 64];
  const int pair = blockIdx.y;
  if (slot_off(g.mask, pair)) return;
  const int line = blockIdx.x;
  const uint32_t* C = g.C + (int64_t)pair * g.cstride;
  uint32_t* S = g.S + (int64_t)pair * g.cstride;
  if (dir == 0) {
    const int64_t base = (int64_t)line * g.nx * g.nd;
    sgm_path<kPer>(g, C + base, S + base, g.nx, g.nd, false, true, prev, red);
    sgm_path<kPer>(g, C + base, S + base, g.nx, g.nd, true, false, prev, red);
  } else {
    const int64_t base = (int64_t)line * g.nd;
    const int64_t ns = (int64_t)g.nx * g.nd;
    sgm_path<kPer>(g, C + base, S + base, g.ny, ns, false, false, prev, red);
    sgm_path<kPer>(g, C + base, S + base, g.ny, ns, true, false, prev, red);
  }
}

// Winner per node: least (S, |dx|+|dy|, dy, dx), as one 64-bit key.
__global__ __launch_bounds__(256) void k_sgm_wta(SgmArgs g) {
  const int pair = blockIdx.y;
  if (slot_off(g.mask, pair)) return;
  const int node = blockIdx.x * 256 + threadIdx.x;
  const int np = g.nx * g.ny;
  if (node >= np) return;
  const uint32_t* S = g.S + (int64_t)pair * g.cstride + (int64_t)node * g.nd;
  const int n1 = 2 * g.R + 1;
  uint64_t best = ~uint64_t(0);
  for (int k = 0; k < g.nd; ++k) {
    const int ky = k / n1, kx = k - (k / n1) * n1;
    const int l = abs(ky - g.R) + abs(kx - g.R);
    const uint64_t key = ((uint64_t)S[k] << 18) | ((uint64_t)l << 12) | ((uint64_t)ky << 6) | (uint64_t)kx;
    best = key < best ? key : best;
  }
  const int ky = (int)((best >> 6) & 63), kx = (int)(best & 63);
  int32_t* o = g.out + (int64_t)pair * g.ostride;
  o[node] = kx - g.R;
  o[np + node] = ky - g.R;
}

}  // namespace

hipError_t launch_sgm_level(const Plan& P, int n, hipStream_t s) {
  const Level& v = P.lv[P.L - 1];
  SgmArgs g;
  const size_t origin = (size_t)v.margin * v.pitch + (size_t)v.margin * P.es;
  g.A = P.ws + v.off_a + origin;
  g.B = P.ws + v.off_b + origin;
  g.pitch = v.pitch;
  g.stride = (int64_t)P.per_pair;
  g.nx = v.nx;
  g.ny = v.ny;
  g.step = P.p.step;
  g.block = P.block;
  g.R = v.R;
  g.nd = (2 * v.R + 1) * (2 * v.R + 1);
  g.C = reinterpret_cast<uint32_t*>(P.ws + P.off_sgm_c);
  g.S = reinterpret_cast<uint32_t*>(P.ws + P.off_sgm_s);
  g.cstride = (int64_t)(P.per_pair / sizeof(uint32_t));
  const uint32_t bb = (uint32_t)(P.block * P.block);
  g.P1 = (uint32_t)P.p.sgm_p1 * bb;
  g.P2 = (uint32_t)P.p.sgm_p2 * bb;
  g.out = reinterpret_cast<int32_t*>(P.ws + v.off_d);
  g.ostride = (int64_t)(P.per_pair / sizeof(int32_t));
  g.mask = P.slot_mask;
  // cost volume: by the cell-shared coarse SAD kernel where its geometry
  // applies, otherwise one thread per node and candidate
  hipError_t ec = launch_sad_cost_cells(P, g.C, g.cstride, n, s);
  if (ec == hipErrorNotSupported) {
    const int64_t total = (int64_t)v.nx * v.ny * g.nd;
    dim3 gc((unsigned)((total + 255) / 256), 1, n);
    if (P.es == 1) hipLaunchKernelGGL(k_sgm_cost<1>, gc, dim3(256), 0, s, g);
    else hipLaunchKernelGGL(k_sgm_cost<2>, gc, dim3(256), 0, s, g);
    ec = hipGetLastError();
  }
  if (ec != hipSuccess) return ec;
  const int per = (g.nd + kAggT - 1) / kAggT;
  for (int dir = 0; dir < 2; ++dir) {
    dim3 ga(dir == 0 ? v.ny : v.nx, n);
#define PIV_SGM_AGG(K_) \
  if (per <= K_) { hipLaunchKernelGGL(k_sgm_aggregate<K_>, ga, dim3(kAggT), 0, s, g, dir); }
    PIV_SGM_AGG(1) else PIV_SGM_AGG(2) else PIV_SGM_AGG(3) else PIV_SGM_AGG(5)
#undef PIV_SGM_AGG
    if (hipError_t e = hipGetLastError()) return e;
  }
  dim3 gw((v.nx * v.ny + 255) / 256, n);
  hipLaunchKernelGGL(k_sgm_wta, gw, dim3(256), 0, s, g);
  return hipGetLastError();
}

}  // namespace piv
