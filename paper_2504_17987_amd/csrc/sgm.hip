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

// Minimum over the wave by DPP (every lane gets it; min is idempotent, so
// lanes of masked rows keeping their own value is harmless)
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  int x = (int)v;
  x = (int)min((uint32_t)x, (uint32_t)PIV_DPP_I(x, 0xB1, 0xF, x));
  x = (int)min((uint32_t)x, (uint32_t)PIV_DPP_I(x, 0x4E, 0xF, x));
  x = (int)min((uint32_t)x, (uint32_t)PIV_DPP_I(x, 0x141, 0xF, x));
  x = (int)min((uint32_t)x, (uint32_t)PIV_DPP_I(x, 0x140, 0xF, x));
  x = (int)min((uint32_t)x, (uint32_t)PIV_DPP_I(x, 0x142, 0xA, x));
  x = (int)min((uint32_t)x, (uint32_t)PIV_DPP_I(x, 0x143, 0xC, x));
  return (uint32_t)__builtin_amdgcn_readlane(x, 63);
}

// The previous node's path costs live in LDS on a (2R+3)^2 grid whose
// one-cell border holds 0xffffffff, so every candidate reads its eight
// neighbours without bounds tests (a border never wins the minimum, and
// every candidate has at least one real neighbour since R >= 1).
constexpr int kMaxR = 16, kPad = 2 * kMaxR + 3, kPrevWords = kPad * kPad + 1;

// Per-lane candidate constants of a wave (kPer candidates per lane).
template <int kPer>
struct Cand {
  int rd[kPer];        // LDS cell read as the candidate's own (a real cell even for padding lanes)
  int wr[kPer];        // LDS cell written (a spare word for padding lanes)
  bool ok[kPer];       // a real candidate (k < nd)
  uint32_t code[kPer]; // tie code (|dx|+|dy|, dy, dx) of the winner search
};

// One path direction over one line of nodes by one wave.  The costs (and
// the running sums) of the node two ahead are requested before a node is
// worked, into two register sets used in turn, so the global reads overlap
// more than one node's work.  The workgroup is the one wave: its LDS reads
// and writes complete in program order, so the exchange of the previous
// node's costs needs no barrier (and none that would wait for the requests
// in flight).  kWrite: the path's costs are stored into S (the first of the
// four passes), otherwise added; kWta (the last pass): the node's total is
// final and its winner, the least (S, |dx|+|dy|, dy, dx), is written.
template <int kPer, bool kWrite, bool kWta>
__device__ void sgm_path(const SgmArgs& g, const Cand<kPer>& cd, const uint32_t* C, uint32_t* S, int len,
                         int64_t nstride, bool reverse, uint32_t* prev, int32_t* out, int node0, int nodestep) {
  const int t = threadIdx.x;
  const int P = 2 * g.R + 3;
  const int np = g.nx * g.ny;
  // (unconditional reads, padding lanes from the node's first candidate and
  // nodes past the end from the last node, so that the requests in flight
  // need no branches; the values are masked where they are used)
  auto request = [&](int s, uint32_t (&c_)[kPer], uint32_t (&s_)[kPer]) __attribute__((always_inline)) {
    const int sc = min(s, len - 1);
    const int pos = reverse ? len - 1 - sc : sc;
    const uint32_t* c = C + pos * nstride;
    const uint32_t* sp = S + pos * nstride;
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const int k = cd.ok[e] ? t + e * 64 : 0;
      c_[e] = c[k];
      if constexpr (!kWrite) s_[e] = sp[k];
    }
  };
  auto node = [&](int s, uint32_t (&cq)[kPer], uint32_t (&sq)[kPer]) __attribute__((always_inline)) {
    const int pos = reverse ? len - 1 - s : s;
    uint32_t* sp = S + pos * nstride;
    uint32_t cv[kPer], sv[kPer], cur[kPer];
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      cv[e] = cd.ok[e] ? cq[e] : 0u;
      sv[e] = kWrite ? 0u : sq[e];
    }
    request(s + 2, cq, sq);
    // (the first node takes its own costs; its reads of prev are unused)
    uint32_t own[kPer], nb[kPer];
    uint32_t lmin = 0xffffffffu;
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      const uint32_t* q = prev + cd.rd[e];
      own[e] = q[0];
      nb[e] = min(min(min(q[-P - 1], q[-P]), min(q[-P + 1], q[-1])), min(min(q[1], q[P - 1]), min(q[P], q[P + 1])));
      lmin = min(lmin, cd.ok[e] ? own[e] : 0xffffffffu);
    }
    const uint32_t m = wave_min_u32(lmin);
#pragma unroll
    for (int e = 0; e < kPer; ++e) cur[e] = s == 0 ? cv[e] : cv[e] + min(min(own[e], nb[e] + g.P1), m + g.P2) - m;
    // (every lane's reads of prev above are issued before these writes)
    __builtin_amdgcn_wave_barrier();
    uint32_t best = 0xffffffffu, code = 0xffffffffu;
#pragma unroll
    for (int e = 0; e < kPer; ++e) {
      prev[cd.wr[e]] = cur[e];
      const uint32_t tot = kWrite ? cur[e] : sv[e] + cur[e];
      if constexpr (kWta) {
        const uint32_t tv = cd.ok[e] ? tot : 0xffffffffu;
        code = tv < best ? cd.code[e] : (tv == best ? min(code, cd.code[e]) : code);
        best = min(best, tv);
      } else {
        if (cd.ok[e]) sp[t + e * 64] = tot;
      }
    }
    if constexpr (kWta) {
      // (the least total, then among the lanes holding it the least code)
      const uint32_t mt = wave_min_u32(best);
      const uint32_t c = wave_min_u32(best == mt ? code : 0xffffffffu);
      if (t == 0) {
        const int nd = node0 + pos * nodestep;
        out[nd] = (int)(c & 63) - g.R;
        out[np + nd] = (int)((c >> 6) & 63) - g.R;
      }
    }
    // (these writes are issued before the next node's reads)
    __builtin_amdgcn_wave_barrier();
  };
  uint32_t c0[kPer], s0[kPer], c1[kPer], s1[kPer];
  request(0, c0, s0);
  request(1, c1, s1);
  int s = 0;
  for (; s + 1 < len; s += 2) {
    node(s, c0, s0);
    node(s + 1, c1, s1);
  }
  if (s < len) node(s, c0, s0);
  // the pass's sums are complete (in memory and LDS) before the next pass
  __syncthreads();
}

// One wave per line.  dir 0: a node row, left to right then right to left;
// dir 1: a node column, top to bottom then bottom to top, the last pass
// taking each node's winner.
template <int kPer>
__global__ __launch_bounds__(64) void k_sgm_aggregate(SgmArgs g, int dir) {
  __shared__ uint32_t prev[kPrevWords];
  const int pair = blockIdx.y;
  if (slot_off(g.mask, pair)) return;
  const int line = blockIdx.x;
  const int t = threadIdx.x;
  const int n1 = 2 * g.R + 1, P = n1 + 2;
  for (int i = t; i < P * P; i += 64) prev[i] = 0xffffffffu;
  Cand<kPer> cd;
#pragma unroll
  for (int e = 0; e < kPer; ++e) {
    const int k = t + e * 64;
    const bool ok = k < g.nd;
    const int ky = ok ? k / n1 : 0, kx = ok ? k - ky * n1 : 0;
    const int cell = (ky + 1) * P + kx + 1;
    cd.ok[e] = ok;
    cd.rd[e] = cell;
    cd.wr[e] = ok ? cell : P * P;
    cd.code[e] = ((uint32_t)(abs(ky - g.R) + abs(kx - g.R)) << 12) | ((uint32_t)ky << 6) | (uint32_t)kx;
  }
  __syncthreads();
  const uint32_t* C = g.C + (int64_t)pair * g.cstride;
  uint32_t* S = g.S + (int64_t)pair * g.cstride;
  int32_t* out = g.out + (int64_t)pair * g.ostride;
  if (dir == 0) {
    const int64_t base = (int64_t)line * g.nx * g.nd;
    sgm_path<kPer, true, false>(g, cd, C + base, S + base, g.nx, g.nd, false, prev, out, 0, 0);
    sgm_path<kPer, false, false>(g, cd, C + base, S + base, g.nx, g.nd, true, prev, out, 0, 0);
  } else {
    const int64_t base = (int64_t)line * g.nd;
    const int64_t ns = (int64_t)g.nx * g.nd;
    sgm_path<kPer, false, false>(g, cd, C + base, S + base, g.ny, ns, false, prev, out, 0, 0);
    sgm_path<kPer, false, true>(g, cd, C + base, S + base, g.ny, ns, true, prev, out, line, g.nx);
  }
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
  const int per = (g.nd + 63) / 64;
  for (int dir = 0; dir < 2; ++dir) {
    dim3 ga(dir == 0 ? v.ny : v.nx, n);
#define PIV_SGM_AGG(K_) \
  if (per <= K_) { hipLaunchKernelGGL(k_sgm_aggregate<K_>, ga, dim3(64), 0, s, g, dir); }
    PIV_SGM_AGG(1) else PIV_SGM_AGG(3) else PIV_SGM_AGG(4) else PIV_SGM_AGG(8) else PIV_SGM_AGG(12) else PIV_SGM_AGG(18)
#undef PIV_SGM_AGG
    if (hipError_t e = hipGetLastError()) return e;
  }
  return hipGetLastError();
}

}  // namespace piv
