// Predictor kernels: padded pyramid, per-level integer SAD block search with
// a packed-key argmin, and the final 3x3 median to the float field.
//
// The predictor stands where the paper (Sec. 2) uses a fixed-function
// optical-flow engine: a coarse, integer-accurate displacement estimate
// that the correlation stage then corrects.
//
// Every level, level 0 included (a copy of the input), is stored in the
// workspace with a zero margin wide enough for the level's whole search
// reach (see Level in piv_internal.h): the SAD kernels read aligned words
// with no bounds checks, and zero outside the image comes from the margin.
#include "dev_common.h"
#include "piv_internal.h"

namespace piv {
namespace {

// ---------------------------------------------------------------------------
// Zero margins of one padded level (both frames, every pair the workspace
// holds): every 4-byte word of a padded row that lies wholly outside the
// image core.  The copy kernels below write the core only (plus the zero
// tail of a ragged last word), so this runs once per bound workspace.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_clear_margins(uint8_t* ws, int64_t stride, int64_t offA, int64_t offB,
                                                       int pitch, int rows, int mbytes, int cbytes, int mrows,
                                                       int H) {
  const int pair = blockIdx.z >> 1, frame = blockIdx.z & 1;
  const int nw = pitch / 4;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int y = (int)(idx / nw);
  const int w = (int)(idx - (int64_t)y * nw);
  if (y >= rows) return;
  const int xb = 4 * w;
  const int core_end = (mbytes + cbytes + 3) & ~3;   // end of the last (maybe ragged) core word
  const bool core_row = y >= mrows && y < mrows + H;
  if (core_row && xb + 4 > mbytes && xb < core_end) return;
  uint8_t* row = ws + (int64_t)pair * stride + (frame ? offB : offA) + (int64_t)y * pitch;
  *reinterpret_cast<uint32_t*>(row + xb) = 0u;
}

// ---------------------------------------------------------------------------
// Level 0 core copy fused with levels 1 and 2.  Every level is
// out(y,x) = floor((in(2y,2x) + in(2y,2x+1) + in(2y+1,2x) + in(2y+1,2x+1) + 2) / 4)
// of the level below, zero outside its image.  One thread per 16-byte column
// chunk and pair of image rows (2k, 2k+1), or with L2 per four image rows:
// it copies the rows into the padded level-0 buffer and writes the chunk's
// level-1 means (and, with L2, the means of those, level 2).  Rows and
// columns past the image read as zero (the level's margin).
// ---------------------------------------------------------------------------
struct PyrDst {
  int64_t offA, offB;   // per-pair offsets of the level's padded buffers
  int pitch, m, W, H;   // bytes per row, margin (px), level size (px)
};

template <typename T, bool L2>
__global__ __launch_bounds__(256) void k_pad_pyr(const uint8_t* __restrict__ A, const uint8_t* __restrict__ B,
                                                 int64_t spitch, int64_t sstride, int W, int H, uint8_t* ws,
                                                 int64_t stride, PyrDst d0, PyrDst d1, PyrDst d2, int do_l1,
                                                 int lframe, const uint8_t* mask) {
  constexpr int ES = (int)sizeof(T);
  constexpr int NP = 16 / ES, NO = NP / 2;   // pixels of a chunk, level-1 pixels they give
  constexpr int NR = L2 ? 2 : 1;             // row pairs per thread
  const int pair = blockIdx.z >> 1, frame = blockIdx.z & 1;
  if (slot_off(mask, pair)) return;
  const int rowbytes = W * ES;
  const int nq = (rowbytes + 15) / 16;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int kk = idx / nq, q = idx - (idx / nq) * nq;
  if (kk >= (H + 2 * NR - 1) / (2 * NR)) return;
  const uint8_t* src = (frame ? B : A) + (int64_t)pair * sstride;
  uint8_t* base = ws + (int64_t)pair * stride;
  // whole chunks of rows inside the image, from 16-byte aligned addresses,
  // take one 16-byte read; the ragged right end and missing last rows are
  // read word by word with zero fill
  const bool whole = 16 * q + 16 <= rowbytes && ((reinterpret_cast<uintptr_t>(src) | spitch) & 15) == 0;
  const int x0 = d0.m * ES + 16 * q;   // byte offset of the chunk in a padded level-0 row (16-aligned)
  // lframe > 0: level 0 is read in place except near its edges, so only the
  // chunks and rows within lframe px of an edge are copied
  const bool col_edge = lframe == 0 || 16 * q < lframe * ES || 16 * q + 16 > (W - lframe) * ES;
  uint32_t s[NR][NO];   // level-1 pixels of the chunk, per row pair
#pragma unroll
  for (int h2 = 0; h2 < NR; ++h2) {
    const int k = NR * kk + h2;   // level-1 row
    uint32_t w[2][4];
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int y = 2 * k + r;
      const uint8_t* row = src + (int64_t)min(y, H - 1) * spitch;
      if (whole && y < H) {
        const uint4 v = *reinterpret_cast<const uint4*>(row + 16 * q);
        w[r][0] = v.x; w[r][1] = v.y; w[r][2] = v.z; w[r][3] = v.w;
      } else {
        const uint32_t ok = y < H ? 0xffffffffu : 0u;
#pragma unroll
        for (int i = 0; i < 4; ++i) w[r][i] = masked_word(row, rowbytes, 16 * q + 4 * i) & ok;
      }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int y = 2 * k + r;
      const bool edge = col_edge || y < lframe || y >= H - lframe;
      uint8_t* row = base + (frame ? d0.offB : d0.offA) + (int64_t)(y + d0.m) * d0.pitch;
      if (edge && x0 + 16 <= d0.pitch) *reinterpret_cast<uint4*>(row + x0) = make_uint4(w[r][0], w[r][1], w[r][2], w[r][3]);
    }
    if (!do_l1) return;
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      uint32_t acc = 2u;
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int px = 2 * j + h;                  // pixel in the chunk
          const int bit = (px * ES * 8) & 31, wd = (px * ES) / 4;
          acc += (w[r][wd] >> bit) & (ES == 1 ? 0xffu : 0xffffu);
        }
      const int x1 = q * NO + j;
      s[h2][j] = (k < d1.H && x1 < d1.W) ? (acc >> 2) : 0u;
    }
    uint32_t o[2] = {0u, 0u};
#pragma unroll
    for (int j = 0; j < NO; ++j) o[(j * ES) / 4] |= s[h2][j] << ((j * ES * 8) & 31);
    uint8_t* row1 = base + (frame ? d1.offB : d1.offA) + (int64_t)(k + d1.m) * d1.pitch;
    const int x1b = d1.m * ES + 8 * q;   // 8-byte aligned
    if (x1b + 8 <= d1.pitch) *reinterpret_cast<uint2*>(row1 + x1b) = make_uint2(o[0], o[1]);
  }
  if constexpr (L2) {
    // the chunk's level-1 2 x NO block -> NO / 2 level-2 pixels (4 bytes)
    uint32_t o = 0u;
#pragma unroll
    for (int j = 0; j < NO / 2; ++j) {
      const uint32_t acc = s[0][2 * j] + s[0][2 * j + 1] + s[1][2 * j] + s[1][2 * j + 1] + 2u;
      const int x2 = q * (NO / 2) + j;
      o |= ((kk < d2.H && x2 < d2.W) ? (acc >> 2) : 0u) << (j * ES * 8);
    }
    uint8_t* row2 = base + (frame ? d2.offB : d2.offA) + (int64_t)(kk + d2.m) * d2.pitch;
    const int x2b = d2.m * ES + 4 * q;   // 4-byte aligned
    if (x2b + 4 <= d2.pitch) *reinterpret_cast<uint32_t*>(row2 + x2b) = o;
  }
}

// ---------------------------------------------------------------------------
// Pyramid level from the padded level below:
// out(y,x) = floor((in(2y,2x) + in(2y,2x+1) + in(2y+1,2x) + in(2y+1,2x+1) + 2) / 4)
// with zero outside the input (its margin).  The core only: the margins
// were zeroed once with the workspace.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_pyr_down(uint8_t* ws, int64_t stride, int64_t sA, int64_t sB,
                                                  int spitch, int smargin, int64_t dA, int64_t dB, int dpitch,
                                                  int dmargin, int dW, int dH, const uint8_t* mask) {
  // one thread: 8 outputs of one row of the level's core from two 16-pixel
  // source rows (aligned 16-byte reads: every level's core starts 16-byte
  // aligned); past the image (a ragged last chunk, inside the margin) it
  // writes 0.
  const int pair = blockIdx.z >> 1, frame = blockIdx.z & 1;
  if (slot_off(mask, pair)) return;
  const int nch = (dW + 7) / 8;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = idx / nch, c = idx - (idx / nch) * nch;
  if (y >= dH) return;
  uint8_t* base = ws + (int64_t)pair * stride;
  const uint8_t* src = base + (frame ? sB : sA) + (int64_t)smargin * spitch + (int64_t)smargin * sizeof(T);
  constexpr int NV = 16 * (int)sizeof(T) / 16;   // 16-byte vectors per 16 source pixels
  const uint4* r0 = reinterpret_cast<const uint4*>(src + (int64_t)(2 * y) * spitch) + NV * c;
  const uint4* r1 = reinterpret_cast<const uint4*>(src + (int64_t)(2 * y + 1) * spitch) + NV * c;
  T a0[16], a1[16];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const uint4 w0 = r0[v], w1 = r1[v];
    __builtin_memcpy(a0 + v * (16 / (int)sizeof(T)), &w0, 16);
    __builtin_memcpy(a1 + v * (16 / (int)sizeof(T)), &w1, 16);
  }
  T o[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const uint32_t sum = (uint32_t)a0[2 * i] + a0[2 * i + 1] + a1[2 * i] + a1[2 * i + 1];
    o[i] = (8 * c + i < dW) ? (T)((sum + 2u) >> 2) : (T)0;
  }
  T* out = reinterpret_cast<T*>(base + (frame ? dB : dA) + (int64_t)(dmargin + y) * dpitch) + dmargin + 8 * c;
  if constexpr (sizeof(T) == 1) {
    uint2 w;
    __builtin_memcpy(&w, o, 8);
    *reinterpret_cast<uint2*>(out) = w;
  } else {
    uint4 w;
    __builtin_memcpy(&w, o, 16);
    *reinterpret_cast<uint4*>(out) = w;
  }
}

// ---------------------------------------------------------------------------
// Shared by the SAD kernels
// ---------------------------------------------------------------------------
// N consecutive 4-byte words at a 4-byte-aligned address, read together
// (wide loads: one instruction per up to four words)
template <int N>
struct __attribute__((aligned(4))) Words {
  uint32_t w[N];
};

struct SadArgs {
  const uint8_t* A;   // padded level image, pair 0, at the core origin (0, 0)
  const uint8_t* B;
  int64_t pitch, stride;
  int nx, ny;         // level grid
  int step, block, R;
  const int32_t* parent;  // parent level field [.][2][pny][pnx] or null (coarsest)
  int64_t pstride;        // int32 elements per pair of the parent field
  int pnx, pny;
  int median;
  int32_t* out;           // this level's field
  int64_t ostride;        // int32 elements per pair
  const uint8_t* mask;
  int npw;                // nodes per workgroup (k_sad)
  int qsplit;             // k_sad: groups of candidate rows per candidate column
  int band;               // k_sad without a parent: staged B band row words (at most), 0 = none
  int margin;             // level margin (px): A - margin (pitch + bytes per px) is padded row 0
  // level 0 read in place (k_sad_lane, k_sad_cols, k_sad_stream, k_sad_cells16_fine): an A block or B span wholly inside
  // the image reads the caller's frames (pair 0 at srcA/srcB); one that
  // crosses the image edge reads the padded copy, of which only a frame of
  // kFrame px along the edges is written
  const uint8_t* srcA;
  const uint8_t* srcB;
  int64_t spitch, sstride;
  int W, H;               // level size (px)
  // cost-volume mode of k_sad_cells (semi-global matching): every node's SAD
  // for every shift, [pair][node][(dy+R)(2R+1) + dx+R], pair stride cstride
  uint32_t* cost;
  int64_t cstride;
  int direct;
};

// Depth of the written frame of the level-0 copy when level 0 is read in
// place: a span that crosses the image edge has all of its in-image pixels
// within its own extent of that edge (at most 2R + 24 <= 28 rows and 28
// columns for the u8 kernels, 30 columns for the streamed u16 kernel).
constexpr int kFrame = 32;

template <int ES>
__device__ __forceinline__ uint32_t sad_word(uint32_t a, uint32_t b, uint32_t c) {
  if constexpr (ES == 1) return __builtin_amdgcn_sad_u8(a, b, c);
  else return __builtin_amdgcn_sad_u16(a, b, c);
}

// 4-byte word of a padded row at a (possibly unaligned) byte offset
__device__ __forceinline__ uint32_t word_at(const uint8_t* row, int xb) {
  const int xa = xb & ~3, sh = xb & 3;
  const uint32_t* p = reinterpret_cast<const uint32_t*>(row + xa);
  return __builtin_amdgcn_alignbyte(p[1], p[0], sh);
}

// Candidate centre component: twice the parent node's result, through the
// 3x3 median of the parent level when enabled (the median after the parent
// level, taken where it is read).
__device__ __forceinline__ int parent_value(const SadArgs& g, const int32_t* par, int comp, int pa, int pb) {
  const int32_t* P = par + (int64_t)comp * g.pnx * g.pny;
  if (!g.median) return P[pa * g.pnx + pb];
  int v[9];
  int k = 0;
#pragma unroll
  for (int i = -1; i <= 1; ++i)
#pragma unroll
    for (int j = -1; j <= 1; ++j) {
      int y = pa + i, x = pb + j;
      bool in = y >= 0 && x >= 0 && y < g.pny && x < g.pnx;
      v[(i + 1) * 3 + j + 1] = in ? P[y * g.pnx + x] : kSlotI;
      k += in;
    }
  return median9_low_i(v, k);
}

// Both components of the candidate centre at once (twice the parent's
// result, through its 3x3 median when enabled): the 18 reads go to clamped,
// always valid addresses and are all in flight before the first is used.
__device__ __forceinline__ void parent_centre(const SadArgs& g, const int32_t* par, int pa, int pb, int& cx,
                                              int& cy) {
  const int np = g.pnx * g.pny;
  if (!g.median) {
    cx = 2 * par[pa * g.pnx + pb];
    cy = 2 * par[np + pa * g.pnx + pb];
    return;
  }
  int vx[9], vy[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int o = min(max(pa + i - 1, 0), g.pny - 1) * g.pnx + min(max(pb + j - 1, 0), g.pnx - 1);
      vx[i * 3 + j] = par[o];
      vy[i * 3 + j] = par[np + o];
    }
  int k = 0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int y = pa + i - 1, x = pb + j - 1;
      const bool in = y >= 0 && x >= 0 && y < g.pny && x < g.pnx;
      if (!in) vx[i * 3 + j] = vy[i * 3 + j] = kSlotI;
      k += in;
    }
  cx = 2 * median9_low_i(vx, k);
  cy = 2 * median9_low_i(vy, k);
}

__device__ __forceinline__ unsigned long long sad_key(uint32_t sad, int dy, int dx) {
  const unsigned l1 = (unsigned)(abs(dx) + abs(dy));
  return ((unsigned long long)sad << 25) | ((unsigned long long)l1 << 16) |
         ((unsigned long long)(dy + 128) << 8) | (unsigned long long)(dx + 128);
}

// ---------------------------------------------------------------------------
// SAD block search for u8 blocks of at most 16 pixels and any R: a group of
// G = 2R+1 lanes per node, lane q owning the candidate row dy = cand_y - R + q
// and every candidate column, four at a time with v_qsad_pk_u16_u8 (four
// 16-bit SADs of one A word against four byte offsets of an 8-byte B span).
// The node's A block is staged in LDS; each lane streams its BLK rows of B.
// Without a parent (the coarsest level) every node of a workgroup searches
// the same rows, so with STAGE the band of B they cover (one span of words
// per row, the nodes step/4 words apart) is staged in LDS too, instead of
// each lane reading its own row from global memory.
// Winner as in the other forms: the minimum packed key over the node's lanes.
// ---------------------------------------------------------------------------
template <int NW, int NGRP, bool STAGE>
__global__ __launch_bounds__(256) void k_sad_q(SadArgs g) {
  constexpr int BLK = 4 * NW, RW = NW + NGRP;
  static_assert(BLK * BLK * 255 <= 65535, "16-bit SAD fields");
  extern __shared__ uint32_t s_ablk[];        // [npw][BLK][NW], then (STAGE) [G + BLK - 1][nwb]
  __shared__ unsigned long long s_key[256];

  const WgIdx wg = xcd_order();
  const int pair = wg.z;
  if (slot_off(g.mask, pair)) return;
  const int G = 2 * g.R + 1;
  const int npw = g.npw;
  const int t = threadIdx.x;
  const int j = t / G, q = t - j * G;
  const int a = wg.y;
  const int b0 = wg.x * npw;
  const int b = b0 + j;
  const bool active = j < npw && b < g.nx;
  const int off = (g.step - BLK) / 2;
  const int oy = a * g.step + off;
  const uint8_t* Ab = g.A + (int64_t)pair * g.stride;
  const uint8_t* Bb = g.B + (int64_t)pair * g.stride;

  const int nblk = min(npw, g.nx - b0);
  for (int idx = t; idx < nblk * BLK * NW; idx += 256) {
    int jj = idx / (BLK * NW), r = (idx / NW) % BLK, w = idx % NW;
    const uint8_t* row = Ab + (int64_t)(oy + r) * g.pitch;
    s_ablk[idx] = word_at(row, (b0 + jj) * g.step + off + 4 * w);
  }
  // (STAGE) the B band: rows oy - R .. oy - R + G + BLK - 2, words from the
  // first node's aligned start; node j's span starts j step/4 words in
  const int nwb = (npw - 1) * (g.step >> 2) + RW + 1;   // words per staged row
  uint32_t* s_b = s_ablk + npw * BLK * NW;
  if constexpr (STAGE) {
    const int x0 = (b0 * g.step + off - g.R) & ~3;
    const int nw = (nblk - 1) * (g.step >> 2) + RW + 1;   // words the active nodes read
    const int nr = G + BLK - 1;
    for (int idx = t; idx < nr * nw; idx += 256) {
      const int r = idx / nw, w = idx - r * nw;
      s_b[r * nwb + w] = *reinterpret_cast<const uint32_t*>(Bb + (int64_t)(oy - g.R + r) * g.pitch + x0 + 4 * w);
    }
  }

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
    const int xs = b * g.step + off + cx - g.R;
    const int xa = xs & ~3, sh = xs & 3;
    const int by = oy + cy - g.R + q;
    // the last group of four candidate columns holds REM real ones; with one
    // or two, plain v_sad_u8 (full rate) replaces the quarter-rate quad SAD
    const int REM = G - 4 * (NGRP - 1);
    const bool tail_sad = REM <= 2;
    unsigned long long acc[NGRP];
    uint32_t tacc[2] = {0u, 0u};
#pragma unroll
    for (int m = 0; m < NGRP; ++m) acc[m] = 0ull;
    const uint32_t* ablk = s_ablk + j * BLK * NW;
#pragma unroll 4
    for (int ar = 0; ar < BLK; ++ar) {
      const uint32_t* row = STAGE ? s_b + (q + ar) * nwb + j * (g.step >> 2)
                                  : reinterpret_cast<const uint32_t*>(Bb + (int64_t)(by + ar) * g.pitch + xa);
      uint32_t w[RW + 1];
#pragma unroll
      for (int i = 0; i <= RW; ++i) w[i] = row[i];
      uint32_t rw[RW];
#pragma unroll
      for (int i = 0; i < RW; ++i) rw[i] = __builtin_amdgcn_alignbyte(w[i + 1], w[i], sh);
      uint32_t aw[NW];
#pragma unroll
      for (int i = 0; i < NW; ++i) aw[i] = ablk[ar * NW + i];
#pragma unroll
      for (int m = 0; m < NGRP; ++m) {
        if (m == NGRP - 1 && tail_sad) {
          // columns 4m and 4m+1: words i+m and (realigned by one byte) i+m..i+m+1
#pragma unroll
          for (int i = 0; i < NW; ++i) {
            tacc[0] = __builtin_amdgcn_sad_u8(aw[i], rw[i + m], tacc[0]);
            if (REM == 2)
              tacc[1] = __builtin_amdgcn_sad_u8(aw[i], __builtin_amdgcn_alignbyte(rw[i + m + 1], rw[i + m], 1), tacc[1]);
          }
          continue;
        }
        unsigned long long s = acc[m];
#pragma unroll
        for (int i = 0; i < NW; ++i) {
          const unsigned long long src = ((unsigned long long)rw[i + m + 1] << 32) | rw[i + m];
          s = __builtin_amdgcn_qsad_pk_u16_u8(src, aw[i], s);
        }
        acc[m] = s;
      }
    }
    const int dy = cy - g.R + q;
#pragma unroll
    for (int m = 0; m < NGRP; ++m)
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) {
        const int k = 4 * m + jj;
        if (k < G) {
          const uint32_t sad = (m == NGRP - 1 && tail_sad) ? tacc[jj & 1] : (uint32_t)(acc[m] >> (16 * jj)) & 0xffffu;
          unsigned long long key = sad_key(sad, dy, cx - g.R + k);
          best = key < best ? key : best;
        }
      }
  }
  s_key[t] = best;
  __syncthreads();
  if (active && q == 0) {
    unsigned long long m = s_key[t];
    for (int k = 1; k < G; ++k) m = s_key[t + k] < m ? s_key[t + k] : m;
    int32_t* out = g.out + (int64_t)pair * g.ostride;
    out[a * g.nx + b] = (int)(m & 0xff) - 128;
    out[g.nx * g.ny + a * g.nx + b] = (int)((m >> 8) & 0xff) - 128;
  }
}

// passes of DYG shift rows over the 2R+1 of a coarse search
template <int R, int DYG>
constexpr int sad_passes() { return (2 * R + 1 + DYG - 1) / DYG; }

// ---------------------------------------------------------------------------
// Coarsest-level SAD search with cell-shared sums (u8, block = 2 step,
// step 8).  Without a parent every node searches the same (2R+1)^2 shifts,
// and a node's 16x16 block is four 8x8 cells that it shares with its
// neighbours, so the SAD of a block is the sum of four cell SADs for the same
// shift: each pixel difference is taken once instead of four times.
// Lane = cell of a 9x7 tile (8x6 nodes per tile); the lane keeps its A cell
// in registers and streams the B rows once per pass of DYG shift rows, four
// shift columns per quad SAD (16-bit
// fields: a cell is at most 64 x 255).  Cell sums become block sums with a
// DPP add of the right-hand cell (lane + 1) and a lane permute of the cell
// below (lane + 9); four cells stay below 2^16, so the packed fields add
// without carries.  Winner: the least (SAD, |dx|+|dy|, dy, dx).  A
// workgroup is one tile; its waves take the passes side by side (a coarse
// level has few tiles) and the first wave merges their winners.
// ---------------------------------------------------------------------------
template <int R, int DYG, bool kCost = false>
__global__ __launch_bounds__(64 * ((2 * R + DYG) / DYG)) void k_sad_cells(SadArgs g) {
  constexpr int G = 2 * R + 1, NGRP = (G + 3) / 4, REM = G - 4 * (NGRP - 1);
  constexpr bool TAIL = REM <= 2;           // last group by full-rate v_sad_u8
  constexpr int NQ = TAIL ? NGRP - 1 : NGRP;  // groups by quad SAD
  constexpr int CWD = 2, RW = CWD + NGRP;     // cell words, realigned B words
  constexpr int CW = 9, CH = 7, NPASS = sad_passes<R, DYG>();
  static_assert(G <= 15, "4-bit shift indices in the key");
  __shared__ uint32_t s_win[NPASS][64];
  const int lane = threadIdx.x & 63;
  const int ps = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // this wave's pass
  const int pair = blockIdx.z;
  if (slot_off(g.mask, pair)) return;
  const int ntx = (g.nx + CW - 2) / (CW - 1), nty = (g.ny + CH - 2) / (CH - 1);
  const int tile = blockIdx.x;
  if (tile >= ntx * nty) return;   // the whole workgroup
  const int ty = tile / ntx, tx = tile - ty * ntx;
  const int lr = lane / CW, lc = lane - lr * CW;
  // cells beyond the last node's read the last needed cell (results unused)
  const int ci = min(ty * (CH - 1) + lr, g.ny), cj = min(tx * (CW - 1) + lc, g.nx);
  const int y = ci * 8 - 4, x = cj * 8 - 4;
  // 32-bit offsets from padded row 0 (the launcher checks that a padded
  // level fits 31 bits): a row costs one add of a uniform step
  const unsigned pitch32 = (unsigned)g.pitch;
  const uint8_t* Ap = g.A + (int64_t)pair * g.stride - ((int64_t)g.margin * g.pitch + g.margin);
  const uint8_t* Bp = g.B + (int64_t)pair * g.stride - ((int64_t)g.margin * g.pitch + g.margin);
  const unsigned aoff = __umul24((unsigned)(y + g.margin), pitch32) + (unsigned)(x + g.margin);
  uint32_t aw[8][CWD];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const Words<CWD> v = *reinterpret_cast<const Words<CWD>*>(Ap + (size_t)(aoff + r * pitch32));
    aw[r][0] = v.w[0];
    aw[r][1] = v.w[1];
  }
  const int xa = (x - R) & ~3, sh = (x - R) & 3;
  const unsigned boff = __umul24((unsigned)(y - R + g.margin), pitch32) + (unsigned)(xa + g.margin);
  const int node_a = ty * (CH - 1) + lr, node_b = tx * (CW - 1) + lc;
  const bool node = lr < CH - 1 && lc < CW - 1 && node_a < g.ny && node_b < g.nx;
  uint32_t best = ~0u;
  // (cost mode: this node's row of the cost volume)
  uint32_t* const crow = kCost && node ? g.cost + (int64_t)pair * g.cstride + (int64_t)(node_a * g.nx + node_b) * (G * G)
                                       : nullptr;
  {
    const int k0 = ps * DYG;                 // first shift row of the pass
    const int nk = min(DYG, G - k0);         // shift rows in the pass
    unsigned long long acc[DYG][NQ > 0 ? NQ : 1];
    uint32_t tacc[DYG][2];
#pragma unroll
    for (int k = 0; k < DYG; ++k) {
#pragma unroll
      for (int m = 0; m < (NQ > 0 ? NQ : 1); ++m) acc[k][m] = 0ull;
      tacc[k][0] = tacc[k][1] = 0u;
    }
#pragma unroll
    for (int rb = 0; rb < 8 + DYG - 1; ++rb) {
      if (rb >= 8 + nk - 1) continue;
      // B row y + (k0 - R) + rb: it meets A row rb - k for shift row k0 + k
      const Words<RW + 1> wv =
          *reinterpret_cast<const Words<RW + 1>*>(Bp + (size_t)(boff + (unsigned)(k0 + rb) * pitch32));
      uint32_t rw[RW];
#pragma unroll
      for (int i = 0; i < RW; ++i) rw[i] = __builtin_amdgcn_alignbyte(wv.w[i + 1], wv.w[i], sh);
#pragma unroll
      for (int k = 0; k < DYG; ++k) {
        const int r = rb - k;
        if (r < 0 || r >= 8 || k0 + k >= G) continue;
#pragma unroll
        for (int i = 0; i < CWD; ++i) {
#pragma unroll
          for (int m = 0; m < NQ; ++m) {
            const unsigned long long src = ((unsigned long long)rw[i + m + 1] << 32) | rw[i + m];
            acc[k][m] = __builtin_amdgcn_qsad_pk_u16_u8(src, aw[r][i], acc[k][m]);
          }
          if constexpr (TAIL) {
            tacc[k][0] = __builtin_amdgcn_sad_u8(aw[r][i], rw[i + NQ], tacc[k][0]);
            if constexpr (REM == 2)
              tacc[k][1] = __builtin_amdgcn_sad_u8(aw[r][i], __builtin_amdgcn_alignbyte(rw[i + NQ + 1], rw[i + NQ], 1),
                                                   tacc[k][1]);
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
    // block sums: + right cell (DPP wave_shl:1), then + the cell row below
    auto quad = [&](uint32_t v) {
      const uint32_t h = v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xF, 0xF, false);
      return h + (uint32_t)__builtin_amdgcn_ds_bpermute((lane + CW) << 2, (int)h);
    };
#pragma unroll
    for (int k = 0; k < DYG; ++k) {
      if (k0 + k >= G) continue;
      const int dy = k0 + k - R;
      const uint32_t kdy = ((uint32_t)abs(dy) << 8) | ((uint32_t)(dy + R) << 4);
#pragma unroll
      for (int m = 0; m < NQ; ++m) {
        const uint32_t lo = quad((uint32_t)acc[k][m]), hi = quad((uint32_t)(acc[k][m] >> 32));
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const int c = 4 * m + f;
          if (c >= G) continue;
          const uint32_t sad = ((f < 2 ? lo : hi) >> (16 * (f & 1))) & 0xffffu;
          const int dx = c - R;
          if constexpr (kCost) {
            if (node) crow[(dy + R) * G + c] = sad;
          } else {
            best = min(best, (sad << 12) | (kdy + ((uint32_t)abs(dx) << 8)) | (uint32_t)(dx + R));
          }
        }
      }
      if constexpr (TAIL) {
#pragma unroll
        for (int f = 0; f < REM; ++f) {
          const int c = 4 * NQ + f, dx = c - R;
          const uint32_t sad = quad(tacc[k][f]);
          if constexpr (kCost) {
            if (node) crow[(dy + R) * G + c] = sad;
          } else {
            best = min(best, (sad << 12) | (kdy + ((uint32_t)abs(dx) << 8)) | (uint32_t)(dx + R));
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);   // one shift row's permutes in flight at a time
    }
  }
  if constexpr (!kCost) {
    // the passes' winners: the least key over them is the sequential search's
    s_win[ps][lane] = best;
    __syncthreads();
    if (ps == 0 && node) {
#pragma unroll
      for (int q = 1; q < NPASS; ++q) best = min(best, s_win[q][lane]);
      int32_t* out = g.out + (int64_t)pair * g.ostride;
      out[node_a * g.nx + node_b] = (int)(best & 15u) - R;
      out[g.nx * g.ny + node_a * g.nx + node_b] = (int)((best >> 4) & 15u) - R;
    }
  }
}

// ---------------------------------------------------------------------------
// Coarsest-level SAD search with cell-shared sums for u16 frames (block =
// 2 step, step 12): as k_sad_cells (every node searches the same shifts, a
// block is four 12x12 cells it shares with its neighbours, block sums by DPP
// and lane permute), with v_sad_u16 on realigned words (an odd shift column
// is a 2-byte realignment).  The lane streams its cell's A rows through a
// ring and the B rows once per pass of DYG shift rows.  A workgroup is one
// tile; its waves take the passes side by side (a coarse level has few
// tiles) and the first wave merges their winners.
// ---------------------------------------------------------------------------
template <int R, int DYG>
__global__ __launch_bounds__(64 * ((2 * R + DYG) / DYG)) void k_sad_cells16(SadArgs g) {
  constexpr int G = 2 * R + 1, CWD = 6, RW = CWD + R;   // cell words, realigned B words
  constexpr int CW = 9, CH = 7, NPASS = sad_passes<R, DYG>();
  __shared__ unsigned long long s_win[NPASS][64];
  const int lane = threadIdx.x & 63;
  const int ps = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // this wave's pass
  const int pair = blockIdx.z;
  if (slot_off(g.mask, pair)) return;
  const int ntx = (g.nx + CW - 2) / (CW - 1), nty = (g.ny + CH - 2) / (CH - 1);
  const int tile = blockIdx.x;
  if (tile >= ntx * nty) return;   // the whole workgroup
  const int ty = tile / ntx, tx = tile - ty * ntx;
  const int lr = lane / CW, lc = lane - lr * CW;
  // cells beyond the last node's read the last needed cell (results unused)
  const int ci = min(ty * (CH - 1) + lr, g.ny), cj = min(tx * (CW - 1) + lc, g.nx);
  const int y = ci * 12 - 6, x = cj * 12 - 6;
  const uint8_t* Ab = g.A + (int64_t)pair * g.stride + (int64_t)y * g.pitch + 2 * x;   // 4-byte aligned
  const int xs = 2 * (x - R), sh = xs & 3;
  const uint8_t* Bb = g.B + (int64_t)pair * g.stride + (int64_t)(y - R) * g.pitch + (xs & ~3);
  const int node_a = ty * (CH - 1) + lr, node_b = tx * (CW - 1) + lc;
  const bool node = lr < CH - 1 && lc < CW - 1 && node_a < g.ny && node_b < g.nx;
  auto quad = [&](uint32_t v) {
    const uint32_t h = v + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xF, 0xF, false);
    return h + (uint32_t)__builtin_amdgcn_ds_bpermute((lane + CW) << 2, (int)h);
  };
  unsigned long long best = ~0ull;
  {
    const int k0 = ps * DYG;             // first shift row of the pass
    const int nk = min(DYG, G - k0);     // shift rows in the pass
    uint32_t acc[DYG][G];
#pragma unroll
    for (int k = 0; k < DYG; ++k)
#pragma unroll
      for (int c = 0; c < G; ++c) acc[k][c] = 0u;
    Words<CWD> aring[DYG];   // A row r sits in aring[r % DYG]
#pragma unroll
    for (int rb = 0; rb < 12 + DYG - 1; ++rb) {
      if (rb >= 12 + nk - 1) continue;
      if (rb < 12) aring[rb % DYG] = *reinterpret_cast<const Words<CWD>*>(Ab + (int64_t)rb * g.pitch);
      // B row y - R + k0 + rb meets A row rb - k for shift row k0 + k
      const Words<RW + 1> wv = *reinterpret_cast<const Words<RW + 1>*>(Bb + (int64_t)(k0 + rb) * g.pitch);
      uint32_t rw[RW];
#pragma unroll
      for (int i = 0; i < RW; ++i) rw[i] = __builtin_amdgcn_alignbyte(wv.w[i + 1], wv.w[i], sh);
#pragma unroll
      for (int c = 0; c < G; ++c) {
        uint32_t bw[CWD];
#pragma unroll
        for (int i = 0; i < CWD; ++i)
          bw[i] = (c & 1) ? __builtin_amdgcn_alignbyte(rw[c / 2 + i + 1], rw[c / 2 + i], 2) : rw[c / 2 + i];
#pragma unroll
        for (int k = 0; k < DYG; ++k) {
          const int r = rb - k;
          if (k >= nk || r < 0 || r >= 12) continue;
          uint32_t sacc = acc[k][c];
#pragma unroll
          for (int i = 0; i < CWD; ++i) sacc = __builtin_amdgcn_sad_u16(aring[r % DYG].w[i], bw[i], sacc);
          acc[k][c] = sacc;
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int k = 0; k < DYG; ++k) {
      if (k >= nk) continue;
      const int dy = k0 + k - R;
#pragma unroll
      for (int c = 0; c < G; ++c) {
        const unsigned long long key = sad_key(quad(acc[k][c]), dy, c - R);
        best = key < best ? key : best;
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  // the passes' winners: the least key over them is the sequential search's
  s_win[ps][lane] = best;
  __syncthreads();
  if (ps == 0 && node) {
#pragma unroll
    for (int q = 1; q < NPASS; ++q) best = min(best, s_win[q][lane]);
    int32_t* out = g.out + (int64_t)pair * g.ostride;
    out[node_a * g.nx + node_b] = (int)(best & 0xff) - 128;
    out[g.nx * g.ny + node_a * g.nx + node_b] = (int)((best >> 8) & 0xff) - 128;
  }
}

// ---------------------------------------------------------------------------
// Finer-level SAD search with cell-shared sums for u16 frames (block =
// 2 step, step 12, R <= 2): the four children of a parent share a 3x3 group
// of 12x12 cells (9 cell SADs per shift instead of 16).  Lane = cell of a
// parent's group (7 parents per wave); the lane streams its 12 A rows
// through a ring of 2R + 1 and the 12 + 2R B rows once, v_sad_u16 on
// realigned words (an odd shift column is a 2-byte realignment).  A child's
// sums: its cell + the right-hand cell (DPP lane + 1) + the pair below (lane
// permute, lane + 3).  Level 0 reads in place as in k_sad_stream.  Winner:
// the least (SAD, |dx|+|dy|, dy, dx).
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(256) void k_sad_cells16_fine(SadArgs g) {
  constexpr int G = 2 * R + 1, CWD = 6, RW = CWD + R, PPW = 7;
  const int lane = threadIdx.x & 63;
  const WgIdx wg = xcd_order();
  const int pair = wg.z;
  if (slot_off(g.mask, pair)) return;
  const int pnx = (g.nx + 1) / 2, pny = (g.ny + 1) / 2;
  const int ntx = (pnx + PPW - 1) / PPW;
  const int tile = wg.x * 4 + (threadIdx.x >> 6);
  if (tile >= ntx * pny) return;   // a whole wave (no barriers below)
  const int pa = tile / ntx, tx = tile - pa * ntx;
  const int grp = min(lane / 9, PPW - 1), cell = lane - 9 * (lane / 9);
  const int u = cell / 3, v = cell - 3 * (cell / 3);
  const int pb = min(tx * PPW + grp, pnx - 1);
  const int32_t* par = g.parent + (int64_t)pair * g.pstride;
  int cx, cy;
  parent_centre(g, par, min(pa, g.pny - 1), min(pb, g.pnx - 1), cx, cy);
  // cells past the last node's read the last needed cell (results unused)
  const int ci = min(2 * pa + u, g.ny), cj = min(2 * pb + v, g.nx);
  const int y = ci * 12 - 6, x = cj * 12 - 6;
  const int y0 = y + cy - R, xs = 2 * (x + cx - R), xa = xs & ~3, sh = xs & 3;
  const int rowbytes = 2 * g.W;
  const bool ain = g.direct && y >= 0 && y + 12 <= g.H && x >= 0 && 2 * x + 4 * CWD <= rowbytes;
  const bool bin = g.direct && y0 >= 0 && y0 + 12 + 2 * R <= g.H && xa >= 0 && xa + 4 * (RW + 1) <= rowbytes;
  const uint8_t* Ab = ain ? g.srcA + (int64_t)pair * g.sstride : g.A + (int64_t)pair * g.stride;
  const uint8_t* Bb = bin ? g.srcB + (int64_t)pair * g.sstride : g.B + (int64_t)pair * g.stride;
  const int64_t apitch = ain ? g.spitch : g.pitch, bpitch = bin ? g.spitch : g.pitch;
  Ab += (int64_t)y * apitch + 2 * x;   // 4-byte aligned
  Bb += (int64_t)y0 * bpitch + xa;
  uint32_t acc[G][G];   // [shift row][shift column]
#pragma unroll
  for (int q = 0; q < G; ++q)
#pragma unroll
    for (int c = 0; c < G; ++c) acc[q][c] = 0u;
  Words<CWD> aring[G];   // A row r sits in aring[r % G]
#pragma unroll
  for (int rb = 0; rb < 12 + 2 * R; ++rb) {
    if (rb < 12) aring[rb % G] = *reinterpret_cast<const Words<CWD>*>(Ab + (int64_t)rb * apitch);
    // B row y0 + rb meets A row rb - q for shift row q
    const Words<RW + 1> wv = *reinterpret_cast<const Words<RW + 1>*>(Bb + (int64_t)rb * bpitch);
    uint32_t rw[RW];
#pragma unroll
    for (int i = 0; i < RW; ++i) rw[i] = __builtin_amdgcn_alignbyte(wv.w[i + 1], wv.w[i], sh);
#pragma unroll
    for (int c = 0; c < G; ++c) {
      uint32_t bw[CWD];
#pragma unroll
      for (int i = 0; i < CWD; ++i)
        bw[i] = (c & 1) ? __builtin_amdgcn_alignbyte(rw[c / 2 + i + 1], rw[c / 2 + i], 2) : rw[c / 2 + i];
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const int r = rb - q;
        if (r < 0 || r >= 12) continue;
        uint32_t sacc = acc[q][c];
#pragma unroll
        for (int i = 0; i < CWD; ++i) sacc = __builtin_amdgcn_sad_u16(aring[r % G].w[i], bw[i], sacc);
        acc[q][c] = sacc;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  auto quad = [&](uint32_t val) {
    const uint32_t h = val + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)val, 0x130, 0xF, 0xF, false);
    return h + (uint32_t)__builtin_amdgcn_ds_bpermute((lane + 3) << 2, (int)h);
  };
  unsigned long long best = ~0ull;
#pragma unroll
  for (int q = 0; q < G; ++q) {
#pragma unroll
    for (int c = 0; c < G; ++c) {
      const unsigned long long key = sad_key(quad(acc[q][c]), cy - R + q, cx - R + c);
      best = key < best ? key : best;
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  const int a = 2 * pa + u, b = 2 * pb + v;
  if (lane < 9 * PPW && u < 2 && v < 2 && tx * PPW + lane / 9 < pnx && a < g.ny && b < g.nx) {
    int32_t* out = g.out + (int64_t)pair * g.ostride;
    out[a * g.nx + b] = (int)(best & 0xff) - 128;
    out[g.nx * g.ny + a * g.nx + b] = (int)((best >> 8) & 0xff) - 128;
  }
}

// ---------------------------------------------------------------------------
// Finer-level SAD search with cell-shared sums (u8, block = 2 step, step 8,
// R <= 2).  The four children of a parent search the same shifts (around
// twice the parent's result), and their 16x16 blocks are the 2x2 windows of
// a 3x3 group of 8x8 cells: 9 cell SADs per shift instead of 16, four shift
// columns per quad SAD (16-bit fields: a cell is at most 64 x 255, four
// cells stay below 2^16).  Lane = (parent, cell column), 21 parents per
// wave: the lane streams the 24 A rows and 24 + 2R B rows of its column once
// (A rows in a ring, both read ahead), keeps the SADs of its three cells, and
// forms its two children's sums as (cell + the cell below, a register add) +
// the same pair of the right-hand column (DPP lane + 1).  The parent's
// centre, the addressing and the winner search are paid once per three
// cells.  Level 0 reads in place as in k_sad_lane.  Winner: the least 31-bit
// key as in k_sad_lane.
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(256) void k_sad_cols(SadArgs g) {
  constexpr int G = 2 * R + 1, NGRP = (G + 3) / 4, REM = G - 4 * (NGRP - 1);
  constexpr bool TAIL = REM <= 2;
  constexpr int NQ = TAIL ? NGRP - 1 : NGRP;
  constexpr int CWD = 2, RW = CWD + NGRP, PPW = 21;   // parents per wave
  constexpr int NA = 24, NB = NA + G - 1;             // A and B rows of the column
  static_assert(G <= 5, "one pass of shift rows");
  const int lane = threadIdx.x & 63;
  const WgIdx wg = xcd_order();
  const int pair = wg.z;
  if (slot_off(g.mask, pair)) return;
  const int pnx = (g.nx + 1) / 2, pny = (g.ny + 1) / 2;
  const int ntx = (pnx + PPW - 1) / PPW;
  const int tile = wg.x * 4 + (threadIdx.x >> 6);
  if (tile >= ntx * pny) return;   // a whole wave (no barriers below)
  const int pa = tile / ntx, tx = tile - pa * ntx;
  const int grp = min(lane / 3, PPW - 1), v = lane - 3 * (lane / 3);
  const int pb = min(tx * PPW + grp, pnx - 1);
  const int32_t* par = g.parent + (int64_t)pair * g.pstride;
  int cx, cy;
  parent_centre(g, par, min(pa, g.pny - 1), min(pb, g.pnx - 1), cx, cy);
  // the column's cells 2pa .. 2pa + 2 (clamped cells past the last node are
  // read but unused)
  const int cj = min(2 * pb + v, g.nx);
  const int y = min(2 * pa, g.ny - 1) * 8 - 4, x = cj * 8 - 4;
  const int y0 = y + cy - R, xs = x + cx - R;
  const int xa = xs & ~3, sh = xs & 3;
  const unsigned pitch32 = (unsigned)g.pitch, spitch32 = (unsigned)g.spitch;
  const bool ain = g.direct && y >= 0 && y + NA <= g.H && x >= 0 && x + 8 <= g.W;
  const bool bin = g.direct && y0 >= 0 && y0 + NB <= g.H && xa >= 0 && xa + 4 * (RW + 1) <= g.W;
  const uint8_t* Apad = g.A + (int64_t)pair * g.stride - ((int64_t)g.margin * g.pitch + g.margin);
  const uint8_t* Bpad = g.B + (int64_t)pair * g.stride - ((int64_t)g.margin * g.pitch + g.margin);
  const uint8_t* Asrc = g.srcA + (int64_t)pair * g.sstride;
  const uint8_t* Bsrc = g.srcB + (int64_t)pair * g.sstride;
  const unsigned pa32 = ain ? spitch32 : pitch32, pb32 = bin ? spitch32 : pitch32;
  const int am = ain ? 0 : g.margin, bm = bin ? 0 : g.margin;
  const unsigned aoff = __umul24((unsigned)(y + am), pa32) + (unsigned)(x + am);
  const unsigned boff = __umul24((unsigned)(y0 + bm), pb32) + (unsigned)(xa + bm);
  auto arow = [&](int r) {
    const unsigned o = aoff + r * pa32;
    return ain ? *reinterpret_cast<const Words<CWD>*>(Asrc + (size_t)o)
               : *reinterpret_cast<const Words<CWD>*>(Apad + (size_t)o);
  };
  auto brow = [&](int rb) {
    const unsigned o = boff + rb * pb32;
    return bin ? *reinterpret_cast<const Words<RW + 1>*>(Bsrc + (size_t)o)
               : *reinterpret_cast<const Words<RW + 1>*>(Bpad + (size_t)o);
  };
  unsigned long long acc[3][G][NQ > 0 ? NQ : 1];
  uint32_t tacc[3][G][2];
#pragma unroll
  for (int u = 0; u < 3; ++u)
#pragma unroll
    for (int q = 0; q < G; ++q) {
#pragma unroll
      for (int m = 0; m < (NQ > 0 ? NQ : 1); ++m) acc[u][q][m] = 0ull;
      tacc[u][q][0] = tacc[u][q][1] = 0u;
    }
  constexpr int PF = 4;   // B and A rows read PF rows ahead of their use
  Words<RW + 1> bring[PF];
  Words<CWD> aring[G + PF];
#pragma unroll
  for (int i = 0; i < PF; ++i) {
    bring[i] = brow(i);
    aring[i] = arow(i);
  }
#pragma unroll
  for (int rb = 0; rb < NB; ++rb) {
    // B row y0 + rb meets A row rb - q (cell (rb - q) / 8) for shift row q
    const Words<RW + 1> wv = bring[rb % PF];
    if (rb + PF < NB) bring[rb % PF] = brow(rb + PF);
    if (rb + PF < NA) aring[(rb + PF) % (G + PF)] = arow(rb + PF);
    uint32_t rw[RW];
#pragma unroll
    for (int i = 0; i < RW; ++i) rw[i] = __builtin_amdgcn_alignbyte(wv.w[i + 1], wv.w[i], sh);
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const int r = rb - q;
      if (r < 0 || r >= NA) continue;
      const int u = r / 8;
      const Words<CWD> aw = aring[r % (G + PF)];
#pragma unroll
      for (int i = 0; i < CWD; ++i) {
#pragma unroll
        for (int m = 0; m < NQ; ++m) {
          const unsigned long long src = ((unsigned long long)rw[i + m + 1] << 32) | rw[i + m];
          acc[u][q][m] = __builtin_amdgcn_qsad_pk_u16_u8(src, aw.w[i], acc[u][q][m]);
        }
        if constexpr (TAIL) {
          tacc[u][q][0] = __builtin_amdgcn_sad_u8(aw.w[i], rw[i + NQ], tacc[u][q][0]);
          if constexpr (REM == 2)
            tacc[u][q][1] = __builtin_amdgcn_sad_u8(aw.w[i], __builtin_amdgcn_alignbyte(rw[i + NQ + 1], rw[i + NQ], 1),
                                                    tacc[u][q][1]);
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  // children (2pa + uc, 2pb + v) for uc = 0, 1 on lanes with v < 2:
  // (cell uc + cell uc + 1) of this column + the same of the next column
  auto pair_sum = [&](uint32_t val) {
    return val + (uint32_t)__builtin_amdgcn_update_dpp(0, (int)val, 0x130, 0xF, 0xF, false);
  };
  uint32_t kx[G], ky[G];
#pragma unroll
  for (int k = 0; k < G; ++k) {
    kx[k] = ((uint32_t)abs(cx - R + k) << 6) | (uint32_t)k;
    ky[k] = ((uint32_t)abs(cy - R + k) << 6) | ((uint32_t)k << 3);
  }
  uint32_t best[2] = {~0u, ~0u};
#pragma unroll
  for (int uc = 0; uc < 2; ++uc) {
#pragma unroll
    for (int q = 0; q < G; ++q) {
#pragma unroll
      for (int m = 0; m < NQ; ++m) {
        const unsigned long long t2 = acc[uc][q][m] + acc[uc + 1][q][m];   // fields stay below 2^15
        const uint32_t lo = pair_sum((uint32_t)t2), hi = pair_sum((uint32_t)(t2 >> 32));
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const int c = 4 * m + f;
          if (c >= G) continue;
          const uint32_t sad = ((f < 2 ? lo : hi) >> (16 * (f & 1))) & 0xffffu;
          best[uc] = min(best[uc], (sad << 15) | (kx[c] + ky[q]));
        }
      }
      if constexpr (TAIL) {
#pragma unroll
        for (int f = 0; f < REM; ++f) {
          const int c = 4 * NQ + f;
          best[uc] = min(best[uc], (pair_sum(tacc[uc][q][f] + tacc[uc + 1][q][f]) << 15) | (kx[c] + ky[q]));
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  const int b = 2 * pb + v;
  const bool col = lane < 3 * PPW && v < 2 && tx * PPW + lane / 3 < pnx && b < g.nx;
  int32_t* out = g.out + (int64_t)pair * g.ostride;
#pragma unroll
  for (int uc = 0; uc < 2; ++uc) {
    const int a = 2 * pa + uc;
    if (col && a < g.ny) {
      out[a * g.nx + b] = cx - R + (int)(best[uc] & 7u);
      out[g.nx * g.ny + a * g.nx + b] = cy - R + (int)((best[uc] >> 3) & 7u);
    }
  }
}

// ---------------------------------------------------------------------------
// SAD block search, one node per lane, A rows streamed (any element size,
// small R): the lane keeps the last G = 2R+1 rows of its A block in a ring of
// registers and streams the rows of B once each; a B row, realigned to the
// leftmost candidate, feeds every candidate column and every candidate row
// whose A row is in the ring.  Neighbouring lanes are neighbouring nodes, so
// a wave's row reads are contiguous.
// ---------------------------------------------------------------------------
template <int ES, int NW, int R>
__global__ __launch_bounds__(256) void k_sad_stream(SadArgs g) {
  constexpr int G = 2 * R + 1;
  constexpr int BLK = 4 * NW / ES;
  constexpr int RWS = NW + (2 * R * ES + 3) / 4;   // realigned words covering every candidate column
  const WgIdx wg = xcd_order();
  const int pair = wg.y;
  if (slot_off(g.mask, pair)) return;
  const int node = wg.x * blockDim.x + threadIdx.x;
  if (node >= g.nx * g.ny) return;
  const int a = node / g.nx, b = node - a * g.nx;
  const int off = (g.step - BLK) / 2;
  const int oy = a * g.step + off, ox = b * g.step + off;
  int cx = 0, cy = 0;
  if (g.parent) {
    const int32_t* par = g.parent + (int64_t)pair * g.pstride;
    int pa = min(a >> 1, g.pny - 1), pb = min(b >> 1, g.pnx - 1);
    cx = 2 * parent_value(g, par, 0, pa, pb);
    cy = 2 * parent_value(g, par, 1, pa, pb);
  }
  uint32_t acc[G][G];   // [candidate row q][candidate column k]
#pragma unroll
  for (int q = 0; q < G; ++q)
#pragma unroll
    for (int k = 0; k < G; ++k) acc[q][k] = 0u;
  const int y0 = oy + cy - R;
  const int xs = (ox + cx - R) * ES, xa = xs & ~3, sh = xs & 3;
  const int axs = ox * ES, axa = axs & ~3, ash = axs & 3;
  // level 0 read in place: a span wholly inside the image reads the caller's
  // frame (the same coordinates, its own pitch), others the padded copy
  const int rowbytes = g.W * ES;
  const bool ain = g.direct && oy >= 0 && oy + BLK <= g.H && axa >= 0 && axa + 4 * (NW + 1) <= rowbytes;
  const bool bin = g.direct && y0 >= 0 && y0 + BLK + 2 * R <= g.H && xa >= 0 && xa + 4 * (RWS + 1) <= rowbytes;
  const uint8_t* Ab = ain ? g.srcA + (int64_t)pair * g.sstride : g.A + (int64_t)pair * g.stride;
  const uint8_t* Bb = bin ? g.srcB + (int64_t)pair * g.sstride : g.B + (int64_t)pair * g.stride;
  const int64_t apitch = ain ? g.spitch : g.pitch, bpitch = bin ? g.spitch : g.pitch;
  uint32_t ring[G][NW];   // A row ar sits in ring[ar % G]
  for (int rb0 = 0; rb0 < BLK + 2 * R; rb0 += G) {
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int rb = rb0 + u;   // rb % G == u
      if (rb < BLK + 2 * R) {
        if (rb < BLK) {
          const uint32_t* row = reinterpret_cast<const uint32_t*>(Ab + (int64_t)(oy + rb) * apitch + axa);
          uint32_t w[NW + 1];
#pragma unroll
          for (int i = 0; i <= NW; ++i) w[i] = row[i];
#pragma unroll
          for (int i = 0; i < NW; ++i) ring[u][i] = __builtin_amdgcn_alignbyte(w[i + 1], w[i], ash);
        }
        const uint32_t* row = reinterpret_cast<const uint32_t*>(Bb + (int64_t)(y0 + rb) * bpitch + xa);
        uint32_t w[RWS + 1];
#pragma unroll
        for (int i = 0; i <= RWS; ++i) w[i] = row[i];
        uint32_t rw[RWS];
#pragma unroll
        for (int i = 0; i < RWS; ++i) rw[i] = __builtin_amdgcn_alignbyte(w[i + 1], w[i], sh);
#pragma unroll
        for (int k = 0; k < G; ++k) {
          const int kb = k * ES, kw = kb >> 2, ks = kb & 3;
          uint32_t bw[NW];
#pragma unroll
          for (int i = 0; i < NW; ++i) bw[i] = ks ? __builtin_amdgcn_alignbyte(rw[kw + i + 1], rw[kw + i], ks) : rw[kw + i];
#pragma unroll
          for (int q = 0; q < G; ++q) {
            const int ar = rb - q;
            if (ar >= 0 && ar < BLK) {
              const int slot = (u - q + G) % G;   // ar % G
              uint32_t s = acc[q][k];
#pragma unroll
              for (int i = 0; i < NW; ++i) s = sad_word<ES>(ring[slot][i], bw[i], s);
              acc[q][k] = s;
            }
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
    }
  }
  unsigned long long best = ~0ull;
#pragma unroll
  for (int q = 0; q < G; ++q)
#pragma unroll
    for (int k = 0; k < G; ++k) {
      unsigned long long key = sad_key(acc[q][k], cy - R + q, cx - R + k);
      best = key < best ? key : best;
    }
  int32_t* out = g.out + (int64_t)pair * g.ostride;
  out[a * g.nx + b] = (int)(best & 0xff) - 128;
  out[g.nx * g.ny + a * g.nx + b] = (int)((best >> 8) & 0xff) - 128;
}

// ---------------------------------------------------------------------------
// SAD block search with a lane per candidate row, for any element size: a
// group of G = 2R+1 lanes per node, lane q owning dy = cand_y - R + q and
// all G candidate columns.  The node's A block is staged in LDS; per block
// row, a lane reads its B row once, realigns it to the leftmost candidate,
// and feeds every candidate column from the same registers (an A row word
// is read once per row, not once per candidate).
// ---------------------------------------------------------------------------
template <int ES, int NW, int KMAX>
__global__ __launch_bounds__(256) void k_sad_r(SadArgs g) {
  constexpr int BLK = 4 * NW / ES;
  constexpr int SPAN = (KMAX - 1) * ES;           // bytes from the first to the last candidate
  constexpr int RWR = NW + (SPAN + 3) / 4;        // realigned words a row needs
  extern __shared__ uint32_t s_ablk[];            // [npw][BLK][NW]
  __shared__ unsigned long long s_key[256];

  const WgIdx wg = xcd_order();
  const int pair = wg.z;
  if (slot_off(g.mask, pair)) return;
  const int G = 2 * g.R + 1;
  const int npw = g.npw;
  const int t = threadIdx.x;
  const int j = t / G, q = t - j * G;
  const int a = wg.y;
  const int b0 = wg.x * npw;
  const int b = b0 + j;
  const bool active = j < npw && b < g.nx;
  const int off = (g.step - BLK) / 2;
  const int oy = a * g.step + off;
  const uint8_t* Ab = g.A + (int64_t)pair * g.stride;
  const uint8_t* Bb = g.B + (int64_t)pair * g.stride;

  const int nblk = min(npw, g.nx - b0);
  for (int idx = t; idx < nblk * BLK * NW; idx += 256) {
    int jj = idx / (BLK * NW), r = (idx / NW) % BLK, w = idx % NW;
    const uint8_t* row = Ab + (int64_t)(oy + r) * g.pitch;
    s_ablk[idx] = word_at(row, ((b0 + jj) * g.step + off) * ES + 4 * w);
  }

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
    const int xs = (b * g.step + off + cx - g.R) * ES;   // byte of candidate column 0
    const int xa = xs & ~3, sh = xs & 3;
    const int by = oy + cy - g.R + q;
    uint32_t acc[KMAX];
#pragma unroll
    for (int k = 0; k < KMAX; ++k) acc[k] = 0u;
    const uint32_t* ablk = s_ablk + j * BLK * NW;
#pragma unroll 2
    for (int ar = 0; ar < BLK; ++ar) {
      const uint32_t* row = reinterpret_cast<const uint32_t*>(Bb + (int64_t)(by + ar) * g.pitch + xa);
      uint32_t w[RWR + 1];
#pragma unroll
      for (int i = 0; i <= RWR; ++i) w[i] = row[i];
      uint32_t rw[RWR];
#pragma unroll
      for (int i = 0; i < RWR; ++i) rw[i] = __builtin_amdgcn_alignbyte(w[i + 1], w[i], sh);
      uint32_t aw[NW];
#pragma unroll
      for (int i = 0; i < NW; ++i) aw[i] = ablk[ar * NW + i];
#pragma unroll
      for (int k = 0; k < KMAX; ++k) {
        if (k < G) {
          const int kb = k * ES, kw = kb >> 2, ks = kb & 3;
          uint32_t s = acc[k];
#pragma unroll
          for (int i = 0; i < NW; ++i) {
            const uint32_t bw = ks ? __builtin_amdgcn_alignbyte(rw[kw + i + 1], rw[kw + i], ks) : rw[kw + i];
            s = sad_word<ES>(aw[i], bw, s);
          }
          acc[k] = s;
        }
      }
    }
    const int dy = cy - g.R + q;
#pragma unroll
    for (int k = 0; k < KMAX; ++k) {
      if (k < G) {
        unsigned long long key = sad_key(acc[k], dy, cx - g.R + k);
        best = key < best ? key : best;
      }
    }
  }
  s_key[t] = best;
  __syncthreads();
  if (active && q == 0) {
    unsigned long long m = s_key[t];
    for (int k = 1; k < G; ++k) m = s_key[t + k] < m ? s_key[t + k] : m;
    int32_t* out = g.out + (int64_t)pair * g.ostride;
    out[a * g.nx + b] = (int)(m & 0xff) - 128;
    out[g.nx * g.ny + a * g.nx + b] = (int)((m >> 8) & 0xff) - 128;
  }
}

// ---------------------------------------------------------------------------
// SAD block search, general form: G = 2R+1 candidate columns per node, each
// split into qsplit groups of at most KMAX candidate rows, one thread per
// (column, group): the thread owns dx = cand_x - R + k and its rows dy, and
// streams only the B rows they meet (realigned to its dx), accumulating
// v_sad_u8 / v_sad_u16; npw nodes of one node row per workgroup.  The node's
// A block is staged in LDS as packed words, and without a parent (every
// node searching the same rows) so is the band of B rows the workgroup
// reads.  The winner minimises the packed key (SAD, |dx|+|dy|, dy, dx): a
// plain u64 min, independent of the reduction order.
// ---------------------------------------------------------------------------
template <int ES, int NW, int KMAX>
__global__ __launch_bounds__(256) void k_sad(SadArgs g) {
  extern __shared__ uint32_t s_ablk[];        // [npw][block][NW], then the staged B band [rows][band]
  __shared__ unsigned long long s_key[256];

  const WgIdx wg = xcd_order();
  const int pair = wg.z;
  if (slot_off(g.mask, pair)) return;
  const int G = 2 * g.R + 1;
  const int QS = g.qsplit, qn = (G + QS - 1) / QS, TPN = G * QS;   // (qn <= KMAX)
  const int npw = g.npw;
  const int t = threadIdx.x;
  const int j = t / TPN, rem = t - j * TPN;
  const int qg = rem / G, k = rem - qg * G;   // candidate-row group, candidate column
  const int a = wg.y;
  const int b0 = wg.x * npw;
  const int b = b0 + j;
  const bool active = j < npw && b < g.nx;
  const int off = (g.step - g.block) / 2;
  const int oy = a * g.step + off;
  const uint8_t* Ab = g.A + (int64_t)pair * g.stride;
  const uint8_t* Bb = g.B + (int64_t)pair * g.stride;

  const int nblk = min(npw, g.nx - b0);
  const int words = g.block * NW;
  const int nrows = g.block + 2 * g.R;
  for (int idx = t; idx < nblk * words; idx += 256) {
    int jj = idx / words, r = (idx / NW) % g.block, w = idx % NW;
    const uint8_t* row = Ab + (int64_t)(oy + r) * g.pitch;
    s_ablk[idx] = word_at(row, ((b0 + jj) * g.step + off) * ES + 4 * w);
  }
  // the band: words xw0 .. the last one a node of the workgroup reads
  uint32_t* const s_band = s_ablk + npw * words;
  const int xw0 = ((b0 * g.step + off - g.R) * ES) >> 2;   // (a floor for negative offsets)
  if (g.band) {
    const int nbw = ((((b0 + nblk - 1) * g.step + off + g.R) * ES) >> 2) + NW - xw0 + 1;
    const uint8_t* Bs = Bb + (int64_t)(oy - g.R) * g.pitch + 4 * (int64_t)xw0;
    for (int idx = t; idx < nrows * nbw; idx += 256) {
      const int r = idx / nbw, w = idx - r * nbw;
      s_band[r * g.band + w] = *reinterpret_cast<const uint32_t*>(Bs + (int64_t)r * g.pitch + 4 * w);
    }
  }

  int cx = 0, cy = 0;
  if (g.parent && active) {
    const int32_t* par = g.parent + (int64_t)pair * g.pstride;
    int pa = min(a >> 1, g.pny - 1), pb = min(b >> 1, g.pnx - 1);
    cx = 2 * parent_value(g, par, 0, pa, pb);
    cy = 2 * parent_value(g, par, 1, pa, pb);
  }
  __syncthreads();

  unsigned long long best = ~0ull;
  const int q0 = qg * qn, q1 = min(q0 + qn, G);   // this thread's candidate rows
  if (active && q0 < q1) {
    const int dx = cx - g.R + k;
    const int xb = (b * g.step + off + dx) * ES;
    const int xa = xb & ~3, sh = xb & 3;
    const int by0 = oy + cy - g.R;
    uint32_t acc[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) acc[q] = 0u;
    const uint32_t* ablk = s_ablk + j * words;
    const uint32_t* brow0 = s_band + ((xa >> 2) - xw0);
    // B row rb meets A row rb - q for candidate row q
    for (int rb = q0; rb < q1 - 1 + g.block; ++rb) {
      uint32_t w[NW + 1];
      if (g.band) {
#pragma unroll
        for (int i = 0; i <= NW; ++i) w[i] = brow0[rb * g.band + i];
      } else {
        const uint32_t* row = reinterpret_cast<const uint32_t*>(Bb + (int64_t)(by0 + rb) * g.pitch + xa);
#pragma unroll
        for (int i = 0; i <= NW; ++i) w[i] = row[i];
      }
      uint32_t bw[NW];
#pragma unroll
      for (int i = 0; i < NW; ++i) bw[i] = __builtin_amdgcn_alignbyte(w[i + 1], w[i], sh);
#pragma unroll
      for (int qi = 0; qi < KMAX; ++qi) {
        const int ar = rb - (q0 + qi);
        if (qi < qn && q0 + qi < q1 && ar >= 0 && ar < g.block) {
          const uint32_t* arow = ablk + ar * NW;
          uint32_t s = acc[qi];
#pragma unroll
          for (int i = 0; i < NW; ++i) s = sad_word<ES>(arow[i], bw[i], s);
          acc[qi] = s;
        }
      }
    }
#pragma unroll
    for (int qi = 0; qi < KMAX; ++qi) {
      if (qi < qn && q0 + qi < q1) {
        unsigned long long key = sad_key(acc[qi], cy - g.R + q0 + qi, dx);
        best = key < best ? key : best;
      }
    }
  }
  // a node's winner: over its row groups per column, then over the columns
  s_key[t] = best;
  __syncthreads();
  if (active && qg == 0) {
    unsigned long long m = s_key[t];
    for (int q = 1; q < QS; ++q) m = s_key[t + q * G] < m ? s_key[t + q * G] : m;
    s_key[t] = m;
  }
  __syncthreads();
  if (active && rem == 0) {
    unsigned long long m = s_key[t];
    for (int q = 1; q < G; ++q) m = s_key[t + q] < m ? s_key[t + q] : m;
    int32_t* out = g.out + (int64_t)pair * g.ostride;
    out[a * g.nx + b] = (int)(m & 0xff) - 128;
    out[g.nx * g.ny + a * g.nx + b] = (int)((m >> 8) & 0xff) - 128;
  }
}

// ---------------------------------------------------------------------------
// SAD block search, one node per lane (small radii, u8 blocks of NW words).
// The lane keeps (2R+1)^2 sums in registers and streams the block + 2R rows
// of B once, fully unrolled so that the pairing of B rows with A rows is
// static.  A row r is loaded just before B row r first needs it and dies
// after B row r + 2R; each B row is realigned to the search origin once and
// every shift dx is a further static alignbyte of the realigned words.
// AAL: every block column starts on a 4-byte boundary (step and block offset
// multiples of 4), so A rows are read as aligned words.  The winner is the
// least 31-bit key (SAD, |dx|+|dy|, candidate row, candidate column): within
// a node the row and column indices order dy and dx, and a block of at most
// 16x16 u8 pixels keeps the SAD below 2^16.
// ---------------------------------------------------------------------------
template <int NW, int R, bool AAL>
__global__ __launch_bounds__(256) void k_sad_lane(SadArgs g) {
  static_assert(NW <= 4 && 2 * R + 1 <= 8, "the 31-bit key holds a SAD of 16x16 u8 pixels and 3-bit indices");
  constexpr int BLK = 4 * NW, G = 2 * R + 1;
  constexpr int RW = NW + (2 * R + 3) / 4 + 1;   // realigned words covering BLK + 2R bytes
  const WgIdx wg = xcd_order();
  const int pair = wg.y;
  if (slot_off(g.mask, pair)) return;
  const int node = wg.x * blockDim.x + threadIdx.x;
  if (node >= g.nx * g.ny) return;
  const int a = node / g.nx, b = node - a * g.nx;
  const int off = (g.step - BLK) / 2;
  const int oy = a * g.step + off, ox = b * g.step + off;
  const uint8_t* Ab = g.A + (int64_t)pair * g.stride;
  const uint8_t* Bb = g.B + (int64_t)pair * g.stride;
  int cx = 0, cy = 0;
  if (g.parent) {
    const int32_t* par = g.parent + (int64_t)pair * g.pstride;
    int pa = min(a >> 1, g.pny - 1), pb = min(b >> 1, g.pnx - 1);
    cx = 2 * parent_value(g, par, 0, pa, pb);
    cy = 2 * parent_value(g, par, 1, pa, pb);
  }
  uint32_t acc[G][G];
#pragma unroll
  for (int q = 0; q < G; ++q)
#pragma unroll
    for (int k = 0; k < G; ++k) acc[q][k] = 0u;
  const int y0 = oy + cy - R, xs = ox + cx - R;
  const int xa = xs & ~3, sh = xs & 3;
  const int axa = ox & ~3, ash = ox & 3;
  // 32-bit offsets from padded row 0 (non-negative; the launcher checks that
  // a padded level fits 31 bits), or from row 0 of the caller's frame for a
  // span wholly inside the image (the launcher checks that a frame fits too)
  const unsigned pitch32 = (unsigned)g.pitch, spitch32 = (unsigned)g.spitch;
  const bool ain = g.direct && oy >= 0 && oy + BLK <= g.H && axa >= 0 && axa + 4 * (AAL ? NW : NW + 1) <= g.W;
  const bool bin = g.direct && y0 >= 0 && y0 + BLK + 2 * R <= g.H && xa >= 0 && xa + 4 * (RW + 1) <= g.W;
  // (two uniform bases, a per-lane choice between loads, so that addresses
  // stay a uniform base plus a 32-bit lane offset)
  const uint8_t* Apad = Ab - ((int64_t)g.margin * g.pitch + g.margin);
  const uint8_t* Bpad = Bb - ((int64_t)g.margin * g.pitch + g.margin);
  const uint8_t* Asrc = g.srcA + (int64_t)pair * g.sstride;
  const uint8_t* Bsrc = g.srcB + (int64_t)pair * g.sstride;
  const unsigned pa = ain ? spitch32 : pitch32, pb = bin ? spitch32 : pitch32;
  const int am = ain ? 0 : g.margin, bm = bin ? 0 : g.margin;
  const unsigned aoff = __umul24((unsigned)(oy + am), pa) + (unsigned)(axa + am);
  const unsigned boff = __umul24((unsigned)(y0 + bm), pb) + (unsigned)(xa + bm);
  uint32_t av[BLK][NW];
#pragma unroll
  for (int rb = 0; rb < BLK + 2 * R; ++rb) {
    if (rb < BLK) {
      const unsigned o = aoff + rb * pa;
      if constexpr (AAL) {
        const Words<NW> w = ain ? *reinterpret_cast<const Words<NW>*>(Asrc + (size_t)o)
                                : *reinterpret_cast<const Words<NW>*>(Apad + (size_t)o);
#pragma unroll
        for (int i = 0; i < NW; ++i) av[rb][i] = w.w[i];
      } else {
        const Words<NW + 1> w = ain ? *reinterpret_cast<const Words<NW + 1>*>(Asrc + (size_t)o)
                                    : *reinterpret_cast<const Words<NW + 1>*>(Apad + (size_t)o);
#pragma unroll
        for (int i = 0; i < NW; ++i) av[rb][i] = __builtin_amdgcn_alignbyte(w.w[i + 1], w.w[i], ash);
      }
    }
    const unsigned ob = boff + rb * pb;
    const Words<RW + 1> w = bin ? *reinterpret_cast<const Words<RW + 1>*>(Bsrc + (size_t)ob)
                                : *reinterpret_cast<const Words<RW + 1>*>(Bpad + (size_t)ob);
    uint32_t rw[RW];
#pragma unroll
    for (int i = 0; i < RW; ++i) rw[i] = __builtin_amdgcn_alignbyte(w.w[i + 1], w.w[i], sh);
#pragma unroll
    for (int k = 0; k < G; ++k) {
      uint32_t bw[NW];
#pragma unroll
      for (int i = 0; i < NW; ++i) {
        const int jj = (k >> 2) + i;
        bw[i] = (k & 3) ? __builtin_amdgcn_alignbyte(rw[jj + 1], rw[jj], k & 3) : rw[jj];
      }
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const int ar = rb - q;
        if (ar >= 0 && ar < BLK) {
          uint32_t s = acc[q][k];
#pragma unroll
          for (int i = 0; i < NW; ++i) s = __builtin_amdgcn_sad_u8(av[ar][i], bw[i], s);
          acc[q][k] = s;
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  // key = SAD << 15 | (|dx| + |dy|) << 6 | q << 3 | k
  uint32_t kx[G], ky[G];
#pragma unroll
  for (int k = 0; k < G; ++k) {
    kx[k] = ((uint32_t)abs(cx - R + k) << 6) | (uint32_t)k;
    ky[k] = ((uint32_t)abs(cy - R + k) << 6) | ((uint32_t)k << 3);
  }
  uint32_t best = ~0u;
#pragma unroll
  for (int q = 0; q < G; ++q)
#pragma unroll
    for (int k = 0; k < G; ++k) best = min(best, (acc[q][k] << 15) | (kx[k] + ky[q]));
  int32_t* out = g.out + (int64_t)pair * g.ostride;
  out[a * g.nx + b] = cx - R + (int)(best & 7u);
  out[g.nx * g.ny + a * g.nx + b] = cy - R + (int)((best >> 3) & 7u);
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
      int v[9];
      int k = 0;
#pragma unroll
      for (int di = -1; di <= 1; ++di)
#pragma unroll
        for (int dj = -1; dj <= 1; ++dj) {
          int y = a + di, x = b + dj;
          bool in = y >= 0 && x >= 0 && y < ny && x < nx;
          v[(di + 1) * 3 + dj + 1] = in ? P[y * nx + x] : kSlotI;
          k += in;
        }
      val = median9_low_i(v, k);
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

// Level 0 is searched reading the caller's frames in place (see SadArgs) by
// the one-node-per-lane or the cell-column kernel (u8, radius <= 2, 8-16 px
// blocks, 32-bit offsets into both the padded copy and one caller frame) or
// by the streamed or cell-shared u16 kernel (radius 1-2, 12-24 px blocks).
static bool level0_in_place(const Plan& P, int64_t pitch) {
  const Level& v = P.lv[0];
  if (P.p.sgm && P.L == 1) return false;   // the semi-global cost reads the padded copy
  const int NW = P.block * P.es / 4;
  if (P.es == 2)   // the streamed u16 kernel (64-bit row addresses)
    return v.R >= 1 && v.R <= 2 && (NW == 6 || NW == 8 || NW == 12);
  const bool off31 = (size_t)v.rows * v.pitch < (1u << 31) && v.pitch < (1 << 24);
  return P.es == 1 && v.R <= 2 && (NW == 2 || NW == 3 || NW == 4) && off31 && pitch < (1 << 24) &&
         (int64_t)P.p.height * pitch < (int64_t(1) << 31);
}

hipError_t launch_clear_margins(const Plan& P, uint8_t* ws, int pairs, hipStream_t s) {
  if (P.p.dtype == PIV_F32 || pairs <= 0) return hipSuccess;   // no pyramid on F32 plans
  // every level's margins, for every pair (grid z holds 2 frames x at most
  // 16384 pairs per launch)
  for (int p0 = 0; p0 < pairs; p0 += 16384) {
    const int np = min(pairs - p0, 16384);
    uint8_t* base = ws + (size_t)p0 * P.per_pair;
    for (int l = 0; l < P.L; ++l) {
      const Level& v = P.lv[l];
      const int64_t words = (int64_t)(v.pitch / 4) * v.rows;
      dim3 grid((unsigned)((words + 255) / 256), 1, 2 * np);
      hipLaunchKernelGGL(k_clear_margins, grid, dim3(256), 0, s, base, (int64_t)P.per_pair, (int64_t)v.off_a,
                         (int64_t)v.off_b, v.pitch, v.rows, v.margin * P.es, v.W * P.es, v.margin, v.H);
      if (hipError_t e = hipGetLastError()) return e;
    }
  }
  return hipSuccess;
}

hipError_t launch_pyramid(const Plan& P, const void* A, const void* B, int64_t pitch, int n,
                          hipStream_t s) {
  const Level& v0 = P.lv[0];
  const bool l2 = P.L > 2;   // levels 1 and 2 from one read of the frames
  {
    auto dst = [&](const Level& v) {
      PyrDst d;
      d.offA = (int64_t)v.off_a;
      d.offB = (int64_t)v.off_b;
      d.pitch = v.pitch;
      d.m = v.margin;
      d.W = v.W;
      d.H = v.H;
      return d;
    };
    const PyrDst d0 = dst(v0), d1 = dst(P.lv[P.L > 1 ? 1 : 0]), d2 = dst(P.lv[l2 ? 2 : 0]);
    const int nq = (v0.W * P.es + 15) / 16;
    const int rows = l2 ? (v0.H + 3) / 4 : (v0.H + 1) / 2;
    dim3 grid((nq * rows + 255) / 256, 1, 2 * n);
    const int lframe = level0_in_place(P, pitch) ? kFrame : 0;
    const int do_l1 = P.L > 1 ? 1 : 0;
#define PIV_PAD_PYR(T_, L2_)                                                                           \
  hipLaunchKernelGGL((k_pad_pyr<T_, L2_>), grid, dim3(256), 0, s, (const uint8_t*)A, (const uint8_t*)B, \
                     pitch, pitch * P.p.height, v0.W, v0.H, P.ws, (int64_t)P.per_pair, d0, d1, d2, do_l1,  \
                     lframe, P.slot_mask)
    if (P.es == 1) {
      if (l2) PIV_PAD_PYR(uint8_t, true);
      else PIV_PAD_PYR(uint8_t, false);
    } else {
      if (l2) PIV_PAD_PYR(uint16_t, true);
      else PIV_PAD_PYR(uint16_t, false);
    }
#undef PIV_PAD_PYR
    if (hipError_t e = hipGetLastError()) return e;
  }
  for (int l = l2 ? 3 : 2; l < P.L; ++l) {
    const Level& u = P.lv[l - 1];
    const Level& v = P.lv[l];
    const int nch = (v.W + 7) / 8;
    dim3 blk(256);
    dim3 grid((unsigned)((nch * v.H + 255) / 256), 1, 2 * n);
    if (P.es == 1)
      hipLaunchKernelGGL(k_pyr_down<uint8_t>, grid, blk, 0, s, P.ws, (int64_t)P.per_pair, (int64_t)u.off_a,
                         (int64_t)u.off_b, u.pitch, u.margin, (int64_t)v.off_a, (int64_t)v.off_b, v.pitch,
                         v.margin, v.W, v.H, P.slot_mask);
    else
      hipLaunchKernelGGL(k_pyr_down<uint16_t>, grid, blk, 0, s, P.ws, (int64_t)P.per_pair, (int64_t)u.off_a,
                         (int64_t)u.off_b, u.pitch, u.margin, (int64_t)v.off_a, (int64_t)v.off_b, v.pitch,
                         v.margin, v.W, v.H, P.slot_mask);
    if (hipError_t e = hipGetLastError()) return e;
  }
  return hipSuccess;
}

hipError_t launch_sad_level(const Plan& P, int l, const void* A, const void* B, int64_t pitch, int n,
                            hipStream_t s) {
  if (P.p.sgm && l == P.L - 1) return launch_sgm_level(P, n, s);
  const Level& v = P.lv[l];
  SadArgs g;
  g.direct = l == 0 && level0_in_place(P, pitch) ? 1 : 0;
  g.srcA = (const uint8_t*)A;
  g.srcB = (const uint8_t*)B;
  g.spitch = pitch;
  g.sstride = pitch * P.p.height;
  g.W = v.W;
  g.H = v.H;
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
  g.npw = 0;
  g.margin = v.margin;
  const int G = 2 * g.R + 1;
  const int NW = P.block * P.es / 4;
  // finer levels, u16, 24x24 blocks at step 12, R <= 2: cell-shared sums per parent
  if (g.parent && P.es == 2 && P.p.step == 12 && P.block == 24 && g.R >= 1 && g.R <= 2) {
    const int tiles = (((v.nx + 1) / 2 + 6) / 7) * ((v.ny + 1) / 2);
    const dim3 grid((tiles + 3) / 4, 1, n);
    if (g.R == 2) hipLaunchKernelGGL((k_sad_cells16_fine<2>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((k_sad_cells16_fine<1>), grid, dim3(256), 0, s, g);
    return hipGetLastError();
  }
  if (P.es == 2 && g.R >= 1 && g.R <= 2 && (NW == 6 || NW == 8 || NW == 12)) {
    dim3 grid((v.nx * v.ny + 255) / 256, n);
#define PIV_SAD_STREAM(NW_, R_) \
  if (NW == NW_ && g.R == R_) { hipLaunchKernelGGL((k_sad_stream<2, NW_, R_>), grid, dim3(256), 0, s, g); return hipGetLastError(); }
    PIV_SAD_STREAM(12, 2) PIV_SAD_STREAM(12, 1) PIV_SAD_STREAM(8, 2) PIV_SAD_STREAM(8, 1)
    PIV_SAD_STREAM(6, 2) PIV_SAD_STREAM(6, 1)
#undef PIV_SAD_STREAM
  }
  // finer levels, u8, 16x16 blocks at step 8, R <= 2: cell-shared sums per parent
  if (g.parent && P.es == 1 && P.p.step == 8 && P.block == 16 && g.R >= 1 && g.R <= 2 &&
      (size_t)v.rows * v.pitch < (1u << 31) && v.pitch < (1 << 24)) {
    const int tiles3 = (((v.nx + 1) / 2 + 20) / 21) * ((v.ny + 1) / 2);
    const dim3 grid3((tiles3 + 3) / 4, 1, n);
    if (g.R == 2) hipLaunchKernelGGL((k_sad_cols<2>), grid3, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((k_sad_cols<1>), grid3, dim3(256), 0, s, g);
    return hipGetLastError();
  }
  const bool off31 = (size_t)v.rows * v.pitch < (1u << 31) && v.pitch < (1 << 24);
  if (P.es == 1 && g.R <= 2 && (NW == 2 || NW == 3 || NW == 4) && off31) {
    dim3 grid((v.nx * v.ny + 255) / 256, n);
    const bool aal = P.p.step % 4 == 0 && ((P.p.step - P.block) / 2) % 4 == 0;
#define PIV_SAD_LANE(NW_, R_)                                                                \
  if (NW == NW_ && g.R == R_) {                                                             \
    if (aal) hipLaunchKernelGGL((k_sad_lane<NW_, R_, true>), grid, dim3(256), 0, s, g);   \
    else hipLaunchKernelGGL((k_sad_lane<NW_, R_, false>), grid, dim3(256), 0, s, g);      \
    return hipGetLastError();                                                               \
  }
    PIV_SAD_LANE(4, 2) PIV_SAD_LANE(4, 1) PIV_SAD_LANE(4, 0)
    PIV_SAD_LANE(3, 2) PIV_SAD_LANE(3, 1) PIV_SAD_LANE(3, 0)
    PIV_SAD_LANE(2, 2) PIV_SAD_LANE(2, 1) PIV_SAD_LANE(2, 0)
#undef PIV_SAD_LANE
  }
  // coarsest level, u16, 24x24 blocks at step 12: cell-shared sums
  if (!g.parent && P.es == 2 && P.p.step == 12 && P.block == 24 && g.R >= 3 && g.R <= 7) {
    const int tiles = ((v.nx + 7) / 8) * ((v.ny + 5) / 6);
    dim3 grid(tiles, 1, n);
#define PIV_SAD16(R_, D_) \
  hipLaunchKernelGGL((k_sad_cells16<R_, D_>), grid, dim3(64 * sad_passes<R_, D_>()), 0, s, g)
    switch (g.R) {
      case 3: PIV_SAD16(3, 4); break;
      case 4: PIV_SAD16(4, 4); break;
      case 5: PIV_SAD16(5, 3); break;
      case 6: PIV_SAD16(6, 3); break;
      default: PIV_SAD16(7, 3); break;
    }
#undef PIV_SAD16
    return hipGetLastError();
  }
  // coarsest level, u8, 16x16 blocks at step 8: cell-shared sums
  if (!g.parent && P.es == 1 && P.p.step == 8 && P.block == 16 && g.R >= 3 && g.R <= 7 &&
      (size_t)v.rows * v.pitch < (1u << 31) && v.pitch < (1 << 24)) {
    const int tiles = ((v.nx + 7) / 8) * ((v.ny + 5) / 6);
    dim3 grid(tiles, 1, n);
#define PIV_SAD8(R_, D_) hipLaunchKernelGGL((k_sad_cells<R_, D_>), grid, dim3(64 * sad_passes<R_, D_>()), 0, s, g)
    switch (g.R) {
      case 3: PIV_SAD8(3, 7); break;
      case 4: PIV_SAD8(4, 5); break;
      case 5: PIV_SAD8(5, 6); break;
      case 6: PIV_SAD8(6, 7); break;
      default: PIV_SAD8(7, 5); break;
    }
#undef PIV_SAD8
    return hipGetLastError();
  }
  // nodes per workgroup: G lanes each, A blocks within 64 KiB of LDS
  const int npw = min(256 / G, 65536 / (P.block * NW * 4));
  if (P.es == 1 && NW >= 1 && NW <= 4 && G <= 4 * 8) {
    g.npw = npw;
    dim3 grid((v.nx + npw - 1) / npw, v.ny, n);
    size_t lds = sizeof(uint32_t) * (size_t)npw * P.block * NW;
    const int ngrp = (G + 3) / 4;
    // the coarsest level stages its common band of B when the nodes' spans
    // stay word-aligned relative to each other and the band fits
    const size_t band = sizeof(uint32_t) * (size_t)(G + P.block - 1) *
                        (size_t)((npw - 1) * (P.p.step / 4) + NW + ngrp + 1);
    const bool stage = !g.parent && P.p.step % 4 == 0 && lds + band <= 60 * 1024;
    if (stage) lds += band;
#define PIV_SAD_Q(NW_, NG_) \
  if (NW == NW_ && ngrp == NG_) { \
    if (stage) hipLaunchKernelGGL((k_sad_q<NW_, NG_, true>), grid, dim3(256), lds, s, g); \
    else hipLaunchKernelGGL((k_sad_q<NW_, NG_, false>), grid, dim3(256), lds, s, g); \
    return hipGetLastError(); }
#define PIV_SAD_Q_NW(NW_) PIV_SAD_Q(NW_, 1) PIV_SAD_Q(NW_, 2) PIV_SAD_Q(NW_, 3) PIV_SAD_Q(NW_, 4) \
  PIV_SAD_Q(NW_, 5) PIV_SAD_Q(NW_, 6) PIV_SAD_Q(NW_, 7) PIV_SAD_Q(NW_, 8)
    PIV_SAD_Q_NW(1) PIV_SAD_Q_NW(2) PIV_SAD_Q_NW(3) PIV_SAD_Q_NW(4)
#undef PIV_SAD_Q_NW
#undef PIV_SAD_Q
  }
  g.npw = npw;
  dim3 grid((v.nx + npw - 1) / npw, v.ny, n);
  size_t lds = sizeof(uint32_t) * (size_t)npw * P.block * NW;
  g.qsplit = 1;
  g.band = 0;
  if (P.es == 2 && G <= 17) {
    // a lane per candidate row (u16 blocks of 8..32 px)
#define PIV_SAD_R(NW_, K_) \
  if (NW == NW_ && G <= K_) { hipLaunchKernelGGL((k_sad_r<2, NW_, K_>), grid, dim3(256), lds, s, g); return hipGetLastError(); }
#define PIV_SAD_R_NW(NW_) PIV_SAD_R(NW_, 5) PIV_SAD_R(NW_, 9) PIV_SAD_R(NW_, 13) PIV_SAD_R(NW_, 17)
    PIV_SAD_R_NW(4) PIV_SAD_R_NW(6) PIV_SAD_R_NW(8) PIV_SAD_R_NW(12) PIV_SAD_R_NW(16)
#undef PIV_SAD_R_NW
#undef PIV_SAD_R
  }
  // k_sad: the candidate rows of a column in groups of about two, each its
  // own thread, so that few nodes still make many threads; and without a
  // parent the workgroup's band of B rows staged in LDS
  {
    int qs = max(1, min((G + 1) / 2, 256 / G));
    const int qn = (G + qs - 1) / qs;
    qs = (G + qn - 1) / qn;   // (no empty group)
    const int npq = max(1, min(256 / (G * qs), 65536 / (P.block * NW * 4)));
    g.qsplit = qs;
    g.npw = npq;
    grid = dim3((v.nx + npq - 1) / npq, v.ny, n);
    lds = sizeof(uint32_t) * (size_t)npq * P.block * NW;
    const int bw = ((npq - 1) * P.p.step + 2 * g.R) * P.es / 4 + NW + 2;
    const size_t bbytes = sizeof(uint32_t) * (size_t)bw * (size_t)(P.block + 2 * g.R);
    if (!g.parent && lds + bbytes <= 60 * 1024) {
      g.band = bw;
      lds += bbytes;
    }
    return P.es == 1 ? sad_dispatch<1>(NW, qn, grid, lds, s, g) : sad_dispatch<2>(NW, qn, grid, lds, s, g);
  }
}

// The coarsest level's SAD of every node and shift into a cost volume
// (semi-global matching) by the cell-shared kernel, where its geometry
// applies (u8, 16x16 blocks at step 8, R 3..7); hipErrorNotSupported
// otherwise.
hipError_t launch_sad_cost_cells(const Plan& P, uint32_t* C, int64_t cstride, int n, hipStream_t s) {
  const int l = P.L - 1;
  const Level& v = P.lv[l];
  if (!(P.es == 1 && P.p.step == 8 && P.block == 16 && v.R >= 3 && v.R <= 7 &&
        (size_t)v.rows * v.pitch < (1u << 31) && v.pitch < (1 << 24)))
    return hipErrorNotSupported;
  SadArgs g = {};
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
  g.parent = nullptr;
  g.out = nullptr;
  g.mask = P.slot_mask;
  g.margin = v.margin;
  g.W = v.W;
  g.H = v.H;
  g.cost = C;
  g.cstride = cstride;
  const int tiles = ((v.nx + 7) / 8) * ((v.ny + 5) / 6);
  dim3 grid(tiles, 1, n);
#define PIV_SADC(R_, D_) \
  hipLaunchKernelGGL((k_sad_cells<R_, D_, true>), grid, dim3(64 * sad_passes<R_, D_>()), 0, s, g)
  switch (g.R) {
    case 3: PIV_SADC(3, 7); break;
    case 4: PIV_SADC(4, 5); break;
    case 5: PIV_SADC(5, 6); break;
    case 6: PIV_SADC(6, 7); break;
    default: PIV_SADC(7, 5); break;
  }
#undef PIV_SADC
  return hipGetLastError();
}

hipError_t launch_pred_out(const Plan& P, int n, float* pred, hipStream_t s) {
  const Level& v = P.lv[0];
  dim3 grid((v.nx * v.ny + 255) / 256, n);
  hipLaunchKernelGGL(k_pred_out, grid, dim3(256), 0, s, reinterpret_cast<const int32_t*>(P.ws + v.off_d),
                     (int64_t)(P.per_pair / sizeof(int32_t)), v.nx, v.ny, P.p.median, pred, P.slot_mask);
  return hipGetLastError();
}

}  // namespace piv
