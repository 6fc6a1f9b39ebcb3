// k_gap.hip -- the GAP problem (section "PACO GAP", equation (gap)):
// D[i][j] = min(D[i-1][j-1] + s(i, j), min over q < j of D[i][q] + w(q, j),
//               min over p < i of D[p][j] + w'(p, i)).
//
// The recursion splits a block of the grid into quadrants: once the top-left
// one is final, its rows update the top-right one and its columns the
// bottom-left one (the external updates, "cubes" of batch x inputs x
// outputs), and so on.  Three kernels: a fill, the base blocks (at most
// GAP_B x GAP_B, one workgroup each, cells finished by anti-diagonals), and
// the cubes (one workgroup per PACO piece).  A row-gap cube reads its inputs
// from D; a column-gap cube reads them from DT, the transposed copy of the
// final values that the base kernel keeps, so that both read their inputs as
// wave-uniform scalars.  Cube outputs combine with atomic minima (exact).
// Values are unsigned 32-bit with INF = 2^30 and weights <= 2^30.
#include "kcommon.h"
#include "kernels.h"

namespace paco {
namespace {

constexpr uint32_t G_INF = 1u << 30;
constexpr uint32_t G_KEY_MUL = 0x9E3779B9u;

__device__ __forceinline__ uint32_t gmin(uint32_t x, uint32_t y) { return x < y ? x : y; }

// MurmurHash3's 32-bit finaliser (Appleby)
__device__ __forceinline__ uint32_t gfmix(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

// weight of a gap from index `from` to index `to` (from < to): WK 0
// affine a + b (to - from), WK 1 hashed a + (fmix32(from K + to ^ seed) & mask)
template <int WK>
__device__ __forceinline__ uint32_t gw(const GapW& w, uint32_t from, uint32_t to) {
  if constexpr (WK == 0) {
    return w.a + w.b * (to - from);
  } else {
    return w.a + (gfmix((from * G_KEY_MUL + to) ^ w.seed) & w.b);
  }
}

__device__ __forceinline__ uint32_t gs(const GapS& s, uint32_t i, uint32_t j) {
  const uint32_t xi = gfmix(i ^ s.seedx) & s.mask;
  const uint32_t yj = gfmix(j ^ s.seedy) & s.mask;
  return xi == yj ? s.match : s.mismatch;
}

// every cell but (0, 0) = INF; (0, 0) clamped to INF
__global__ __launch_bounds__(256) void k_gap_fill(uint32_t* __restrict__ D, int64_t ld, int64_t rows, int64_t cols) {
  const int64_t total = rows * cols;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e / cols, j = e - i * cols;
    uint32_t* p = D + i * ld + j;
    *p = e == 0 ? gmin(*p, G_INF) : G_INF;
  }
}

// One base block per workgroup: rows [r0, r0 + R), columns [c0, c0 + C),
// R, C <= GAP_B, whose cells already hold every update from outside the
// block.  LDS holds the block twice, row-major (hr) and column-major (hc),
// each with a one-cell halo (the row above and the column to the left,
// final already, for the diagonal term); hashed weights also get tables
// (wrt[j][q] = w(q, j), wct[i][p] = w'(p, i)), affine ones are stepped in
// registers.  Anti-diagonal dd holds the cells with local row + column = dd;
// each is final once the diagonals before it are.  GAP_TPC threads per cell
// take every GAP_TPC-th row and column predecessor; the
// group's minimum joins the cell's own value and diagonal term.  Rows are
// GAP_LS words apart (GAP_TPC mod 64 banks): the 64 lanes of a wave read 64
// different banks.
constexpr int GAP_TPC = 16;   // threads per cell (measured: 16 beats 8 and 4)
constexpr int GAP_THREADS = GAP_B * GAP_TPC;
constexpr int GAP_LS = 80;    // LDS row stride in words (16 mod 64 banks)

// minimum over each row of 16 lanes
__device__ __forceinline__ uint32_t min16(uint32_t v) {
  v = gmin(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));    // quad_perm [1,0,3,2]
  v = gmin(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));    // quad_perm [2,3,0,1]
  v = gmin(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x124, 0xF, 0xF, false));   // row_ror:4
  v = gmin(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false));   // row_ror:8
  return v;
}

// a cell's partial minimum over its row (q = u, u + 4, ... < lj) or column
// predecessors; `val` the row (or column) in LDS, `wt` the weight table row
// (hashed) or, affine, weight w0 at the first slot and step down by step
// (all slots read, indices inside the arrays, so that the reads are in
// flight together; slots at or past lim are discarded)
template <int WK>
__device__ __forceinline__ uint32_t scan_slots(uint32_t acc, const uint32_t* val, const uint32_t* wt, int u, int lim,
                                               uint32_t w0, uint32_t step) {
#pragma unroll
  for (int k = 0; k < GAP_B / GAP_TPC; ++k) {
    const int q = u + GAP_TPC * k;
    const uint32_t wq = WK == 0 ? w0 - step * (uint32_t)k : wt[q];
    const uint32_t c = val[q] + wq;
    acc = q < lim ? gmin(acc, c) : acc;
  }
  return acc;
}

template <int WKR, int WKC>
__global__ __launch_bounds__(GAP_THREADS) void k_gap_base(uint32_t* __restrict__ D, int64_t ld,
                                                          uint32_t* __restrict__ DT, int64_t ldt,
                                                          const GapBlock* __restrict__ blocks, GapW wr, GapW wc,
                                                          GapS s) {
  __shared__ uint32_t hr[(GAP_B + 1) * GAP_LS];   // hr[(li + 1) * LS + lj + 1]
  __shared__ uint32_t hc[(GAP_B + 1) * GAP_LS];   // hc[(lj + 1) * LS + li + 1]
  __shared__ uint32_t wrt[WKR == 1 ? GAP_B * GAP_LS : 1];   // wrt[lj * LS + q] = w(c0 + q, c0 + lj)
  __shared__ uint32_t wct[WKC == 1 ? GAP_B * GAP_LS : 1];   // wct[li * LS + p] = w'(r0 + p, r0 + li)
  const GapBlock b = blocks[blockIdx.x];
  const int R = (int)(b.r1 - b.r0), C = (int)(b.c1 - b.c0);
  const int tid = threadIdx.x;
  for (int e = tid; e < (R + 1) * (C + 1); e += GAP_THREADS) {
    const int hi = e / (C + 1), hj = e - hi * (C + 1);
    const int64_t gi = b.r0 + hi - 1, gj = b.c0 + hj - 1;
    const uint32_t v = (gi >= 0 && gj >= 0) ? gmin(D[gi * ld + gj], G_INF) : G_INF;
    hr[hi * GAP_LS + hj] = v;
    hc[hj * GAP_LS + hi] = v;
  }
  for (int e = tid; e < GAP_B * GAP_B; e += GAP_THREADS) {
    const int x = e / GAP_B, y = e - x * GAP_B;   // target x, source y
    if constexpr (WKR == 1) wrt[x * GAP_LS + y] = gw<1>(wr, (uint32_t)(b.c0 + y), (uint32_t)(b.c0 + x));
    if constexpr (WKC == 1) wct[x * GAP_LS + y] = gw<1>(wc, (uint32_t)(b.r0 + y), (uint32_t)(b.r0 + x));
  }
  __syncthreads();
  const int u = tid & (GAP_TPC - 1);
  const int cell = tid / GAP_TPC;
  for (int dd = 0; dd <= R + C - 2; ++dd) {
    const int li = (dd - (C - 1) > 0 ? dd - (C - 1) : 0) + cell;
    const int lj = dd - li;
    const bool live = li < R && lj >= 0 && li <= dd;
    uint32_t acc = G_INF;
    if (live) {
      const int64_t gi = b.r0 + li, gj = b.c0 + lj;
      acc = hr[(li + 1) * GAP_LS + lj + 1];
      if (u == 0 && gi >= 1 && gj >= 1) acc = gmin(acc, hr[li * GAP_LS + lj] + gs(s, (uint32_t)gi, (uint32_t)gj));
      // affine: w(c0 + u + T k, c0 + lj) = a + b (lj - u) - T b k, T = GAP_TPC
      acc = scan_slots<WKR>(acc, hr + (li + 1) * GAP_LS + 1, wrt + (WKR == 1 ? lj * GAP_LS : 0), u, lj,
                       wr.a + wr.b * (uint32_t)(lj - u), wr.b * GAP_TPC);
      acc = scan_slots<WKC>(acc, hc + (lj + 1) * GAP_LS + 1, wct + (WKC == 1 ? li * GAP_LS : 0), u, li,
                       wc.a + wc.b * (uint32_t)(li - u), wc.b * GAP_TPC);
    }
    acc = gmin(min16(acc), G_INF);
    if (live && u == 0) {
      hr[(li + 1) * GAP_LS + lj + 1] = acc;
      hc[(lj + 1) * GAP_LS + li + 1] = acc;
    }
    __syncthreads();
  }
  for (int e = tid; e < R * C; e += GAP_THREADS) {
    const int li = e / C, lj = e - li * C;
    D[(b.r0 + li) * ld + b.c0 + lj] = hr[(li + 1) * GAP_LS + lj + 1];
  }
  for (int e = tid; e < R * C; e += GAP_THREADS) {
    const int lj = e / R, li = e - lj * R;
    DT[(b.c0 + lj) * ldt + b.r0 + li] = hc[(lj + 1) * GAP_LS + li + 1];
  }
}

// One cube piece per workgroup.  Row-gap piece (col = 0): for rows
// t in [t0, t1), D[t][o] = min over inputs x in [x0, x1) of D[t][x] + w(x, o),
// outputs o in [o0, o1).  Column-gap piece (col = 1): for columns t,
// D[o][t] = min over x of DT[t][x] + w'(x, o).  A wave takes one batch index,
// four 64-output strips (four outputs per lane; one strip when the piece is
// at most 128 outputs wide) and a slice of the inputs, read 8 at a time as
// wave-uniform values.
constexpr int GR = 4;

template <int WK, int NR>
__device__ __forceinline__ void cube_unit(uint32_t* __restrict__ D, int64_t ld, const uint32_t* __restrict__ src,
                                          bool col, int64_t t, int64_t ob, int64_t o1, int64_t xa, int64_t xb,
                                          const GapW& w) {
  uint32_t ou[NR], acc[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    ou[r] = (uint32_t)(ob + 64 * r);
    acc[r] = G_INF;
  }
  int64_t x = xa;
  for (; x + 8 <= xb; x += 8) {
    uint32_t dv[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) dv[k] = src[x + k];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
#pragma unroll
      for (int r = 0; r < NR; ++r) acc[r] = gmin(acc[r], dv[k] + gw<WK>(w, (uint32_t)(x + k), ou[r]));
    }
  }
  for (; x < xb; ++x) {
    const uint32_t dx = src[x];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = gmin(acc[r], dx + gw<WK>(w, (uint32_t)x, ou[r]));
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int64_t o = ob + 64 * r;
    if (o < o1) atomicMin(col ? D + o * ld + t : D + t * ld + o, gmin(acc[r], G_INF));
  }
}

__global__ __launch_bounds__(256) void k_gap_cube(uint32_t* __restrict__ D, int64_t ld, const uint32_t* __restrict__ DT,
                                                  int64_t ldt, const GapPiece* __restrict__ pieces, GapW wr, GapW wc) {
  const GapPiece pc = pieces[blockIdx.x];
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t T = pc.t1 - pc.t0, W = pc.o1 - pc.o0, H = pc.x1 - pc.x0;
  if (T <= 0 || W <= 0 || H <= 0) return;
  const bool col = pc.col != 0;
  const GapW w = col ? wc : wr;
  // narrow pieces (at most two strips) take one 64-output strip per unit
  const int nr = W <= 128 ? 1 : GR;
  const int64_t groups = (W + 64 * nr - 1) / (64 * nr);
  const int S = T * groups >= 4 ? 1 : (T * groups >= 2 ? 2 : 4);
  const int64_t units = T * groups * S;
  for (int64_t un = wv; un < units; un += 4) {
    const int slice = (int)(un % S);
    const int64_t rest = un / S;
    const int64_t t = pc.t0 + rest / groups;
    const int64_t g = rest % groups;
    const int64_t ob = pc.o0 + g * 64 * nr + lane;
    const int64_t xa = pc.x0 + H * slice / S, xb = pc.x0 + H * (slice + 1) / S;
    const uint32_t* src = col ? DT + t * ldt : D + t * ld;
    if (nr == 1) {
      if (w.kind == 0) {
        cube_unit<0, 1>(D, ld, src, col, t, ob, pc.o1, xa, xb, w);
      } else {
        cube_unit<1, 1>(D, ld, src, col, t, ob, pc.o1, xa, xb, w);
      }
    } else if (w.kind == 0) {
      cube_unit<0, GR>(D, ld, src, col, t, ob, pc.o1, xa, xb, w);
    } else {
      cube_unit<1, GR>(D, ld, src, col, t, ob, pc.o1, xa, xb, w);
    }
  }
}

}  // namespace

hipError_t launch_gap_fill(uint32_t* D, int64_t ld, int64_t rows, int64_t cols, hipStream_t s) {
  if (rows <= 0 || cols <= 0 || ld < cols) return hipErrorInvalidValue;
  const int64_t blocks = (rows * cols + 255) / 256;
  hipLaunchKernelGGL(k_gap_fill, dim3((unsigned)(blocks < 4096 ? blocks : 4096)), dim3(256), 0, s, D, ld, rows, cols);
  return hipGetLastError();
}

hipError_t launch_gap_base(uint32_t* D, int64_t ld, uint32_t* DT, int64_t ldt, const GapBlock* blocks, int nblocks,
                           const GapW& wr, const GapW& wc, const GapS& sub, hipStream_t s) {
  if (nblocks <= 0) return hipErrorInvalidValue;
  const dim3 g(nblocks), t(GAP_THREADS);
  if (wr.kind == 0 && wc.kind == 0) {
    hipLaunchKernelGGL((k_gap_base<0, 0>), g, t, 0, s, D, ld, DT, ldt, blocks, wr, wc, sub);
  } else if (wr.kind == 0) {
    hipLaunchKernelGGL((k_gap_base<0, 1>), g, t, 0, s, D, ld, DT, ldt, blocks, wr, wc, sub);
  } else if (wc.kind == 0) {
    hipLaunchKernelGGL((k_gap_base<1, 0>), g, t, 0, s, D, ld, DT, ldt, blocks, wr, wc, sub);
  } else {
    hipLaunchKernelGGL((k_gap_base<1, 1>), g, t, 0, s, D, ld, DT, ldt, blocks, wr, wc, sub);
  }
  return hipGetLastError();
}

hipError_t launch_gap_cube(uint32_t* D, int64_t ld, const uint32_t* DT, int64_t ldt, const GapPiece* pieces,
                           int npieces, const GapW& wr, const GapW& wc, hipStream_t s) {
  if (npieces <= 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_gap_cube, dim3(npieces), dim3(256), 0, s, D, ld, DT, ldt, pieces, wr, wc);
  return hipGetLastError();
}

}  // namespace paco
