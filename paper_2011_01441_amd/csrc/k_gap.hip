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
// final already, for the diagonal term) and padded with INF to GAP_B + 1
// cells a side; two weight tables (wrt[j][q] = w(q, j), wct[i][p] = w'(p, i))
// hold GAP_NOPE where the source is not before the target, so that a
// candidate from outside the cell's predecessors can never win and the
// candidate reads need no bounds test; the two sequences' symbols sit in
// sx / sy.  Anti-diagonal dd holds the cells with local row + column = dd;
// each is final once the diagonals before it are.  GAP_TPC threads per cell
// take every GAP_TPC-th row and column predecessor, as many slots as the
// diagonal's longest row or column needs (a block-uniform count, so the
// reads are issued together); the group's minimum joins the cell's own
// value and diagonal term.  Waves that hold no cell of the diagonal go
// straight to the barrier.  Rows are GAP_LS words apart (GAP_TPC mod 64
// banks): the 64 lanes of a wave read 64 different banks.
constexpr int GAP_TPC = 16;   // threads per cell (4, 8 or 16; measured: 16 is fastest)
static_assert(GAP_TPC == 4 || GAP_TPC == 8 || GAP_TPC == 16, "lane groups of 4, 8 or 16");
constexpr int GAP_THREADS = GAP_B * GAP_TPC;
constexpr int GAP_WAVES = GAP_THREADS / 64;
constexpr int GAP_CPW = 64 / GAP_TPC;   // cells per wave
constexpr int GAP_LS = GAP_B + GAP_TPC;   // LDS row stride in words (GAP_TPC mod 64 banks)
constexpr int GAP_SLOTS = GAP_B / GAP_TPC;   // slots a side at most
constexpr int GAP_HROWS = (GAP_B + 1 + GAP_WAVES - 1) / GAP_WAVES;   // halo rows per wave
// weight-table entry of a source at or after the target: values are at most
// INF = 2^30, so value + GAP_NOPE > INF and stays below 2^32
constexpr uint32_t GAP_NOPE = 1u << 31;

// minimum over each aligned group of GAP_TPC lanes (every lane of the group
// gets it): quad swaps, then the other quad of each half-row (mirror), then
// the other half of each row (rotate by 8)
__device__ __forceinline__ uint32_t min_group(uint32_t v) {
  v = gmin(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));    // quad_perm [1,0,3,2]
  v = gmin(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));    // quad_perm [2,3,0,1]
  if constexpr (GAP_TPC >= 8)
    v = gmin(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));  // row_half_mirror
  if constexpr (GAP_TPC >= 16)
    v = gmin(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x128, 0xF, 0xF, false));  // row_ror:8
  return v;
}

// LDS of a base block, one array so that regions read with the same index
// sit within an instruction's offset range of each other: hr / wct (indexed
// by the row) and hc / wrt (indexed by the column)
constexpr int GAP_HSZ = (GAP_B + 1) * GAP_LS, GAP_WSZ = GAP_B * GAP_LS;
constexpr int GAP_HR = 0;                      // hr[(li + 1) * LS + lj + 1]
constexpr int GAP_WCT = GAP_HR + GAP_HSZ;      // wct[li * LS + p] = w'(r0 + p, r0 + li), p < li
constexpr int GAP_HC = GAP_WCT + GAP_WSZ;      // hc[(lj + 1) * LS + li + 1]
constexpr int GAP_WRT = GAP_HC + GAP_HSZ;      // wrt[lj * LS + q] = w(c0 + q, c0 + lj), q < lj
constexpr int GAP_SX = GAP_WRT + GAP_WSZ;      // symbols of rows r0 + li
constexpr int GAP_SY = GAP_SX + GAP_B;         // symbols of columns c0 + lj
constexpr int GAP_LDS = GAP_SY + GAP_B;

// One anti-diagonal dd for one thread, N slots a side: the cell's own value,
// its diagonal term (the value up-left plus the substitution cost), N slots
// of its row predecessors and N of its column predecessors (slot k at
// GAP_TPC k), every read issued before the first sum; the group's minimum is
// stored by its first two lanes (row-major and column-major copy).
template <int N>
__device__ __forceinline__ void gap_diag(uint32_t* L, int dd, int R, int C, int wv, int cell, int u,
                                         const GapS& s) {
  const int lo = dd - (C - 1) > 0 ? dd - (C - 1) : 0;   // first and last row on the diagonal
  const int hi = dd < R - 1 ? dd : R - 1;
  if (GAP_CPW * wv > hi - lo) return;                   // no cell of this wave on the diagonal
  const int li0 = lo + cell;
  const bool live = li0 <= hi;
  const int li = li0 < hi ? li0 : hi, lj = dd - li;    // lanes past the diagonal's end read a real cell
  const int rc = li * GAP_LS + lj;                      // (li + 1, lj + 1) in hr, less LS + 1
  const int ru = li * GAP_LS + u, cu = lj * GAP_LS + u;
  uint32_t v[2 * N + 1], w[2 * N + 1];
  const uint32_t own = L[GAP_HR + rc + GAP_LS + 1], sxv = L[GAP_SX + li], syv = L[GAP_SY + lj];
  v[2 * N] = L[GAP_HR + rc];   // the halo's INF row / column covers the grid's first row and column
#pragma unroll
  for (int k = 0; k < N; ++k) {
    v[k] = L[GAP_HR + ru + GAP_LS + 1 + GAP_TPC * k];
    w[k] = L[GAP_WRT + cu + GAP_TPC * k];
    v[N + k] = L[GAP_HC + cu + GAP_LS + 1 + GAP_TPC * k];
    w[N + k] = L[GAP_WCT + ru + GAP_TPC * k];
  }
  w[2 * N] = sxv == syv ? s.match : s.mismatch;
  uint32_t acc = own;
#pragma unroll
  for (int k = 0; k < 2 * N + 1; ++k) acc = gmin(acc, v[k] + w[k]);
  acc = gmin(min_group(acc), G_INF);
  if (live && u < 2) L[u == 0 ? GAP_HR + rc + GAP_LS + 1 : GAP_HC + lj * GAP_LS + li + GAP_LS + 1] = acc;
}

template <int WKR, int WKC>
__global__ __launch_bounds__(GAP_THREADS) void k_gap_base(uint32_t* __restrict__ D, int64_t ld,
                                                          uint32_t* __restrict__ DT, int64_t ldt,
                                                          const GapBlock* __restrict__ blocks, GapW wr, GapW wc,
                                                          GapS s) {
  __shared__ uint32_t L[GAP_LDS];
  uint32_t* hr = L + GAP_HR;
  uint32_t* hc = L + GAP_HC;
  const GapBlock b = blocks[blockIdx.x];
  const int R = (int)(b.r1 - b.r0), C = (int)(b.c1 - b.c0);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  // halo and block: wave wv takes rows wv, wv + GAP_WAVES, ...; every load first
  {
    uint32_t hv[GAP_HROWS][2];
#pragma unroll
    for (int a = 0; a < GAP_HROWS; ++a) {
#pragma unroll
      for (int c2 = 0; c2 < 2; ++c2) {
        const int hi = wv + GAP_WAVES * a, hj = lane + 64 * c2;
        const int64_t gi = b.r0 + hi - 1, gj = b.c0 + hj - 1;
        hv[a][c2] = (hi <= R && hj <= C && gi >= 0 && gj >= 0) ? gmin(D[gi * ld + gj], G_INF) : G_INF;
      }
    }
#pragma unroll
    for (int a = 0; a < GAP_HROWS; ++a) {
#pragma unroll
      for (int c2 = 0; c2 < 2; ++c2) {
        const int hi = wv + GAP_WAVES * a, hj = lane + 64 * c2;
        if (hi <= GAP_B && hj <= GAP_B) {
          hr[hi * GAP_LS + hj] = hv[a][c2];
          hc[hj * GAP_LS + hi] = hv[a][c2];
        }
      }
    }
  }
  for (int e = tid; e < GAP_B * GAP_B; e += GAP_THREADS) {
    const int x = e / GAP_B, y = e - x * GAP_B;   // target x, source y
    L[GAP_WRT + x * GAP_LS + y] = y < x ? gw<WKR>(wr, (uint32_t)(b.c0 + y), (uint32_t)(b.c0 + x)) : GAP_NOPE;
    L[GAP_WCT + x * GAP_LS + y] = y < x ? gw<WKC>(wc, (uint32_t)(b.r0 + y), (uint32_t)(b.r0 + x)) : GAP_NOPE;
  }
  if (tid < GAP_B) {
    L[GAP_SX + tid] = gfmix((uint32_t)(b.r0 + tid) ^ s.seedx) & s.mask;
  } else if (tid < 2 * GAP_B) {
    L[GAP_SY + tid - GAP_B] = gfmix((uint32_t)(b.c0 + tid - GAP_B) ^ s.seedy) & s.mask;
  }
  __syncthreads();
  const int u = tid & (GAP_TPC - 1);
  const int cell = tid / GAP_TPC;
  // The slot count a diagonal needs, ceil(min(dd, max(R, C) - 1) / GAP_TPC),
  // grows with dd and then stays: the diagonals run in segments of one count
  // (segment N ends at dd = GAP_TPC N, the last one at the block's end).
  const int last = R + C - 2;
  const int mx = (R > C ? R : C) - 1;
  const int nmax = (mx + GAP_TPC - 1) / GAP_TPC;
  int dd = 0;
#define GAP_SEGMENT(N)                                                        \
  if constexpr (N <= GAP_SLOTS) {                                             \
    if (N <= nmax) {                                                          \
      const int end = N == nmax ? last + 1 : GAP_TPC * N + 1;                 \
      for (; dd < end; ++dd) {                                                \
        gap_diag<N>(L, dd, R, C, wv, cell, u, s);                             \
        __syncthreads();                                                      \
      }                                                                       \
    }                                                                         \
  }
  GAP_SEGMENT(0) GAP_SEGMENT(1) GAP_SEGMENT(2) GAP_SEGMENT(3) GAP_SEGMENT(4)
  GAP_SEGMENT(5) GAP_SEGMENT(6) GAP_SEGMENT(7) GAP_SEGMENT(8)
  GAP_SEGMENT(9) GAP_SEGMENT(10) GAP_SEGMENT(11) GAP_SEGMENT(12)
  GAP_SEGMENT(13) GAP_SEGMENT(14) GAP_SEGMENT(15) GAP_SEGMENT(16)
#undef GAP_SEGMENT
#pragma unroll
  for (int a = 0; a < GAP_B / GAP_WAVES; ++a) {
    const int li = wv + GAP_WAVES * a, lj = lane;
    if (li < R && lj < C) D[(b.r0 + li) * ld + b.c0 + lj] = hr[(li + 1) * GAP_LS + lj + 1];
  }
#pragma unroll
  for (int a = 0; a < GAP_B / GAP_WAVES; ++a) {
    const int lj = wv + GAP_WAVES * a, li = lane;
    if (lj < C && li < R) DT[(b.c0 + lj) * ldt + b.r0 + li] = hc[(lj + 1) * GAP_LS + li + 1];
  }
}

// One cube piece per workgroup.  Row-gap piece (col = 0): for rows
// t in [t0, t1), D[t][o] = min over inputs x in [x0, x1) of D[t][x] + w(x, o),
// outputs o in [o0, o1).  Column-gap piece (col = 1): for columns t,
// D[o][t] = min over x of DT[t][x] + w'(x, o).  A wave takes one batch index,
// four 64-output strips (four outputs per lane; one strip when the piece is
// at most 128 outputs wide) and a slice of the inputs, read 8 at a time as
// wave-uniform values (affine weights: 16 at a time, in two alternating sets).
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
  if constexpr (WK == 0) {
    // affine weights cost about two instructions a pair, too few to cover a
    // load from HBM: two sets of 16 inputs alternate, each requested while
    // the other is applied
    constexpr int CH = 16;
    if (x + 2 * CH <= xb) {
      uint32_t va[CH], vb[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k) va[k] = src[x + k];
      for (; x + 2 * CH <= xb; x += 2 * CH) {
#pragma unroll
        for (int k = 0; k < CH; ++k) vb[k] = src[x + CH + k];
#pragma unroll
        for (int k = 0; k < CH; ++k) {
#pragma unroll
          for (int r = 0; r < NR; ++r) acc[r] = gmin(acc[r], va[k] + gw<WK>(w, (uint32_t)(x + k), ou[r]));
        }
        if (x + 4 * CH <= xb) {
#pragma unroll
          for (int k = 0; k < CH; ++k) va[k] = src[x + 2 * CH + k];
        }
#pragma unroll
        for (int k = 0; k < CH; ++k) {
#pragma unroll
          for (int r = 0; r < NR; ++r) acc[r] = gmin(acc[r], vb[k] + gw<WK>(w, (uint32_t)(x + CH + k), ou[r]));
        }
      }
    }
  }
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

// one piece's units with the weight kind WK of its direction
template <int WK>
__device__ __forceinline__ void cube_piece(uint32_t* __restrict__ D, int64_t ld, const uint32_t* __restrict__ DT,
                                           int64_t ldt, const GapPiece& pc, const GapW& w) {
  const int lane = threadIdx.x & 63;
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t T = pc.t1 - pc.t0, W = pc.o1 - pc.o0, H = pc.x1 - pc.x0;
  const bool col = pc.col != 0;
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
    if (nr == 1) cube_unit<WK, 1>(D, ld, src, col, t, ob, pc.o1, xa, xb, w);
    else cube_unit<WK, GR>(D, ld, src, col, t, ob, pc.o1, xa, xb, w);
  }
}

// One piece per workgroup; WKR / WKC the weight kinds of the row and column
// directions (one instantiation each, so that a kind's registers do not
// limit the other's occupancy).
template <int WKR, int WKC>
__global__ __launch_bounds__(256) void k_gap_cube(uint32_t* __restrict__ D, int64_t ld, const uint32_t* __restrict__ DT,
                                                  int64_t ldt, const GapPiece* __restrict__ pieces, GapW wr, GapW wc) {
  const GapPiece pc = pieces[blockIdx.x];
  if (pc.t1 <= pc.t0 || pc.o1 <= pc.o0 || pc.x1 <= pc.x0) return;
  if (pc.col != 0) cube_piece<WKC>(D, ld, DT, ldt, pc, wc);
  else cube_piece<WKR>(D, ld, DT, ldt, pc, wr);
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
  const dim3 g(npieces), t(256);
  if (wr.kind == 0 && wc.kind == 0) {
    hipLaunchKernelGGL((k_gap_cube<0, 0>), g, t, 0, s, D, ld, DT, ldt, pieces, wr, wc);
  } else if (wr.kind == 0) {
    hipLaunchKernelGGL((k_gap_cube<0, 1>), g, t, 0, s, D, ld, DT, ldt, pieces, wr, wc);
  } else if (wc.kind == 0) {
    hipLaunchKernelGGL((k_gap_cube<1, 0>), g, t, 0, s, D, ld, DT, ldt, pieces, wr, wc);
  } else {
    hipLaunchKernelGGL((k_gap_cube<1, 1>), g, t, 0, s, D, ld, DT, ldt, pieces, wr, wc);
  }
  return hipGetLastError();
}

}  // namespace paco
