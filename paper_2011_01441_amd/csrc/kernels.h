// kernels.h -- host-callable launchers of the HIP kernels (one per family).
#pragma once
#include <hip/hip_runtime.h>

#include "device_types.h"

namespace paco {

// Tile shapes of the integer (VALU) semiring kernel: output tile TM x TN,
// k-step 32, 256 threads.
enum IntTile : int { INT_T128x128 = 0, INT_T256x64 = 1, INT_T64x64 = 2, INT_T64x128 = 3, INT_T128x64 = 4 };
constexpr int kIntTiles = 5;
struct IntTileShape { int tm, tn; };
IntTileShape int_tile_shape(int tile);
// Workgroups of the kernel that fit on one compute unit at once (1 when the
// runtime cannot tell, e.g. without a device).
int int_occupancy(int sr, int tile);

// Persistent semiring kernel: `nwg` workgroups; workgroup w runs the items
// wg_off[q] .. wg_off[q+1] of processor q = remap(w).
hipError_t launch_semiring_int(int sr, int tile, const ProbRef& pr, const WorkItem* items,
                               const int32_t* wg_off, int nwg, int xcd_remap, void* ws,
                               hipStream_t s);

// Boolean OR-AND kernel on bit-packed words.
// Tile shapes of the boolean kernel: TM rows x TNW words, 128 bits per step.
enum BoolTile : int { BOOL_T512x32W = 0, BOOL_T128x128W = 1, BOOL_T256x64W = 2, BOOL_T64x64W = 3 };
struct BoolTileShape { int tm, tnw; };
BoolTileShape bool_tile_shape(int tile);
int bool_occupancy(int tile);
hipError_t launch_semiring_bool(int tile, const ProbRef& pr, const WorkItem* items,
                                const int32_t* wg_off, int nwg, int xcd_remap, void* ws,
                                hipStream_t s);

// (+,x) ring kernel on matrix cores.
// Tile shapes of the ring kernel (32 k per step): 8 waves (4 x 2, or 2 x 4
// for 256 x 256) unless marked W4 (4 waves, 2 x 2).
enum RingTile : int {
  RING_T256x128 = 0, RING_T128x128 = 1, RING_T128x64 = 2, RING_T128x128W4 = 3, RING_T256x256 = 4
};
struct RingTileShape { int tm, tn, bk; };
RingTileShape ring_tile_shape(int tile, int prec);
hipError_t launch_ring(int prec, int tile, const ProbRef& pr, const WorkItem* items,
                       const int32_t* wg_off, int nwg, int xcd_remap, void* ws, hipStream_t s);

// Fold temporary faces into C (ascending k), one workgroup per tile; a tile
// spans at most 256 * vec columns.  vec = 4 needs every C row segment and
// source face 16-byte aligned (HostPlan::red_vec).
hipError_t launch_reduce(int sr, const ProbRef& pr, const RedTile* tiles, int ntiles,
                         const RedSrc* srcs, const void* ws, hipStream_t s, int vec);

// C = semiring zero (or unchanged when accumulating) for k = 0.
hipError_t launch_fill_zero(int sr, void* C, int64_t rows, int64_t cols, int64_t ldc,
                            hipStream_t s);

// Float64 check of sampled rows: each of verify_blocks(m, nrows) blocks
// writes 4 doubles to `part` (device): max rel, max abs, sum of squared
// differences, sum of squared float64 values (see paco_verify_rows_f64).
int64_t verify_blocks(int64_t m, int64_t nrows);
hipError_t launch_verify_f64(int64_t n, int64_t m, int64_t k, const float* A, int64_t lda,
                             const float* B, int64_t ldb, const float* C, int64_t ldc,
                             const int64_t* rows, int64_t nrows, double* part, hipStream_t s);

// Strassen fused L-level (1..3) pre-add and combine (see k_strassen.hip):
// n x n A, B -> 7^L S, T blocks of (n/2^L)^2; 7^L M blocks -> n x n C.
hipError_t launch_strassen_preadd(int levels, int64_t n, const float* A, const float* B,
                                  float* S, float* T, hipStream_t s);
hipError_t launch_strassen_combine(int levels, int64_t n, const float* M, float* C,
                                   hipStream_t s);
// The same over nb dense n x n parents: parent y is A + y*xs (and B + y*xs),
// its 7^L blocks start at S + y*os (T + y*os); the combine writes parent y
// at C + y*cs with leading dimension ldc from M + y*ms.
hipError_t launch_strassen_preadd_batch(int levels, int64_t n, int nb, const float* A, const float* B,
                                        float* S, float* T, int64_t xs, int64_t os, hipStream_t s);
hipError_t launch_strassen_combine_batch(int levels, int64_t n, int nb, const float* M, float* C,
                                         int64_t ldc, int64_t ms, int64_t cs, hipStream_t s);

// Calibration: nwg workgroups of 256 threads each run `iters` rounds of four
// bf16 matrix-core products per wave; workgroup w writes its start and end
// (100 MHz real-time counter) to stamps[2w], stamps[2w+1].  `sink` (256
// floats) is never written in practice.
// 1D problem (section "PACO 1D"): weight parameters (b is the slope for
// affine weights, the mask for hashed ones) and one external-update piece
struct DpW {
  uint32_t a, b, seed, pad;
};
struct DpPiece {
  int64_t i0, i1, j0, j1;   // inputs [i0, i1) -> outputs [j0, j1)
  int32_t atomic, pad;      // 1: the inputs were cut, combine with an atomic minimum
};
constexpr int DP_TRI_MAX = 1024;   // longest base triangle (one workgroup, LDS)
// D[1..n] = INF, then the base triangle [0, tri_len); cnt: one zeroed
// counter (left zeroed)
hipError_t launch_dp1d_fill(int wk, uint32_t* D, int64_t n, uint32_t* cnt, int tri_len, const DpW& w,
                            hipStream_t s);
// one square's pieces, then the base triangle [tri_lo, tri_lo + tri_len),
// run after the first `ntri` pieces (those reaching into it) have finished
hipError_t launch_dp1d_rect(int wk, uint32_t* D, const DpPiece* pieces, int npieces, int ntri, uint32_t* cnt,
                            int64_t tri_lo, int tri_len, const DpW& w, hipStream_t s);

// GAP problem (section "PACO GAP"): a weight function (kind 0 affine with
// b the slope, kind 1 hashed with b the mask), the substitution cost, a base
// block and one cube piece
struct GapW {
  uint32_t kind, a, b, seed;
};
struct GapS {
  uint32_t match, mismatch, mask, seedx, seedy, pad;
};
struct GapBlock {
  int64_t r0, r1, c0, c1;   // rows [r0, r1) x columns [c0, c1)
};
struct GapPiece {
  int64_t t0, t1;   // batch: rows (row gaps) or columns (column gaps)
  int64_t x0, x1;   // inputs (columns q, or rows p)
  int64_t o0, o1;   // outputs (columns j, or rows i)
  int32_t col, pad; // 1: column-gap piece (inputs read from DT)
};
constexpr int GAP_B = 64;   // largest base block side
hipError_t launch_gap_fill(uint32_t* D, int64_t ld, int64_t rows, int64_t cols, hipStream_t s);
hipError_t launch_gap_base(uint32_t* D, int64_t ld, uint32_t* DT, int64_t ldt, const GapBlock* blocks, int nblocks,
                           const GapW& wr, const GapW& wc, const GapS& sub, hipStream_t s);
hipError_t launch_gap_cube(uint32_t* D, int64_t ld, const uint32_t* DT, int64_t ldt, const GapPiece* pieces,
                           int npieces, const GapW& wr, const GapW& wc, hipStream_t s);

hipError_t launch_calib(int nwg, int iters, uint64_t* stamps, float* sink, hipStream_t s);
hipError_t launch_peak_valu_i32(int nwg, int iters, uint32_t* sink, hipStream_t s);
hipError_t launch_peak_valu_f32(int nwg, int iters, float* sink, hipStream_t s);
hipError_t launch_peak_copy(const void* src, void* dst, int64_t bytes, int nwg, hipStream_t s);

}  // namespace paco
