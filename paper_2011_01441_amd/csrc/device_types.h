// device_types.h -- descriptors shared by the host planner and the kernels.
//
// A piece of the n-by-m-by-k iteration cuboid (section "PACO MM", cuboid
// view) becomes one or more WorkItems; a workgroup runs the items of the
// processor it stands for.  Pieces whose k-range does not start at 0 write
// a temporary face (the upper cuboid of a cut on height), which a reduction
// pass folds into C in ascending-k order.
#pragma once
#include <stdint.h>

namespace paco {

enum Semiring : int32_t { SR_RING = 0, SR_MINPLUS = 1, SR_MAXPLUS = 2, SR_BOOL = 3 };
enum Prec : int32_t { PREC_FP32 = 0, PREC_BF16X3 = 1, PREC_BF16X6 = 2 };

constexpr int32_t kMinPlusInf = 1 << 30;        // (min,+) zero
constexpr int32_t kMaxPlusNegInf = -(1 << 30);  // (max,+) zero
// Every (max,+) sum with a NEG_INF factor is below this; every finite sum of
// two entries of the finite domain [-2^28, 2^28] is at or above it.
constexpr int32_t kMaxPlusThreshold = -(1 << 29);

// One multiplication C = A (x) B.  Boolean matrices count words in m, k for
// their leading dimensions only; n, m, k are always logical (bit) sizes.
struct Problem {
  const void* A;
  const void* B;
  void* C;
  int64_t lda, ldb, ldc;
  int32_t n, m, k;
  int32_t accumulate;
};

// Problems of one launch: an explicit device table, or `count` problems laid
// out at fixed element strides from `base` (batched Strassen leaves).
struct ProbRef {
  const Problem* table;
  Problem base;
  int64_t sA, sB, sC;  // element strides between consecutive problems
  int32_t vec_ok;      // set by the host: every problem's A and B rows are
                       // 16-byte aligned with lengths multiple of 4, and
                       // for the integer kernel every work item starts on
                       // a multiple of 4 in k and m (128-bit loads)
  int32_t stamp_cap;   // processors with a slot in `stamps`
  uint64_t* stamps;    // null, or 4 words per processor: start and end of
                       // its work on the device's 100 MHz clock, its XCC_ID
                       // and HW_ID hardware registers
  // Fused folding of temporary faces (null item_fold: a separate launch
  // folds them): item i covers the reduction cells fold_list[item_fold[2i]
  // .. + item_fold[2i+1]); cell c is fold_tiles[c] (its pad holds the
  // number of pieces covering it) with sources in fold_srcs; fold_cnt
  // holds one counter per cell, zero between calls.
  const int32_t* item_fold;
  const int32_t* fold_list;
  const struct RedTile* fold_tiles;
  const struct RedSrc* fold_srcs;
  uint32_t* fold_cnt;
  int32_t fold_vec;    // 4: cells and faces allow 128-bit access
  int32_t fold_pad;
};

// A sub-cuboid [n0,n1) x [m0,m1) x [k0,k1) of problem `prob`.  out_off < 0:
// write C directly; otherwise write a dense temporary face of (n1-n0) rows
// and (m1-m0) columns (words for boolean) at element offset out_off of the
// workspace.
struct WorkItem {
  int32_t prob;
  int32_t n0, n1, m0, m1, k0, k1;
  int32_t pad;
  int64_t out_off;
};

// Reduction: rectangle [i0,i1) x [j0,j1) of problem `prob`'s C gets the
// sources src[s0..s1) folded in, in that (ascending-k) order.
struct RedTile {
  int32_t prob;
  int32_t i0, i1, j0, j1;
  int32_t s0, s1;
  int32_t pad;
};

// A temporary face: element (i, j) of C's coordinates lives at
// ws[off + (i - r0) * ld + (j - c0)].
struct RedSrc {
  int64_t off;
  int32_t ld, r0, c0, pad;
};

}  // namespace paco
