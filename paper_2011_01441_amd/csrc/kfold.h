// kfold.h -- folding the temporary faces of k-cuts into C.
//
// Section "PACO MM": a cut on the height (k) of a cuboid gives the upper
// half a temporary face the size of the bottom face, and the halves are
// combined by (+) afterwards.  A reduction cell is a rectangle of one
// problem's C covered by the same ordered list of faces; its fold starts
// from the value the lowest-k piece wrote into C and applies the faces in
// ascending k, so a fixed partition gives bit-reproducible float results.
// The fold runs either in its own launch (one workgroup per cell tile) or,
// in a fused plan, inside the product kernel: every piece covering a cell
// counts itself in the cell's counter once its writes are visible, and the
// piece that completes the count folds the cell and resets the counter.
#pragma once
#include "kcommon.h"

namespace paco {

struct RSum {
  using T = float;
  static __device__ __forceinline__ T op(T a, T b) { return a + b; }
};
struct RMin {
  using T = uint32_t;
  static __device__ __forceinline__ T op(T a, T b) { return a < b ? a : b; }
};
struct RMax {
  using T = int32_t;
  static __device__ __forceinline__ T op(T a, T b) { return a > b ? a : b; }
};
struct ROr {
  using T = uint32_t;
  static __device__ __forceinline__ T op(T a, T b) { return a | b; }
};

template <class T, int VEC>
__device__ __forceinline__ void load_vec(const T* p, T x[VEC]) {
  if constexpr (VEC == 4) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 q = gload((const u32x4*)p);
    // copy each lane to a scalar before the bit cast (a bit cast applied to
    // a vector component expression reads component 0)
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const uint32_t w = q[e];
      x[e] = __builtin_bit_cast(T, w);
    }
  } else {
#pragma unroll
    for (int e = 0; e < VEC; ++e) x[e] = gload(p + e);
  }
}

// Fold the sources of one cell tile into C with NT threads: the tile's
// (row, VEC-column group) units are spread over the threads, sources read
// in batches of 8 so their loads are in flight together and folded strictly
// in list (ascending-k) order.
template <class R, int VEC, int NT>
__device__ __forceinline__ void fold_tile(const ProbRef& pr, const RedTile& tl, const RedSrc* __restrict__ srcs,
                                          const typename R::T* __restrict__ ws) {
  using T = typename R::T;
  const Problem P = uni(get_prob(pr, uni(tl.prob)));
  const int i0 = uni(tl.i0), i1 = uni(tl.i1), j0 = uni(tl.j0), j1 = uni(tl.j1);
  const int s0 = uni(tl.s0), s1 = uni(tl.s1);
  T* C = (T*)P.C;
  const int wv = (j1 - j0 + VEC - 1) / VEC;
  const int units = wv * (i1 - i0);
  for (int u = (int)threadIdx.x; u < units; u += NT) {
    const int i = i0 + u / wv, j = j0 + (u % wv) * VEC;
    T* cp = C + (int64_t)i * P.ldc + j;
    T v[VEC];
    load_vec<T, VEC>(cp, v);
    auto src_ptr = [&](int s) {
      const RedSrc S = srcs[s];
      return ws + S.off + (int64_t)(i - S.r0) * S.ld + (j - S.c0);
    };
    int s = s0;
    for (; s + 8 <= s1; s += 8) {
      T x[8][VEC];
#pragma unroll
      for (int q = 0; q < 8; ++q) load_vec<T, VEC>(src_ptr(s + q), x[q]);
#pragma unroll
      for (int q = 0; q < 8; ++q)
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[e] = R::op(v[e], x[q][e]);
    }
    for (; s < s1; ++s) {
      T x[VEC];
      load_vec<T, VEC>(src_ptr(s), x);
#pragma unroll
      for (int e = 0; e < VEC; ++e) v[e] = R::op(v[e], x[e]);
    }
#pragma unroll
    for (int e = 0; e < VEC; ++e) gstore(cp + e, v[e]);
  }
}

// Fused fold after work item `it` of a workgroup of NT threads: count the
// item in each reduction cell it covers; fold the cells it completes.  A
// plan without fused folding (pr.item_fold null) or an item covering no
// cell does nothing.  Every branch is uniform over the workgroup.
template <class R, int NT>
__device__ __forceinline__ void fold_after_item(const ProbRef& pr, int it, const typename R::T* __restrict__ ws) {
  if (!pr.item_fold) return;
  const int f0 = uni(pr.item_fold[2 * it]), fc = uni(pr.item_fold[2 * it + 1]);
  if (fc <= 0) return;
  __shared__ int s_last;
  // release: every wave waits until its writes of this item (C or its
  // face) have left it; after the barrier one device-scope fence (which
  // writes back this die's cache) publishes them before the item is counted
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) __threadfence();
  for (int q = 0; q < fc; ++q) {
    const int cell = uni(pr.fold_list[f0 + q]);
    if (threadIdx.x == 0) {
      const uint32_t total = (uint32_t)pr.fold_tiles[cell].pad;
      const uint32_t old = atomicAdd(pr.fold_cnt + cell, 1u);
      s_last = old + 1 == total;
      if (s_last) {
        atomicExch(pr.fold_cnt + cell, 0u);   // ready for the next call
        __threadfence();   // acquire: the other contributors' writes
      }
    }
    __syncthreads();
    if (s_last) {
      // the narrow fold: a wider one (every load of four units in flight)
      // measured 2 us faster a call but cost the 64 x 64 (min,+) kernel a
      // wave per SIMD (121 -> 130 registers), fused or not
      const RedTile tl = pr.fold_tiles[cell];
      if (pr.fold_vec == 4) fold_tile<R, 4, NT>(pr, tl, pr.fold_srcs, ws);
      else fold_tile<R, 1, NT>(pr, tl, pr.fold_srcs, ws);
    }
    __syncthreads();
  }
}

}  // namespace paco
