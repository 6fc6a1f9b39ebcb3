// k_reduce.hip -- fold the temporary faces of k-cuts into C, and the k = 0 fill.
//
// Section "PACO MM": a cut on the height (k) of a cuboid gives the upper
// half a temporary face the size of the bottom face; the halves are then
// combined by a fully parallel (+) of the faces.  Here every output element
// folds all temporary faces that cover it in ascending-k order onto the
// value the lowest-k piece already wrote into C, so a fixed partition gives
// bit-reproducible float results.  One workgroup per rectangle tile; threads
// walk the tile row-major, so each source read is coalesced.
#include "kcommon.h"
#include "kernels.h"

namespace paco {
namespace {

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

// One workgroup per tile; the tile's (row, VEC columns) units are spread
// over the threads.  Sources are read in batches of 8 so their loads are in
// flight together, and folded strictly in list (ascending-k) order.
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

template <class R, int VEC>
__global__ __launch_bounds__(256) void k_reduce(ProbRef pr, const RedTile* __restrict__ tiles,
                                                const RedSrc* __restrict__ srcs,
                                                const typename R::T* __restrict__ ws) {
  using T = typename R::T;
  const RedTile tl = tiles[blockIdx.x];
  const Problem P = uni(get_prob(pr, uni(tl.prob)));
  const int i0 = uni(tl.i0), i1 = uni(tl.i1), j1 = uni(tl.j1);
  const int s0 = uni(tl.s0), s1 = uni(tl.s1);
  T* C = (T*)P.C;
  // work unit = (row, VEC-column group) of the tile; 256 units in flight
  const int j0 = uni(tl.j0);
  const int wv = (j1 - j0 + VEC - 1) / VEC;
  const int units = wv * (i1 - i0);
  for (int u = (int)threadIdx.x; u < units; u += 256) {
    const int i = i0 + u / wv, j = j0 + (u % wv) * VEC;
    T* cp = C + (int64_t)i * P.ldc + j;
    T v[VEC];
    load_vec<T, VEC>(cp, v);
    auto src_ptr = [&](int s) {
      const RedSrc S = srcs[s];
      return ws + S.off + (int64_t)(i - S.r0) * S.ld + (j - S.c0);
    };
    int s = s0;
    for (; s + 8 <= s1; s += 8) {  // eight loads in flight, folded in order
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

template <class T>
__global__ __launch_bounds__(256) void k_fill(T* C, int64_t rows, int64_t cols, int64_t ldc, T v) {
  int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256)
    C[(e / cols) * ldc + e % cols] = v;
}

}  // namespace

hipError_t launch_reduce(int sr, const ProbRef& pr, const RedTile* tiles, int ntiles,
                         const RedSrc* srcs, const void* ws, hipStream_t s, int vec) {
  if (ntiles <= 0) return hipSuccess;
  dim3 g(ntiles), b(256);
#define PACO_RED(R, T)                                                                   \
  if (vec == 4) hipLaunchKernelGGL((k_reduce<R, 4>), g, b, 0, s, pr, tiles, srcs, (const T*)ws); \
  else hipLaunchKernelGGL((k_reduce<R, 1>), g, b, 0, s, pr, tiles, srcs, (const T*)ws);
  switch (sr) {
    case SR_RING: PACO_RED(RSum, float); break;
    case SR_MINPLUS: PACO_RED(RMin, uint32_t); break;
    case SR_MAXPLUS: PACO_RED(RMax, int32_t); break;
    case SR_BOOL: PACO_RED(ROr, uint32_t); break;
    default: return hipErrorInvalidValue;
  }
#undef PACO_RED
  return hipGetLastError();
}

hipError_t launch_fill_zero(int sr, void* C, int64_t rows, int64_t cols, int64_t ldc, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  int64_t total = rows * cols;
  int blocks = (int)std::min<int64_t>((total + 255) / 256, 4096);
  uint32_t v = 0;
  if (sr == SR_MINPLUS) v = (uint32_t)kMinPlusInf;
  else if (sr == SR_MAXPLUS) v = (uint32_t)kMaxPlusNegInf;
  hipLaunchKernelGGL(k_fill<uint32_t>, dim3(blocks), dim3(256), 0, s, (uint32_t*)C, rows, cols, ldc, v);
  return hipGetLastError();
}

}  // namespace paco
