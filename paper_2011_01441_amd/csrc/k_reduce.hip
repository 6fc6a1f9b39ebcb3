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

template <class R>
__global__ __launch_bounds__(256) void k_reduce(ProbRef pr, const RedTile* __restrict__ tiles,
                                                const RedSrc* __restrict__ srcs,
                                                const typename R::T* __restrict__ ws) {
  using T = typename R::T;
  const RedTile tl = tiles[blockIdx.x];
  const Problem P = uni(get_prob(pr, uni(tl.prob)));
  const int i0 = uni(tl.i0), j0 = uni(tl.j0);
  const int w = uni(tl.j1) - j0, h = uni(tl.i1) - i0;
  const int s0 = uni(tl.s0), s1 = uni(tl.s1);
  T* C = (T*)P.C;
  for (int e = threadIdx.x; e < w * h; e += 256) {
    const int i = i0 + e / w, j = j0 + e % w;
    T* cp = C + (int64_t)i * P.ldc + j;
    T v = gload(cp);
    for (int s = s0; s < s1; ++s) {
      const RedSrc S = srcs[s];
      v = R::op(v, gload(ws + S.off + (int64_t)(i - S.r0) * S.ld + (j - S.c0)));
    }
    gstore(cp, v);
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
                         const RedSrc* srcs, const void* ws, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  dim3 g(ntiles), b(256);
  switch (sr) {
    case SR_RING: hipLaunchKernelGGL(k_reduce<RSum>, g, b, 0, s, pr, tiles, srcs, (const float*)ws); break;
    case SR_MINPLUS: hipLaunchKernelGGL(k_reduce<RMin>, g, b, 0, s, pr, tiles, srcs, (const uint32_t*)ws); break;
    case SR_MAXPLUS: hipLaunchKernelGGL(k_reduce<RMax>, g, b, 0, s, pr, tiles, srcs, (const int32_t*)ws); break;
    case SR_BOOL: hipLaunchKernelGGL(k_reduce<ROr>, g, b, 0, s, pr, tiles, srcs, (const uint32_t*)ws); break;
    default: return hipErrorInvalidValue;
  }
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
