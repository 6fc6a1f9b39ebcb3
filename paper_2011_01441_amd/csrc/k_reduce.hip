// k_reduce.hip -- fold the temporary faces of k-cuts into C, and the k = 0 fill.
//
// Section "PACO MM": a cut on the height (k) of a cuboid gives the upper
// half a temporary face the size of the bottom face; the halves are then
// combined by a fully parallel (+) of the faces.  Here every output element
// folds all temporary faces that cover it in ascending-k order onto the
// value the lowest-k piece already wrote into C, so a fixed partition gives
// bit-reproducible float results.  One workgroup per rectangle tile; threads
// walk the tile row-major, so each source read is coalesced.  (Plans with
// small cells fold inside the product kernel instead: kfold.h.)
#include "kcommon.h"
#include "kernels.h"
#include "kfold.h"

namespace paco {
namespace {

// One workgroup per cell tile.
template <class R, int VEC>
__global__ __launch_bounds__(256) void k_reduce(ProbRef pr, const RedTile* __restrict__ tiles,
                                                const RedSrc* __restrict__ srcs,
                                                const typename R::T* __restrict__ ws) {
  fold_tile<R, VEC, 256>(pr, tiles[blockIdx.x], srcs, ws);
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
