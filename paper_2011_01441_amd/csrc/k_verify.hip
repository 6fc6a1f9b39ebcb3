// k_verify.hip -- float64 recomputation of sampled rows of a float32 ring
// product, for the error report attached to a result.
//
// For each sampled row i and column j: C64 = sum_l A[i][l] B[l][j] and
// S = sum_l |A[i][l] B[l][j]| in float64 (exact products of float32 values),
// then per-block partial maxima of |C - C64| / S and |C - C64| and sums of
// (C - C64)^2 and C64^2.  A NaN or infinite entry of C counts as an
// infinite error.  A block covers 8 sampled rows x 256 columns so B
// is streamed once per 8 rows.
#include <cfloat>

#include "kcommon.h"
#include "kernels.h"

namespace paco {
namespace {

constexpr int kRows = 8;

__global__ __launch_bounds__(256) void k_verify(int64_t m, int64_t k, const float* __restrict__ A, int64_t lda,
                                                const float* __restrict__ B, int64_t ldb,
                                                const float* __restrict__ C, int64_t ldc,
                                                const int64_t* __restrict__ rows, int64_t nrows,
                                                double* __restrict__ part) {
  const int64_t r0 = (int64_t)blockIdx.y * kRows;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  int64_t ri[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) ri[r] = (r0 + r < nrows) ? rows[r0 + r] : -1;
  double acc[kRows], sab[kRows];
#pragma unroll
  for (int r = 0; r < kRows; ++r) acc[r] = sab[r] = 0.0;
  if (j < m) {
    for (int64_t l = 0; l < k; ++l) {
      const double b = (double)B[l * ldb + j];
#pragma unroll
      for (int r = 0; r < kRows; ++r) {
        if (ri[r] < 0) continue;
        const double p = (double)A[ri[r] * lda + l] * b;
        acc[r] += p;
        sab[r] += fabs(p);
      }
    }
  }
  double mrel = 0.0, mabs = 0.0, sd = 0.0, sr = 0.0;
  if (j < m) {
#pragma unroll
    for (int r = 0; r < kRows; ++r) {
      if (ri[r] < 0) continue;
      // a non-finite result (NaN or infinity in C) is an infinite error:
      // fmax below would otherwise drop a NaN
      double d = fabs((double)C[ri[r] * ldc + j] - acc[r]);
      if (!(d <= DBL_MAX)) d = INFINITY;
      if (sab[r] > 0.0) mrel = fmax(mrel, d / sab[r]);
      else if (d > 0.0) mrel = INFINITY;
      mabs = fmax(mabs, d);
      sd += d * d;
      sr += acc[r] * acc[r];
    }
  }
  __shared__ double red[4][256];
  red[0][threadIdx.x] = mrel;
  red[1][threadIdx.x] = mabs;
  red[2][threadIdx.x] = sd;
  red[3][threadIdx.x] = sr;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + w]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w]);
      red[2][threadIdx.x] += red[2][threadIdx.x + w];
      red[3][threadIdx.x] += red[3][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double* o = part + 4 * ((int64_t)blockIdx.y * gridDim.x + blockIdx.x);
    o[0] = red[0][0]; o[1] = red[1][0]; o[2] = red[2][0]; o[3] = red[3][0];
  }
}

}  // namespace

int64_t verify_blocks(int64_t m, int64_t nrows) {
  return ((m + 255) / 256) * ((nrows + kRows - 1) / kRows);
}

hipError_t launch_verify_f64(int64_t n, int64_t m, int64_t k, const float* A, int64_t lda, const float* B,
                             int64_t ldb, const float* C, int64_t ldc, const int64_t* rows, int64_t nrows,
                             double* part, hipStream_t s) {
  (void)n;
  if (nrows <= 0 || m <= 0) return hipSuccess;
  dim3 g((unsigned)((m + 255) / 256), (unsigned)((nrows + kRows - 1) / kRows));
  hipLaunchKernelGGL(k_verify, g, dim3(256), 0, s, m, k, A, lda, B, ldb, C, ldc, rows, nrows, part);
  return hipGetLastError();
}

}  // namespace paco
