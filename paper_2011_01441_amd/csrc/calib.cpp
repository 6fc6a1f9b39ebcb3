// calib.cpp -- paco_calibrate: measured processor throughputs for the
// heterogeneous split.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/paco.h"
#include "ctx.h"
#include "kernels.h"

using namespace paco;

extern "C" paco_status paco_calibrate(paco_ctx ctx, int32_t p, int32_t iters, double* rates) {
  if (!ctx) return PACO_ERR_INVALID_ARG;
  if (p <= 0 || p % 8 != 0 || p > 8 * ctx->num_cus || iters < 0 || !rates) {
    set_err(ctx, "calibrate: p must be a positive multiple of 8 (at most 8 x compute units), rates non-null");
    return PACO_ERR_INVALID_ARG;
  }
  // about 50 ms at 1.7 GHz: 128 cycles per round of four products
  const int it = iters > 0 ? iters : 650000;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  uint64_t* d_st = nullptr;
  float* d_sink = nullptr;
  if ((e = hipMalloc(&d_st, sizeof(uint64_t) * 2 * p)) != hipSuccess) return hip_fail(ctx, e, "calibrate alloc");
  if ((e = hipMalloc(&d_sink, sizeof(float) * 256)) != hipSuccess) {
    (void)hipFree(d_st);
    return hip_fail(ctx, e, "calibrate alloc");
  }
  std::vector<uint64_t> st(2 * p);
  // untimed run first: clocks and power settle under the same load
  e = launch_calib(p, it, d_st, d_sink, ctx->stream);
  if (e == hipSuccess) e = launch_calib(p, it, d_st, d_sink, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  if (e == hipSuccess) e = hipMemcpy(st.data(), d_st, sizeof(uint64_t) * 2 * p, hipMemcpyDeviceToHost);
  (void)hipFree(d_st);
  (void)hipFree(d_sink);
  if (e != hipSuccess) return hip_fail(ctx, e, "calibrate run");
  // workgroup w runs on XCD w % 8 and stands for processor
  // (w % 8) * (p / 8) + w / 8; a processor's rate is its XCD's mean
  const double flops = (double)it * 4 * 4 * 2.0 * 32 * 32 * 16;   // waves x products x flops
  double sum[8] = {0}, cnt[8] = {0};
  for (int w = 0; w < p; ++w) {
    const double sec = (double)(st[2 * w + 1] - st[2 * w]) / 100e6;
    if (!(sec > 0)) {
      set_err(ctx, "calibrate: non-positive duration");
      return PACO_ERR_INTERNAL;
    }
    sum[w % 8] += flops / sec;
    cnt[w % 8] += 1;
  }
  const int per = p / 8;
  for (int q = 0; q < p; ++q) rates[q] = sum[q / per] / cnt[q / per] / 1e12;
  return PACO_OK;
}

extern "C" paco_status paco_set_processor_weights(paco_ctx ctx, int32_t p, const double* weights) {
  if (!ctx) return PACO_ERR_INVALID_ARG;
  if (p == 0 || !weights) {
    ctx->weights.clear();
    return PACO_OK;
  }
  if (p != ctx->num_cus) {
    set_err(ctx, "processor weights: p must equal the compute units");
    return PACO_ERR_INVALID_ARG;
  }
  for (int i = 0; i < p; ++i)
    if (!(weights[i] > 0) || !std::isfinite(weights[i])) {
      set_err(ctx, "processor weights must be positive and finite");
      return PACO_ERR_INVALID_ARG;
    }
  ctx->weights.assign(weights, weights + p);
  return PACO_OK;
}
