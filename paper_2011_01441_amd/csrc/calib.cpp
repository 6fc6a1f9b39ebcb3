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

namespace {

// runs `launch` twice (the first untimed) and returns the seconds of the
// second run between events on the context stream
template <class F>
hipError_t time_twice(paco_ctx ctx, F launch, double* sec) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e0, ctx->stream);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(e1, ctx->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  *sec = ms * 1e-3;
  return e;
}

}  // namespace

extern "C" paco_status paco_peak(paco_ctx ctx, paco_peak_kind kind, double* rate) {
  if (!ctx || !rate) return PACO_ERR_INVALID_ARG;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  const int nwg = 4 * ctx->num_cus;   // four workgroups (16 waves) per compute unit
  double sec = 0, work = 0;
  void* buf = nullptr;
  switch (kind) {
    case PACO_PEAK_MFMA_BF16: {
      const int it = 100000;
      if ((e = hipMalloc(&buf, sizeof(uint64_t) * 2 * nwg + 1024)) != hipSuccess) break;
      uint64_t* st = (uint64_t*)buf;
      float* sink = (float*)(st + 2 * nwg);
      e = time_twice(ctx, [&] { return launch_calib(nwg, it, st, sink, ctx->stream); }, &sec);
      work = (double)nwg * it * 4 * 4 * 2.0 * 32 * 32 * 16;   // flops
      break;
    }
    case PACO_PEAK_VALU_I32: {
      const int it = 100000;
      if ((e = hipMalloc(&buf, 1024)) != hipSuccess) break;
      e = time_twice(ctx, [&] { return launch_peak_valu_i32(nwg, it, (uint32_t*)buf, ctx->stream); }, &sec);
      work = (double)nwg * 256 * it * 8 * 2;   // lane-instructions
      break;
    }
    case PACO_PEAK_VALU_F32: {
      const int it = 100000;
      if ((e = hipMalloc(&buf, 1024)) != hipSuccess) break;
      e = time_twice(ctx, [&] { return launch_peak_valu_f32(nwg, it, (float*)buf, ctx->stream); }, &sec);
      work = (double)nwg * 256 * it * 8 * 2;   // flops (one FMA = 2)
      break;
    }
    case PACO_PEAK_HBM_COPY: {
      const int cwg = 4 * ctx->num_cus;
      const int64_t bytes = (int64_t)1 << 30;
      if ((e = hipMalloc(&buf, 2 * bytes)) != hipSuccess) break;
      char* src = (char*)buf;
      char* dst = src + bytes;
      if ((e = hipMemsetAsync(src, 1, bytes, ctx->stream)) != hipSuccess) break;
      e = time_twice(ctx, [&] { return launch_peak_copy(src, dst, bytes, cwg, ctx->stream); }, &sec);
      work = 2.0 * bytes;   // bytes read + written
      break;
    }
    default:
      set_err(ctx, "peak: unknown kind");
      return PACO_ERR_INVALID_ARG;
  }
  if (buf) (void)hipFree(buf);
  if (e != hipSuccess) return hip_fail(ctx, e, "peak probe");
  if (!(sec > 0)) {
    set_err(ctx, "peak: non-positive duration");
    return PACO_ERR_INTERNAL;
  }
  *rate = work / sec / (kind == PACO_PEAK_HBM_COPY ? 1e9 : 1e12);
  return PACO_OK;
}

