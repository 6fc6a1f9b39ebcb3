// graph.cpp -- a library call captured once into a hipGraph and replayed.
//
// A call first runs eagerly (its plan is built and uploaded, the workspace
// sized); the same call is then captured on a private stream, where it only
// launches kernels, and instantiated.  Each replay repeats exactly those
// launches on the operand buffers of the capture.
#include <hip/hip_runtime.h>

#include <cstring>

#include "../../include/paco.h"
#include "ctx.h"

using namespace paco;

struct paco_graph_s {
  paco_ctx ctx = nullptr;
  uint64_t ws_gen = 0;   // workspace generation the launches point into
  hipGraph_t g = nullptr;
  hipGraphExec_t ge = nullptr;
};

namespace {

template <class F>
paco_status capture(paco_ctx ctx, F call, int repeat, paco_graph* out) {
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  // eager run: plans, uploads and workspace growth happen here, not in the
  // capture (none of them may be recorded)
  paco_status st = call();
  if (st != PACO_OK) return st;
  if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hip_fail(ctx, e, "graph warm-up");
  hipStream_t cs = nullptr;
  if ((e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking)) != hipSuccess)
    return hip_fail(ctx, e, "capture stream");
  hipStream_t old = ctx->stream;
  const bool timing = ctx->timing;
  ctx->stream = cs;
  ctx->timing = false;
  hipGraph_t g = nullptr;
  e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    for (int r = 0; r < repeat && st == PACO_OK; ++r) st = call();
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e2 != hipSuccess && st == PACO_OK) {
      e = e2;
      st = PACO_ERR_HIP;
    }
  }
  ctx->stream = old;
  ctx->timing = timing;
  (void)hipStreamDestroy(cs);
  if (e != hipSuccess || st != PACO_OK) {
    if (g) (void)hipGraphDestroy(g);
    if (st == PACO_OK) st = hip_fail(ctx, e, "graph capture");
    return st;
  }
  hipGraphExec_t ge = nullptr;
  if ((e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0)) != hipSuccess) {
    (void)hipGraphDestroy(g);
    return hip_fail(ctx, e, "graph instantiate");
  }
  paco_graph_s* gr = new paco_graph_s;
  gr->ctx = ctx;
  gr->ws_gen = ctx->ws_gen;
  gr->g = g;
  gr->ge = ge;
  *out = gr;
  return PACO_OK;
}

}  // namespace

extern "C" paco_status paco_graph_create(paco_ctx ctx, const paco_mm_desc* d, int32_t repeat, paco_graph* out) {
  if (!ctx || !d || !out || repeat < 1 || repeat > 4096) return PACO_ERR_INVALID_ARG;
  *out = nullptr;
  if (d->verify_rows != 0) {
    set_err(ctx, "a captured call cannot verify (it synchronises)");
    return PACO_ERR_INVALID_ARG;
  }
  paco_mm_desc dc = *d;
  return capture(ctx, [&] { return paco_semiring_mm_ex(ctx, &dc, nullptr); }, repeat, out);
}

extern "C" paco_status paco_graph_create_strassen(paco_ctx ctx, const paco_strassen_desc* d, int32_t repeat,
                                                  paco_graph* out) {
  if (!ctx || !d || !out || repeat < 1 || repeat > 4096) return PACO_ERR_INVALID_ARG;
  *out = nullptr;
  paco_strassen_desc dc = *d;
  return capture(ctx, [&] { return paco_strassen_pbfs(ctx, &dc, nullptr); }, repeat, out);
}

extern "C" paco_status paco_graph_launch(paco_graph g, void* stream) {
  if (!g) return PACO_ERR_INVALID_ARG;
  if (g->ws_gen != g->ctx->ws_gen) {   // the workspace it points into was replaced
    set_err(g->ctx, "graph is stale: the context workspace or plans were replaced after capture");
    return PACO_ERR_INVALID_ARG;
  }
  hipError_t e = hipGraphLaunch(g->ge, stream ? (hipStream_t)stream : g->ctx->stream);
  return e == hipSuccess ? PACO_OK : hip_fail(g->ctx, e, "graph launch");
}

extern "C" paco_status paco_graph_destroy(paco_graph g) {
  if (!g) return PACO_ERR_INVALID_ARG;
  if (g->ge) (void)hipGraphExecDestroy(g->ge);
  if (g->g) (void)hipGraphDestroy(g->g);
  delete g;
  return PACO_OK;
}
