// tune.cpp -- paco_tune: measured choice of partition mode, processor count,
// k-cut cost and kernel tile for one shape.
//
// The default plan comes from a cost model; the tuner times it and its
// alternatives on the caller's operands and keeps the fastest for the shape
// in the context, where later default calls of that shape pick it up.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/paco.h"
#include "ctx.h"
#include "kernels.h"

using namespace paco;

namespace {

struct Cand {
  int part, p, tile;
  double kc;
  bool weighted;
};

// Average milliseconds of the call over a few repetitions after one
// untimed call (which builds and uploads its plan); < 0 on failure.
template <class F>
double time_call(paco_ctx ctx, F call) {
  if (call() != PACO_OK) return -1;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return -1;
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return -1;
  }
  double ms = -1;
  int reps = 1;
  for (int round = 0; round < 2; ++round) {
    (void)hipEventRecord(a, ctx->stream);
    bool ok = true;
    for (int r = 0; r < reps && ok; ++r) ok = call() == PACO_OK;
    (void)hipEventRecord(b, ctx->stream);
    float t = 0;
    if (!ok || hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&t, a, b) != hipSuccess) {
      ms = -1;
      break;
    }
    ms = t / reps;
    // second round: enough repetitions for about 3 ms, 2 to 10 of them
    reps = std::min(10, std::max(2, (int)std::ceil(3.0 / std::max(ms, 1e-3))));
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return ms;
}

}  // namespace

extern "C" paco_status paco_tune(paco_ctx ctx, const paco_mm_desc* d, paco_tune_result* out) {
  if (!ctx || !d) return PACO_ERR_INVALID_ARG;
  if (d->part != PACO_PART_PACO || d->p != 0 || d->kcut_cost != 0 || d->weights || d->verify_rows != 0 ||
      d->accumulate) {
    set_err(ctx, "tune: give a default PACO call (p, kcut_cost, weights, verify_rows, accumulate all 0)");
    return PACO_ERR_INVALID_ARG;
  }
  if (d->n <= 0 || d->m <= 0 || d->k <= 0) {
    set_err(ctx, "tune: empty shape");
    return PACO_ERR_INVALID_ARG;
  }
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  const bool ring = d->sr == PACO_SR_PLUS_TIMES_F32;
  const int prec = ring ? (d->precision == PACO_PREC_AUTO ? auto_precision(d->k) : (int)d->precision) : -1;
  const std::string key = tune_key(d, prec);
  ctx->tuned.erase(key);
  const double t_def = time_call(ctx, [&] { return run_mm(ctx, d, nullptr, -1); });
  if (t_def < 0) {
    if (ctx->last_error.empty()) set_err(ctx, "tune: the default call failed");
    return PACO_ERR_INTERNAL;
  }

  std::vector<Cand> cands;
  const int C = ctx->num_cus;
  if (ring) {
    const bool wts = (int)ctx->weights.size() == C;
    const int tiles[4] = {RING_T256x256, RING_T256x128, RING_T128x128, RING_T128x64};
    for (int part : {(int)PACO_PART_PACO, (int)PACO_PART_MULTI})
      for (double kc : {1.0, 4.0, 16.0, 64.0})
        for (int t : tiles) {
          if (t == RING_T256x256 && prec == PREC_BF16X6) continue;
          cands.push_back({part, C, t, kc, wts && part == PACO_PART_PACO});
        }
  } else {
    const bool is_bool = d->sr == PACO_SR_OR_AND_B1;
    for (int t = 0; t < (is_bool ? 4 : kIntTiles); ++t) {
      int occ = is_bool ? bool_occupancy(t) : int_occupancy((int)d->sr, t);
      occ = std::min(std::max(occ, 1), 8);
      for (int f : {1, 2, 4, 8, 16})
        for (double kc : {1.0, 16.0, 64.0})
          if (C * occ * f <= 65536) cands.push_back({(int)PACO_PART_PACO, C * occ * f, t, kc, false});
    }
  }
  Cand best{-1, 0, -1, 0.0, false};
  double t_best = t_def;
  int tried = 0;
  for (const Cand& c : cands) {
    paco_mm_desc dc = *d;
    dc.part = (paco_part_mode)c.part;
    dc.p = c.p;
    dc.kcut_cost = c.kc;
    dc.weights = c.weighted ? ctx->weights.data() : nullptr;
    const double t = time_call(ctx, [&] { return run_mm(ctx, &dc, nullptr, c.tile); });
    if (t < 0) continue;   // e.g. a plan whose temporary faces exceed the budget
    ++tried;
    if (t < t_best) {
      t_best = t;
      best = c;
    }
  }
  ctx->last_error.clear();
  if (best.part >= 0) {
    paco_ctx_s::Tuned tu;
    tu.part = best.part;
    tu.p = best.p;
    tu.tile = best.tile;
    tu.kcut = best.kc;
    tu.weighted = best.weighted;
    ctx->tuned[key] = tu;
  }
  if (out) {
    memset(out, 0, sizeof *out);
    out->tuned = best.part >= 0 ? 1 : 0;
    out->part = (paco_part_mode)(best.part >= 0 ? best.part : PACO_PART_PACO);
    out->p = best.p;
    out->tile = best.tile;
    out->kcut_cost = best.kc;
    out->weighted = best.weighted ? 1 : 0;
    out->best_ms = t_best;
    out->default_ms = t_def;
    out->candidates = tried;
  }
  return PACO_OK;
}

extern "C" paco_status paco_tune_clear(paco_ctx ctx) {
  if (!ctx) return PACO_ERR_INVALID_ARG;
  ctx->tuned.clear();
  return PACO_OK;
}
