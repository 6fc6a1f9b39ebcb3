// strassen.cpp -- paco_strassen_mm: multi-level Strassen with all leaf
// products run as one PACO-partitioned batch.
//
// Section "PACO Strassen": all intermediate S, T and M matrices live in
// temporary space so every product of a depth can run concurrently; the
// 7^L leaf products of L levels are the nodes handed to processors.  Here
// the leaves form one batch that MM-1-Piece splits over the compute units:
// the leaf cuboids are stacked along n (they share no face), the stacked
// cuboid is partitioned, and a piece that crosses a leaf boundary becomes
// one work item per leaf on the same processor.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>

#include "../../include/paco.h"
#include "ctx.h"
#include "kernels.h"

using namespace paco;

namespace {

paco_status ensure_sws(paco_ctx ctx, uint64_t bytes) {
  if (bytes <= ctx->sws_bytes) return PACO_OK;
  if (bytes + ctx->ws_bytes > ctx->budget) {
    set_err(ctx, "Strassen temporaries exceed the workspace budget");
    return PACO_ERR_BUDGET;
  }
  hipError_t e;
  if (ctx->sws) {
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hip_fail(ctx, e, "workspace sync");
    (void)hipFree(ctx->sws);
    ctx->sws = nullptr;
    ctx->sws_bytes = 0;
  }
  if ((e = hipMalloc(&ctx->sws, bytes)) != hipSuccess) return hip_fail(ctx, e, "Strassen workspace alloc");
  ctx->sws_bytes = bytes;
  return PACO_OK;
}

}  // namespace

namespace paco {
void destroy_ctx_extras(paco_ctx ctx) {
  if (ctx->sws) (void)hipFree(ctx->sws);
  if (ctx->d_rows) (void)hipFree(ctx->d_rows);
  ctx->sws = nullptr;
  ctx->d_rows = nullptr;
}
}  // namespace paco

extern "C" paco_status paco_strassen_mm(paco_ctx ctx, int64_t n, const float* A, const float* B, float* C,
                                        int levels, paco_precision leaf) {
  if (!ctx) return PACO_ERR_INVALID_ARG;
  if (n < 0 || levels < 0 || levels > 3 || leaf < PACO_PREC_FP32 || leaf > PACO_PREC_AUTO) {
    set_err(ctx, "invalid Strassen arguments (levels in [0,3])");
    return PACO_ERR_INVALID_ARG;
  }
  if (n == 0) return PACO_OK;
  if (!A || !B || !C) {
    set_err(ctx, "null operand");
    return PACO_ERR_INVALID_ARG;
  }
  if (n % (1ll << levels) != 0) {
    set_err(ctx, "n must be divisible by 2^levels");
    return PACO_ERR_UNSUPPORTED;
  }
  if (levels == 0) {
    paco_mm_desc d;
    memset(&d, 0, sizeof d);
    d.n = d.m = d.k = n;
    d.sr = PACO_SR_PLUS_TIMES_F32;
    d.A = A; d.B = B; d.C = C;
    d.precision = leaf;
    d.part = PACO_PART_PACO;
    return paco_semiring_mm_ex(ctx, &d, nullptr);
  }
  const int64_t h = n >> levels;
  if (h >= (1ll << 22) || n >= (1ll << 31)) {
    set_err(ctx, "Strassen leaf dimension too large");
    return PACO_ERR_UNSUPPORTED;
  }
  int nleaf = 1;
  for (int l = 0; l < levels; ++l) nleaf *= 7;
  const int prec = leaf == PACO_PREC_AUTO ? (h >= 4096 ? PREC_BF16X3 : PREC_BF16X6) : (int)leaf;
  const int p = ctx->num_cus;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");

  char key[160];
  snprintf(key, sizeof key, "strassen/%lld/%d/%d/%d", (long long)n, levels, prec, p);
  DevPlan* dp = nullptr;
  auto itp = ctx->plans.find(key);
  if (itp != ctx->plans.end()) {
    dp = itp->second.get();
  } else {
    std::unique_ptr<DevPlan> np(new DevPlan());
    PartOpts po;
    po.p = p;
    po.q[0] = 16; po.q[1] = 16; po.q[2] = 32;
    po.kcut_cost = default_kcut_cost(PACO_SR_PLUS_TIMES_F32);
    std::vector<Piece> pcs = partition_mm1((int64_t)nleaf * h, h, h, po);
    std::vector<TaggedPiece> tp;
    std::vector<Piece> local;
    for (const Piece& pc : pcs) {
      if (pc.empty()) continue;
      for (int64_t r = pc.n0 / h; r * h < pc.n1; ++r) {
        Piece q = pc;
        q.n0 = std::max(pc.n0, r * h) - r * h;
        q.n1 = std::min(pc.n1, (r + 1) * h) - r * h;
        if (q.n1 <= q.n0) continue;
        tp.push_back({q, (int32_t)r, pc.proc});
        local.push_back(q);
      }
    }
    std::vector<ProbGeom> geom(nleaf, ProbGeom{h, h, h});
    np->h = build_plan(tp, p, true, geom);
    np->tile = choose_ring_tile(local, prec);
    np->fam = 2;
    np->p = p;
    paco_status st = upload_plan(ctx, np.get());
    if (st != PACO_OK) return st;
    dp = np.get();
    ctx->plans[key] = std::move(np);
  }

  const uint64_t blk = (uint64_t)h * h;
  paco_status st = ensure_sws(ctx, 3ull * nleaf * blk * 4);
  if (st != PACO_OK) return st;
  st = ensure_ws(ctx, (uint64_t)dp->h.temp_elems * 4);
  if (st != PACO_OK) return st;
  float* S = (float*)ctx->sws;
  float* T = S + nleaf * blk;
  float* M = T + nleaf * blk;

  {
    TimeScope ts(ctx, 2);
    e = launch_strassen_preadd(levels, n, A, B, S, T, ctx->stream);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "Strassen pre-add");
  ProbRef pr;
  memset(&pr, 0, sizeof pr);
  pr.base.A = S; pr.base.B = T; pr.base.C = M;
  pr.base.lda = pr.base.ldb = pr.base.ldc = h;
  pr.base.n = pr.base.m = pr.base.k = (int32_t)h;
  pr.sA = pr.sB = pr.sC = (int64_t)blk;
  pr.vec_ok = (h % 4 == 0) ? 1 : 0;   // S, T blocks start 16-byte aligned when h % 4 == 0
  {
    TimeScope ts(ctx, 0);
    e = launch_ring(prec, dp->tile, pr, dp->d_items, dp->d_wg_off, dp->h.nwg, dp->h.xcd_remap, ctx->ws,
                    ctx->stream);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "Strassen leaf launch");
  if (!dp->h.tiles.empty()) {
    {
      TimeScope ts(ctx, 1);
      e = launch_reduce(SR_RING, pr, dp->d_tiles, (int)dp->h.tiles.size(), dp->d_srcs, ctx->ws, ctx->stream,
                        dp->h.red_vec);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "Strassen leaf reduce");
  }
  {
    TimeScope ts(ctx, 2);
    e = launch_strassen_combine(levels, n, M, C, ctx->stream);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "Strassen combine");
  return PACO_OK;
}
