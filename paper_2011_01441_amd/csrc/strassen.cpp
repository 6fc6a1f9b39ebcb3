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
#include <array>
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
  ctx->ws_gen += 1;
  if ((e = hipMalloc(&ctx->sws, bytes)) != hipSuccess) return hip_fail(ctx, e, "Strassen workspace alloc");
  ctx->sws_bytes = bytes;
  return PACO_OK;
}

}  // namespace

namespace paco {
void destroy_ctx_extras(paco_ctx ctx) {
  if (ctx->gws) (void)hipFree(ctx->gws);
  ctx->gws = nullptr;
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
    trim_plans(ctx);
    std::unique_ptr<DevPlan> np(new DevPlan());
    // Two schedules of the 7^L leaf products.  Sequenced: one leaf split
    // over all p processors (MM-1-Piece on the tile grid), processor q
    // running its piece of every leaf, leaf after leaf, so all processors
    // work on the same leaf at a time and its S and T blocks stay in the
    // last-level cache.  Stacked: the leaves concatenated along n and split
    // as one product, pieces straddling leaves; each piece then streams its
    // own leaves' T blocks, and every row tile re-reads its column panel.
    // Sequenced is taken unless its busiest processor has over 2% more
    // padded work than the stacked one's.
    const double kc = default_kcut_cost(PACO_SR_PLUS_TIMES_F32);
    auto crit = [&](const std::vector<Piece>& v, int t, double mult) {
      const RingTileShape ts = ring_tile_shape(t, prec);
      std::vector<double> load(p, 0.0);
      double worst = 0;
      for (const Piece& pc : v) {
        if (pc.empty()) continue;
        load[pc.proc] += mult * (double)((pc.n1 - pc.n0 + ts.tm - 1) / ts.tm) *
                         (double)((pc.m1 - pc.m0 + ts.tn - 1) / ts.tn) * ts.tm * ts.tn *
                         (double)((pc.k1 - pc.k0 + ts.bk - 1) / ts.bk * ts.bk + 64);
        worst = std::max(worst, load[pc.proc]);
      }
      return worst;
    };
    int tile_seq = -1, tile_stk = -1;
    std::vector<Piece> one = ring_partition(h, h, h, p, prec, kc, nullptr, -1, &tile_seq);
    std::vector<Piece> pcs = ring_partition((int64_t)nleaf * h, h, h, p, prec, kc, nullptr, -1, &tile_stk);
    std::vector<TaggedPiece> tp;
    int tile = tile_stk;
    if (crit(one, tile_seq, (double)nleaf) <= 1.02 * crit(pcs, tile_stk, 1.0)) {
      tile = tile_seq;
      for (int r = 0; r < nleaf; ++r)
        for (const Piece& pc : one)
          if (!pc.empty()) tp.push_back({pc, (int32_t)r, pc.proc});
    } else {
      for (const Piece& pc : pcs) {
        if (pc.empty()) continue;
        for (int64_t r = pc.n0 / h; r * h < pc.n1; ++r) {
          Piece q = pc;
          q.n0 = std::max(pc.n0, r * h) - r * h;
          q.n1 = std::min(pc.n1, (r + 1) * h) - r * h;
          if (q.n1 <= q.n0) continue;
          tp.push_back({q, (int32_t)r, pc.proc});
        }
      }
    }
    std::vector<ProbGeom> geom(nleaf, ProbGeom{h, h, h});
    np->h = build_plan(tp, p, true, geom);
    np->tile = tile;
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
  pr.stamps = ctx->stamps;
  pr.stamp_cap = ctx->stamps ? ctx->stamp_cap : 0;
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

// ------------------------------------------------------------------------
// Pruned-BFS PACO Strassen (paco_strassen_pbfs).

#include <cmath>

#include "strassen_sched.h"

namespace {

// Plan of one (n, p, gamma, base, precision): the schedule, where each
// depth's S, T and M live in the Strassen workspace, and the leaf launch.
struct SPlan : paco::DevPlan {
  paco::SSchedule sched;
  int fused = 0;                      // depths 1..fused come from one fused pre-add
  int first = 0;                      // first depth that hands out nodes
  std::vector<int64_t> s_off, t_off, m_off;   // per depth, in floats (depth >= fused)
  int64_t total = 0;                  // floats of S, T, M
  std::vector<std::array<int64_t, 4>> prob;   // (depth, node, h, unused) per leaf problem
  paco::Problem* d_probs = nullptr;
  const void* probs_base = nullptr;   // workspace address d_probs points into
  int prec = 0;
  ~SPlan() override {
    if (d_probs) (void)hipFree(d_probs);
  }
};

paco_status strassen_args(paco_ctx ctx, const paco_strassen_desc* d, int* p, int64_t* base) {
  if (!d || d->n < 0 || d->gamma < 0 || d->base < 0 || d->p < 0 || d->leaf < PACO_PREC_FP32 ||
      d->leaf > PACO_PREC_AUTO) {
    set_err(ctx, "invalid Strassen descriptor");
    return PACO_ERR_INVALID_ARG;
  }
  if (d->n >= (1ll << 31)) {
    set_err(ctx, "Strassen dimension too large");
    return PACO_ERR_UNSUPPORTED;
  }
  *p = d->p > 0 ? d->p : std::max(1, ctx->num_cus / 32);
  if (*p > ctx->num_cus) {
    set_err(ctx, "Strassen processors exceed the compute units");
    return PACO_ERR_INVALID_ARG;
  }
  *base = d->base > 0 ? d->base : 256;
  return PACO_OK;
}

}  // namespace

extern "C" paco_status paco_strassen_schedule(int64_t n, int32_t p, int32_t gamma, int64_t base,
                                              paco_strassen_level* levels, int32_t cap, int32_t* n_levels,
                                              double* work_classic, double* work_strassen) {
  if (n < 1 || n >= (1ll << 31) || p < 1 || p > 65536 || gamma < 0 || base < 1 || !n_levels || cap < 0 ||
      (cap > 0 && !levels))
    return PACO_ERR_INVALID_ARG;
  SSchedule s = strassen_schedule(n, p, gamma, base);
  *n_levels = (int32_t)s.levels.size();
  for (int32_t i = 0; i < cap && i < (int32_t)s.levels.size(); ++i) {
    const SLevel& lv = s.levels[i];
    levels[i].depth = lv.depth;
    levels[i].super_round = lv.super_round ? 1 : 0;
    levels[i].h = lv.h;
    levels[i].nodes = lv.nodes;
    levels[i].assigned = lv.assigned;
  }
  const double omega = std::log2(7.0);
  for (int j = 0; j < p; ++j) {
    double wc = 0, ws = 0;
    for (const auto& dn : s.per_proc[j]) {
      const double h = (double)s.levels[dn.first].h;
      wc += h * h * h;
      ws += std::pow(h, omega);
    }
    if (work_classic) work_classic[j] = wc;
    if (work_strassen) work_strassen[j] = ws;
  }
  return PACO_OK;
}

extern "C" paco_status paco_strassen_pbfs(paco_ctx ctx, const paco_strassen_desc* d, paco_strassen_result* out) {
  if (!ctx) return PACO_ERR_INVALID_ARG;
  int p;
  int64_t base;
  paco_status st = strassen_args(ctx, d, &p, &base);
  if (st != PACO_OK) return st;
  const int64_t n = d->n;
  if (n == 0) return PACO_OK;
  if (!d->A || !d->B || !d->C) {
    set_err(ctx, "null operand");
    return PACO_ERR_INVALID_ARG;
  }
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");

  // ---- plan
  SSchedule sched = strassen_schedule(n, p, d->gamma, base);
  int first = 0;
  while (sched.levels[first].assigned == 0) ++first;
  const int prec = d->leaf == PACO_PREC_AUTO ? (sched.levels[first].h >= 1024 ? PREC_BF16X3 : PREC_BF16X6)
                                              : (int)d->leaf;
  if (out) {
    memset(out, 0, sizeof *out);
    out->p = p;
    out->super_rounds = sched.super_rounds;
    out->max_depth = sched.levels.back().depth;
    out->leaf = (paco_precision)prec;
    double mx = 0, mn = 1e300;
    for (int j = 0; j < p; ++j) {
      double w = 0;
      for (const auto& dn : sched.per_proc[j]) {
        const double h = (double)sched.levels[dn.first].h;
        w += h * h * h;
        out->nodes += 1;
      }
      mx = std::max(mx, w);
      mn = std::min(mn, w);
    }
    out->max_work = mx;
    out->min_work = mn;
  }
  if (first == 0) {   // the root itself is handed out: one classic product on all compute units
    paco_mm_desc md;
    memset(&md, 0, sizeof md);
    md.n = md.m = md.k = n;
    md.sr = PACO_SR_PLUS_TIMES_F32;
    md.A = d->A; md.B = d->B; md.C = d->C;
    md.precision = (paco_precision)prec;
    md.part = PACO_PART_PACO;
    return paco_semiring_mm_ex(ctx, &md, nullptr);
  }

  char key[200];
  snprintf(key, sizeof key, "spbfs/%lld/%d/%d/%lld/%d", (long long)n, p, d->gamma, (long long)base, prec);
  SPlan* sp = nullptr;
  auto itp = ctx->plans.find(key);
  if (itp != ctx->plans.end()) {
    sp = static_cast<SPlan*>(itp->second.get());
  } else {
    trim_plans(ctx);
    std::unique_ptr<SPlan> np(new SPlan());
    np->sched = sched;
    np->first = first;
    np->fused = std::min(first, 3);
    np->prec = prec;
    const int nd = (int)sched.levels.size();
    np->s_off.assign(nd, -1);
    np->t_off.assign(nd, -1);
    np->m_off.assign(nd, -1);
    int64_t off = 0;
    for (int dd = np->fused; dd < nd; ++dd) {
      const int64_t blk = sched.levels[dd].nodes * sched.levels[dd].h * sched.levels[dd].h;
      np->s_off[dd] = off; off += blk;
      np->t_off[dd] = off; off += blk;
      np->m_off[dd] = off; off += blk;
    }
    np->total = off;
    // leaf problems: processor group g = compute units [g C / p, (g+1) C / p)
    // runs its nodes in depth order, each split over the group by MM-1-Piece
    const int C = ctx->num_cus;
    std::vector<TaggedPiece> tp;
    std::vector<Piece> local;
    std::vector<ProbGeom> geom;
    for (int g = 0; g < p; ++g) {
      const int c0 = (int)((int64_t)g * C / p), c1 = (int)((int64_t)(g + 1) * C / p);
      for (const auto& dn : sched.per_proc[g]) {
        const int64_t h = sched.levels[dn.first].h;
        const int32_t pi = (int32_t)np->prob.size();
        np->prob.push_back({dn.first, dn.second, h, 0});
        geom.push_back(ProbGeom{h, h, h});
        PartOpts po;
        po.p = c1 - c0;
        po.q[0] = 16; po.q[1] = 16; po.q[2] = 32;
        po.kcut_cost = default_kcut_cost(PACO_SR_PLUS_TIMES_F32);
        for (const Piece& pc : partition_mm1(h, h, h, po)) {
          if (pc.empty()) continue;
          tp.push_back({pc, pi, c0 + pc.proc});
          local.push_back(pc);
        }
      }
    }
    np->h = build_plan(tp, C, true, geom);
    np->tile = choose_ring_tile(local, prec);
    np->fam = 2;
    np->p = p;
    st = upload_plan(ctx, np.get());
    if (st != PACO_OK) return st;
    if ((e = hipMalloc(&np->d_probs, sizeof(Problem) * np->prob.size())) != hipSuccess)
      return hip_fail(ctx, e, "Strassen problem table");
    sp = np.get();
    ctx->plans[key] = std::move(np);
  }

  // ---- workspace and the leaf problem table
  st = ensure_sws(ctx, (uint64_t)sp->total * 4);
  if (st != PACO_OK) return st;
  st = ensure_ws(ctx, (uint64_t)sp->h.temp_elems * 4);
  if (st != PACO_OK) return st;
  float* W = (float*)ctx->sws;
  if (sp->probs_base != ctx->sws) {
    std::vector<Problem> probs(sp->prob.size());
    for (size_t i = 0; i < probs.size(); ++i) {
      const int dd = (int)sp->prob[i][0];
      const int64_t j = sp->prob[i][1], h = sp->prob[i][2];
      Problem& q = probs[i];
      q.A = W + sp->s_off[dd] + j * h * h;
      q.B = W + sp->t_off[dd] + j * h * h;
      q.C = W + sp->m_off[dd] + j * h * h;
      q.lda = q.ldb = q.ldc = h;
      q.n = q.m = q.k = (int32_t)h;
      q.accumulate = 0;
    }
    // the stream may still read the old table: wait before replacing it
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hip_fail(ctx, e, "Strassen table sync");
    if ((e = hipMemcpy(sp->d_probs, probs.data(), sizeof(Problem) * probs.size(), hipMemcpyHostToDevice)) !=
        hipSuccess)
      return hip_fail(ctx, e, "Strassen table upload");
    sp->probs_base = ctx->sws;
  }
  if (out) out->temp_bytes = (uint64_t)sp->total * 4;

  const auto& lv = sp->sched.levels;
  const int nd = (int)lv.size();
  // ---- pre-additions, top down
  {
    TimeScope ts(ctx, 2);
    e = launch_strassen_preadd(sp->fused, n, d->A, d->B, W + sp->s_off[sp->fused], W + sp->t_off[sp->fused],
                               ctx->stream);
    for (int dd = sp->fused + 1; dd < nd && e == hipSuccess; ++dd) {
      const int64_t hp = lv[dd - 1].h, hc = lv[dd].h;
      const int64_t a = lv[dd - 1].assigned, cnt = lv[dd - 1].nodes - a;
      e = launch_strassen_preadd_batch(1, hp, (int)cnt, W + sp->s_off[dd - 1] + a * hp * hp,
                                       W + sp->t_off[dd - 1] + a * hp * hp, W + sp->s_off[dd], W + sp->t_off[dd],
                                       hp * hp, 7 * hc * hc, ctx->stream);
    }
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "Strassen pre-add");
  // ---- every handed-out node, one persistent launch
  ProbRef pr;
  memset(&pr, 0, sizeof pr);
  pr.table = sp->d_probs;
  bool v4 = true;
  for (const auto& q : sp->prob) v4 = v4 && q[2] % 4 == 0;
  pr.vec_ok = v4 ? 1 : 0;
  {
    TimeScope ts(ctx, 0);
    e = launch_ring(sp->prec, sp->tile, pr, sp->d_items, sp->d_wg_off, sp->h.nwg, sp->h.xcd_remap, ctx->ws,
                    ctx->stream);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "Strassen node launch");
  if (!sp->h.tiles.empty()) {
    TimeScope ts(ctx, 1);
    e = launch_reduce(SR_RING, pr, sp->d_tiles, (int)sp->h.tiles.size(), sp->d_srcs, ctx->ws, ctx->stream,
                      sp->h.red_vec);
    if (e != hipSuccess) return hip_fail(ctx, e, "Strassen node reduce");
  }
  // ---- combines, bottom up
  {
    TimeScope ts(ctx, 2);
    for (int dd = nd - 1; dd > sp->fused && e == hipSuccess; --dd) {
      const int64_t hp = lv[dd - 1].h, hc = lv[dd].h;
      const int64_t a = lv[dd - 1].assigned, cnt = lv[dd - 1].nodes - a;
      e = launch_strassen_combine_batch(1, hp, (int)cnt, W + sp->m_off[dd], W + sp->m_off[dd - 1] + a * hp * hp,
                                        hp, 7 * hc * hc, hp * hp, ctx->stream);
    }
    if (e == hipSuccess) e = launch_strassen_combine(sp->fused, n, W + sp->m_off[sp->fused], d->C, ctx->stream);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "Strassen combine");
  return PACO_OK;
}
