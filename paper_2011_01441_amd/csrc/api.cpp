// api.cpp -- the C ABI of libpaco (include/paco.h): contexts, plan cache,
// workspace, and the semiring MM entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/paco.h"
#include "ctx.h"
#include "kernels.h"
#include "partition.h"
#include "plan.h"

using namespace paco;

namespace paco {

void set_err(paco_ctx ctx, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
}

paco_status hip_fail(paco_ctx ctx, hipError_t e, const char* what) {
  set_err(ctx, std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? PACO_ERR_OUT_OF_MEMORY : PACO_ERR_HIP;
}

DevPlan::~DevPlan() {
  if (d_items) (void)hipFree(d_items);
  if (d_wg_off) (void)hipFree(d_wg_off);
  if (d_tiles) (void)hipFree(d_tiles);
  if (d_srcs) (void)hipFree(d_srcs);
  if (d_item_fold) (void)hipFree(d_item_fold);
  if (d_fold_list) (void)hipFree(d_fold_list);
  if (d_fold_cnt) (void)hipFree(d_fold_cnt);
}

template <class T>
static hipError_t upload(T** dst, const std::vector<T>& v) {
  *dst = nullptr;
  if (v.empty()) return hipSuccess;
  hipError_t e = hipMalloc((void**)dst, sizeof(T) * v.size());
  if (e != hipSuccess) return e;
  return hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
}

paco_status upload_plan(paco_ctx ctx, DevPlan* dp) {
  hipError_t e;
  if ((e = upload(&dp->d_items, dp->h.items)) != hipSuccess) return hip_fail(ctx, e, "plan upload");
  if ((e = upload(&dp->d_wg_off, dp->h.wg_off)) != hipSuccess) return hip_fail(ctx, e, "plan upload");
  if ((e = upload(&dp->d_tiles, dp->h.tiles)) != hipSuccess) return hip_fail(ctx, e, "plan upload");
  if ((e = upload(&dp->d_srcs, dp->h.srcs)) != hipSuccess) return hip_fail(ctx, e, "plan upload");
  if (dp->h.fused) {
    if ((e = upload(&dp->d_item_fold, dp->h.item_fold)) != hipSuccess) return hip_fail(ctx, e, "plan upload");
    if ((e = upload(&dp->d_fold_list, dp->h.fold_list)) != hipSuccess) return hip_fail(ctx, e, "plan upload");
    // one counter per cell, zero between calls (each call's folding
    // workgroups reset the counters they complete)
    if ((e = upload(&dp->d_fold_cnt, std::vector<uint32_t>(dp->h.tiles.size(), 0u))) != hipSuccess)
      return hip_fail(ctx, e, "plan upload");
  }
  return PACO_OK;
}

paco_status ensure_ws(paco_ctx ctx, uint64_t bytes) {
  if (bytes <= ctx->ws_bytes) return PACO_OK;
  if (bytes > ctx->budget) {
    char buf[160];
    snprintf(buf, sizeof buf, "workspace of %llu bytes exceeds the budget of %llu bytes",
             (unsigned long long)bytes, (unsigned long long)ctx->budget);
    set_err(ctx, buf);
    return PACO_ERR_BUDGET;
  }
  hipError_t e;
  if (ctx->ws) {
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hip_fail(ctx, e, "workspace sync");
    (void)hipFree(ctx->ws);
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  // round up to 64 MiB so small growth steps do not reallocate every call
  uint64_t want = (bytes + (64ull << 20) - 1) & ~((64ull << 20) - 1);
  if (want > ctx->budget) want = bytes;
  ctx->ws_gen += 1;
  if ((e = hipMalloc(&ctx->ws, want)) != hipSuccess) return hip_fail(ctx, e, "workspace alloc");
  ctx->ws_bytes = want;
  return PACO_OK;
}

int choose_int_tile(const std::vector<Piece>& pcs) {
  // critical-path padded work of each tile shape, small tiles weighted by
  // their lower efficiency
  const int cand[5] = {INT_T128x128, INT_T256x64, INT_T64x128, INT_T64x64, INT_T128x64};
  const double eff[5] = {1.0, 1.0, 1.15, 1.35, 1.1};
  int best = INT_T128x128;
  double bestc = 1e300;
  for (int c = 0; c < 5; ++c) {
    IntTileShape ts = int_tile_shape(cand[c]);
    double worst = 0;
    for (const Piece& p : pcs) {
      if (p.empty()) continue;
      double tiles = (double)((p.n1 - p.n0 + ts.tm - 1) / ts.tm) * (double)((p.m1 - p.m0 + ts.tn - 1) / ts.tn);
      worst = std::max(worst, tiles * ts.tm * ts.tn * (double)(p.k1 - p.k0) * eff[c]);
    }
    if (worst < bestc) {
      bestc = worst;
      best = cand[c];
    }
  }
  return best;
}

static hipEvent_t take_event(paco_ctx ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void trim_plans(paco_ctx ctx) {
  if (ctx->plans.size() < PACO_PLAN_CACHE_MAX) return;
  // kernels in flight, on whichever stream the calls used, may still read
  // the plans' device tables
  (void)hipDeviceSynchronize();
  ctx->plans.clear();
  ctx->ws_gen += 1;   // captured graphs that point into them refuse to replay
}

TimeScope::TimeScope(paco_ctx c, int r) : ctx(c), role(r) {
  if (!ctx->timing) return;
  a = take_event(ctx);
  if (a) (void)hipEventRecord(a, ctx->stream);
}

TimeScope::~TimeScope() {
  if (!a) return;
  hipEvent_t b = take_event(ctx);
  if (!b) {
    ctx->event_pool.push_back(a);
    return;
  }
  (void)hipEventRecord(b, ctx->stream);
  ctx->marks.push_back({a, b, role});
}

}  // namespace paco

extern "C" paco_status paco_timing_enable(paco_ctx ctx, int enable) {
  if (!ctx) return PACO_ERR_INVALID_ARG;
  ctx->timing = enable != 0;
  return PACO_OK;
}

extern "C" paco_status paco_timing_read(paco_ctx ctx, paco_timing* out) {
  if (!ctx || !out) return PACO_ERR_INVALID_ARG;
  memset(out, 0, sizeof *out);
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_fail(ctx, e, "timing sync");
  for (auto& mk : ctx->marks) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, mk.a, mk.b) == hipSuccess) {
      if (mk.role == 0) {
        out->main_ms += ms;
        out->launches += 1;
      } else if (mk.role == 1) {
        out->reduce_ms += ms;
      } else {
        out->other_ms += ms;
      }
    }
    ctx->event_pool.push_back(mk.a);
    ctx->event_pool.push_back(mk.b);
  }
  ctx->marks.clear();
  return PACO_OK;
}

// ------------------------------------------------------------------ context

extern "C" paco_status paco_create(paco_ctx* out, int device, uint64_t budget) {
  if (!out) return PACO_ERR_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return PACO_ERR_HIP;
  if (device < 0 || device >= ndev) return PACO_ERR_INVALID_ARG;
  if (hipSetDevice(device) != hipSuccess) return PACO_ERR_HIP;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return PACO_ERR_HIP;
  auto* c = new paco_ctx_s();
  c->device = device;
  c->num_cus = prop.multiProcessorCount;
  c->budget = budget ? budget : (64ull << 30);
  if (noalloc_init(c) != PACO_OK) {
    delete c;
    return PACO_ERR_HIP;
  }
  *out = c;
  return PACO_OK;
}

extern "C" paco_status paco_destroy(paco_ctx ctx) {
  if (!ctx) return PACO_ERR_INVALID_ARG;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  ctx->plans.clear();
  for (auto& mk : ctx->marks) {
    (void)hipEventDestroy(mk.a);
    (void)hipEventDestroy(mk.b);
  }
  for (hipEvent_t ev : ctx->event_pool) (void)hipEventDestroy(ev);
  if (ctx->switch_ev) (void)hipEventDestroy(ctx->switch_ev);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->d_verify) (void)hipFree(ctx->d_verify);
  destroy_ctx_extras(ctx);
  delete ctx;
  return PACO_OK;
}

extern "C" paco_status paco_set_stream(paco_ctx ctx, void* stream) {
  if (!ctx) return PACO_ERR_INVALID_ARG;
  hipStream_t ns = (hipStream_t)stream;
  if (ns == ctx->stream) return PACO_OK;
  // the workspace is shared by every call of the context: the new stream
  // waits for what was launched on the old one
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess && !ctx->switch_ev) e = hipEventCreateWithFlags(&ctx->switch_ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(ctx->switch_ev, ctx->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(ns, ctx->switch_ev, 0);
  if (e != hipSuccess) return hip_fail(ctx, e, "stream change");
  ctx->stream = ns;
  return PACO_OK;
}

extern "C" int paco_num_cus(paco_ctx ctx) { return ctx ? ctx->num_cus : 0; }

extern "C" paco_status paco_set_piece_stamps(paco_ctx ctx, void* stamps, int32_t capacity) {
  if (!ctx || capacity < 0 || (stamps && capacity == 0)) return PACO_ERR_INVALID_ARG;
  ctx->stamps = (uint64_t*)stamps;
  ctx->stamp_cap = stamps ? capacity : 0;
  return PACO_OK;
}

extern "C" const char* paco_status_string(paco_status s) {
  switch (s) {
    case PACO_OK: return "ok";
    case PACO_ERR_INVALID_ARG: return "invalid argument";
    case PACO_ERR_UNSUPPORTED: return "unsupported";
    case PACO_ERR_OUT_OF_MEMORY: return "out of device memory";
    case PACO_ERR_BUDGET: return "budget exceeded";
    case PACO_ERR_HIP: return "HIP runtime error";
    case PACO_ERR_INTERNAL: return "internal error";
    case PACO_ERR_NOT_FOUND: return "not found";
  }
  return "unknown status";
}

extern "C" const char* paco_last_error(paco_ctx ctx) {
  return ctx ? ctx->last_error.c_str() : "null context";
}

// --------------------------------------------------------------- partition

extern "C" paco_status paco_partition(int64_t n, int64_t m, int64_t k, const paco_part_opts* o,
                                      paco_piece* out, int64_t cap, int64_t* n_out) {
  if (!o || !n_out || n < 0 || m < 0 || k < 0 || o->p < 1 || o->p > (1 << 20)) return PACO_ERR_INVALID_ARG;
  if (cap > 0 && !out) return PACO_ERR_INVALID_ARG;
  PartOpts po;
  po.p = o->p;
  po.q[0] = o->q_n > 0 ? o->q_n : 1;
  po.q[1] = o->q_m > 0 ? o->q_m : 1;
  po.q[2] = o->q_k > 0 ? o->q_k : 1;
  po.weights = o->weights;
  po.kcut_cost = o->kcut_cost > 0 ? o->kcut_cost : 1.0;
  if (!(po.kcut_cost >= 1.0) || !std::isfinite(po.kcut_cost) || o->max_rounds < 0) return PACO_ERR_INVALID_ARG;
  po.max_rounds = o->max_rounds;
  po.tile_balance = o->tile_balance != 0;
  if (o->weights)
    for (int i = 0; i < o->p; ++i)
      if (!(o->weights[i] > 0) || !std::isfinite(o->weights[i])) return PACO_ERR_INVALID_ARG;
  std::vector<Piece> pcs = o->multi_piece ? partition_multi(n, m, k, po) : partition_mm1(n, m, k, po);
  *n_out = (int64_t)pcs.size();
  for (int64_t i = 0; i < std::min<int64_t>(cap, (int64_t)pcs.size()); ++i) {
    const Piece& p = pcs[i];
    out[i].n0 = p.n0; out[i].n1 = p.n1;
    out[i].m0 = p.m0; out[i].m1 = p.m1;
    out[i].k0 = p.k0; out[i].k1 = p.k1;
    out[i].proc = p.proc;
    out[i].temp = (!p.empty() && p.k0 > 0) ? 1 : 0;
    out[i].round = p.round;
    out[i].depth = p.depth;
  }
  return PACO_OK;
}

// -------------------------------------------------------------- semiring MM

namespace paco {

// k-cut cost of the PACO partition when the caller gives none.  A k-cut
// makes the upper cuboid write a temporary face that is read back by the
// reduction; next to the matrix-core ring kernel that round trip costs about
// as much as the piece's work on a face 16 times larger, while the VALU
// semirings spend far longer per element and keep the paper's rule (1).
// Measured on (2048, 1024, 65536) and 8192^3 (ring) and on the (min,+) and
// boolean shapes; PACO_KCUT_COST in the environment overrides it.
double default_kcut_cost(int sr) {
  const char* e = getenv("PACO_KCUT_COST");
  if (e) {
    double v = atof(e);
    return v >= 1.0 ? v : 1.0;
  }
  return sr == PACO_SR_PLUS_TIMES_F32 ? 16.0 : 1.0;
}

// k-cut cost a PACO call plans with when the caller gives none: the
// environment override, else 16 for the ring; 0 (choose among 1, 4 and 16
// with the tile and p) for the VALU semirings.
double plan_kcut_cost(int sr) {
  if (getenv("PACO_KCUT_COST") || sr == PACO_SR_PLUS_TIMES_F32) return default_kcut_cost(sr);
  return 0.0;
}

int64_t words(int64_t bits) { return (bits + 31) / 32; }

// Float32 componentwise-error model of bf16x3 at depth k (see paco.h, AUTO).
int auto_precision(int64_t k) {
  // measured/emulated max normalised error of bf16x3 falls like 1/sqrt(k):
  // about 2^-17.2 at k = 32 and 2^-20 at k = 1024; bf16x3 is chosen when the
  // predicted value is at most 2^-21, i.e. k >= 4096.
  return k >= 4096 ? PREC_BF16X3 : PREC_BF16X6;
}

bool ring_vec_ok(const void* A, int64_t lda, const void* B, int64_t ldb, int64_t m, int64_t k) {
  return (uintptr_t)A % 16 == 0 && (uintptr_t)B % 16 == 0 && lda % 4 == 0 && ldb % 4 == 0 && k % 4 == 0 &&
         m % 4 == 0;
}

}  // namespace paco

namespace {

struct Norm {  // normalised call
  paco_semiring sr;
  int64_t n, m, k;           // logical sizes
  int64_t mu, ku;            // kernel units of m and k-words (bool: words)
  int64_t lda, ldb, ldc;     // kernel units
  int prec;
};

}  // namespace

namespace paco {

// Tile override for experiments (PACO_*_TILE = index into the kernel's tile
// list); out-of-range values are ignored.
static int env_tile(const char* name, int count, int dflt) {
  const char* v = getenv(name);
  if (!v) return dflt;
  int t = atoi(v);
  return (t >= 0 && t < count) ? t : dflt;
}

// MM-1-Piece of a ring product on the matrix-core kernel's tile grid: for
// each tile shape the cuts of n and m land on whole tiles (when the
// dimension holds two), k on the 32-deep step, with the tile-balanced
// dimension choice; the tile whose busiest processor has the least padded
// work (weighted by the tile's measured relative cost, plus a prologue and
// epilogue of two steps per tile) wins.  force_tile >= 0 tries that one only.
std::vector<Piece> ring_partition(int64_t n, int64_t m, int64_t k, int p, int prec, double kcut_cost,
                                  const double* weights, int force_tile, int* tile_out, double min_gain_s) {
  // tile shapes tried and their measured relative cost per padded element;
  // a forced tile (any of the kernel's shapes) is the only candidate
  // (three bf16 parts of a 256 x 256 tile do not fit the LDS: that forced
  // tile is ignored like an out-of-range one)
  const int dcand[4] = {RING_T256x256, RING_T256x128, RING_T128x128, RING_T128x64};
  const double deff[4] = {1.0, 1.1, 1.25, 1.6};
  const bool forced = force_tile >= 0 && force_tile < 5 && !(force_tile == RING_T256x256 && prec == PREC_BF16X6);
  const double k_ovh = 64.0;
  double wsum = 0;
  for (int i = 0; i < p; ++i) wsum += weights ? weights[i] : 1.0;
  struct Cand {
    int tile;
    double eff, lb;
  };
  std::vector<Cand> cands;
  for (int c = 0; c < (forced ? 1 : 4); ++c) {
    const int t = forced ? force_tile : dcand[c];
    if (!forced && t == RING_T256x256 && prec == PREC_BF16X6) continue;
    const RingTileShape ts = ring_tile_shape(t, prec);
    // no partition does better than the whole padded product spread evenly
    const double lb = (double)((n + ts.tm - 1) / ts.tm * ts.tm) * (double)((m + ts.tn - 1) / ts.tn * ts.tn) *
                      ((double)((k + ts.bk - 1) / ts.bk * ts.bk) + k_ovh) / wsum * (forced ? 1.0 : deff[c]);
    cands.push_back({t, forced ? 1.0 : deff[c], lb});
  }
  auto options = [&](int t, bool search) {
    const RingTileShape ts = ring_tile_shape(t, prec);
    PartOpts po;
    po.p = p;
    po.kcut_cost = kcut_cost;
    po.weights = weights;
    po.q[0] = n >= 2 * ts.tm ? ts.tm : 16;
    po.q[1] = m >= 2 * ts.tn ? ts.tn : 16;
    po.q[2] = ts.bk;
    po.tile_balance = search;
    po.tile_n = ts.tm;
    po.tile_m = ts.tn;
    po.tile_k_ovh = k_ovh;
    return po;
  };
  auto cost = [&](const std::vector<Piece>& v, const Cand& c) {
    const RingTileShape ts = ring_tile_shape(c.tile, prec);
    double worst = 0;
    for (const Piece& pc : v) {
      if (pc.empty()) continue;
      const double tiles = (double)((pc.n1 - pc.n0 + ts.tm - 1) / ts.tm) * (double)((pc.m1 - pc.m0 + ts.tn - 1) / ts.tn);
      const double kk = (double)((pc.k1 - pc.k0 + ts.bk - 1) / ts.bk * ts.bk);
      const double w = weights ? weights[pc.proc] : 1.0;
      worst = std::max(worst, tiles * ts.tm * ts.tn * (kk + k_ovh) * c.eff / w);
    }
    return worst;
  };
  // The paper's rule on each tile grid first (microseconds); a plan within
  // 3% of its tile's lower bound is kept as it is.  Otherwise the search
  // (tens of microseconds) runs on the tile with the best lower bound, and
  // on the next one if that still leaves more than 3%.
  std::vector<Piece> best;
  double bestc = 1e300;
  int bt = -1;
  for (const Cand& c : cands) {
    std::vector<Piece> v = partition_mm1(n, m, k, options(c.tile, false));
    const double cs = cost(v, c);
    if (cs < bestc) {
      bestc = cs;
      best = std::move(v);
      bt = c.tile;
    }
  }
  double best_lb = 1e300;
  for (const Cand& c : cands)
    if (c.tile == bt) best_lb = c.lb;
  // the search costs tens to hundreds of microseconds of host time: run it
  // when the busiest processor's estimated time above the bound exceeds
  // min_gain_s (padded element-steps at about 8.5e11 a second per processor
  // for bf16x3 on matrix cores, half that for bf16x6, a fifth for float32)
  const double rate = prec == PREC_BF16X6 ? 4.2e11 : (prec == PREC_FP32 ? 1.6e11 : 8.5e11);
  if (bestc > 1.03 * best_lb && (bestc - best_lb) / rate > min_gain_s) {
    std::sort(cands.begin(), cands.end(), [](const Cand& a, const Cand& b) { return a.lb < b.lb; });
    for (size_t i = 0; i < cands.size() && i < 2; ++i) {
      if (cands[i].lb >= bestc) break;
      std::vector<Piece> v = partition_mm1(n, m, k, options(cands[i].tile, true));
      const double cs = cost(v, cands[i]);
      if (cs < bestc) {
        bestc = cs;
        best = std::move(v);
        bt = cands[i].tile;
      }
      if (bestc <= 1.03 * cands[i].lb) break;
    }
  }
  *tile_out = bt;
  return best;
}

// Host part of a semiring MM plan: partition, tile choice, work lists.
// Relative time of f pieces per workgroup slot of a VALU plan: with one
// piece per slot the slowest slot sets the end, with more the dispatcher
// evens out the slots' speeds.
// (f may be fractional: piece counts that are not a multiple of the slots)
static double slot_spread(double f) {
  if (f < 2) return 1.2;
  if (f < 4) return 1.1;
  if (f < 8) return 1.045;
  if (f < 16) return 1.02;
  return 1.0;
}

void make_mm_plan(int sr, int64_t n, int64_t m, int64_t k, int part, int p, int split_k, int prec,
                  int num_cus, DevPlan* np, double kcut_cost, const double* weights, int force_tile,
                  double search_min_gain_s) {
  const bool is_bool = sr == PACO_SR_OR_AND_B1;
  const int64_t mu = is_bool ? words(m) : m, ku = is_bool ? words(k) : k;
  const int fam = sr == PACO_SR_PLUS_TIMES_F32 ? 2 : (is_bool ? 1 : 0);
  std::vector<Piece> pcs;
  int tile = 0, tm = 0, tn = 0, bk = 32;
  double kcut_cost_used = 0.0;
  if (part != PACO_PART_GRID) {
    PartOpts po;
    po.kcut_cost = kcut_cost;
    po.max_rounds = 4;
    po.weights = weights;   // explicit p only (checked by the caller)
    // weighted ratio cuts land anywhere on the quantum grid; for the ring
    // kernel's 256-wide tiles an n or m cut off that grid pads every tile
    // it crosses, so weighted ring cuts in n and m stay on tile multiples
    // (k cuts keep the 32-deep step)
    const bool wring = weights && fam == 2;
    // integer cuts in m and k land on multiples of four, so the work items
    // start 16-byte aligned for the kernel's 128-bit loads
    if (fam == 0) { po.q[1] = 4; po.q[2] = 4; }
    else if (fam == 1) { po.q[0] = 1; po.q[1] = 32; po.q[2] = 32; }
    else if (fam == 2) { po.q[0] = wring ? 256 : 16; po.q[1] = wring ? 256 : 16; po.q[2] = 32; }
    auto part_for = [&](int pp) {
      po.p = pp;
      std::vector<Piece> v = part == PACO_PART_MULTI ? partition_multi(n, m, k, po) : partition_mm1(n, m, k, po);
      if (fam == 1)  // bits -> words in m
        for (Piece& pc : v) { pc.m0 /= 32; pc.m1 = words(pc.m1); }
      return v;
    };
    const char* tile_env = fam == 0 ? "PACO_INT_TILE" : (fam == 1 ? "PACO_BOOL_TILE" : "PACO_RING_TILE");
    if (p <= 0 && fam != 2) {
      // Default p of the VALU kernels.  A single workgroup per compute unit
      // leaves each SIMD one wave to hide latency with, so a processor is a
      // workgroup slot: each candidate tile is tried with p = CUs x (its
      // resident workgroups per CU) -- when the problem gives every slot a
      // few tiles -- and with two to sixteen times as many pieces as
      // slots, which the hardware dispatcher hands to slots as they free up
      // (the slots do not run at one speed, the XCD clocks alone differ by
      // 3%: on (min,+) 8192^3 one, four and sixteen pieces per slot measured
      // 25.96, 22.65 and 21.64 ms, the factors 1.2 / 1.045 / 1 below, the
      // last equal to the tile grid's 16384 workgroups).  Unless the caller fixed it, the
      // k-cut cost is tried at 1 (the paper's rule), 4, 16 and 64.  The
      // plan with the shortest estimated time wins: the worst piece's
      // padded tiles, each costing its k-range plus a fixed
      // prologue/epilogue overhead, at the tile's measured rate per compute
      // unit shared by the workgroups on it, times the rounds of pieces per
      // slot, plus the temporary faces written and read back at HBM speed.
      // (Two and eight pieces per slot, between the measured points, take
      // 1.1 and 1.02; on boolean 8192^3 two pieces per slot of the 512 x 32
      // word tile measured 0.593 ms of kernel time against 0.614 for one.)
      // These kernels stream about 8 elements per byte, so a k-cut also
      // costs L2 reuse (concurrent pieces no longer walk k in step); the
      // overhead term and the face traffic stand for that.
      // relative time per padded element of each integer tile at its own
      // occupancy, from full-size (min,+) 8192^3 and 4096^3 runs (64 x 64
      // at four workgroups per CU = 0.95; 64 x 128 at three 2.5% faster,
      // 128 x 64 at two 11% slower, 128 x 128 and 256 x 64 at one 28% and
      // 36% slower)
      const int ci[5] = {INT_T128x128, INT_T256x64, INT_T64x128, INT_T64x64, INT_T128x64};
      const double ei[5] = {1.22, 1.29, 0.926, 0.95, 1.06};
      const int cb[4] = {BOOL_T512x32W, BOOL_T128x128W, BOOL_T256x64W, BOOL_T64x64W};
      const double eb[4] = {1.0, 1.0, 0.98, 1.08};
      const int ncand = fam == 0 ? 5 : 4;
      const double rate_cu = fam == 0 ? 70e9 : 110e9;      // elements (words) per second per CU
      const double k_ovh = fam == 0 ? 64.0 : 128.0;        // prologue + epilogue, in k units
      const double kcs[4] = {1.0, 4.0, 16.0, 64.0};
      const int nkc = kcut_cost > 0 ? 1 : 4;
      const int forced = force_tile >= 0 ? force_tile : env_tile(tile_env, ncand, -1);
      const double work = (double)n * (double)mu * (double)k;
      double bestc = 1e300;
      for (int ik = 0; ik < nkc; ++ik) {
        po.kcut_cost = kcut_cost > 0 ? kcut_cost : kcs[ik];
        for (int c = 0; c < ncand; ++c) {
          const int t = fam == 0 ? ci[c] : cb[c];
          if (forced >= 0 && t != forced) continue;
          int tm_, tn_;
          if (fam == 0) { IntTileShape ts = int_tile_shape(t); tm_ = ts.tm; tn_ = ts.tn; }
          else { BoolTileShape ts = bool_tile_shape(t); tm_ = ts.tm; tn_ = ts.tnw; }
          int occ = fam == 0 ? int_occupancy(sr, t) : bool_occupancy(t);
          occ = std::min(std::max(occ, 1), 8);
          const double tile_work = (double)tm_ * tn_ * 256;   // one tile, 256 deep
          const int slots = (occ > 1 && work >= (double)num_cus * occ * 4 * tile_work) ? num_cus * occ : num_cus;
          // piece counts: one to sixteen per slot, and power-of-two multiples
          // of the CUs (with three slots per CU those are the counts whose
          // cuts of power-of-two sizes land on whole tiles)
          std::vector<int> counts;
          for (int f : {1, 2, 4, 8, 16}) counts.push_back(slots * f);
          for (int j = 0; j <= 6; ++j)
            if (std::find(counts.begin(), counts.end(), num_cus << j) == counts.end() && (num_cus << j) >= slots)
              counts.push_back(num_cus << j);
          for (int pt : counts) {
            const double f = (double)pt / slots;
            // more pieces than slots only while each keeps a tile's worth of
            // work (the per-tile overhead term prices smaller ones)
            if (pt > slots && work < (double)pt * tile_work) continue;
            if (pt > 65536) continue;
            std::vector<Piece> v = part_for(pt);
            std::vector<double> load(pt, 0.0);   // per processor (multi-piece: several pieces)
            double worst = 0, temps = 0;
            for (const Piece& pc : v) {
              if (pc.empty()) continue;
              const double tl =
                  (double)((pc.n1 - pc.n0 + tm_ - 1) / tm_) * (double)((pc.m1 - pc.m0 + tn_ - 1) / tn_);
              load[pc.proc] += tl * tm_ * tn_ * ((double)(pc.k1 - pc.k0) + k_ovh);
              worst = std::max(worst, load[pc.proc]);
              if (pc.k0 > 0) temps += (double)(pc.n1 - pc.n0) * (double)(pc.m1 - pc.m0);  // upper k-part
            }
            const double rounds = (double)pt / slots;
            const double cost = worst * ((double)slots / num_cus) * rounds * (fam == 0 ? ei[c] : eb[c]) /
                                    rate_cu * slot_spread(f) +
                                temps * 8.0 / 5e12;
            if (cost < bestc) {
              bestc = cost;
              tile = t;
              p = pt;
              kcut_cost_used = po.kcut_cost;
              pcs = std::move(v);
            }
          }
        }
      }
    } else if (fam == 2 && part == PACO_PART_PACO) {
      if (p <= 0) p = num_cus;
      if (kcut_cost <= 0) kcut_cost = 1.0;
      kcut_cost_used = kcut_cost;
      const int forced = force_tile >= 0 ? force_tile : env_tile(tile_env, 5, -1);
      pcs = ring_partition(n, m, k, p, prec, kcut_cost, weights, forced, &tile, search_min_gain_s);
    } else {
      if (p <= 0) p = num_cus;
      if (kcut_cost <= 0) po.kcut_cost = 1.0;
      kcut_cost_used = po.kcut_cost;
      pcs = part_for(p);
      if (fam == 0) tile = choose_int_tile(pcs);
      else if (fam == 1) tile = choose_bool_tile(pcs);
      else tile = choose_ring_tile(pcs, prec);
      tile = env_tile(tile_env, fam == 2 ? 5 : (fam == 0 ? kIntTiles : 4), tile);
      if (force_tile >= 0) tile = force_tile;
    }
  } else {
    if (fam == 0) {
      tile = m <= 64 ? INT_T256x64 : (n <= 64 ? INT_T64x128 : INT_T128x128);
      tile = env_tile("PACO_INT_TILE", kIntTiles, tile);
      IntTileShape ts = int_tile_shape(tile);
      tm = ts.tm; tn = ts.tn;
    } else if (fam == 1) {
      tile = BOOL_T128x128W;
      tile = env_tile("PACO_BOOL_TILE", 4, tile);
      BoolTileShape ts = bool_tile_shape(tile);
      tm = ts.tm; tn = ts.tnw * 32;
    } else {
      // the largest tile the output fills (the same microkernels PACO uses)
      tile = (n >= 256 && m >= 256 && prec != PREC_BF16X6) ? RING_T256x256
             : (n >= 256 ? RING_T256x128 : (m >= 128 ? RING_T128x128 : RING_T128x64));
      tile = env_tile("PACO_RING_TILE", 5, tile);
      RingTileShape ts = ring_tile_shape(tile, prec);
      tm = ts.tm; tn = ts.tn; bk = ts.bk;
    }
    int64_t tiles = ((n + tm - 1) / tm) * ((m + tn - 1) / tn);
    int64_t kb = (k + bk - 1) / bk;
    int sk = split_k;
    if (sk <= 0) sk = (int)std::max<int64_t>(1, std::min<int64_t>(kb, (num_cus + tiles - 1) / tiles));
    pcs = partition_grid(n, m, k, tm, tn, bk, sk);
    if (fam == 1)
      for (Piece& pc : pcs) { pc.m0 /= 32; pc.m1 = words(pc.m1); }
  }
  std::vector<TaggedPiece> tp(pcs.size());
  for (size_t i = 0; i < pcs.size(); ++i) tp[i] = {pcs[i], 0, part != PACO_PART_GRID ? pcs[i].proc : (int)i};
  const int nwg = part != PACO_PART_GRID ? p : (int)pcs.size();
  std::vector<ProbGeom> geom{{n, mu, ku}};
  // the temporary faces are folded by a separate launch: folding inside
  // the product kernel (the last piece to finish a cell folds it) measured
  // slower on this device, 22.5 against 16.0 us a call on the (min,+)
  // 384 x 256 x 320 product, since the device-scope release and acquire
  // around every counted item and the one-workgroup fold cost more than the
  // second launch, whose start overlaps the first one's tail.
  // PACO_FUSE_FOLD=1 fuses, 2 fuses plans whose cells are all small.
  int fuse = 0;
  if (const char* ef = getenv("PACO_FUSE_FOLD")) fuse = std::min(2, std::max(0, atoi(ef)));
  np->h = build_plan(tp, nwg, part != PACO_PART_GRID, geom, 0, 4, fuse);
  np->tile = tile;
  np->fam = fam;
  np->p = p;
  np->kcut = kcut_cost_used;
}

}  // namespace paco

extern "C" paco_status paco_plan_export(int64_t n, int64_t m, int64_t k, paco_semiring sr, paco_part_mode part,
                                        int32_t p, int32_t split_k, paco_precision prec, int32_t num_cus,
                                        paco_plan_info* info, int64_t* items, int32_t* wg_off, int32_t* tiles,
                                        int64_t* srcs) {
  if (!info || n <= 0 || m <= 0 || k <= 0 || n >= (1ll << 31) || m >= (1ll << 31) || k >= (1ll << 31) ||
      sr < PACO_SR_PLUS_TIMES_F32 || sr > PACO_SR_OR_AND_B1 || part < PACO_PART_PACO || part > PACO_PART_MULTI ||
      p < 0 || (p == 0 && part == PACO_PART_GRID) || p > 65536 || split_k < 0 || num_cus < 1 ||
      prec < PACO_PREC_FP32 || prec > PACO_PREC_AUTO)
    return PACO_ERR_INVALID_ARG;
  int pr = -1;
  if (sr == PACO_SR_PLUS_TIMES_F32) pr = prec == PACO_PREC_AUTO ? auto_precision(k) : (int)prec;
  DevPlan dp;
  // p = 0: the default choice of a call (p, tile and, for the VALU
  // semirings, the k-cut cost); occupancies come from the runtime, 1 where
  // it has no device
  make_mm_plan((int)sr, n, m, k, (int)part, p, split_k, pr, num_cus, &dp,
               p == 0 ? plan_kcut_cost((int)sr) : default_kcut_cost((int)sr));
  const HostPlan& h = dp.h;
  const bool fill = items && wg_off && tiles && srcs;
  if (fill) {
    if (info->n_items < (int32_t)h.items.size() || info->n_wg < h.nwg || info->n_tiles < (int32_t)h.tiles.size() ||
        info->n_srcs < (int32_t)h.srcs.size())
      return PACO_ERR_INVALID_ARG;
    for (size_t i = 0; i < h.items.size(); ++i) {
      const WorkItem& w = h.items[i];
      int64_t* o = items + 8 * i;
      o[0] = w.prob; o[1] = w.n0; o[2] = w.n1; o[3] = w.m0; o[4] = w.m1; o[5] = w.k0; o[6] = w.k1; o[7] = w.out_off;
    }
    for (int i = 0; i <= h.nwg; ++i) wg_off[i] = h.wg_off[i];
    for (size_t i = 0; i < h.tiles.size(); ++i) {
      const RedTile& t = h.tiles[i];
      int32_t* o = tiles + 7 * i;
      o[0] = t.prob; o[1] = t.i0; o[2] = t.i1; o[3] = t.j0; o[4] = t.j1; o[5] = t.s0; o[6] = t.s1;
    }
    for (size_t i = 0; i < h.srcs.size(); ++i) {
      const RedSrc& r = h.srcs[i];
      int64_t* o = srcs + 4 * i;
      o[0] = r.off; o[1] = r.ld; o[2] = r.r0; o[3] = r.c0;
    }
  }
  info->n_wg = h.nwg;
  info->n_items = (int32_t)h.items.size();
  info->n_tiles = (int32_t)h.tiles.size();
  info->n_srcs = (int32_t)h.srcs.size();
  info->tile = dp.tile;
  info->red_vec = h.red_vec;
  info->xcd_remap = h.xcd_remap ? 1 : 0;
  info->temp_elems = h.temp_elems;
  info->fused = h.fused ? 1 : 0;
  info->n_fold_list = (int32_t)h.fold_list.size();
  return PACO_OK;
}

extern "C" paco_status paco_plan_export_fold(int64_t n, int64_t m, int64_t k, paco_semiring sr, paco_part_mode part,
                                             int32_t p, int32_t split_k, paco_precision prec, int32_t num_cus,
                                             paco_plan_info* info, int32_t* pads, int32_t* item_fold,
                                             int32_t* fold_list) {
  paco_plan_info in = info ? *info : paco_plan_info{};
  paco_status st = paco_plan_export(n, m, k, sr, part, p, split_k, prec, num_cus, &in, nullptr, nullptr, nullptr,
                                    nullptr);
  if (st != PACO_OK) return st;
  const bool fill = pads && item_fold && fold_list;
  if (fill && info && (info->n_tiles < in.n_tiles || info->n_items < in.n_items ||
                       info->n_fold_list < in.n_fold_list))
    return PACO_ERR_INVALID_ARG;
  if (fill) {
    int pr = -1;
    if (sr == PACO_SR_PLUS_TIMES_F32) pr = prec == PACO_PREC_AUTO ? auto_precision(k) : (int)prec;
    DevPlan dp;
    make_mm_plan((int)sr, n, m, k, (int)part, p, split_k, pr, num_cus, &dp,
                 p == 0 ? plan_kcut_cost((int)sr) : default_kcut_cost((int)sr));
    const HostPlan& h = dp.h;
    for (size_t i = 0; i < h.tiles.size(); ++i) pads[i] = h.tiles[i].pad;
    for (size_t i = 0; i < h.item_fold.size(); ++i) item_fold[i] = h.item_fold[i];
    for (size_t i = 0; i < h.fold_list.size(); ++i) fold_list[i] = h.fold_list[i];
  }
  if (info) *info = in;
  return PACO_OK;
}

extern "C" paco_status paco_semiring_mm(paco_ctx ctx, int64_t n, int64_t m, int64_t k,
                                        paco_semiring sr, const void* A, const void* B, void* C) {
  paco_mm_desc d;
  memset(&d, 0, sizeof d);
  d.n = n; d.m = m; d.k = k; d.sr = sr;
  d.A = A; d.B = B; d.C = C;
  d.precision = PACO_PREC_AUTO;
  d.part = PACO_PART_PACO;
  return paco_semiring_mm_ex(ctx, &d, nullptr);
}

extern "C" paco_status paco_semiring_mm_ex(paco_ctx ctx, const paco_mm_desc* d, paco_mm_result* res) {
  if (!ctx) return PACO_ERR_INVALID_ARG;
  if (!d) {
    set_err(ctx, "null descriptor");
    return PACO_ERR_INVALID_ARG;
  }
  return run_mm(ctx, d, res);
}

std::string paco::tune_key(const paco_mm_desc* d, int prec) {
  char key[128];
  snprintf(key, sizeof key, "%d/%lld/%lld/%lld/%d", (int)d->sr, (long long)d->n, (long long)d->m, (long long)d->k,
           prec);
  return key;
}

namespace {

// Argument validation of a semiring MM descriptor (no device is touched):
// the status the call returns for it, the reason, and the normalised sizes.
paco_status check_desc(const paco_mm_desc* d, Norm* zo, std::string* why) {
  if (d->sr < PACO_SR_PLUS_TIMES_F32 || d->sr > PACO_SR_OR_AND_B1) {
    *why = "unknown semiring";
    return PACO_ERR_INVALID_ARG;
  }
  if (d->n < 0 || d->m < 0 || d->k < 0 || d->n >= (1ll << 31) || d->m >= (1ll << 31) ||
      d->k >= (1ll << 31)) {
    *why = "sizes must lie in [0, 2^31)";
    return PACO_ERR_INVALID_ARG;
  }
  if (d->precision < PACO_PREC_FP32 || d->precision > PACO_PREC_AUTO || d->part < PACO_PART_PACO ||
      d->part > PACO_PART_MULTI || d->p < 0 || d->grid_split_k < 0 || d->verify_rows < 0 ||
      !(d->kcut_cost == 0 || (d->kcut_cost >= 1 && std::isfinite(d->kcut_cost)))) {
    *why = "invalid option";
    return PACO_ERR_INVALID_ARG;
  }
  const bool is_bool = d->sr == PACO_SR_OR_AND_B1;
  Norm& z = *zo;
  z.sr = d->sr;
  z.n = d->n; z.m = d->m; z.k = d->k;
  z.mu = is_bool ? words(d->m) : d->m;
  z.ku = is_bool ? words(d->k) : d->k;
  z.lda = d->lda ? d->lda : z.ku;
  z.ldb = d->ldb ? d->ldb : z.mu;
  z.ldc = d->ldc ? d->ldc : z.mu;
  if (z.lda < z.ku || z.ldb < z.mu || z.ldc < z.mu) {
    *why = "leading dimension smaller than the row length";
    return PACO_ERR_INVALID_ARG;
  }
  // the kernels form 32-bit byte offsets within a block of rows of each
  // operand (64-bit row bases)
  if (z.lda >= (1ll << 22) || z.ldb >= (1ll << 22) || z.ldc >= (1ll << 22)) {
    *why = "leading dimensions of A, B and C must be below 2^22 elements";
    return PACO_ERR_UNSUPPORTED;
  }
  if (d->verify_rows > 0 && d->sr != PACO_SR_PLUS_TIMES_F32) {
    *why = "verify_rows applies to the ring only";
    return PACO_ERR_INVALID_ARG;
  }
  if (z.n == 0 || z.m == 0) return PACO_OK;
  if (!d->C || (z.k > 0 && (!d->A || !d->B))) {
    *why = "null operand";
    return PACO_ERR_INVALID_ARG;
  }
  return PACO_OK;
}

}  // namespace

namespace paco {

// Lays the plan's device tables out in one host block (each table 256-byte
// aligned) and places the temporary faces after it.
void pack_tables(HostTables* t) {
  const HostPlan& h = t->plan.h;
  auto al = [](uint64_t x) { return (x + 255) & ~(uint64_t)255; };
  t->items_off = 0;
  t->wg_off = al(t->items_off + h.items.size() * sizeof(WorkItem));
  t->tiles_off = al(t->wg_off + h.wg_off.size() * sizeof(int32_t));
  t->srcs_off = al(t->tiles_off + h.tiles.size() * sizeof(RedTile));
  t->item_fold_off = al(t->srcs_off + h.srcs.size() * sizeof(RedSrc));
  t->fold_list_off = al(t->item_fold_off + h.item_fold.size() * sizeof(int32_t));
  // fold counters: zeros, copied with the tables at every call
  t->fold_cnt_off = al(t->fold_list_off + h.fold_list.size() * sizeof(int32_t));
  const uint64_t end = t->fold_cnt_off + (h.fused ? h.tiles.size() * sizeof(uint32_t) : 0);
  t->faces_off = al(end);
  t->blob.assign(end, 0);
  auto put = [&](uint64_t off, const void* src, size_t bytes) {
    if (bytes) memcpy(t->blob.data() + off, src, bytes);
  };
  put(t->items_off, h.items.data(), h.items.size() * sizeof(WorkItem));
  put(t->wg_off, h.wg_off.data(), h.wg_off.size() * sizeof(int32_t));
  put(t->tiles_off, h.tiles.data(), h.tiles.size() * sizeof(RedTile));
  put(t->srcs_off, h.srcs.data(), h.srcs.size() * sizeof(RedSrc));
  put(t->item_fold_off, h.item_fold.data(), h.item_fold.size() * sizeof(int32_t));
  put(t->fold_list_off, h.fold_list.data(), h.fold_list.size() * sizeof(int32_t));
}

}  // namespace paco

extern "C" paco_status paco_mm_validate(const paco_mm_desc* d) {
  if (!d) return PACO_ERR_INVALID_ARG;
  Norm z;
  std::string why;
  return check_desc(d, &z, &why);
}

paco_status paco::run_mm(paco_ctx ctx, const paco_mm_desc* d, paco_mm_result* res, int force_tile,
                         const FixedScratch* fx) {
  if (res) {
    memset(res, 0, sizeof *res);
    res->verify_max_rel = -1;
    res->verify_max_abs = -1;
  }
  Norm z;
  std::string why;
  paco_status vst = check_desc(d, &z, &why);
  if (vst != PACO_OK) {
    set_err(ctx, why);
    return vst;
  }
  if (fx && d->verify_rows > 0) {
    set_err(ctx, "verify_rows needs device buffers of its own: use paco_semiring_mm_ex");
    return PACO_ERR_UNSUPPORTED;
  }
  if (z.n == 0 || z.m == 0) return PACO_OK;
  const bool is_bool = d->sr == PACO_SR_OR_AND_B1;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  if (z.k == 0) {
    if (d->accumulate) return PACO_OK;
    TimeScope ts(ctx, 2);
    e = launch_fill_zero(is_bool ? SR_BOOL : (int)d->sr, d->C, z.n, z.mu, z.ldc, ctx->stream);
    return e == hipSuccess ? PACO_OK : hip_fail(ctx, e, "fill");
  }
  z.prec = -1;
  if (d->sr == PACO_SR_PLUS_TIMES_F32) {
    if (d->precision == PACO_PREC_AUTO) z.prec = auto_precision(z.k);
    else z.prec = (int)d->precision;
  }
  const double* weights = d->weights;
  int p = d->p > 0 ? d->p : (d->part != PACO_PART_GRID ? 0 : ctx->num_cus);
  int part = (int)d->part;
  double kc_in = d->kcut_cost;
  bool use_ctx_weights = d->sr == PACO_SR_PLUS_TIMES_F32 && (int)ctx->weights.size() == ctx->num_cus;
  if (force_tile < 0 && d->part == PACO_PART_PACO && d->p == 0 && d->kcut_cost == 0 && !d->weights &&
      !ctx->tuned.empty()) {
    auto it = ctx->tuned.find(tune_key(d, z.prec));
    if (it != ctx->tuned.end()) {   // paco_tune measured this shape
      part = it->second.part;
      p = it->second.p;
      kc_in = it->second.kcut;
      force_tile = it->second.tile;
      use_ctx_weights = use_ctx_weights && it->second.weighted;
    }
  }
  if (!weights && d->p == 0 && part == PACO_PART_PACO && use_ctx_weights) {
    weights = ctx->weights.data();   // the context's measured throughputs
    p = ctx->num_cus;
  }
  uint64_t whash = 0;
  if (weights) {
    if (part != PACO_PART_PACO || p <= 0) {
      set_err(ctx, "processor weights need PACO mode and an explicit p");
      return PACO_ERR_INVALID_ARG;
    }
    whash = 1469598103934665603ull;   // FNV-1a over the weights' bytes, for the plan key
    for (int i = 0; i < p; ++i) {
      if (!(weights[i] > 0) || !std::isfinite(weights[i])) {
        set_err(ctx, "processor weights must be positive and finite");
        return PACO_ERR_INVALID_ARG;
      }
      unsigned char b[8];
      memcpy(b, &weights[i], 8);
      for (unsigned char c : b) whash = (whash ^ c) * 1099511628211ull;
    }
  }
  if (p > 65536) {
    set_err(ctx, "p above 65536");
    return PACO_ERR_INVALID_ARG;
  }

  // ---- plan
  char key[256];
  // 0 = chosen with the tile and p (VALU semirings, see make_mm_plan)
  const double kc = kc_in > 0 ? kc_in : plan_kcut_cost((int)d->sr);
  const char* tenv = getenv(is_bool ? "PACO_BOOL_TILE" : (d->sr == PACO_SR_PLUS_TIMES_F32 ? "PACO_RING_TILE"
                                                                                           : "PACO_INT_TILE"));
  const char* fenv = getenv("PACO_FUSE_FOLD");
  snprintf(key, sizeof key, "mm/%d/%lld/%lld/%lld/%d/%d/%d/%d/%g/%.8s/%.2s/%llx/%d", (int)d->sr, (long long)z.n,
           (long long)z.m, (long long)z.k, part, p, d->grid_split_k, z.prec, kc, tenv ? tenv : "",
           fenv ? fenv : "", (unsigned long long)whash, force_tile);
  DevPlan* dp = nullptr;
  // device tables of the plan and the temporary faces: the plan's own
  // allocations and the context's workspace, or (fx) the caller's fixed
  // scratch, into which the host copies of the tables are written
  const WorkItem* d_items = nullptr;
  const int32_t* d_wg_off = nullptr;
  const RedTile* d_tiles = nullptr;
  const RedSrc* d_srcs = nullptr;
  const int32_t* d_item_fold = nullptr;
  const int32_t* d_fold_list = nullptr;
  uint32_t* d_fold_cnt = nullptr;
  void* ws = nullptr;
  paco_status st = PACO_OK;
  if (!fx) {
    auto itp = ctx->plans.find(key);
    if (itp != ctx->plans.end()) {
      dp = itp->second.get();
    } else {
      trim_plans(ctx);
      std::unique_ptr<DevPlan> np(new DevPlan());
      make_mm_plan((int)d->sr, z.n, z.m, z.k, part, p, d->grid_split_k, z.prec, ctx->num_cus, np.get(), kc,
                   weights, force_tile, ctx->search_min_gain);
      st = upload_plan(ctx, np.get());
      if (st != PACO_OK) return st;
      dp = np.get();
      ctx->plans[key] = std::move(np);
    }
    // ---- workspace
    st = ensure_ws(ctx, (uint64_t)dp->h.temp_elems * 4);
    if (st != PACO_OK) return st;
    d_items = dp->d_items;
    d_wg_off = dp->d_wg_off;
    d_tiles = dp->d_tiles;
    d_srcs = dp->d_srcs;
    d_item_fold = dp->d_item_fold;
    d_fold_list = dp->d_fold_list;
    d_fold_cnt = dp->d_fold_cnt;
    ws = ctx->ws;
  } else {
    auto itp = ctx->host_plans.find(key);
    HostTables* ht = nullptr;
    if (itp != ctx->host_plans.end()) {
      ht = itp->second.get();
    } else {
      if (ctx->host_plans.size() >= PACO_PLAN_CACHE_MAX) {
        // a copy from one of these host tables may still be pending
        if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hip_fail(ctx, e, "plan cache sync");
        ctx->host_plans.clear();
      }
      std::unique_ptr<HostTables> nt(new HostTables());
      make_mm_plan((int)d->sr, z.n, z.m, z.k, part, p, d->grid_split_k, z.prec, ctx->num_cus, &nt->plan, kc,
                   weights, force_tile, ctx->search_min_gain);
      pack_tables(nt.get());
      ht = nt.get();
      ctx->host_plans[key] = std::move(nt);
    }
    dp = &ht->plan;
    const uint64_t need = ht->faces_off + (uint64_t)dp->h.temp_elems * 4;
    if (need > fx->bytes) {
      char buf[256];
      snprintf(buf, sizeof buf,
               "the plan needs %llu bytes of scratch (tables and %lld temporary-face elements); the fixed "
               "scratch holds %llu: use paco_semiring_mm_ex, or a partition with fewer k-cuts (kcut_cost)",
               (unsigned long long)need, (long long)dp->h.temp_elems, (unsigned long long)fx->bytes);
      set_err(ctx, buf);
      return PACO_ERR_BUDGET;
    }
    char* base = (char*)fx->ptr;
    if (!ht->blob.empty() &&
        (e = hipMemcpyAsync(base, ht->blob.data(), ht->blob.size(), hipMemcpyHostToDevice, ctx->stream)) !=
            hipSuccess)
      return hip_fail(ctx, e, "plan table copy");
    d_items = (const WorkItem*)(base + ht->items_off);
    d_wg_off = (const int32_t*)(base + ht->wg_off);
    d_tiles = (const RedTile*)(base + ht->tiles_off);
    d_srcs = (const RedSrc*)(base + ht->srcs_off);
    if (dp->h.fused) {
      d_item_fold = (const int32_t*)(base + ht->item_fold_off);
      d_fold_list = (const int32_t*)(base + ht->fold_list_off);
      d_fold_cnt = (uint32_t*)(base + ht->fold_cnt_off);
    }
    ws = base + ht->faces_off;
  }

  // ---- launch
  ProbRef pr;
  memset(&pr, 0, sizeof pr);
  pr.base.A = d->A; pr.base.B = d->B; pr.base.C = d->C;
  pr.base.lda = z.lda; pr.base.ldb = z.ldb; pr.base.ldc = z.ldc;
  pr.base.n = (int32_t)z.n; pr.base.m = (int32_t)z.m; pr.base.k = (int32_t)z.k;
  pr.base.accumulate = d->accumulate ? 1 : 0;
  // 128-bit operand loads: aligned rows of multiples of four elements, and
  // for the integer kernel work items that start on such multiples
  pr.vec_ok = ring_vec_ok(d->A, z.lda, d->B, z.ldb, z.m, z.k) && (dp->fam != 0 || dp->h.aligned4) ? 1 : 0;
  pr.stamps = ctx->stamps;
  pr.stamp_cap = ctx->stamps ? ctx->stamp_cap : 0;
  const int rvec = (dp->h.red_vec == 4 && (uintptr_t)d->C % 16 == 0 && z.ldc % 4 == 0) ? 4 : 1;
  if (dp->h.fused) {
    pr.item_fold = d_item_fold;
    pr.fold_list = d_fold_list;
    pr.fold_tiles = d_tiles;
    pr.fold_srcs = d_srcs;
    pr.fold_cnt = d_fold_cnt;
    pr.fold_vec = rvec;
  }
  {
  TimeScope ts(ctx, 0);
  if (dp->fam == 0)
    e = launch_semiring_int((int)d->sr, dp->tile, pr, d_items, d_wg_off, dp->h.nwg, dp->h.xcd_remap, ws,
                            ctx->stream);
  else if (dp->fam == 1)
    e = launch_semiring_bool(dp->tile, pr, d_items, d_wg_off, dp->h.nwg, dp->h.xcd_remap, ws, ctx->stream);
  else
    e = launch_ring(z.prec, dp->tile, pr, d_items, d_wg_off, dp->h.nwg, dp->h.xcd_remap, ws, ctx->stream);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "semiring kernel launch");
  if (!dp->h.tiles.empty() && !dp->h.fused) {
    TimeScope ts(ctx, 1);
    e = launch_reduce(is_bool ? SR_BOOL : (int)d->sr, pr, d_tiles, (int)dp->h.tiles.size(), d_srcs, ws,
                      ctx->stream, rvec);
    if (e != hipSuccess) return hip_fail(ctx, e, "reduce launch");
  }
  if (res) {
    res->precision = (paco_precision)(z.prec < 0 ? PACO_PREC_FP32 : z.prec);
    res->p = part != PACO_PART_GRID ? dp->p : dp->h.nwg;
    res->n_pieces = dp->h.n_pieces;
    res->max_piece_volume = dp->h.vmax;
    res->min_piece_volume = dp->h.vmin;
    res->temp_elems = dp->h.temp_elems;
    res->n_kcuts = dp->h.n_kcuts;
    res->kcut_cost = dp->kcut;
  }
  if (d->verify_rows > 0) {
    st = verify_sampled(ctx, z.n, z.m, z.k, (const float*)d->A, z.lda, (const float*)d->B, z.ldb,
                        (const float*)d->C, z.ldc, d->verify_rows, d->verify_seed, res);
    if (st != PACO_OK) return st;
  }
  return PACO_OK;
}
