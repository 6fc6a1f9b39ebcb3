// gap.cpp -- paco_gap: the GAP problem (section "PACO GAP") on the GPU.
//
// The recursion of the section on the (m+1) x (n+1) grid: a block splits
// into quadrants X00, X01, X10, X11 (halves rounded to 64; a side of at most
// GAP_B is not split).  Once X00 is final, its rows update X01 (row gaps)
// and its columns update X10 (column gaps); X01 and X10 are then solved;
// X10's rows and X01's columns update X11; X11 is solved.  Subproblems that
// are independent run in the same launches: the host walks the recursion
// over lists of blocks, so a launch holds every base block, or every cube,
// of one phase.  Each cube is cut by the MM-1-Piece rule over its share of
// the processors by the section's rule: slabs of whole batch rows, so that
// every piece updates a region of its own.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/paco.h"
#include "ctx.h"
#include "kernels.h"

using namespace paco;

namespace {

constexpr int64_t G_INF64 = (int64_t)1 << 30;

struct GapLaunch {
  int base;           // 1: base blocks, 0: cubes
  int64_t off, cnt;   // its entries in the block or piece table
};

struct GapPlan : DevPlan {
  std::vector<GapLaunch> launches;
  std::vector<GapBlock> blocks;
  std::vector<GapPiece> pieces;
  GapBlock* d_blocks = nullptr;
  GapPiece* d_pieces = nullptr;
  int64_t cubes = 0;
  ~GapPlan() override {
    if (d_blocks) (void)hipFree(d_blocks);
    if (d_pieces) (void)hipFree(d_pieces);
  }
};

struct Cube {
  int col;
  int64_t t0, t1, x0, x1, o0, o1;
  double vol() const { return (double)(t1 - t0) * (double)(x1 - x0) * (double)(o1 - o0); }
};

int64_t gsplit(int64_t lo, int64_t hi) {
  const int64_t len = hi - lo;
  int64_t h = ((len + 1) / 2 + 63) / 64 * 64;
  if (h >= len) h = len / 2;
  return lo + h;
}

struct GapBuilder {
  GapPlan* pl;
  int part, p;
  int64_t min_piece;

  void emit_base(const std::vector<GapBlock>& L) {
    if (L.empty()) return;
    pl->launches.push_back({1, (int64_t)pl->blocks.size(), (int64_t)L.size()});
    pl->blocks.insert(pl->blocks.end(), L.begin(), L.end());
  }

  // one launch for a list of cubes, processors shared by volume.  PACO (the
  // section's rule): a cube's share pc cuts its batch into pc slabs of whole
  // rows (or columns), so every piece updates its own outputs; a batch of
  // fewer than pc also cuts each slab's outputs (64-wide quanta).  Grid
  // baseline: fixed tiles of 16 batch rows x 256 outputs, all inputs.
  void emit_cubes(const std::vector<Cube>& U) {
    if (U.empty()) return;
    double tot = 0;
    for (const Cube& c : U) tot += c.vol();
    const int64_t off = (int64_t)pl->pieces.size();
    for (const Cube& c : U) {
      ++pl->cubes;
      const int64_t T = c.t1 - c.t0, O = c.o1 - c.o0;
      if (part == PACO_PART_GRID) {
        for (int64_t t = c.t0; t < c.t1; t += 16)
          for (int64_t o = c.o0; o < c.o1; o += 256)
            pl->pieces.push_back({t, std::min(t + 16, c.t1), c.x0, c.x1, o, std::min(o + 256, c.o1), c.col, 0});
        continue;
      }
      const int64_t pc = (int64_t)std::max(1.0, std::min(std::min((double)p * c.vol() / tot, (double)p),
                                                          c.vol() / (double)min_piece));
      const int64_t slabs = std::min(pc, T);
      const int64_t ocut = std::max<int64_t>(1, std::min<int64_t>(pc / slabs, (O + 63) / 64));
      for (int64_t q = 0; q < slabs; ++q) {
        const int64_t a = c.t0 + T * q / slabs, b = c.t0 + T * (q + 1) / slabs;
        for (int64_t r = 0; r < ocut; ++r) {
          const int64_t o0 = c.o0 + (O * r / ocut) / 64 * 64;
          const int64_t o1 = r + 1 == ocut ? c.o1 : c.o0 + (O * (r + 1) / ocut) / 64 * 64;
          if (b > a && o1 > o0) pl->pieces.push_back({a, b, c.x0, c.x1, o0, o1, c.col, 0});
        }
      }
    }
    pl->launches.push_back({0, off, (int64_t)pl->pieces.size() - off});
  }

  void solve(const std::vector<GapBlock>& L) {
    if (L.empty()) return;
    std::vector<GapBlock> A, C, E, base;
    std::vector<Cube> U1, U2;
    for (const GapBlock& x : L) {
      const bool sr = x.r1 - x.r0 > GAP_B, sc = x.c1 - x.c0 > GAP_B;
      if (!sr && !sc) {
        base.push_back(x);
        continue;
      }
      const int64_t rm = sr ? gsplit(x.r0, x.r1) : x.r1;
      const int64_t cm = sc ? gsplit(x.c0, x.c1) : x.c1;
      if (sr && sc) {
        const GapBlock x00{x.r0, rm, x.c0, cm}, x01{x.r0, rm, cm, x.c1}, x10{rm, x.r1, x.c0, cm}, x11{rm, x.r1, cm, x.c1};
        A.push_back(x00);
        U1.push_back({0, x.r0, rm, x.c0, cm, cm, x.c1});   // rows of X00 -> X01
        U1.push_back({1, x.c0, cm, x.r0, rm, rm, x.r1});   // columns of X00 -> X10
        C.push_back(x01);
        C.push_back(x10);
        U2.push_back({0, rm, x.r1, x.c0, cm, cm, x.c1});   // rows of X10 -> X11
        U2.push_back({1, cm, x.c1, x.r0, rm, rm, x.r1});   // columns of X01 -> X11
        E.push_back(x11);
      } else if (sc) {
        A.push_back({x.r0, x.r1, x.c0, cm});
        U1.push_back({0, x.r0, x.r1, x.c0, cm, cm, x.c1});
        C.push_back({x.r0, x.r1, cm, x.c1});
      } else {
        A.push_back({x.r0, rm, x.c0, x.c1});
        U1.push_back({1, x.c0, x.c1, x.r0, rm, rm, x.r1});
        C.push_back({rm, x.r1, x.c0, x.c1});
      }
    }
    if (A.empty()) {   // only base blocks
      emit_base(base);
      return;
    }
    A.insert(A.end(), base.begin(), base.end());
    solve(A);
    emit_cubes(U1);
    solve(C);
    emit_cubes(U2);
    solve(E);
  }
};

void build_gap_plan(GapPlan* pl, int64_t m, int64_t n, int part, int p, int64_t min_piece) {
  GapBuilder b{pl, part, p, min_piece};
  b.solve({GapBlock{0, m + 1, 0, n + 1}});
}

bool gap_weight(const paco_weight& w, int64_t span, GapW* out) {
  if (w.a < 0 || w.b < 0) return false;
  if (w.kind == PACO_W_AFFINE) {
    if ((int64_t)w.a + (int64_t)w.b * span > G_INF64) return false;
    *out = {0u, (uint32_t)w.a, (uint32_t)w.b, w.seed};
  } else if (w.kind == PACO_W_HASH) {
    if (w.b > 29 || (int64_t)w.a + ((int64_t)1 << w.b) > G_INF64) return false;
    *out = {1u, (uint32_t)w.a, (uint32_t)(((uint64_t)1 << w.b) - 1), w.seed};
  } else {
    return false;
  }
  return true;
}

paco_status ensure_gws(paco_ctx ctx, uint64_t bytes) {
  if (bytes <= ctx->gws_bytes) return PACO_OK;
  if (bytes + ctx->ws_bytes + ctx->sws_bytes > ctx->budget) {
    set_err(ctx, "GAP problem: the transposed copy exceeds the workspace budget");
    return PACO_ERR_BUDGET;
  }
  hipError_t e;
  if (ctx->gws) {
    if ((e = hipStreamSynchronize(ctx->stream)) != hipSuccess) return hip_fail(ctx, e, "workspace sync");
    (void)hipFree(ctx->gws);
    ctx->gws = nullptr;
    ctx->gws_bytes = 0;
  }
  ctx->ws_gen += 1;
  if ((e = hipMalloc(&ctx->gws, bytes)) != hipSuccess) return hip_fail(ctx, e, "GAP workspace alloc");
  ctx->gws_bytes = bytes;
  return PACO_OK;
}

}  // namespace

extern "C" paco_status paco_gap(paco_ctx ctx, const paco_gap_desc* d, paco_gap_result* res) {
  if (!ctx) return PACO_ERR_INVALID_ARG;
  if (!d || d->m < 0 || d->n < 0 || !d->D || d->ldd < d->n + 1 || d->p < 0 || d->min_piece < 0 ||
      (d->part != PACO_PART_PACO && d->part != PACO_PART_GRID) || d->s_bits < 0 || d->s_bits > 30 ||
      d->s_match < 0 || d->s_mismatch < 0) {
    set_err(ctx, "invalid GAP-problem descriptor");
    return PACO_ERR_INVALID_ARG;
  }
  if (d->m >= ((int64_t)1 << 31) - 1 || d->n >= ((int64_t)1 << 31) - 1) {
    set_err(ctx, "GAP problem: sides too large");
    return PACO_ERR_UNSUPPORTED;
  }
  GapW wr, wc;
  if (!gap_weight(d->w_row, d->n, &wr) || !gap_weight(d->w_col, d->m, &wc) ||
      (int64_t)d->s_match > G_INF64 || (int64_t)d->s_mismatch > G_INF64) {
    set_err(ctx, "GAP problem: weights must be non-negative and at most INF = 2^30 "
                 "(affine: a + b side <= 2^30; hash: b <= 29, a + 2^b <= 2^30)");
    return PACO_ERR_UNSUPPORTED;
  }
  GapS sub{(uint32_t)d->s_match, (uint32_t)d->s_mismatch,
           (uint32_t)(d->s_bits >= 32 ? 0xFFFFFFFFull : (((uint64_t)1 << d->s_bits) - 1)), d->s_seed_x,
           d->s_seed_y, 0u};
  const int p = d->p > 0 ? d->p : 4 * ctx->num_cus;
  const int64_t min_piece = d->min_piece > 0 ? d->min_piece : 16384;
  if (res) memset(res, 0, sizeof *res);
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");
  const int64_t rows = d->m + 1, cols = d->n + 1;
  const int64_t ldt = (rows + 63) / 64 * 64;
  paco_status st = ensure_gws(ctx, (uint64_t)cols * ldt * 4);
  if (st != PACO_OK) return st;

  char key[160];
  snprintf(key, sizeof key, "gap/%lld/%lld/%d/%d/%lld", (long long)d->m, (long long)d->n, d->part, p,
           (long long)min_piece);
  GapPlan* pl = nullptr;
  auto it = ctx->plans.find(key);
  if (it != ctx->plans.end()) {
    pl = static_cast<GapPlan*>(it->second.get());
  } else {
    trim_plans(ctx);
    std::unique_ptr<GapPlan> np(new GapPlan());
    build_gap_plan(np.get(), d->m, d->n, d->part, p, min_piece);
    if (!np->blocks.empty() && (e = hipMalloc(&np->d_blocks, sizeof(GapBlock) * np->blocks.size())) != hipSuccess)
      return hip_fail(ctx, e, "GAP plan alloc");
    if (!np->pieces.empty() && (e = hipMalloc(&np->d_pieces, sizeof(GapPiece) * np->pieces.size())) != hipSuccess)
      return hip_fail(ctx, e, "GAP plan alloc");
    if (!np->blocks.empty() &&
        (e = hipMemcpy(np->d_blocks, np->blocks.data(), sizeof(GapBlock) * np->blocks.size(),
                       hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(ctx, e, "GAP plan upload");
    if (!np->pieces.empty() &&
        (e = hipMemcpy(np->d_pieces, np->pieces.data(), sizeof(GapPiece) * np->pieces.size(),
                       hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(ctx, e, "GAP plan upload");
    pl = np.get();
    ctx->plans[key] = std::move(np);
  }

  uint32_t* D = reinterpret_cast<uint32_t*>(d->D);
  uint32_t* DT = reinterpret_cast<uint32_t*>(ctx->gws);
  {
    TimeScope ts(ctx, 2);
    e = launch_gap_fill(D, d->ldd, rows, cols, ctx->stream);
  }
  for (size_t q = 0; q < pl->launches.size() && e == hipSuccess; ++q) {
    const GapLaunch& L = pl->launches[q];
    if (L.base) {
      TimeScope ts(ctx, 1);
      e = launch_gap_base(D, d->ldd, DT, ldt, pl->d_blocks + L.off, (int)L.cnt, wr, wc, sub, ctx->stream);
    } else {
      TimeScope ts(ctx, 0);
      e = launch_gap_cube(D, d->ldd, DT, ldt, pl->d_pieces + L.off, (int)L.cnt, wr, wc, ctx->stream);
    }
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "GAP launch");
  if (res) {
    res->p = p;
    res->launches = (int32_t)(pl->launches.size() + 1);
    res->base_blocks = (int64_t)pl->blocks.size();
    res->cubes = pl->cubes;
    res->pieces = (int64_t)pl->pieces.size();
  }
  return PACO_OK;
}

extern "C" paco_status paco_gap_plan_export(int64_t m, int64_t n, int32_t part, int32_t p, int32_t min_piece,
                                            int64_t* info, int64_t* launches, int64_t* blocks, int64_t* pieces) {
  if (m < 0 || n < 0 || p <= 0 || min_piece <= 0 || (part != PACO_PART_PACO && part != PACO_PART_GRID) || !info)
    return PACO_ERR_INVALID_ARG;
  GapPlan pl;
  build_gap_plan(&pl, m, n, part, p, min_piece);
  const int64_t cl = info[0], cb = info[1], cp = info[2];
  info[0] = (int64_t)pl.launches.size();
  info[1] = (int64_t)pl.blocks.size();
  info[2] = (int64_t)pl.pieces.size();
  info[3] = pl.cubes;
  if (launches) {
    if (cl < info[0]) return PACO_ERR_INVALID_ARG;
    for (size_t q = 0; q < pl.launches.size(); ++q) {
      launches[3 * q] = pl.launches[q].base;
      launches[3 * q + 1] = pl.launches[q].off;
      launches[3 * q + 2] = pl.launches[q].cnt;
    }
  }
  if (blocks) {
    if (cb < info[1]) return PACO_ERR_INVALID_ARG;
    for (size_t q = 0; q < pl.blocks.size(); ++q) {
      const GapBlock& b = pl.blocks[q];
      const int64_t row[4] = {b.r0, b.r1, b.c0, b.c1};
      memcpy(blocks + 4 * q, row, sizeof row);
    }
  }
  if (pieces) {
    if (cp < info[2]) return PACO_ERR_INVALID_ARG;
    for (size_t q = 0; q < pl.pieces.size(); ++q) {
      const GapPiece& c = pl.pieces[q];
      const int64_t row[7] = {c.col, c.t0, c.t1, c.x0, c.x1, c.o0, c.o1};
      memcpy(pieces + 7 * q, row, sizeof row);
    }
  }
  return PACO_OK;
}
