// dp1d.cpp -- paco_dp1d: the 1D problem (section "PACO 1D") on the GPU.
//
// The host walks the recursion once per shape and keeps, in order, the
// squares with the base triangle that follows each of them, and every
// square's pieces in one device table.  A call is one fill launch (which
// ends with the first triangle) and one launch per square (which ends with
// the next triangle): see k_dp1d.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/paco.h"
#include "ctx.h"
#include "kernels.h"
#include "partition.h"

using namespace paco;

namespace {

constexpr int64_t DP_INF = (int64_t)1 << 30;

struct DpSquare {
  int64_t lo, mid, hi;   // inputs [lo, mid), outputs [mid, hi)
  int64_t off, cnt;      // its pieces in the table
  int64_t tri_lo;        // the base triangle that follows it
  int32_t tri_len;
  int32_t ntri;          // its first ntri pieces reach into that triangle
};

struct Dp1dPlan : DevPlan {
  int first_len = 0;   // the first base triangle, [0, first_len)
  std::vector<DpSquare> sq;
  std::vector<DpPiece> pieces;
  DpPiece* d_pieces = nullptr;
  uint32_t* d_cnt = nullptr;   // one launch counter per launch, zero between calls
  int64_t triangles = 0;
  int max_pieces = 0;
  int64_t atomic_pieces = 0;
  ~Dp1dPlan() override {
    if (d_pieces) (void)hipFree(d_pieces);
    if (d_cnt) (void)hipFree(d_cnt);
  }
};

// cut point of [lo, hi): half the length rounded up to a multiple of 64
int64_t split_at(int64_t lo, int64_t hi) {
  const int64_t len = hi - lo;
  int64_t h = ((len + 1) / 2 + 63) / 64 * 64;
  if (h >= len) h = len / 2;
  return lo + h;
}

struct Builder {
  Dp1dPlan* pl;
  int part, p;
  int64_t base, min_piece;
  bool pending_first = true;

  void tri(int64_t lo, int64_t hi) {
    ++pl->triangles;
    if (pending_first) {
      pl->first_len = (int)(hi - lo);
      pending_first = false;
    } else {
      pl->sq.back().tri_lo = lo;
      pl->sq.back().tri_len = (int32_t)(hi - lo);
    }
  }

  void square(int64_t lo, int64_t mid, int64_t hi) {
    const int64_t H = mid - lo, W = hi - mid;
    const double area = (double)H * (double)W;
    const int pe = (int)std::max<double>(1.0, std::min<double>(p, area / (double)min_piece));
    DpSquare s{lo, mid, hi, (int64_t)pl->pieces.size(), 0, 0, 0, 0};
    if (part == PACO_PART_GRID) {
      const int64_t strips = std::max<int64_t>(1, std::min<int64_t>(pe, W / 64));
      for (int64_t t = 0; t < strips; ++t) {
        const int64_t j0 = mid + W * t / strips / 64 * 64;
        const int64_t j1 = t + 1 == strips ? hi : mid + W * (t + 1) / strips / 64 * 64;
        if (j1 > j0) pl->pieces.push_back({lo, mid, j0, j1, 0, 0});
      }
    } else {
      // MM-1-Piece on the 1 x W x H cuboid: m = outputs (quantum 64, one
      // wave's lanes), k = inputs (quantum 8); ties cut the outputs
      PartOpts po;
      po.p = pe;
      po.q[0] = 1; po.q[1] = 64; po.q[2] = 8;
      po.kcut_cost = 1.0;
      for (const Piece& pc : partition_mm1(1, W, H, po)) {
        if (pc.empty()) continue;
        const int at = (pc.k1 - pc.k0) < H ? 1 : 0;
        pl->atomic_pieces += at;
        pl->pieces.push_back({lo + pc.k0, lo + pc.k1, mid + pc.m0, mid + pc.m1, at, 0});
      }
    }
    s.cnt = (int64_t)pl->pieces.size() - s.off;
    pl->max_pieces = std::max<int>(pl->max_pieces, (int)s.cnt);
    pl->sq.push_back(s);
  }

  // each square's pieces that reach into the base triangle after it go
  // first (the triangle waits for those only)
  void order_pieces() {
    for (DpSquare& s : pl->sq) {
      const int64_t end = s.tri_lo + s.tri_len;
      auto b = pl->pieces.begin() + s.off;
      auto mid = std::stable_partition(b, b + s.cnt, [end](const DpPiece& c) { return c.j0 < end; });
      s.ntri = (int32_t)(mid - b);
    }
  }

  // in order: left half, its square, right half; a square is always
  // followed by a base triangle (the first leaf of its right half)
  void rec(int64_t lo, int64_t hi) {
    if (hi - lo <= base) {
      tri(lo, hi);
      return;
    }
    const int64_t mid = split_at(lo, hi);
    rec(lo, mid);
    square(lo, mid, hi);
    rec(mid, hi);
  }
};

}  // namespace

extern "C" paco_status paco_dp1d(paco_ctx ctx, const paco_dp1d_desc* d, paco_dp1d_result* res) {
  if (!ctx) return PACO_ERR_INVALID_ARG;
  if (!d || d->n < 0 || !d->D || d->a < 0 || d->b < 0 || d->p < 0 || d->base < 0 || d->min_piece < 0 ||
      (d->part != PACO_PART_PACO && d->part != PACO_PART_GRID) ||
      (d->w_kind != PACO_W_AFFINE && d->w_kind != PACO_W_HASH)) {
    set_err(ctx, "invalid 1D-problem descriptor");
    return PACO_ERR_INVALID_ARG;
  }
  if (d->base != 0 && (d->base < 64 || d->base > DP_TRI_MAX)) {
    set_err(ctx, "1D problem: base must lie in 64..1024");
    return PACO_ERR_INVALID_ARG;
  }
  if (d->n >= ((int64_t)1 << 31) - 1) {
    set_err(ctx, "1D problem: n too large");
    return PACO_ERR_UNSUPPORTED;
  }
  if (d->w_kind == PACO_W_AFFINE ? (int64_t)d->a + (int64_t)d->b * d->n > DP_INF
                                 : (d->b > 29 || (int64_t)d->a + ((int64_t)1 << d->b) > DP_INF)) {
    set_err(ctx, "1D problem: weights exceed INF = 2^30 (affine: a + b n <= 2^30; hash: b <= 29, a + 2^b <= 2^30)");
    return PACO_ERR_UNSUPPORTED;
  }
  const int p = d->p > 0 ? d->p : 4 * ctx->num_cus;
  const int64_t base = d->base > 0 ? d->base : 512;
  const int64_t min_piece = d->min_piece > 0 ? d->min_piece : 65536;
  if (res) memset(res, 0, sizeof *res);
  if (d->n == 0) {
    if (res) res->p = p;
    return PACO_OK;
  }
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(ctx, e, "hipSetDevice");

  char key[160];
  snprintf(key, sizeof key, "dp1d/%lld/%d/%d/%lld/%lld", (long long)d->n, d->part, p, (long long)base,
           (long long)min_piece);
  Dp1dPlan* pl = nullptr;
  auto it = ctx->plans.find(key);
  if (it != ctx->plans.end()) {
    pl = static_cast<Dp1dPlan*>(it->second.get());
  } else {
    trim_plans(ctx);
    std::unique_ptr<Dp1dPlan> np(new Dp1dPlan());
    Builder b{np.get(), d->part, p, base, min_piece};
    b.rec(0, d->n + 1);
    b.order_pieces();
    const size_t nc = np->sq.size() + 1;
    if (!np->pieces.empty() &&
        (e = hipMalloc(&np->d_pieces, sizeof(DpPiece) * np->pieces.size())) != hipSuccess)
      return hip_fail(ctx, e, "1D plan alloc");
    if ((e = hipMalloc(&np->d_cnt, sizeof(uint32_t) * nc)) != hipSuccess) return hip_fail(ctx, e, "1D plan alloc");
    if (!np->pieces.empty() &&
        (e = hipMemcpy(np->d_pieces, np->pieces.data(), sizeof(DpPiece) * np->pieces.size(),
                       hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(ctx, e, "1D plan upload");
    if ((e = hipMemset(np->d_cnt, 0, sizeof(uint32_t) * nc)) != hipSuccess) return hip_fail(ctx, e, "1D plan counters");
    pl = np.get();
    ctx->plans[key] = std::move(np);
  }

  DpW w;
  w.a = (uint32_t)d->a;
  w.b = d->w_kind == PACO_W_AFFINE ? (uint32_t)d->b : (uint32_t)(((uint64_t)1 << d->b) - 1);
  w.seed = d->seed;
  w.pad = 0;
  uint32_t* D = reinterpret_cast<uint32_t*>(d->D);
  const int wk = d->w_kind;
  {
    TimeScope ts(ctx, 2);
    e = launch_dp1d_fill(wk, D, d->n, pl->d_cnt, pl->first_len, w, ctx->stream);
  }
  for (size_t q = 0; q < pl->sq.size() && e == hipSuccess; ++q) {
    const DpSquare& s = pl->sq[q];
    TimeScope ts(ctx, 0);
    e = launch_dp1d_rect(wk, D, pl->d_pieces + s.off, (int)s.cnt, s.ntri, pl->d_cnt + q + 1, s.tri_lo, s.tri_len,
                         w, ctx->stream);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "1D launch");
  if (res) {
    res->p = p;
    res->launches = (int32_t)(pl->sq.size() + 1);
    res->triangles = pl->triangles;
    res->squares = (int64_t)pl->sq.size();
    res->pieces = (int64_t)pl->pieces.size();
    res->max_pieces = pl->max_pieces;
    res->atomic_pieces = (int32_t)pl->atomic_pieces;
  }
  return PACO_OK;
}

extern "C" paco_status paco_dp1d_plan_export(int64_t n, int32_t part, int32_t p, int32_t base, int32_t min_piece,
                                             int64_t* info, int64_t* squares, int64_t* pieces) {
  if (n < 0 || p <= 0 || base < 64 || base > DP_TRI_MAX || min_piece <= 0 ||
      (part != PACO_PART_PACO && part != PACO_PART_GRID) || !info)
    return PACO_ERR_INVALID_ARG;
  Dp1dPlan pl;
  if (n > 0) {
    Builder b{&pl, part, p, base, min_piece};
    b.rec(0, n + 1);
    b.order_pieces();
  }
  const int64_t cap_sq = info[0], cap_pc = info[1];
  info[0] = (int64_t)pl.sq.size();
  info[1] = (int64_t)pl.pieces.size();
  info[2] = pl.first_len;
  info[3] = pl.triangles;
  if (squares) {
    if (cap_sq < (int64_t)pl.sq.size()) return PACO_ERR_INVALID_ARG;
    for (size_t q = 0; q < pl.sq.size(); ++q) {
      const DpSquare& s = pl.sq[q];
      const int64_t row[8] = {s.lo, s.mid, s.hi, s.off, s.cnt, s.tri_lo, s.tri_len, s.ntri};
      memcpy(squares + 8 * q, row, sizeof row);
    }
  }
  if (pieces) {
    if (cap_pc < (int64_t)pl.pieces.size()) return PACO_ERR_INVALID_ARG;
    for (size_t q = 0; q < pl.pieces.size(); ++q) {
      const DpPiece& c = pl.pieces[q];
      const int64_t row[5] = {c.i0, c.i1, c.j0, c.j1, c.atomic};
      memcpy(pieces + 5 * q, row, sizeof row);
    }
  }
  return PACO_OK;
}

