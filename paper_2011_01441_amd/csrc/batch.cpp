// batch.cpp -- processor split over a batch of requests.
//
// The heterogeneous variant of the experiments section cuts a cuboid in the
// ratio of the summed throughputs of the two halves of the processor list.
// For a batch the roles are mirrored: the processors are identical and the
// work is a list of independent cuboids, so the list is cut into two parts
// of about equal work and the processors in the ratio of the parts' work;
// this recursion ends in single requests, each then split by MM-1-Piece
// over its own processors (contiguous, so siblings share an XCD).
#include "batch.h"

#include <algorithm>
#include <cmath>

#include "ctx.h"
#include "device_types.h"
#include "kernels.h"

namespace paco {

int batch_group(const BatchReq& r) {
  switch (r.sr) {
    case 0: return r.prec == PREC_FP32 ? G_RING_FP32 : (r.prec == PREC_BF16X6 ? G_RING_X6 : G_RING_X3);
    case 1: return G_MINPLUS;
    case 2: return G_MAXPLUS;
    default: return G_BOOL;
  }
}

double batch_weight(const BatchReq& r) {
  // time per (i, j, l) relative to bf16x3 on matrix cores: bf16x6 issues
  // twice the products, float32 matrix cores run at about a fifth of the
  // bf16x3 rate, an int32 (min,+)/(max,+) pair costs 1.5 VALU lane-ops, a
  // boolean pair 1/32 of a word and-or.  The (min,+) weight is measured on
  // the server's mixed batches: one batch of the 4096 benchmark requests
  // took 193.5 ms at 10, 151.5 at 13 and 164.8 at 15
  static const double cost[G_COUNT] = {5.3, 1.0, 2.0, 13.0, 13.0, 0.35};
  const double fixed = 4.0e6;  // one tile pass of latency, whatever the size
  return (double)r.n * (double)r.m * (double)r.k * cost[batch_group(r)] + fixed;
}

namespace {

void split_rec(const std::vector<BatchReq>& reqs, const std::vector<int>& ids, size_t a, size_t b, int p0, int p1,
               const std::vector<double>& w, int tile, std::vector<TaggedPiece>& out) {
  if (b <= a) return;
  const int P = p1 - p0;
  if (b - a == 1 || P == 1) {
    if (b - a == 1 && P > 1) {
      const BatchReq& r = reqs[ids[a]];
      PartOpts po;
      po.p = P;
      po.kcut_cost = default_kcut_cost(r.sr);
      const int g = batch_group(r);
      if (g == G_BOOL) { po.q[0] = 1; po.q[1] = 32; po.q[2] = 32; }
      if (g == G_MINPLUS || g == G_MAXPLUS) { po.q[1] = 4; po.q[2] = 4; }   // 128-bit loads (as a call's plan)
      std::vector<Piece> pcs;
      if (g <= G_RING_X6 && tile >= 0) {
        int t = tile;
        pcs = ring_partition(r.n, r.m, r.k, P, r.prec, po.kcut_cost, nullptr, tile, &t, 2e-4);
      } else {
        pcs = partition_mm1(r.n, r.m, r.k, po);
      }
      for (Piece& pc : pcs) {
        if (pc.empty()) continue;
        TaggedPiece t{pc, ids[a], p0 + pc.proc};
        out.push_back(t);
      }
    } else {
      for (size_t i = a; i < b; ++i) {
        const BatchReq& r = reqs[ids[i]];
        if (r.n == 0 || r.m == 0 || r.k == 0) continue;
        Piece pc;
        pc.n0 = 0; pc.n1 = r.n; pc.m0 = 0; pc.m1 = r.m; pc.k0 = 0; pc.k1 = r.k;
        pc.proc = 0; pc.round = 0; pc.depth = 0;
        out.push_back({pc, ids[i], p0});
      }
    }
    return;
  }
  double tot = 0;
  for (size_t i = a; i < b; ++i) tot += w[ids[i]];
  // split point: prefix weight closest to half
  double acc = 0;
  size_t c = a + 1;
  double best = 1e300;
  for (size_t i = a; i + 1 < b; ++i) {
    acc += w[ids[i]];
    double d = std::fabs(acc - tot / 2);
    if (d < best) {
      best = d;
      c = i + 1;
    }
  }
  double wl = 0;
  for (size_t i = a; i < c; ++i) wl += w[ids[i]];
  int pl = (int)std::llround(P * wl / tot);
  pl = std::min(std::max(pl, 1), P - 1);
  split_rec(reqs, ids, a, c, p0, p0 + pl, w, tile, out);
  split_rec(reqs, ids, c, b, p0 + pl, p1, w, tile, out);
}

// Tile of a ring group: the shape whose padded work over the group's
// requests (each whole, n and m rounded up to the tile, weighted by the
// tile's relative cost per element) is least.
int group_ring_tile(const std::vector<BatchReq>& reqs, const std::vector<int>& ids, int prec) {
  const int cand[4] = {RING_T256x256, RING_T256x128, RING_T128x128, RING_T128x64};
  const double eff[4] = {1.0, 1.1, 1.25, 1.6};
  int best = RING_T256x128;
  double bestc = 1e300;
  for (int c = 0; c < 4; ++c) {
    if (cand[c] == RING_T256x256 && prec == PREC_BF16X6) continue;
    const RingTileShape ts = ring_tile_shape(cand[c], prec);
    double tot = 0;
    for (int i : ids) {
      const BatchReq& r = reqs[i];
      tot += (double)((r.n + ts.tm - 1) / ts.tm * ts.tm) * (double)((r.m + ts.tn - 1) / ts.tn * ts.tn) *
             (double)r.k * eff[c];
    }
    if (tot < bestc) {
      bestc = tot;
      best = cand[c];
    }
  }
  return best;
}

}  // namespace

BatchSplit batch_partition(const std::vector<BatchReq>& reqs, int p) {
  BatchSplit bs;
  std::vector<double> w(reqs.size());
  double gw[G_COUNT] = {0};
  std::vector<int> ids[G_COUNT];
  for (size_t i = 0; i < reqs.size(); ++i) {
    w[i] = batch_weight(reqs[i]);
    int g = batch_group(reqs[i]);
    gw[g] += w[i];
    ids[g].push_back((int)i);
  }
  double tot = 0;
  int ng = 0;
  for (int g = 0; g < G_COUNT; ++g)
    if (!ids[g].empty()) {
      tot += gw[g];
      ++ng;
    }
  // largest remainder with a floor of one processor per non-empty group
  int cnt[G_COUNT] = {0};
  if (ng > 0) {
    int left = p;
    double rem[G_COUNT] = {0};
    for (int g = 0; g < G_COUNT; ++g) {
      if (ids[g].empty()) continue;
      double share = p * gw[g] / tot;
      cnt[g] = std::max(1, (int)std::floor(share));
      rem[g] = share - std::floor(share);
      left -= cnt[g];
    }
    while (left > 0) {
      int best = -1;
      for (int g = 0; g < G_COUNT; ++g)
        if (!ids[g].empty() && (best < 0 || rem[g] > rem[best])) best = g;
      cnt[best] += 1;
      rem[best] = -1;
      left -= 1;
    }
    while (left < 0) {  // more groups than processors: take from the largest
      int best = -1;
      for (int g = 0; g < G_COUNT; ++g)
        if (cnt[g] > 1 && (best < 0 || cnt[g] > cnt[best])) best = g;
      if (best < 0) break;
      cnt[best] -= 1;
      left += 1;
    }
  }
  int cur = 0;
  for (int g = 0; g < G_COUNT; ++g) {
    bs.g0[g] = cur;
    bs.tile[g] = -1;
    if (!ids[g].empty()) {
      if (g <= G_RING_X6)
        bs.tile[g] = group_ring_tile(reqs, ids[g], g == G_RING_FP32 ? PREC_FP32 : (g == G_RING_X3 ? PREC_BF16X3
                                                                                                   : PREC_BF16X6));
      split_rec(reqs, ids[g], 0, ids[g].size(), cur, cur + cnt[g], w, bs.tile[g], bs.pieces);
      cur += cnt[g];
    }
    bs.g1[g] = cur;
  }
  return bs;
}

}  // namespace paco
