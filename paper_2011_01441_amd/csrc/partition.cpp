// partition.cpp -- PACO partitioning of the MM iteration cuboid.
//
// Section "PACO MM": the n-by-m-by-k cuboid has A and B as side faces and C
// as bottom face; a processor's share is a sub-cuboid.  Two schemes:
//  * MM-1-Piece (corollary mm-1-piece): cut the longest dimension in the
//    ratio floor(p/2):ceil(p/2), split the processor list the same way,
//    recurse until one processor is left.  The dimension is chosen on a
//    same-sized virtual cuboid that is always halved evenly, so the order of
//    cut dimensions is the one of the multi-piece scheme.  With processor
//    throughputs (the heterogeneous variant of the experiments section) the
//    ratio is the two halves' summed throughput instead of their counts.
//  * Multi-piece pruned BFS (theorem mm, figure of the pruned BFS): cut all
//    unassigned cuboids of a depth evenly; once a depth holds >= p of them,
//    the first p in BFS order go to processors 0..p-1 and the rest go on;
//    cuboids that can no longer be cut are dealt out round-robin.
// Readings where the paper is silent: ties among equally long dimensions go
// n, then m, then k (a k-cut costs a temporary face); cuts land on multiples
// of a per-dimension quantum, rounded to nearest; a dimension shorter than
// two quanta is not cut while another one can be.  An optional k-cut cost
// divides k's virtual length in that choice (1 keeps the paper's rule).
#include "partition.h"

#include <algorithm>
#include <cmath>
#include <deque>

namespace paco {

namespace {

struct Box {
  int64_t lo[3], hi[3];
  int64_t len(int d) const { return hi[d] - lo[d]; }
};

// Longest virtual dimension (ties n, m, k) among those whose real length
// still allows a cut on the quantum grid; if none does, the longest one.
int pick_dim(const double v_in[3], const Box& b, const int64_t q[3], double kcost) {
  const double v[3] = {v_in[0], v_in[1], v_in[2] / kcost};
  int best = -1;
  for (int d = 0; d < 3; ++d) {
    if (b.len(d) < 2 * q[d]) continue;
    if (best < 0 || v[d] > v[best]) best = d;
  }
  if (best >= 0) return best;
  best = 0;
  for (int d = 1; d < 3; ++d)
    if (v[d] > v[best]) best = d;
  return best;
}

// Offset of a cut giving fraction f of length L to the left part, on the
// quantum grid q, keeping both parts non-empty when L allows it.
int64_t cut_offset(int64_t L, double f, int64_t q) {
  if (L <= 0) return 0;
  if (L < 2 * q) return f >= 0.5 ? L : 0;  // no cut on the grid: one side gets all
  int64_t c = q * (int64_t)std::llround(((double)L * f) / (double)q);
  int64_t cmax = q * ((L - 1) / q);
  return std::min(std::max(c, q), cmax);
}

Piece make_piece(const Box& b, int proc, int round, int depth) {
  Piece p;
  p.n0 = b.lo[0]; p.n1 = b.hi[0];
  p.m0 = b.lo[1]; p.m1 = b.hi[1];
  p.k0 = b.lo[2]; p.k1 = b.hi[2];
  p.proc = proc; p.round = round; p.depth = depth;
  return p;
}

void mm1_rec(const Box& b, const double v[3], int p0, int p1, int depth, const PartOpts& o,
             const std::vector<double>& wprefix, std::vector<Piece>& out) {
  int P = p1 - p0;
  if (P == 1) {
    out.push_back(make_piece(b, p0, 0, depth));
    return;
  }
  int d = pick_dim(v, b, o.q, o.kcut_cost);
  int pl = P / 2;
  double wl = wprefix[p0 + pl] - wprefix[p0];
  double wa = wprefix[p1] - wprefix[p0];
  double f = wa > 0 ? wl / wa : (double)pl / (double)P;
  int64_t c = cut_offset(b.len(d), f, o.q[d]);
  Box l = b, r = b;
  l.hi[d] = b.lo[d] + c;
  r.lo[d] = b.lo[d] + c;
  double vh[3] = {v[0], v[1], v[2]};
  vh[d] = v[d] / 2.0;
  mm1_rec(l, vh, p0, p0 + pl, depth + 1, o, wprefix, out);
  mm1_rec(r, vh, p0 + pl, p1, depth + 1, o, wprefix, out);
}

}  // namespace

std::vector<Piece> partition_mm1(int64_t n, int64_t m, int64_t k, const PartOpts& o) {
  std::vector<Piece> out;
  out.reserve(o.p);
  std::vector<double> wprefix(o.p + 1, 0.0);
  for (int i = 0; i < o.p; ++i) wprefix[i + 1] = wprefix[i] + (o.weights ? o.weights[i] : 1.0);
  Box b{{0, 0, 0}, {n, m, k}};
  double v[3] = {(double)n, (double)m, (double)k};
  mm1_rec(b, v, 0, o.p, 0, o, wprefix, out);
  return out;
}

std::vector<Piece> partition_multi(int64_t n, int64_t m, int64_t k, const PartOpts& o) {
  std::vector<Piece> out;
  struct Node { Box b; int depth; };
  std::vector<Node> level{{Box{{0, 0, 0}, {n, m, k}}, 0}};
  int round = 0;
  while (!level.empty()) {
    if ((int64_t)level.size() >= o.p) {
      for (int j = 0; j < o.p; ++j) out.push_back(make_piece(level[j].b, j, round, level[j].depth));
      level.erase(level.begin(), level.begin() + o.p);
      ++round;
      if (level.empty()) break;
      if (o.max_rounds > 0 && round >= o.max_rounds) {   // the rest round-robin
        for (size_t j = 0; j < level.size(); ++j)
          out.push_back(make_piece(level[j].b, (int)(j % o.p), round, level[j].depth));
        break;
      }
    }
    bool any_cuttable = false;
    for (const Node& nd : level)
      for (int d = 0; d < 3; ++d)
        if (nd.b.len(d) >= 2 * o.q[d]) any_cuttable = true;
    if (!any_cuttable) {  // base cases: round-robin
      for (size_t j = 0; j < level.size(); ++j)
        out.push_back(make_piece(level[j].b, (int)(j % o.p), round, level[j].depth));
      break;
    }
    std::vector<Node> next;
    next.reserve(level.size() * 2);
    for (const Node& nd : level) {
      // even division of the longest side (the cuboid's own dimensions)
      double v[3] = {(double)nd.b.len(0), (double)nd.b.len(1), (double)nd.b.len(2)};
      int d = pick_dim(v, nd.b, o.q, o.kcut_cost);
      if (nd.b.len(d) < 2 * o.q[d]) {  // this one is a base case already
        next.push_back({nd.b, nd.depth});
        continue;
      }
      int64_t c = cut_offset(nd.b.len(d), 0.5, o.q[d]);
      Node l = nd, r = nd;
      l.b.hi[d] = nd.b.lo[d] + c;
      r.b.lo[d] = nd.b.lo[d] + c;
      l.depth = r.depth = nd.depth + 1;
      next.push_back(l);
      next.push_back(r);
    }
    level.swap(next);
  }
  return out;
}

std::vector<Piece> partition_grid(int64_t n, int64_t m, int64_t k, int64_t tm, int64_t tn,
                                  int64_t bk, int split_k) {
  std::vector<Piece> out;
  int64_t kb = (k + bk - 1) / bk;  // k blocks
  int s = std::max(1, (int)std::min<int64_t>(split_k, std::max<int64_t>(kb, 1)));
  int proc = 0;
  for (int64_t i = 0; i < n; i += tm)
    for (int64_t j = 0; j < m; j += tn)
      for (int t = 0; t < s; ++t) {
        int64_t kb0 = kb * t / s, kb1 = kb * (t + 1) / s;
        Box b{{i, j, std::min(k, kb0 * bk)}, {std::min(n, i + tm), std::min(m, j + tn), std::min(k, kb1 * bk)}};
        out.push_back(make_piece(b, proc++, 0, 0));
      }
  return out;
}

}  // namespace paco
