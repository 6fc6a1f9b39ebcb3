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
// On a kernel's tile grid (tile_balance) the quanta are whole tiles and
// the dimension of each ratio cut is searched for (TileSearch below): the
// paper's bounds assume cuts at any position, while a tile kernel pads
// every partial tile, and the padding of one uneven cut compounds down the
// tree.
#include "partition.h"

#include <algorithm>
#include <cmath>
#include <deque>
#include <unordered_map>

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
  int pl = P / 2;
  double wl = wprefix[p0 + pl] - wprefix[p0];
  double wa = wprefix[p1] - wprefix[p0];
  double f = wa > 0 ? wl / wa : (double)pl / (double)P;
  int d = pick_dim(v, b, o.q, o.kcut_cost);
  int64_t c = cut_offset(b.len(d), f, o.q[d]);
  Box l = b, r = b;
  l.hi[d] = b.lo[d] + c;
  r.lo[d] = b.lo[d] + c;
  double vh[3] = {v[0], v[1], v[2]};
  vh[d] = v[d] / 2.0;
  mm1_rec(l, vh, p0, p0 + pl, depth + 1, o, wprefix, out);
  mm1_rec(r, vh, p0 + pl, p1, depth + 1, o, wprefix, out);
}

// MM-1-Piece on a tile grid.  The recursion is the paper's (cut in the
// processor ratio, recurse on both halves), but the cut dimension is found
// by a search: cost(box, P, face) is the busiest processor's cost below
// the box, min over cuttable dimensions of max(cost(left), cost(right)).
// Cut positions depend only on the lengths and P, so the search is memoised
// on (lengths, P, whether the box starts above k = 0, i.e. writes faces).
// Ties (within 0.1%) keep the paper's choice.  Processor weights make each
// subrange's ratio differ, so the search is keyed on the first processor
// too.
struct TileSearch {
  const PartOpts& o;
  const std::vector<double>& wprefix;
  int64_t tn, tm;
  struct Key {
    int64_t len[3];
    int p0, P;
    bool face;
    bool operator==(const Key& b) const {
      return len[0] == b.len[0] && len[1] == b.len[1] && len[2] == b.len[2] && p0 == b.p0 && P == b.P &&
             face == b.face;
    }
  };
  struct KeyHash {
    size_t operator()(const Key& k) const {
      uint64_t h = 1469598103934665603ull;
      auto mix = [&](uint64_t v) { h = (h ^ v) * 1099511628211ull; };
      mix((uint64_t)k.len[0]); mix((uint64_t)k.len[1]); mix((uint64_t)k.len[2]);
      mix((uint64_t)(uint32_t)k.p0 << 32 | (uint32_t)k.P); mix(k.face);
      return (size_t)h;
    }
  };
  std::unordered_map<Key, std::pair<double, int>, KeyHash> memo;

  double leaf(const int64_t len[3], bool face, int p0) const {
    if (len[0] <= 0 || len[1] <= 0 || len[2] <= 0) return 0.0;
    const double tiles = (double)((len[0] + tn - 1) / tn) * (double)((len[1] + tm - 1) / tm);
    const double kk = (double)((len[2] + o.q[2] - 1) / o.q[2] * o.q[2]);
    const double w = o.weights ? o.weights[p0] : 1.0;
    return tiles * (double)tn * (double)tm * (kk + o.tile_k_ovh + (face ? o.tile_face : 0.0)) / w;
  }
  double frac(int p0, int P) const {
    const int pl = P / 2;
    const double wl = wprefix[p0 + pl] - wprefix[p0], wa = wprefix[p0 + P] - wprefix[p0];
    return wa > 0 ? wl / wa : (double)pl / (double)P;
  }
  // (cost, dimension) of the best cut of a box with these lengths
  std::pair<double, int> solve(const int64_t len[3], const double v[3], int p0, int P, bool face) {
    if (P == 1) return {leaf(len, face, p0), -1};
    Key key{{len[0], len[1], len[2]}, o.weights ? p0 : 0, P, face};
    auto it = memo.find(key);
    if (it != memo.end()) return it->second;
    Box b{{0, 0, 0}, {len[0], len[1], len[2]}};
    const int d0 = pick_dim(v, b, o.q, o.kcut_cost);
    const double f = frac(p0, P);
    const int pl = P / 2;
    std::pair<double, int> best{1e300, d0};
    for (int pass = 0; pass < 2; ++pass) {
      for (int d = 0; d < 3; ++d) {
        if ((pass == 0) != (d == d0)) continue;   // the paper's choice first
        if (d != d0 && len[d] < 2 * o.q[d]) continue;
        const int64_t c = cut_offset(len[d], f, o.q[d]);
        int64_t ll[3] = {len[0], len[1], len[2]}, lr[3] = {len[0], len[1], len[2]};
        ll[d] = c;
        lr[d] = len[d] - c;
        double vh[3] = {v[0], v[1], v[2]};
        vh[d] = v[d] / 2.0;
        const double cl = solve(ll, vh, p0, pl, face).first;
        const double cr = solve(lr, vh, p0 + pl, P - pl, face || (d == 2 && c > 0)).first;
        const double cst = std::max(cl, cr);
        if (cst < best.first * (1.0 - 1e-3)) best = {cst, d};
      }
    }
    memo[key] = best;
    return best;
  }
  void build(const Box& b, const double v[3], int p0, int P, int depth, std::vector<Piece>& out) {
    if (P == 1) {
      out.push_back(make_piece(b, p0, 0, depth));
      return;
    }
    const int64_t len[3] = {b.len(0), b.len(1), b.len(2)};
    const int d = solve(len, v, p0, P, b.lo[2] > 0).second;
    const int pl = P / 2;
    const int64_t c = cut_offset(b.len(d), frac(p0, P), o.q[d]);
    Box l = b, r = b;
    l.hi[d] = b.lo[d] + c;
    r.lo[d] = b.lo[d] + c;
    double vh[3] = {v[0], v[1], v[2]};
    vh[d] = v[d] / 2.0;
    build(l, vh, p0, pl, depth + 1, out);
    build(r, vh, p0 + pl, P - pl, depth + 1, out);
  }
};

}  // namespace

std::vector<Piece> partition_mm1(int64_t n, int64_t m, int64_t k, const PartOpts& o) {
  std::vector<Piece> out;
  out.reserve(o.p);
  std::vector<double> wprefix(o.p + 1, 0.0);
  for (int i = 0; i < o.p; ++i) wprefix[i + 1] = wprefix[i] + (o.weights ? o.weights[i] : 1.0);
  Box b{{0, 0, 0}, {n, m, k}};
  double v[3] = {(double)n, (double)m, (double)k};
  if (o.tile_balance) {
    TileSearch ts{o, wprefix, o.tile_n > 0 ? o.tile_n : o.q[0], o.tile_m > 0 ? o.tile_m : o.q[1], {}};
    ts.build(b, v, 0, o.p, 0, out);
    return out;
  }
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
