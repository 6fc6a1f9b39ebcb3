// plan.cpp -- work lists and k-cut reduction plan from partition pieces.
//
// Section "PACO MM": when a cuboid is cut on its height, the lower cuboid
// keeps the parent's output face and the upper one writes a temporary face
// of the same size; the faces are combined by (+) afterwards.  Flattened
// over the whole partition tree this means: the piece of an output element
// with the lowest k-range writes C, every other piece covering it writes
// its own temporary face, and the reduction folds the faces of each element
// in ascending k order.  The overlay of the temporary faces' rectangles cuts
// C into cells with one fixed, ordered list of faces each.
#include "plan.h"

#include <algorithm>
#include <numeric>

namespace paco {

namespace {

// The cells of one problem's temporary faces: the overlay of the faces' row
// boundaries rb and column boundaries cb; cell (r, c) lists the faces that
// cover it, in ascending k, at list[start[r * Cn + c] .. start[r * Cn + c + 1]).
// Flat arrays filled by counting: a server plans every lone request anew,
// and per-cell containers cost more than the rest of the plan.
struct Overlay {
  std::vector<int64_t> rb, cb;
  std::vector<int32_t> start, list;
  size_t R = 0, Cn = 0;
};

// Sorted distinct values of v.  A partition's faces share few boundaries
// (hundreds of values, a handful distinct): insertion into the short sorted
// list beats sorting them all; past 64 distinct values, sort.
void sorted_unique(std::vector<int64_t>& v) {
  size_t d = 0;
  for (size_t i = 0; i < v.size(); ++i) {
    const int64_t x = v[i];
    size_t at = std::lower_bound(v.begin(), v.begin() + d, x) - v.begin();
    if (at < d && v[at] == x) continue;
    if (d == 64) {
      std::sort(v.begin(), v.end());
      v.erase(std::unique(v.begin(), v.end()), v.end());
      return;
    }
    // v[i] is read already, and i >= d, so the shift only overwrites
    // values that are in the sorted prefix or done with
    for (size_t j = d; j > at; --j) v[j] = v[j - 1];
    v[at] = x;
    ++d;
  }
  v.resize(d);
}

void overlay(const std::vector<TaggedPiece>& pieces, const std::vector<int>& faces, Overlay& o) {
  o.rb.clear();
  o.cb.clear();
  for (int i : faces) {
    o.rb.push_back(pieces[i].pc.n0); o.rb.push_back(pieces[i].pc.n1);
    o.cb.push_back(pieces[i].pc.m0); o.cb.push_back(pieces[i].pc.m1);
  }
  sorted_unique(o.rb);
  sorted_unique(o.cb);
  o.R = o.rb.size() - 1;
  o.Cn = o.cb.size() - 1;
  // each face's span of cells
  std::vector<int32_t> span(4 * faces.size());
  for (size_t f = 0; f < faces.size(); ++f) {
    const Piece& p = pieces[faces[f]].pc;
    span[4 * f + 0] = (int32_t)(std::lower_bound(o.rb.begin(), o.rb.end(), p.n0) - o.rb.begin());
    span[4 * f + 1] = (int32_t)(std::lower_bound(o.rb.begin(), o.rb.end(), p.n1) - o.rb.begin());
    span[4 * f + 2] = (int32_t)(std::lower_bound(o.cb.begin(), o.cb.end(), p.m0) - o.cb.begin());
    span[4 * f + 3] = (int32_t)(std::lower_bound(o.cb.begin(), o.cb.end(), p.m1) - o.cb.begin());
  }
  o.start.assign(o.R * o.Cn + 1, 0);
  for (size_t f = 0; f < faces.size(); ++f)
    for (int32_t r = span[4 * f]; r < span[4 * f + 1]; ++r)
      for (int32_t c = span[4 * f + 2]; c < span[4 * f + 3]; ++c) o.start[r * o.Cn + c + 1] += 1;
  std::partial_sum(o.start.begin(), o.start.end(), o.start.begin());
  o.list.resize(o.start.back());
  std::vector<int32_t> pos(o.start.begin(), o.start.end() - 1);
  for (size_t f = 0; f < faces.size(); ++f)
    for (int32_t r = span[4 * f]; r < span[4 * f + 1]; ++r)
      for (int32_t c = span[4 * f + 2]; c < span[4 * f + 3]; ++c) o.list[pos[r * o.Cn + c]++] = faces[f];
  // fold order: faces covering one cell are disjoint in k, so their k0
  // differ; the lists are short (one per k-cut above the cell)
  for (size_t cell = 0; cell + 1 < o.start.size(); ++cell)
    for (int32_t a = o.start[cell] + 1; a < o.start[cell + 1]; ++a) {
      const int32_t x = o.list[a];
      const int64_t kx = pieces[x].pc.k0;
      int32_t b = a;
      for (; b > o.start[cell] && pieces[o.list[b - 1]].pc.k0 > kx; --b) o.list[b] = o.list[b - 1];
      o.list[b] = x;
    }
}

}  // namespace

HostPlan build_plan(const std::vector<TaggedPiece>& pieces, int nwg, bool xcd_remap,
                    const std::vector<ProbGeom>& geom, int64_t temp_base, int red_vec, int fuse) {
  (void)geom;
  HostPlan hp;
  hp.nwg = nwg;
  hp.xcd_remap = xcd_remap && nwg % 8 == 0;

  // temporary faces
  std::vector<int64_t> off(pieces.size(), -1);
  int64_t cur = temp_base;
  int32_t nprob = 0;
  for (size_t i = 0; i < pieces.size(); ++i) {
    const Piece& p = pieces[i].pc;
    if (p.empty()) continue;
    ++hp.n_pieces;
    int64_t v = p.vol();
    hp.vmax = std::max(hp.vmax, v);
    hp.vmin = hp.n_pieces == 1 ? v : std::min(hp.vmin, v);
    nprob = std::max(nprob, pieces[i].prob + 1);
    if (p.k0 % 4 || p.m0 % 4) hp.aligned4 = false;
    if (p.k0 > 0) {
      off[i] = cur;
      // faces start on 16-byte boundaries
      cur += ((p.n1 - p.n0) * (p.m1 - p.m0) + 3) / 4 * 4;
      ++hp.n_kcuts;
    }
  }
  hp.temp_elems = cur - temp_base;

  // items grouped by workgroup, in piece order within a workgroup
  hp.wg_off.assign(nwg + 1, 0);
  for (size_t i = 0; i < pieces.size(); ++i)
    if (!pieces[i].pc.empty()) hp.wg_off[pieces[i].wg + 1] += 1;
  std::partial_sum(hp.wg_off.begin(), hp.wg_off.end(), hp.wg_off.begin());
  std::vector<int> item_piece(hp.wg_off[nwg]);   // piece of each item
  hp.items.resize(hp.wg_off[nwg]);
  {
    std::vector<int32_t> pos(hp.wg_off.begin(), hp.wg_off.end() - 1);
    for (size_t i = 0; i < pieces.size(); ++i) {
      const Piece& p = pieces[i].pc;
      if (p.empty()) continue;
      const int32_t at = pos[pieces[i].wg]++;
      item_piece[at] = (int)i;
      WorkItem& it = hp.items[at];
      it.prob = pieces[i].prob;
      it.n0 = (int32_t)p.n0; it.n1 = (int32_t)p.n1;
      it.m0 = (int32_t)p.m0; it.m1 = (int32_t)p.m1;
      it.k0 = (int32_t)p.k0; it.k1 = (int32_t)p.k1;
      it.pad = 0;
      it.out_off = off[i];
    }
  }
  if (hp.n_kcuts == 0) return hp;
  int vec = red_vec == 4 ? 4 : 1;
  for (size_t i = 0; i < pieces.size() && vec == 4; ++i) {
    if (off[i] < 0) continue;
    const Piece& p = pieces[i].pc;
    if ((p.m1 - p.m0) % 4 || p.m0 % 4 || off[i] % 4) vec = 1;
  }
  hp.red_vec = vec;

  // reduction cells per problem, problems in ascending order
  std::vector<std::vector<int>> temps_of(nprob);
  for (size_t i = 0; i < pieces.size(); ++i)
    if (off[i] >= 0) temps_of[pieces[i].prob].push_back((int)i);
  Overlay ov;
  if (fuse == 2) {   // fused unless some cell's fold is large
    fuse = 1;
    for (const std::vector<int>& tp : temps_of) {
      if (tp.empty()) continue;
      overlay(pieces, tp, ov);
      for (size_t r = 0; r < ov.R; ++r)
        for (size_t c = 0; c < ov.Cn; ++c) {
          const int64_t ns = ov.start[r * ov.Cn + c + 1] - ov.start[r * ov.Cn + c];
          if (ns > 0 && (ov.rb[r + 1] - ov.rb[r]) * (ov.cb[c + 1] - ov.cb[c]) * (ns + 1) * 4 > kFuseCellBytes)
            fuse = 0;
        }
    }
  }
  hp.fused = fuse == 1;
  // about one tile per 1024 face elements, and the cells' sources
  hp.tiles.reserve((size_t)(hp.temp_elems / 1024) + 64);
  hp.srcs.reserve(4 * (size_t)hp.n_kcuts + 64);
  std::vector<std::vector<int32_t>> piece_cells(hp.fused ? pieces.size() : 0);
  for (int32_t prob = 0; prob < nprob; ++prob) {
    const std::vector<int>& tp = temps_of[prob];
    if (tp.empty()) continue;
    overlay(pieces, tp, ov);
    for (size_t r = 0; r < ov.R; ++r)
      for (size_t c = 0; c < ov.Cn; ++c) {
        const int32_t l0 = ov.start[r * ov.Cn + c], l1 = ov.start[r * ov.Cn + c + 1];
        if (l0 == l1) continue;
        int32_t s0 = (int32_t)hp.srcs.size();
        for (int32_t l = l0; l < l1; ++l) {
          const int i = ov.list[l];
          const Piece& p = pieces[i].pc;
          RedSrc s;
          s.off = off[i];
          s.ld = (int32_t)(p.m1 - p.m0);
          s.r0 = (int32_t)p.n0;
          s.c0 = (int32_t)p.m0;
          s.pad = 0;
          hp.srcs.push_back(s);
        }
        int32_t s1 = (int32_t)hp.srcs.size();
        int64_t i0 = ov.rb[r], i1 = ov.rb[r + 1], j0 = ov.cb[c], j1 = ov.cb[c + 1];
        if (hp.fused) {
          // one tile per cell; every piece of the problem meeting the cell
          // (its faces' pieces and the lowest-k ones writing C) counts
          const int32_t cell = (int32_t)hp.tiles.size();
          RedTile t;
          t.prob = prob;
          t.i0 = (int32_t)i0; t.i1 = (int32_t)i1;
          t.j0 = (int32_t)j0; t.j1 = (int32_t)j1;
          t.s0 = s0; t.s1 = s1; t.pad = 0;
          for (size_t i = 0; i < pieces.size(); ++i) {
            const Piece& p = pieces[i].pc;
            if (pieces[i].prob != prob || p.empty()) continue;
            if (p.n0 < i1 && p.n1 > i0 && p.m0 < j1 && p.m1 > j0) {
              piece_cells[i].push_back(cell);
              t.pad += 1;
            }
          }
          hp.tiles.push_back(t);
          continue;
        }
        // split the cell into tiles of at most 256*vec columns and about
        // 1024 elements: a 256-thread workgroup folds one or four elements
        // per thread (many workgroups: the fold is bandwidth-bound)
        int64_t cw = std::min<int64_t>(j1 - j0, 256 * vec);
        int64_t rh = std::max<int64_t>(1, 1024 / cw);
        for (int64_t ii = i0; ii < i1; ii += rh)
          for (int64_t jj = j0; jj < j1; jj += cw) {
            RedTile t;
            t.prob = prob;
            t.i0 = (int32_t)ii; t.i1 = (int32_t)std::min(i1, ii + rh);
            t.j0 = (int32_t)jj; t.j1 = (int32_t)std::min(j1, jj + cw);
            t.s0 = s0; t.s1 = s1; t.pad = 0;
            hp.tiles.push_back(t);
          }
      }
  }
  if (hp.fused) {
    hp.item_fold.assign(2 * hp.items.size(), 0);
    for (size_t it = 0; it < hp.items.size(); ++it) {
      const std::vector<int32_t>& cl = piece_cells[item_piece[it]];
      hp.item_fold[2 * it] = (int32_t)hp.fold_list.size();
      hp.item_fold[2 * it + 1] = (int32_t)cl.size();
      hp.fold_list.insert(hp.fold_list.end(), cl.begin(), cl.end());
    }
  }
  return hp;
}

}  // namespace paco
