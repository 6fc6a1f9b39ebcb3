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
#include <map>

namespace paco {

HostPlan build_plan(const std::vector<TaggedPiece>& pieces, int nwg, bool xcd_remap,
                    const std::vector<ProbGeom>& geom, int64_t temp_base, int red_vec, int fuse) {
  HostPlan hp;
  hp.nwg = nwg;
  hp.xcd_remap = xcd_remap && nwg % 8 == 0;

  // items grouped by workgroup, in piece order within a workgroup
  std::vector<std::vector<int>> by_wg(nwg);
  for (size_t i = 0; i < pieces.size(); ++i)
    if (!pieces[i].pc.empty()) by_wg[pieces[i].wg].push_back((int)i);

  // temporary faces
  std::vector<int64_t> off(pieces.size(), -1);
  int64_t cur = temp_base;
  for (size_t i = 0; i < pieces.size(); ++i) {
    const Piece& p = pieces[i].pc;
    if (p.empty()) continue;
    ++hp.n_pieces;
    int64_t v = p.vol();
    hp.vmax = std::max(hp.vmax, v);
    hp.vmin = hp.n_pieces == 1 ? v : std::min(hp.vmin, v);
    if (p.k0 > 0) {
      off[i] = cur;
      // faces start on 16-byte boundaries
      cur += ((p.n1 - p.n0) * (p.m1 - p.m0) + 3) / 4 * 4;
      ++hp.n_kcuts;
    }
  }
  hp.temp_elems = cur - temp_base;

  std::vector<int> item_piece;   // piece of each item
  hp.wg_off.assign(nwg + 1, 0);
  for (int w = 0; w < nwg; ++w) {
    hp.wg_off[w] = (int32_t)hp.items.size();
    for (int i : by_wg[w]) {
      item_piece.push_back(i);
      const Piece& p = pieces[i].pc;
      WorkItem it;
      it.prob = pieces[i].prob;
      it.n0 = (int32_t)p.n0; it.n1 = (int32_t)p.n1;
      it.m0 = (int32_t)p.m0; it.m1 = (int32_t)p.m1;
      it.k0 = (int32_t)p.k0; it.k1 = (int32_t)p.k1;
      it.pad = 0;
      it.out_off = off[i];
      hp.items.push_back(it);
    }
  }
  hp.wg_off[nwg] = (int32_t)hp.items.size();
  if (hp.n_kcuts == 0) return hp;
  int vec = red_vec == 4 ? 4 : 1;
  for (size_t i = 0; i < pieces.size() && vec == 4; ++i) {
    if (off[i] < 0) continue;
    const Piece& p = pieces[i].pc;
    if ((p.m1 - p.m0) % 4 || p.m0 % 4 || off[i] % 4) vec = 1;
  }
  hp.red_vec = vec;

  // reduction cells per problem
  std::map<int, std::vector<int>> temps_of;  // prob -> temp piece indices
  for (size_t i = 0; i < pieces.size(); ++i)
    if (off[i] >= 0) temps_of[pieces[i].prob].push_back((int)i);
  if (fuse == 2) {   // fused unless some cell's fold is large
    fuse = 1;
    for (auto& kv : temps_of) {
      std::vector<int64_t> rb, cb;
      for (int i : kv.second) {
        rb.push_back(pieces[i].pc.n0); rb.push_back(pieces[i].pc.n1);
        cb.push_back(pieces[i].pc.m0); cb.push_back(pieces[i].pc.m1);
      }
      std::sort(rb.begin(), rb.end()); rb.erase(std::unique(rb.begin(), rb.end()), rb.end());
      std::sort(cb.begin(), cb.end()); cb.erase(std::unique(cb.begin(), cb.end()), cb.end());
      const size_t Cn = cb.size() - 1;
      std::vector<int64_t> nsrc((rb.size() - 1) * Cn, 0);
      for (int i : kv.second) {
        const Piece& p = pieces[i].pc;
        size_t r0 = std::lower_bound(rb.begin(), rb.end(), p.n0) - rb.begin();
        size_t r1 = std::lower_bound(rb.begin(), rb.end(), p.n1) - rb.begin();
        size_t c0 = std::lower_bound(cb.begin(), cb.end(), p.m0) - cb.begin();
        size_t c1 = std::lower_bound(cb.begin(), cb.end(), p.m1) - cb.begin();
        for (size_t r = r0; r < r1; ++r)
          for (size_t c = c0; c < c1; ++c) nsrc[r * Cn + c] += 1;
      }
      for (size_t r = 0; r + 1 < rb.size(); ++r)
        for (size_t c = 0; c < Cn; ++c)
          if (nsrc[r * Cn + c] > 0 &&
              (rb[r + 1] - rb[r]) * (cb[c + 1] - cb[c]) * (nsrc[r * Cn + c] + 1) * 4 > kFuseCellBytes)
            fuse = 0;
    }
  }
  hp.fused = fuse == 1;
  // about one tile per 1024 face elements, and the cells' sources
  hp.tiles.reserve((size_t)(hp.temp_elems / 1024) + 64);
  hp.srcs.reserve(4 * (size_t)hp.n_kcuts + 64);
  std::vector<std::vector<int32_t>> piece_cells(hp.fused ? pieces.size() : 0);
  for (auto& kv : temps_of) {
    const int prob = kv.first;
    const std::vector<int>& tp = kv.second;
    std::vector<int64_t> rb, cb;
    for (int i : tp) {
      rb.push_back(pieces[i].pc.n0); rb.push_back(pieces[i].pc.n1);
      cb.push_back(pieces[i].pc.m0); cb.push_back(pieces[i].pc.m1);
    }
    std::sort(rb.begin(), rb.end()); rb.erase(std::unique(rb.begin(), rb.end()), rb.end());
    std::sort(cb.begin(), cb.end()); cb.erase(std::unique(cb.begin(), cb.end()), cb.end());
    const size_t R = rb.size() - 1, Cn = cb.size() - 1;
    std::vector<std::vector<int>> cell(R * Cn);
    for (int i : tp) {
      const Piece& p = pieces[i].pc;
      size_t r0 = std::lower_bound(rb.begin(), rb.end(), p.n0) - rb.begin();
      size_t r1 = std::lower_bound(rb.begin(), rb.end(), p.n1) - rb.begin();
      size_t c0 = std::lower_bound(cb.begin(), cb.end(), p.m0) - cb.begin();
      size_t c1 = std::lower_bound(cb.begin(), cb.end(), p.m1) - cb.begin();
      for (size_t r = r0; r < r1; ++r)
        for (size_t c = c0; c < c1; ++c) cell[r * Cn + c].push_back(i);
    }
    for (size_t r = 0; r < R; ++r)
      for (size_t c = 0; c < Cn; ++c) {
        std::vector<int>& lst = cell[r * Cn + c];
        if (lst.empty()) continue;
        std::sort(lst.begin(), lst.end(),
                  [&](int a, int b) { return pieces[a].pc.k0 < pieces[b].pc.k0; });
        int32_t s0 = (int32_t)hp.srcs.size();
        for (int i : lst) {
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
        int64_t i0 = rb[r], i1 = rb[r + 1], j0 = cb[c], j1 = cb[c + 1];
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
    (void)geom;
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
