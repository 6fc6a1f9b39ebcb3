// plan.h -- turn partition pieces into device work lists and a k-cut
// reduction plan.
#pragma once
#include <stdint.h>

#include <vector>

#include "device_types.h"
#include "partition.h"

namespace paco {

// Geometry of one problem in kernel units (words for boolean m).
struct ProbGeom {
  int64_t n, m, k;
};

struct HostPlan {
  int nwg = 0;                     // workgroups launched
  bool xcd_remap = false;
  std::vector<WorkItem> items;
  std::vector<int32_t> wg_off;     // nwg + 1
  std::vector<RedTile> tiles;
  std::vector<RedSrc> srcs;
  int64_t temp_elems = 0;          // workspace elements for temporary faces
  int red_vec = 1;                 // reduction vector width (4 when aligned)
  // fused folding (the product kernel folds the cells; `tiles` are whole
  // cells, each tile's pad the number of pieces covering it): per item
  // (begin, count) into fold_list, the cells the item covers
  bool fused = false;
  std::vector<int32_t> item_fold;
  std::vector<int32_t> fold_list;
  // every non-empty item starts on a multiple of four in k and m (the
  // integer kernel's 128-bit loads need it)
  bool aligned4 = true;
  // statistics over non-empty pieces
  int32_t n_pieces = 0, n_kcuts = 0;
  int64_t vmax = 0, vmin = 0;
};

// A piece tagged with the problem it belongs to (batched launches).
struct TaggedPiece {
  Piece pc;          // coordinates in the problem's kernel units
  int32_t prob;
  int32_t wg;        // workgroup (processor) index
};

// Build work lists for `nwg` workgroups from tagged pieces.  A piece whose
// k0 > 0 writes its own temporary face (allocated after `temp_base`
// elements); every covered C element then folds its faces in ascending-k
// order.  `geom` gives each problem's C size (rows, cols in kernel units).
// `red_vec` 4 asks for 4-wide reduction tiles; the plan falls back to 1
// unless every face offset, width and column origin is a multiple of 4
// (the caller checks the alignment of C itself).
// fuse: 0 a separate fold launch (cells cut into tiles of about 1024
// elements); 1 fused folding; 2 fused when no cell's fold reads more than
// kFuseCellBytes (one workgroup folds each cell).  The library's calls use
// 0 unless PACO_FUSE_FOLD says otherwise.
constexpr int64_t kFuseCellBytes = 256 << 10;
HostPlan build_plan(const std::vector<TaggedPiece>& pieces, int nwg, bool xcd_remap,
                    const std::vector<ProbGeom>& geom, int64_t temp_base = 0, int red_vec = 4,
                    int fuse = 0);

}  // namespace paco
