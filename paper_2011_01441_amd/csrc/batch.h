// batch.h -- splitting processors over a batch of independent requests.
#pragma once
#include <stdint.h>

#include <vector>

#include "partition.h"
#include "plan.h"

namespace paco {

// One request of a batch in kernel units.
struct BatchReq {
  int64_t n, m, k;     // logical sizes (bits for boolean)
  int sr;              // paco_semiring
  int prec;            // ring precision (Prec), -1 otherwise
};

// Kernel group of a request: requests of one group share one launch.
enum BatchGroup : int { G_RING_FP32 = 0, G_RING_X3 = 1, G_RING_X6 = 2, G_MINPLUS = 3, G_MAXPLUS = 4, G_BOOL = 5,
                        G_COUNT = 6 };
int batch_group(const BatchReq& r);

// Relative time of one request on one processor: n m k times the group's
// cost per (i, j, l) plus a fixed per-request term.
double batch_weight(const BatchReq& r);

struct BatchSplit {
  int g0[G_COUNT], g1[G_COUNT];          // processor range of each group
  int tile[G_COUNT];                     // ring groups: the kernel tile the group runs; else -1
  std::vector<TaggedPiece> pieces;       // prob = request index, wg = processor
};

// Processors go to groups in proportion to their weight (largest
// remainder, at least one per non-empty group while processors last).
// Within a group the request list (in arrival order) is split recursively
// into two parts of about equal weight and the processors in the ratio of
// the parts' weights; a request left alone with several processors is
// partitioned with MM-1-Piece over them (ring requests on the group's tile
// grid, the tile chosen first from the group's requests), requests left on
// one processor run there whole.
BatchSplit batch_partition(const std::vector<BatchReq>& reqs, int p);

}  // namespace paco
