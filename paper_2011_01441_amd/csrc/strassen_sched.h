// strassen_sched.h -- the pruned BFS of PACO Strassen over processor groups.
#pragma once
#include <stdint.h>

#include <vector>

namespace paco {

// One depth of the 7-way recursion tree.  Its `nodes` are the children, in
// order, of the nodes of the previous depth that were left unassigned there
// (node j's parent is node first_left(d-1) + j / 7, its Strassen index
// j % 7); the first `assigned` of them are handed out, node i to processor
// i % p, the rest are divided again.
struct SLevel {
  int depth;
  int64_t h;          // node dimension n / 2^depth
  int64_t nodes;      // nodes at this depth
  int64_t assigned;   // nodes handed out at this depth
  bool super_round;   // this depth assigned floor(nodes / p) * p nodes
};

struct SSchedule {
  int p = 1;
  int super_rounds = 0;
  std::vector<SLevel> levels;
  // per processor: the (depth, node) pairs it runs, in order of depth
  std::vector<std::vector<std::pair<int, int64_t>>> per_proc;
};

// Section "PACO Strassen": expand the tree breadth-first; at a depth with at
// least p unassigned nodes hand out floor(nodes / p) * p of them (each
// processor gets the same number, at most 6 since the depth before had
// fewer than p) and divide the rest; after `gamma` such super-rounds
// (Strassen-Const-Pieces; 0 = no limit), or when the next depth would have
// nodes smaller than `base` or of odd size, hand out everything left.
SSchedule strassen_schedule(int64_t n, int p, int gamma, int64_t base);

}  // namespace paco
