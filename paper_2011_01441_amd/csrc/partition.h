// partition.h -- host-side PACO partitioner of the n-by-m-by-k MM cuboid.
#pragma once
#include <stdint.h>
#include <vector>

namespace paco {

struct Piece {
  int64_t n0, n1, m0, m1, k0, k1;
  int32_t proc, round, depth;
  int64_t vol() const { return (n1 - n0) * (m1 - m0) * (k1 - k0); }
  bool empty() const { return n1 <= n0 || m1 <= m0 || k1 <= k0; }
};

struct PartOpts {
  int32_t p = 1;
  int64_t q[3] = {1, 1, 1};      // cut quanta for n, m, k
  const double* weights = nullptr;
  bool multi_piece = false;
  // k counts as k / kcut_cost when the longest dimension is chosen (1 = the
  // paper's rule; larger values prefer n and m cuts, which need no
  // temporary face)
  double kcut_cost = 1.0;
  // multi-piece: rounds of p pieces before the rest goes out round-robin
  // (0 = none; division then stops at the quanta)
  int max_rounds = 0;
  // MM-1-Piece on a kernel's tile grid (see partition.cpp): cuts still
  // split each cuboid in the processor ratio, on the quanta, but the
  // dimension of each cut is chosen to minimise the busiest processor's
  // cost: its output tiles (tile_n x tile_m, 0 = the quanta) times its
  // k-range padded to q[2], plus a per-tile overhead of tile_k_ovh and, for
  // a piece that writes a temporary face, tile_face (both in units of k)
  bool tile_balance = false;
  int64_t tile_n = 0, tile_m = 0;
  double tile_k_ovh = 64.0;
  double tile_face = 128.0;
};

// MM-1-Piece (corollary mm-1-piece): exactly p pieces, piece j on proc j.
std::vector<Piece> partition_mm1(int64_t n, int64_t m, int64_t k, const PartOpts& o);
// PACO MM multi-piece pruned BFS (theorem mm): every cuboid of a depth with
// at least p unassigned cuboids is cut evenly; exactly p get assigned.
std::vector<Piece> partition_multi(int64_t n, int64_t m, int64_t k, const PartOpts& o);
// Plain grid baseline: tm-by-tn output tiles, each split into `split_k`
// k-chunks aligned to bk; piece j runs on workgroup j.
std::vector<Piece> partition_grid(int64_t n, int64_t m, int64_t k, int64_t tm, int64_t tn,
                                  int64_t bk, int split_k);

}  // namespace paco
