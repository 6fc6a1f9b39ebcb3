// strassen_sched.cpp -- pruned-BFS schedule of PACO Strassen (host).
#include "strassen_sched.h"

namespace paco {

SSchedule strassen_schedule(int64_t n, int p, int gamma, int64_t base) {
  SSchedule s;
  s.p = p;
  s.per_proc.resize(p);
  int64_t nodes = 1, h = n;
  for (int d = 0;; ++d) {
    SLevel lv{d, h, nodes, 0, false};
    if (nodes >= p) {
      lv.assigned = (nodes / p) * p;
      lv.super_round = true;
      s.super_rounds += 1;
    }
    const int64_t left = nodes - lv.assigned;
    const bool divide = left > 0 && h % 2 == 0 && h / 2 >= base && (gamma <= 0 || s.super_rounds < gamma) &&
                        left * 7 < (int64_t)1 << 40;
    if (left > 0 && !divide) lv.assigned = nodes;   // round-robin, the last assignment
    for (int64_t i = 0; i < lv.assigned; ++i) s.per_proc[i % p].push_back({d, i});
    s.levels.push_back(lv);
    if (lv.assigned == nodes) break;
    nodes = left * 7;
    h /= 2;
  }
  return s;
}

}  // namespace paco
