// Prefix-scan planner (host only).
#pragma once

#include <vector>

namespace rs {

struct PlanOp {
  int level, out, a, b, i, j, k;
};

// Returns 0 on success, -1 for invalid arguments.
int build_plan(int M, int algo, int chunk, int global_algo, std::vector<PlanOp>& out, int& n_levels);

}  // namespace rs
