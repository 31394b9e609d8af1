// Host planner: validates a tree + epoch structure and turns it into the
// flat schedules the kernels consume.  Pure C++ (no HIP), so it also runs in
// CPU-only builds.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace epochlik {

struct TreePlan {
  int n_tips = 0;
  int n_nodes = 0;  // 2N-1
  int root = -1;
  std::vector<int32_t> parent;       // [n_nodes]
  std::vector<int32_t> left, right;  // children of internal nodes, -1 for tips
  std::vector<double> height;        // [n_nodes]
  std::vector<double> rate;          // [n_nodes], rate of the branch above each node
  std::vector<double> tau;           // [n_nodes], branch duration (height units), root 0
  // internal nodes in a valid post-order (children before parents)
  std::vector<int32_t> post;
  // internal nodes grouped by level (level = 1 + max level of the children,
  // tips at level 0); level_nodes[level_offset[l] .. level_offset[l+1]) for l >= 1
  std::vector<int32_t> level;
  std::vector<int32_t> level_offset;
  std::vector<int32_t> level_nodes;
  int n_levels = 0;  // highest level (the root's)
  // per-branch segments, CSR by child node, parent side first
  std::vector<int32_t> seg_offset;   // [n_nodes + 1]
  std::vector<int32_t> seg_process;  // [n_seg]
  std::vector<double> seg_time;      // [n_seg] duration in height units
  std::vector<double> seg_frac;      // [n_seg] duration / tau (0 when tau == 0)
  int max_segments = 0;              // longest segment list of any branch
  // Strahler-ordered post-order walk for the register-stack kernels:
  // for every internal node in walk order, which child is visited first
  std::vector<int32_t> walk;          // internal nodes, children before parents
  int stack_depth = 0;                // max simultaneously pending partials
};

// Validates and plans.  Returns 0 on success; on failure returns -1 and sets err.
int plan_tree(int n_tips, const int32_t* parent, const double* height, const double* branch_rate,
              int n_intervals, const double* boundaries, const int32_t* interval_process,
              int n_processes, TreePlan& out, std::string& err);

}  // namespace epochlik
