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
  std::vector<int32_t> seg_interval; // [n_seg] interval index of each segment
  int max_segments = 0;              // longest segment list of any branch
  std::vector<double> boundaries;          // [M-1] ascending boundary heights
  std::vector<int32_t> interval_process;   // [M] process of each interval
};

// Programs of the four-state tree-walk kernels (one wavefront carries a tile of
// patterns through the whole tree).  Each operation is four int32:
//   info: bit 0 PRE (else POST), bit 1 ROOT, bit 2 STORE (POST: write the partial
//         to HBM), bits 3-4 / 5-6 source of child a / b (kWalkTip, kWalkHbm,
//         kWalkStack), bits 8-13 / 14-19 stack slot of child a / b, bits 20-25
//         output slot (POST) or slot of q_u that receives q_a (PRE), bits 26-31
//         slot receiving q_b (PRE); an output nobody reads (the root's partial,
//         q of a tip) goes to slot number "slots" of its program;
//   a, b: the children (a first), u: the node.
// POST computes the partial of u from its children; PRE consumes the outside
// vector q_u and the children's partials and produces the children's outside
// vectors and their branches' dlogL/dl shares.
enum { kWalkTip = 0, kWalkHbm = 1, kWalkStack = 2 };
constexpr int kWalkPre = 1, kWalkRoot = 2, kWalkStore = 4;
constexpr int kWalkMaxSlots = 62;  // live slots; one more slot takes the outputs an operation discards
constexpr int kWalkTrash = 63;     // placeholder while building

struct WalkProgram {
  std::vector<int32_t> post, pre;  // 4 int32 per operation
  int post_slots = 0, pre_slots = 0;
  std::vector<uint8_t> stored;     // [n_nodes]: 1 if the post program writes the node's partial
};

// Builds both programs.  Internal nodes whose subtree holds at most
// recompute_tips tips (>= 2) are not stored: the pre-order program recomputes
// them from the tip states.  post_slots / pre_slots count the live slots (the
// kernels reserve one more).  Fails (returns -1) when a program would need more
// than kWalkMaxSlots live slots.
int build_walk_programs(const TreePlan& plan, int recompute_tips, WalkProgram& out);

// Validates and plans.  Returns 0 on success; on failure returns -1 and sets err.
int plan_tree(int n_tips, const int32_t* parent, const double* height, const double* branch_rate,
              int n_intervals, const double* boundaries, const int32_t* interval_process,
              int n_processes, TreePlan& out, std::string& err);

}  // namespace epochlik
