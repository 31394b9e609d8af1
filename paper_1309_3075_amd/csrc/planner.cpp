// Host planner: tree validation, post-order and level schedules, and the
// per-branch epoch segmentation (Methods, "Relaxing time-homogeneity";
// "Coarse-grain parallel implementation": the time each process is active
// on a branch).
#include "planner.h"

#include <algorithm>
#include <cmath>
#include <cstdio>

namespace epochlik {

namespace {

bool fail(std::string& err, const char* msg, long a = -1, long b = -1) {
  char buf[256];
  if (a >= 0 && b >= 0)
    snprintf(buf, sizeof(buf), "%s (%ld, %ld)", msg, a, b);
  else if (a >= 0)
    snprintf(buf, sizeof(buf), "%s (%ld)", msg, a);
  else
    snprintf(buf, sizeof(buf), "%s", msg);
  err = buf;
  return false;
}

// Segments of one branch from parent height hu down to child height hv.
// Interval k covers heights [b_{k-1}, b_k) with b_{-1} = -inf and b_{M-1} = +inf
// (0-based boundaries b_0..b_{M-2}).  Walk from the interval holding the
// stretch just below hu down to the one holding the stretch just above hv.
void segment_branch(double hu, double hv, int M, const double* b, const int32_t* phi,
                    std::vector<int32_t>& proc, std::vector<double>& dur) {
  if (!(hu > hv)) return;
  // k_top: number of boundaries strictly below hu
  int k_top = 0;
  while (k_top < M - 1 && b[k_top] < hu) ++k_top;
  for (int k = k_top; k >= 0; --k) {
    double lo = (k == 0) ? -INFINITY : b[k - 1];
    double hi = (k == M - 1) ? INFINITY : b[k];
    double top = std::min(hu, hi);
    double bot = std::max(hv, lo);
    if (top > bot) {
      proc.push_back(phi[k]);
      dur.push_back(top - bot);
    }
    if (lo <= hv) break;
  }
}

}  // namespace

int plan_tree(int n_tips, const int32_t* parent, const double* height, const double* branch_rate,
              int n_intervals, const double* boundaries, const int32_t* interval_process,
              int n_processes, TreePlan& out, std::string& err) {
  auto bad = [&](const char* m, long a = -1, long b = -1) {
    fail(err, m, a, b);
    return -1;
  };
  if (n_tips < 2) return bad("n_tips must be >= 2");
  if (!parent || !height) return bad("parent and height are required");
  if (n_intervals < 1) return bad("n_intervals must be >= 1");
  if (n_intervals > 1 && !boundaries) return bad("boundaries required when n_intervals > 1");
  if (!interval_process) return bad("interval_process is required");
  const int N = n_tips, n = 2 * n_tips - 1;
  for (int k = 0; k + 1 < n_intervals; ++k) {
    if (!std::isfinite(boundaries[k])) return bad("boundary is not finite", k);
    if (k > 0 && !(boundaries[k] > boundaries[k - 1]))
      return bad("boundaries must be strictly ascending", k);
  }
  for (int k = 0; k < n_intervals; ++k)
    if (interval_process[k] < 0 || interval_process[k] >= n_processes)
      return bad("interval_process out of range", k, interval_process[k]);

  TreePlan P;
  P.n_tips = N;
  P.n_nodes = n;
  P.parent.assign(parent, parent + n);
  P.height.assign(height, height + n);
  P.rate.assign(n, 1.0);
  P.left.assign(n, -1);
  P.right.assign(n, -1);
  for (int v = 0; v < n; ++v) {
    if (!std::isfinite(height[v])) return bad("height is not finite", v);
    if (branch_rate) {
      if (!(branch_rate[v] > 0.0) || !std::isfinite(branch_rate[v]))
        if (parent[v] >= 0) return bad("branch_rate must be finite and > 0", v);
      P.rate[v] = branch_rate[v];
    }
    int u = parent[v];
    if (u == -1) {
      if (P.root >= 0) return bad("more than one root", P.root, v);
      P.root = v;
      continue;
    }
    if (u < N || u >= n) return bad("parent must be an internal node index", v, u);
    if (u == v) return bad("node is its own parent", v);
    if (P.left[u] < 0)
      P.left[u] = v;
    else if (P.right[u] < 0)
      P.right[u] = v;
    else
      return bad("node has more than two children", u);
  }
  if (P.root < N) return bad("root must be an internal node");
  for (int u = N; u < n; ++u)
    if (P.left[u] < 0 || P.right[u] < 0) return bad("internal node without two children", u);
  for (int v = 0; v < n; ++v) {
    int u = parent[v];
    if (u >= 0 && !(height[u] >= height[v]))
      return bad("parent is younger than child", u, v);
  }
  // post-order by iterative DFS; also detects cycles / disconnected nodes
  P.level.assign(n, 0);
  {
    std::vector<int32_t> stack;
    std::vector<char> state(n, 0);
    stack.push_back(P.root);
    while (!stack.empty()) {
      int u = stack.back();
      if (u < N) {
        stack.pop_back();
        state[u] = 2;
        continue;
      }
      if (state[u] == 0) {
        state[u] = 1;
        for (int c : {P.left[u], P.right[u]}) {
          if (state[c] != 0) {
            fail(err, "tree has a cycle", u, c);
            return -1;
          }
          stack.push_back(c);
        }
      } else {
        stack.pop_back();
        state[u] = 2;
        P.level[u] = 1 + std::max(P.level[P.left[u]], P.level[P.right[u]]);
        P.post.push_back(u);
      }
    }
    for (int v = 0; v < n; ++v)
      if (state[v] != 2) return bad("node not reachable from the root", v);
  }
  // level schedule
  P.n_levels = P.level[P.root];
  P.level_offset.assign(P.n_levels + 2, 0);
  for (int u : P.post) P.level_offset[P.level[u] + 1]++;
  for (int l = 1; l <= P.n_levels + 1; ++l) P.level_offset[l] += P.level_offset[l - 1];
  P.level_nodes.assign(P.post.size(), 0);
  {
    std::vector<int32_t> fill(P.level_offset.begin(), P.level_offset.end());
    for (int u = N; u < n; ++u) P.level_nodes[fill[P.level[u]]++] = u;  // ascending index in a level
  }
  // segments
  P.tau.assign(n, 0.0);
  P.seg_offset.assign(n + 1, 0);
  for (int v = 0; v < n; ++v) {
    P.seg_offset[v] = (int32_t)P.seg_process.size();
    int u = parent[v];
    if (u < 0) continue;
    double tau = height[u] - height[v];
    P.tau[v] = tau;
    size_t before = P.seg_process.size();
    segment_branch(height[u], height[v], n_intervals, boundaries, interval_process, P.seg_process,
                   P.seg_time);
    for (size_t k = before; k < P.seg_process.size(); ++k)
      P.seg_frac.push_back(tau > 0 ? P.seg_time[k] / tau : 0.0);
    P.max_segments = std::max<int>(P.max_segments, (int)(P.seg_process.size() - before));
  }
  P.seg_offset[n] = (int32_t)P.seg_process.size();
  // Strahler-ordered walk: visit the child needing more stack slots first.
  {
    std::vector<int32_t> need(n, 0);
    for (int u : P.post) {
      int a = need[P.left[u]], b = need[P.right[u]];
      if (P.left[u] < N && P.right[u] < N)
        need[u] = 1;
      else
        need[u] = (a == b) ? a + 1 : std::max(a, b);
    }
    P.stack_depth = need[P.root];
    std::vector<std::pair<int, int>> st;  // (node, expanded)
    st.push_back({P.root, 0});
    while (!st.empty()) {
      auto& top = st.back();
      int u = top.first;
      if (top.second) {
        P.walk.push_back(u);
        st.pop_back();
        continue;
      }
      top.second = 1;
      int a = P.left[u], b = P.right[u];
      if (need[b] > need[a]) std::swap(a, b);
      // push second child first so the first child is processed first
      if (b >= N) st.push_back({b, 0});
      if (a >= N) st.push_back({a, 0});
    }
  }
  out = std::move(P);
  return 0;
}

}  // namespace epochlik
