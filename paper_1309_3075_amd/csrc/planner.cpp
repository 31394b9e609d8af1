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
                    std::vector<int32_t>& proc, std::vector<double>& dur, std::vector<int32_t>& interval) {
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
      interval.push_back(k);
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
                   P.seg_time, P.seg_interval);
    for (size_t k = before; k < P.seg_process.size(); ++k)
      P.seg_frac.push_back(tau > 0 ? P.seg_time[k] / tau : 0.0);
    P.max_segments = std::max<int>(P.max_segments, (int)(P.seg_process.size() - before));
  }
  P.seg_offset[n] = (int32_t)P.seg_process.size();
  if (n_intervals > 1) P.boundaries.assign(boundaries, boundaries + n_intervals - 1);
  P.interval_process.assign(interval_process, interval_process + n_intervals);
  out = std::move(P);
  return 0;
}

namespace {

struct SlotPool {
  std::vector<char> used;
  int peak = 0;
  int get() {
    for (int s = 0;; ++s) {
      if (s == (int)used.size()) used.push_back(0);
      if (!used[s]) {
        used[s] = 1;
        peak = std::max(peak, s + 1);
        return s;
      }
    }
  }
  void put(int s) {
    if (s >= 0) used[s] = 0;
  }
};

int32_t encode(int flags, int src_a, int src_b, int s0, int s1, int s2, int s3) {
  const uint32_t v = (uint32_t)flags | ((uint32_t)src_a << 3) | ((uint32_t)src_b << 5) |
                     ((uint32_t)(s0 & 63) << 8) | ((uint32_t)(s1 & 63) << 14) | ((uint32_t)(s2 & 63) << 20) |
                     ((uint32_t)(s3 & 63) << 26);
  return (int32_t)v;
}

void emit(std::vector<int32_t>& prog, int32_t info, int a, int b, int u) {
  prog.push_back(info);
  prog.push_back(a);
  prog.push_back(b);
  prog.push_back(u);
}

}  // namespace

int build_walk_programs(const TreePlan& P, int recompute_tips, WalkProgram& out) {
  const int N = P.n_tips, n = P.n_nodes;
  out = WalkProgram{};
  std::vector<int32_t> tipcount(n, 1), need(n, 0);
  for (int u : P.post) {
    tipcount[u] = tipcount[P.left[u]] + tipcount[P.right[u]];
    const int a = need[P.left[u]], b = need[P.right[u]];
    need[u] = (a == b) ? a + 1 : std::max(a, b);
  }
  // children in visiting order: the one needing more stack slots first
  auto first = [&](int u) { return need[P.right[u]] > need[P.left[u]] ? P.right[u] : P.left[u]; };
  auto second = [&](int u) { return need[P.right[u]] > need[P.left[u]] ? P.left[u] : P.right[u]; };
  out.stored.assign(n, 0);
  for (int u = N; u < n; ++u) out.stored[u] = (u == P.root || tipcount[u] > recompute_tips) ? 1 : 0;

  // Post-order over the subtree of v (children before parents, first child
  // first); calls f(u) for every internal node.
  auto post_walk = [&](int v, auto&& f) {
    std::vector<std::pair<int, int>> st{{v, 0}};
    while (!st.empty()) {
      auto& top = st.back();
      const int u = top.first;
      if (top.second) {
        st.pop_back();
        f(u);
        continue;
      }
      top.second = 1;
      const int a = first(u), b = second(u);
      if (b >= N) st.push_back({b, 0});
      if (a >= N) st.push_back({a, 0});
    }
  };
  // POST operations for the subtree of v; returns the slot holding x_v (-1 for the root).
  auto emit_post = [&](std::vector<int32_t>& prog, SlotPool& pool, std::vector<int>& slot, int v, bool main) {
    post_walk(v, [&](int u) {
      const int a = first(u), b = second(u);
      const int sa = a >= N ? slot[a] : -1, sb = b >= N ? slot[b] : -1;
      pool.put(sa);
      pool.put(sb);
      int flags = 0, so = kWalkTrash;
      if (main && u == P.root) {
        flags = kWalkRoot | kWalkStore;
      } else {
        so = pool.get();
        slot[u] = so;
        if (main && out.stored[u]) flags = kWalkStore;
      }
      emit(prog, encode(flags, a >= N ? kWalkStack : kWalkTip, b >= N ? kWalkStack : kWalkTip, sa, sb, so, 0), a, b,
           u);
    });
    return slot[v];
  };

  {
    SlotPool pool;
    std::vector<int> slot(n, -1);
    emit_post(out.post, pool, slot, P.root, true);
    out.post_slots = pool.peak;
  }
  {
    SlotPool pool;
    std::vector<int> slot(n, -1);
    std::vector<std::pair<int, int>> st{{P.root, -1}};  // (node, slot holding its outside vector)
    while (!st.empty()) {
      const int u = st.back().first, qs = st.back().second;
      st.pop_back();
      // the child needing fewer slots first: the other's outside vector waits meanwhile
      const int a = second(u), b = first(u);
      int src[2], s[2] = {-1, -1};
      const int ch[2] = {a, b};
      for (int k = 0; k < 2; ++k) {
        if (ch[k] < N) {
          src[k] = kWalkTip;
        } else if (out.stored[ch[k]]) {
          src[k] = kWalkHbm;
        } else {
          src[k] = kWalkStack;
          s[k] = emit_post(out.pre, pool, slot, ch[k], false);
        }
      }
      int sqa = qs;
      if (a >= N && sqa < 0) sqa = pool.get();
      const int sqb = b >= N ? pool.get() : -1;
      const int flags = kWalkPre | (u == P.root ? kWalkRoot : 0);
      // q_u is read from, and q_a written to, the same slot; for a tip a the write
      // lands in q_u's slot, free after this operation (at the root: the discard slot)
      emit(out.pre, encode(flags, src[0], src[1], s[0], s[1], sqa >= 0 ? sqa : kWalkTrash, b >= N ? sqb : kWalkTrash),
           a, b, u);
      pool.put(s[0]);
      pool.put(s[1]);
      if (a < N) pool.put(sqa);
      if (b >= N) st.push_back({b, sqb});
      if (a >= N) st.push_back({a, sqa});
    }
    out.pre_slots = pool.peak;
  }
  if (out.post_slots > kWalkMaxSlots || out.pre_slots > kWalkMaxSlots) return -1;
  // unused outputs go to the slot just past the last one (every write is then unconditional)
  auto patch = [](std::vector<int32_t>& prog, int trash) {
    for (size_t k = 0; k < prog.size(); k += 4) {
      uint32_t v = (uint32_t)prog[k];
      for (int sh : {20, 26})
        if (((v >> sh) & 63u) == (uint32_t)kWalkTrash) v = (v & ~(63u << sh)) | ((uint32_t)trash << sh);
      prog[k] = (int32_t)v;
    }
  };
  patch(out.post, out.post_slots);
  patch(out.pre, out.pre_slots);
  return 0;
}

}  // namespace epochlik
