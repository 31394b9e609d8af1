// Incremental re-evaluation for MCMC proposals.
//
// A Metropolis-Hastings proposal changes one parameter at a time (a branch
// length, or the rates of one process), and the sampler then needs the new
// log-likelihood (Introduction; Results, run time analysis).  Only the
// transition matrices of the branches that parameter touches change (Eq. 6-7:
// a branch's product contains process s's factor only where the branch spends
// time in an interval assigned to s), and with them only the partials of the
// nodes above those branches (Eq. 4: a node's partial depends on its subtree
// alone).  The instance therefore remembers which branches changed since the
// last complete post-order pass and re-forms exactly those matrices and the
// partials on their paths to the root, as the usual level launches restricted
// to the dirty nodes.  The root reduction always runs in full; the gradient
// passes, when requested, run in full over the updated partials.
//
// The restricted launches use the same kernels on the same inputs, so the
// result equals a full evaluation; on the matrix-core P stage a long chain
// that the full launch would cut into parts is formed whole, which rounds
// differently.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "instance.h"

namespace epochlik {

void mark_dirty_all(EpochInstance* in) {
  in->dirty_all = true;
  in->inc_active = false;
}

// Every branch with a stretch in an interval whose process is s (Eq. 6-7).
void mark_dirty_process(EpochInstance* in, int s) {
  if (!in->have_tree || in->dirty_all) return;
  const auto& pl = in->plan;
  in->dirty.resize(in->n_nodes, 0);
  for (int v = 0; v < in->n_nodes; ++v)
    for (int g = pl.seg_offset[v]; g < pl.seg_offset[v + 1]; ++g)
      if (pl.seg_process[g] == s) {
        in->dirty[v] = 1;
        break;
      }
}

bool incremental_eligible(const EpochInstance* in) {
  if (!in->inc_enable || in->dirty_all || !in->inc_base || !in->have_tree) return false;
  // only a recorded change is re-evaluated in part: evaluating an unchanged state runs in full
  if (std::find(in->dirty.begin(), in->dirty.end(), (uint8_t)1) == in->dirty.end()) return false;
  // the dlogL/dQ adjoint reads per-segment products the P stage keeps for every chain
  if (in->cfg.flags & EPOCH_GRAD_Q) return false;
  switch (in->path) {
    case 1: return !in->walk_ok && in->budget == 0;  // 4-state level kernels (the tree walk redoes the tree)
    case 2: return in->codon_nchunks == 1;           // 64-state kernels, all patterns at once
    default: return in->gen_nchunks == 1;            // generic kernels, all patterns at once
  }
}

namespace {

size_t align16(size_t b) { return (b + 15) / 16 * 16; }

// Host lists of one restricted pass, uploaded in one copy.
int build_lists(EpochInstance* in) {
  const auto& pl = in->plan;
  auto& L = in->inc;
  const int n = in->n_nodes;
  std::vector<uint8_t> up(n, 0);  // internal nodes whose partial is formed again
  L.pnodes.clear();
  L.chain_items.clear();
  in->dirty.resize(n, 0);
  for (int v = 0; v < n; ++v) {
    if (!in->dirty[v] || v == pl.root) continue;
    L.pnodes.push_back(v);
    for (int u = pl.parent[v]; u >= 0 && !up[u]; u = pl.parent[u]) up[u] = 1;
  }
  // whole-chain items, longest chain first (as the full matrix-core launch orders them)
  for (int v : L.pnodes) L.chain_items.push_back(make_int4(v, 0, pl.seg_offset[v + 1] - pl.seg_offset[v], 0));
  std::stable_sort(L.chain_items.begin(), L.chain_items.end(),
                   [](const int4& a, const int4& b) { return a.z > b.z; });
  // partials, grouped by level like the plan's level lists
  L.post_nodes.clear();
  L.post_level_off.assign(pl.n_levels + 2, 0);
  for (int l = 1; l <= pl.n_levels; ++l) {
    L.post_level_off[l] = (int32_t)L.post_nodes.size();
    for (int k = pl.level_offset[l]; k < pl.level_offset[l + 1]; ++k)
      if (up[pl.level_nodes[k]]) L.post_nodes.push_back(pl.level_nodes[k]);
  }
  L.post_level_off[pl.n_levels + 1] = (int32_t)L.post_nodes.size();
  // the 64-state schedule keeps its per-level tile shapes and drops the clean nodes
  std::vector<int2> citems;
  if (in->path == 2) {
    const auto& sc = in->codon_sched;
    L.codon = sc;
    L.codon.amb = in->tips_amb;
    L.codon.items.clear();
    L.codon.level_off.assign(1, 0);
    for (int l = 1; l <= sc.n_levels; ++l) {
      for (int k = sc.level_off[l - 1]; k < sc.level_off[l]; ++k)
        if (up[sc.items[k].y]) L.codon.items.push_back(sc.items[k]);
      L.codon.level_off.push_back((int)L.codon.items.size());
    }
    citems = L.codon.items;
  }
  L.off_chain = align16(L.pnodes.size() * sizeof(int32_t));
  L.off_post = L.off_chain + align16(L.chain_items.size() * sizeof(int4));
  L.off_codon = L.off_post + align16(L.post_nodes.size() * sizeof(int32_t));
  const size_t bytes = L.off_codon + citems.size() * sizeof(int2);
  int rc = ensure(in->inc_dev, std::max<size_t>(bytes, 256));
  if (rc) return rc;
  std::vector<char> h(bytes, 0);
  if (!L.pnodes.empty()) memcpy(h.data(), L.pnodes.data(), L.pnodes.size() * sizeof(int32_t));
  if (!L.chain_items.empty()) memcpy(h.data() + L.off_chain, L.chain_items.data(), L.chain_items.size() * sizeof(int4));
  if (!L.post_nodes.empty()) memcpy(h.data() + L.off_post, L.post_nodes.data(), L.post_nodes.size() * sizeof(int32_t));
  if (!citems.empty()) memcpy(h.data() + L.off_codon, citems.data(), citems.size() * sizeof(int2));
  if (bytes) {
    rc = hip_check(hipMemcpyAsync(in->inc_dev.ptr, h.data(), bytes, hipMemcpyHostToDevice, in->stream),
                   "incremental list upload");
    if (!rc) rc = hip_check(hipStreamSynchronize(in->stream), "incremental list sync");  // h is a local copy
  }
  return rc;
}

}  // namespace

int launch_pstage_incremental(EpochInstance* in) {
  int rc = build_lists(in);
  if (rc) return rc;
  const auto& L = in->inc;
  const char* base = static_cast<const char*>(in->inc_dev.ptr);
  in->work_P = (int64_t)L.pnodes.size() * in->C;
  in->inc_active = true;
  if (L.pnodes.empty()) return EPOCH_OK;
  if (in->cfg.kernel_path == EPOCH_KERNEL_AUTO && pstage_mfma_supported(in))
    return launch_pstage_mfma_items(in, reinterpret_cast<const int4*>(base + L.off_chain), (int)L.chain_items.size());
  return launch_pstage_generic_nodes(in, reinterpret_cast<const int32_t*>(base), (int)L.pnodes.size());
}

int launch_post_incremental(EpochInstance* in) {
  const auto& L = in->inc;
  const auto& pl = in->plan;
  const char* base = static_cast<const char*>(in->inc_dev.ptr);
  const int32_t* d_post = reinterpret_cast<const int32_t*>(base + L.off_post);
  int64_t formed = 0;
  for (int l = (in->path == 1 && pl.n_levels > 1) ? 2 : 1; l <= pl.n_levels; ++l)
    formed += L.post_level_off[l + 1] - L.post_level_off[l];  // 4-state cherries are never stored
  in->work_partials = formed;
  if (L.post_nodes.empty()) return EPOCH_OK;
  switch (in->path) {
    case 1: return launch_nuc_post_nodes(in, d_post, L.post_level_off.data());
    case 2: return launch_codon_post_schedule(in, L.codon, reinterpret_cast<const int2*>(base + L.off_codon));
    default: return launch_post_generic_nodes(in, d_post, L.post_level_off.data());
  }
}

void incremental_done(EpochInstance* in) {
  in->dirty.assign(in->n_nodes, 0);
  in->dirty_all = false;
  in->inc_base = true;
  in->inc_active = false;
}

}  // namespace epochlik

using namespace epochlik;

extern "C" {

int epoch_set_branch_rates(EpochInstance* in, int32_t n, const int32_t* nodes, const double* rates) {
  if (!in) return set_error(EPOCH_ERR_ARG, "NULL instance");
  if (!in->have_tree) return set_error(EPOCH_ERR_STATE, "set_tree_epochs has not been called");
  if (n < 0 || (n > 0 && (!nodes || !rates))) return set_error(EPOCH_ERR_ARG, "n >= 0 nodes and rates required");
  for (int k = 0; k < n; ++k) {
    if (nodes[k] < 0 || nodes[k] >= in->n_nodes)
      return set_error(EPOCH_ERR_ARG, "node %d outside [0, %d)", nodes[k], in->n_nodes);
    if (!std::isfinite(rates[k]) || !(rates[k] > 0))
      return set_error(EPOCH_ERR_ARG, "rate %d must be finite and > 0", k);
  }
  in->dirty.resize(in->n_nodes, 0);
  for (int k = 0; k < n; ++k) {
    const int v = nodes[k];
    if (v == in->plan.root) continue;  // the root has no branch
    in->plan.rate[v] = rates[k];
    in->dirty[v] = 1;
  }
  int rc = hip_check(hipMemcpyAsync(in->d_rate, in->plan.rate.data(), in->plan.rate.size() * sizeof(double),
                                    hipMemcpyHostToDevice, in->stream), "branch rate upload");
  if (!rc) rc = hip_check(hipStreamSynchronize(in->stream), "branch rate sync");
  if (rc) return rc;
  in->P_valid = in->partials_valid = in->logL_valid = false;
  return EPOCH_OK;
}

int epoch_get_work_counts(EpochInstance* in, int64_t* out) {
  if (!in || !out) return set_error(EPOCH_ERR_ARG, "NULL argument");
  out[0] = in->work_P;
  out[1] = in->work_partials;
  return EPOCH_OK;
}

}  // extern "C"
