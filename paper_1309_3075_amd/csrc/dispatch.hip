// Kernel selection for each step of the path: the specialised 4-state
// kernels when K == 4 (unless the generic path is forced), the generic any-K
// kernels otherwise.
#include <algorithm>
#include <vector>

#include "fastpath.h"

namespace epochlik {

namespace {
bool nuc(const EpochInstance* in) { return in->path == 1; }
bool codon(const EpochInstance* in) { return in->path == 2; }
}  // namespace

int fastpath_init(EpochInstance* in) {
  in->path = 0;
  if (in->cfg.kernel_path == EPOCH_KERNEL_AUTO) {
    if (in->K == 4) in->path = 1;
    else if (((in->Kp == 64 && in->K > 48) || (in->Kp == 32 && in->K > 16)) &&
             (in->budget == 0 || (in->C == 1 && !in->fp64)))
      in->path = 2;
  }
  const bool grad = (in->cfg.flags & (EPOCH_GRAD_BRANCH | EPOCH_GRAD_Q)) != 0;
  in->root_slot = 0;
  if (nuc(in) && grad && in->budget == 0) {
    in->nuc_slots = nuc_slots(in->P, in->C, in->nuc_rmin);
    const size_t bytes = (size_t)in->nuc_slots * in->n_nodes * in->C * 16 * sizeof(double);
    int rc = ensure(in->Gpart, std::max(bytes, in->Gpart.bytes));
    if (rc) return rc;
    return ensure(in->gslots, (size_t)in->n_nodes * sizeof(int32_t));
  }
  return EPOCH_OK;
}
void fastpath_release(EpochInstance*) {}
int fastpath_tips_changed(EpochInstance*) { return EPOCH_OK; }
int fastpath_tree_changed(EpochInstance* in) {
  if (codon(in)) return codon_prepare(in);
  if (nuc(in)) {
    int rc = walk_prepare(in);
    if (rc) return rc;
  }
  if (!nuc(in) || !in->gslots.ptr) return EPOCH_OK;
  std::vector<int32_t> slots, nodes;
  nuc_pre_order_nodes(in, nodes, in->nuc_fuse);
  nuc_slots_per_node(in, nodes, in->nuc_fuse, slots);
  int rc = ensure(in->nuc_nodes, std::max<size_t>(1, nodes.size()) * sizeof(int32_t));
  if (!rc) rc = hip_check(hipMemcpyAsync(in->gslots.ptr, slots.data(), slots.size() * sizeof(int32_t),
                                         hipMemcpyHostToDevice, in->stream), "gslots upload");
  if (!rc && !nodes.empty())
    rc = hip_check(hipMemcpyAsync(in->nuc_nodes.ptr, nodes.data(), nodes.size() * sizeof(int32_t),
                                  hipMemcpyHostToDevice, in->stream), "pre-order node upload");
  if (rc) return rc;
  return hip_check(hipStreamSynchronize(in->stream), "gslots sync");
}

#define EPOCH_PHASE(k, expr)            \
  do {                                  \
    int _rc = phase_begin(in, k);       \
    if (!_rc) _rc = (expr);             \
    if (!_rc) _rc = phase_end(in, k);   \
    if (_rc) return _rc;                \
  } while (0)

int launch_pstage(EpochInstance* in) {
  if (in->cfg.kernel_path == EPOCH_KERNEL_AUTO && pstage_mfma_supported(in)) return launch_pstage_mfma(in);
  return launch_pstage_generic(in);
}

int launch_grad_Q(EpochInstance* in) {
  if (in->cfg.kernel_path == EPOCH_KERNEL_AUTO && grad_Q_mfma_supported(in)) return launch_grad_Q_mfma(in);
  return launch_grad_Q_generic(in);
}

int fastpath_after_pstage(EpochInstance* in) { return (nuc(in) && in->walk_ok) ? launch_walk_tipcol(in) : EPOCH_OK; }

namespace {
int pstage_then_tip_columns(EpochInstance* in) {
  const int rc = launch_pstage(in);
  return rc ? rc : fastpath_after_pstage(in);
}

// internal-node partials a full post-order pass forms (4-state level kernels recompute cherries)
int64_t full_post_count(const EpochInstance* in) {
  const auto& pl = in->plan;
  if (nuc(in) && !in->walk_ok && pl.n_levels > 1) return (int64_t)(in->N - 1) - (pl.level_offset[2] - pl.level_offset[1]);
  return in->N - 1;
}
}  // namespace

int fastpath_pstage(EpochInstance* in) {
  if (incremental_eligible(in)) {  // only the branches changed since the last post-order pass
    EPOCH_PHASE(0, launch_pstage_incremental(in));
    return EPOCH_OK;
  }
  in->inc_active = false;
  in->work_P = (int64_t)(in->n_nodes - 1) * in->C;
  EPOCH_PHASE(0, pstage_then_tip_columns(in));
  return EPOCH_OK;
}

namespace {
// Generic path under an HBM budget: select pattern chunk j (or all patterns, j < 0).
void set_view(EpochInstance* in, int j, bool accumulate) {
  if (j < 0) {
    in->view_P = in->view_p0 = in->view_j = 0;
    in->view_accumulate = false;
    return;
  }
  in->view_p0 = j * in->gen_pc;
  in->view_P = std::min(in->P - in->view_p0, in->gen_pc);
  in->view_j = j;
  in->view_accumulate = accumulate;
}

// Post-order pass of the generic path; in pattern chunks, each chunk's share of
// logL follows its partials (the next chunk overwrites them), then the shares
// are summed in order.
int launch_post_generic_chunks(EpochInstance* in) {
  if (in->gen_nchunks == 1) return launch_post_generic(in);
  for (int j = 0; j < in->gen_nchunks; ++j) {
    set_view(in, j, false);
    int rc = launch_post_generic(in);
    if (!rc) rc = launch_root_generic(in);
    if (rc) {
      set_view(in, -1, false);
      return rc;
    }
  }
  set_view(in, -1, false);
  return launch_chunk_sum(in, in->gen_nchunks);
}

// Pre-order pass and dlogL/dP of the generic path; in pattern chunks, each
// chunk's partials are formed again first and dlogL/dP accumulates over chunks.
int launch_pre_grad_generic_chunks(EpochInstance* in) {
  for (int j = 0; j < in->gen_nchunks; ++j) {
    if (in->gen_nchunks > 1) set_view(in, j, j > 0);
    int rc = in->gen_nchunks > 1 ? launch_post_generic(in) : EPOCH_OK;
    if (!rc) rc = launch_pre_generic(in);
    if (!rc) rc = launch_grad_branch_generic(in);
    if (rc) {
      set_view(in, -1, false);
      return rc;
    }
  }
  set_view(in, -1, false);
  return EPOCH_OK;
}
}  // namespace

int launch_post(EpochInstance* in) {
  if (nuc(in) && in->budget > 0 && !in->walk_ok)
    return set_error(EPOCH_ERR_STATE, "no tree-walk schedule for the HBM budget");
  if (nuc(in)) return in->walk_ok ? launch_walk_post(in) : launch_nuc_post(in);
  return codon(in) ? launch_codon_post(in) : launch_post_generic_chunks(in);
}

int fastpath_post(EpochInstance* in) {
  if (in->inc_active) {
    EPOCH_PHASE(1, launch_post_incremental(in));
  } else {
    in->work_partials = full_post_count(in);
    EPOCH_PHASE(1, launch_post(in));
  }
  incremental_done(in);
  in->eval_gen++;
  return EPOCH_OK;
}

int fastpath_root(EpochInstance* in) {
  in->eval_gen++;  // new weights or root frequencies change the branch adjoints too
  if (!nuc(in) && !codon(in) && in->gen_nchunks > 1) return EPOCH_OK;  // formed with the chunks' partials
  EPOCH_PHASE(2, nuc(in) ? launch_nuc_root(in) : (codon(in) ? launch_codon_root(in) : launch_root_generic(in)));
  return EPOCH_OK;
}

int fastpath_gradient(EpochInstance* in, bool want_Q) {
  if (nuc(in) && in->walk_ok && in->walk_pre_ok && !want_Q) {
    EPOCH_PHASE(3, launch_walk_pre_grad(in));
  } else if (nuc(in)) {
    EPOCH_PHASE(3, launch_nuc_pre_grad(in));
    EPOCH_PHASE(4, launch_grad_reduce(in, in->nuc_slots, static_cast<const int32_t*>(in->gslots.ptr)));
  } else if (codon(in)) {
    EPOCH_PHASE(3, launch_codon_pre_grad(in));
  } else if (in->gen_nchunks > 1) {
    EPOCH_PHASE(3, launch_pre_grad_generic_chunks(in));
  } else {
    EPOCH_PHASE(3, launch_pre_generic(in));
    EPOCH_PHASE(4, launch_grad_branch_generic(in));
  }
  if (want_Q) EPOCH_PHASE(5, launch_grad_Q(in));
  in->G_gen = in->eval_gen;
  return EPOCH_OK;
}

}  // namespace epochlik
