// Kernel selection for each step of the path: the specialised 4-state
// kernels when K == 4 (unless the generic path is forced), the generic any-K
// kernels otherwise.
#include <algorithm>
#include <vector>

#include "fastpath.h"

namespace epochlik {

namespace {
bool nuc(const EpochInstance* in) { return in->path == 1; }
}  // namespace

int fastpath_init(EpochInstance* in) {
  in->path = (in->K == 4 && in->cfg.kernel_path == EPOCH_KERNEL_AUTO) ? 1 : 0;
  if (nuc(in) && (in->cfg.flags & (EPOCH_GRAD_BRANCH | EPOCH_GRAD_Q))) {
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
  if (!nuc(in) || !in->gslots.ptr) return EPOCH_OK;
  std::vector<int32_t> slots;
  nuc_slots_per_node(in, slots);
  int rc = hip_check(hipMemcpyAsync(in->gslots.ptr, slots.data(), slots.size() * sizeof(int32_t),
                                    hipMemcpyHostToDevice, in->stream), "gslots upload");
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

int fastpath_pstage(EpochInstance* in) {
  EPOCH_PHASE(0, launch_pstage_generic(in));
  return EPOCH_OK;
}

int fastpath_post(EpochInstance* in) {
  EPOCH_PHASE(1, nuc(in) ? launch_nuc_post(in) : launch_post_generic(in));
  return EPOCH_OK;
}

int fastpath_root(EpochInstance* in) {
  EPOCH_PHASE(2, nuc(in) ? launch_nuc_root(in) : launch_root_generic(in));
  return EPOCH_OK;
}

int fastpath_gradient(EpochInstance* in, bool want_Q) {
  if (nuc(in)) {
    EPOCH_PHASE(3, launch_nuc_pre_grad(in));
    EPOCH_PHASE(4, launch_grad_reduce(in, in->nuc_slots, static_cast<const int32_t*>(in->gslots.ptr)));
  } else {
    EPOCH_PHASE(3, launch_pre_generic(in));
    EPOCH_PHASE(4, launch_grad_branch_generic(in));
  }
  if (want_Q) EPOCH_PHASE(5, launch_grad_Q_generic(in));
  return EPOCH_OK;
}

}  // namespace epochlik
