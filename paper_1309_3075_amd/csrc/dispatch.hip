// Kernel selection for each step of the path.
#include "fastpath.h"

namespace epochlik {

int fastpath_init(EpochInstance*) { return EPOCH_OK; }
void fastpath_release(EpochInstance*) {}
int fastpath_tips_changed(EpochInstance*) { return EPOCH_OK; }
int fastpath_tree_changed(EpochInstance*) { return EPOCH_OK; }

int fastpath_pstage(EpochInstance* in) { return launch_pstage_generic(in); }
int fastpath_post(EpochInstance* in) { return launch_post_generic(in); }
int fastpath_root(EpochInstance* in) { return launch_root_generic(in); }

int fastpath_gradient(EpochInstance* in, bool want_Q) {
  int rc = launch_pre_generic(in);
  if (rc) return rc;
  rc = launch_grad_branch_generic(in);
  if (rc) return rc;
  if (want_Q) rc = launch_grad_Q_generic(in);
  return rc;
}

}  // namespace epochlik
