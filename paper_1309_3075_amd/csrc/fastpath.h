// Kernel selection: which implementation runs each step of the path.
#pragma once
#include "instance.h"

namespace epochlik {

int fastpath_init(EpochInstance* in);
void fastpath_release(EpochInstance* in);
int fastpath_tips_changed(EpochInstance* in);
int fastpath_tree_changed(EpochInstance* in);
int fastpath_pstage(EpochInstance* in);
int fastpath_after_pstage(EpochInstance* in);  // work that follows the P stage (4-state tip columns)
int fastpath_post(EpochInstance* in);
int fastpath_root(EpochInstance* in);
int fastpath_gradient(EpochInstance* in, bool want_Q);

}  // namespace epochlik
