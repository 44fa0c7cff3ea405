// Random-walk chain kernels (the alternative inner kernel) and their
// launcher, compiled on their own so that they build in parallel with the
// slice-chain groups.
#include "ns_kernels.h"

namespace ns {

hipError_t launch_walk(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB, const RunDev& R,
                       hipStream_t st) {
  if (M.likelihood == LK_GAUSS) return launch_walk_t<1, LK_GAUSS, false>(M, Md, T, RB, R, st);
  switch (M.n_det) {
    case 1: return launch_walk_det<1>(M, Md, T, RB, R, st);
    case 2: return launch_walk_det<2>(M, Md, T, RB, R, st);
    default: return launch_walk_det<3>(M, Md, T, RB, R, st);
  }
}

}  // namespace ns
