// Chain kernels of 2-detector runs: their launcher, compiled on its own so that the
// groups of chain-kernel instantiations build in parallel.
#include "ns_kernels.h"

namespace ns {

hipError_t launch_slice_d2(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                           const RunDev& R, const LaunchCfg& C, hipStream_t st) {
  return launch_slice_det<2>(M, Md, T, RB, R, C, st);
}

}  // namespace ns
