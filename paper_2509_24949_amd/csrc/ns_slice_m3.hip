// Move-counting chain kernels of 3-detector runs (64 threads per chain),
// compiled on their own so that they build in parallel with the others.
#include "ns_kernels.h"

namespace ns {

hipError_t launch_slice_mv_d3(const ModelDev& M, const ModelDev* Md, const Tables& T, const RBTables& RB,
                              const RunDev& R, const LaunchCfg& C, hipStream_t st) {
  return launch_slice_nt<3, 64, true>(M, Md, T, RB, R, C, st);
}

}  // namespace ns
