// Chain kernels of the packed serving launches with one-wave chains: their launcher, compiled on its own so that the
// groups of chain-kernel instantiations build in parallel.
#include "ns_kernels.h"

namespace ns {

hipError_t launch_slice_packed64(const PackedRun* runs, const int* slice_off, int nr, int slice_blocks, int lk,
                                 size_t slice_lds, hipStream_t st) {
  return launch_slice_packed_nt<64>(runs, slice_off, nr, slice_blocks, lk, slice_lds, st);
}

}  // namespace ns
