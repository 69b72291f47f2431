// Parity hop kernels for FP64 spinors, FP64 links.
#include "dslash_kernels.h"

namespace wl {
template hipError_t launch_hop_r<P64, P64>(const HopArgs &, const LaunchCfg &, hipStream_t);
}  // namespace wl
