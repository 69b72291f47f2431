// Parity hop kernels for FP16 spinors, FP16 links.
#include "dslash_kernels.h"

namespace wl {
template hipError_t launch_hop_r<P16, P16>(const HopArgs &, const LaunchCfg &, hipStream_t);
}  // namespace wl
