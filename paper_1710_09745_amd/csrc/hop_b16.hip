// Hop kernels instantiated for B16 storage (see hop_kernels.h).
#include "hop_kernels.h"

namespace bcg {
template void launch_hop_s<B16>(int, const void*, const void*, void*, const void*, double, int, const Geom&, int,
                                int, const HopShape&, const int*, double*, double2*, int*,
                                hipStream_t);
}  // namespace bcg
