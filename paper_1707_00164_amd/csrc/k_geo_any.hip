// Instantiates the L2L kernels whose near blocks are computed on the device
// from the points (every tile shape, every kernel kind), for one row alignment.
#include "kernels.hpp"

namespace gofmm {
namespace dev {
void kernels_geo_any(KernelFn* table) { fill_geo<false>(table); }
}  // namespace dev
}  // namespace gofmm
