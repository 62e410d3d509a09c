// Instantiates the gather-GEMM kernels for one operator precision.
#include "kernels.hpp"

namespace gofmm {
namespace dev {
void kernels_x3(KernelFn* table) { fill_table<PREC_BF16X3>(table); }
}  // namespace dev
}  // namespace gofmm
