// Instantiates the gather-GEMM kernels for one operator precision.
#include "kernels.hpp"

namespace gofmm {
namespace dev {
void kernels_x3(KernelFn* table, BatchedFn* batched) { fill_table<PREC_BF16X3>(table, batched); }
}  // namespace dev
}  // namespace gofmm
