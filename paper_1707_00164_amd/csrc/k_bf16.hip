// Instantiates the gather-GEMM kernels for one operator precision.
#include "kernels.hpp"

namespace gofmm {
namespace dev {
void kernels_bf16(KernelFn* table, BatchedFn* batched) { fill_table<PREC_BF16>(table, batched); }
}  // namespace dev
}  // namespace gofmm
