// Instantiates the gather-GEMM kernels for one operator precision and row
// alignment.
#include "kernels.hpp"

namespace gofmm {
namespace dev {
void kernels_x3_any(KernelFn* table, BatchedFn* batched) { fill_table<PREC_BF16X3, false>(table, batched); }
}  // namespace dev
}  // namespace gofmm
