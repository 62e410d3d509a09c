// Instantiates the gather-GEMM kernels for one operator precision and row
// alignment.
#include "kernels.hpp"

namespace gofmm {
namespace dev {
void kernels_f32_vec(KernelFn* table, BatchedFn* batched) { fill_table<PREC_F32, true>(table, batched); }
}  // namespace dev
}  // namespace gofmm
