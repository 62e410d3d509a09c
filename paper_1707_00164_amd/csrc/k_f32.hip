// Instantiates the gather-GEMM kernels for one operator precision.
#include "kernels.hpp"

namespace gofmm {
namespace dev {
void kernels_f32(KernelFn* table, BatchedFn* batched) { fill_table<PREC_F32>(table, batched); }
}  // namespace dev
}  // namespace gofmm
