// Instantiates the gather-GEMM kernels for one operator precision.
#include "kernels.hpp"

namespace gofmm {
namespace dev {
void kernels_f32(KernelFn* table) { fill_table<PREC_F32>(table); }
}  // namespace dev
}  // namespace gofmm
