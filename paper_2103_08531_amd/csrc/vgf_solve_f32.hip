// FP32 instantiations of the per-solve passes.
#include "vgf_solve_kernels.hpp"

namespace vgf {
#define VGF_T float
VGF_DEFINE_DISPATCH(float)
#undef VGF_T
}  // namespace vgf
