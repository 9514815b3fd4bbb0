// FP64 instantiations of the per-solve passes.
#include "vgf_solve_kernels.hpp"

namespace vgf {
#define VGF_T double
VGF_DEFINE_DISPATCH(double)
#undef VGF_T
}  // namespace vgf
