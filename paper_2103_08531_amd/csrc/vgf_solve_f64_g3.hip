// FP64 per-solve passes of the FFT lengths of group 3 (VGF_P_GROUP3).
#include "vgf_solve_kernels.hpp"

namespace vgf {
#define VGF_T double
VGF_P_GROUP3(VGF_INSTANTIATE_P)
#undef VGF_T
}  // namespace vgf
