// FP32 per-solve passes of the FFT lengths of group 1 (VGF_P_GROUP1).
#include "vgf_solve_kernels.hpp"

namespace vgf {
#define VGF_T float
VGF_P_GROUP1(VGF_INSTANTIATE_P)
#undef VGF_T
}  // namespace vgf
