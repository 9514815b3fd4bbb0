// FP64 passes of the longer 2D FFT lengths of group 5 (VGF_P_GROUP5): the
// axis-0 R2C / C2R and the multiply pass along the contiguous axis.
#include "vgf_solve_kernels.hpp"

namespace vgf {
#define VGF_T double
VGF_P_GROUP5(VGF_INSTANTIATE_P_WIDE)
#undef VGF_T
}  // namespace vgf
