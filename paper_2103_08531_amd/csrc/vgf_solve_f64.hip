// FP64 dispatch of the per-solve passes: a switch over the FFT length per
// launcher; the launchers of each length are instantiated in the group units
// vgf_solve_f64_g1.hip .. vgf_solve_f64_g6.hip.
#include "vgf_solve_kernels.hpp"

namespace vgf {
#define VGF_T double
VGF_FOR_EACH_P(VGF_EXTERN_P)
VGF_FOR_EACH_P_WIDE(VGF_EXTERN_P_WIDE)
VGF_DEFINE_DISPATCH(double)
#undef VGF_T
}  // namespace vgf
