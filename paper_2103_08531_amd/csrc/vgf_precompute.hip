// vgf_precompute.hip -- plan-time kernels, all in FP64.
//
// VGF (Sec. II of the paper): the closed-form spectrum of the kernel
// truncated at radius L (Eq. 7 in 2D, Eq. 8 in 3D) is sampled on the
// non-negative octant of the 4N-oversampled frequency grid; its inverse DFT
// restricted to offsets |n_a| < N_a is the numerical Green's function. Both
// that restricted inverse DFT and the 2N DFT of the resulting even kernel are
// separable cosine transforms of real even data, applied one axis at a time
// (k_axis_apply) with FP64 cosine tables built on the host.
//
// HE (Eq. 3 and the text after it): the kernel h^d G(|n h|) with the
// singular factor at the origin replaced by 1.
#include <hip/hip_runtime.h>

#include "vgf_internal.hpp"

namespace vgf {

namespace {

constexpr double kPi = 3.14159265358979323846264338327950288;

// F{G^L}(k): 3D  2 (sin(L k / 2) / k)^2,                 k = 0: L^2 / 2
//            2D  (1 - J0(L k)) / k^2 - L ln L J1(L k) / k, k = 0: L^2/4 - L^2 ln(L)/2
__device__ double ghat(int dim, double L, double k) {
  if (dim == 3) {
    if (k == 0.0) return 0.5 * L * L;
    const double s = sin(0.5 * L * k) / k;
    return 2.0 * s * s;
  }
  const double lnL = log(L);
  if (k == 0.0) return 0.25 * L * L - 0.5 * L * L * lnL;
  const double x = L * k;
  return (1.0 - j0(x)) / (k * k) - L * lnL * j1(x) / k;
}

__global__ void k_ghat(double* __restrict__ out, int dim, int64_t e0, int64_t e1, int64_t e2,
                       double dk0, double dk1, double dk2, double L, int64_t total) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  double k2;
  if (dim == 3) {
    const int64_t m2 = i % e2, m1 = (i / e2) % e1, m0 = i / (e1 * e2);
    const double a = (double)m0 * dk0, b = (double)m1 * dk1, c = (double)m2 * dk2;
    k2 = a * a + b * b + c * c;
  } else {
    const int64_t m1 = i % e1, m0 = i / e1;
    const double a = (double)m0 * dk0, b = (double)m1 * dk1;
    k2 = a * a + b * b;
  }
  out[i] = ghat(dim, L, sqrt(k2));
}

__global__ void k_he(double* __restrict__ out, int dim, int64_t n0, int64_t n1, int64_t n2,
                     double h0, double h1, double h2, int64_t total, double origin) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  double r2, vol;
  if (dim == 3) {
    const int64_t a2 = i % n2, a1 = (i / n2) % n1, a0 = i / (n1 * n2);
    const double x = (double)a0 * h0, y = (double)a1 * h1, z = (double)a2 * h2;
    r2 = x * x + y * y + z * z;
    vol = h0 * h1 * h2;
  } else {
    const int64_t a1 = i % n1, a0 = i / n1;
    const double x = (double)a0 * h0, y = (double)a1 * h1;
    r2 = x * x + y * y;
    vol = h0 * h1;
  }
  if (i == 0) {
    out[0] = origin;
    return;
  }
  const double g = (dim == 3) ? 1.0 / (4.0 * kPi * sqrt(r2)) : -0.5 * log(r2) / (2.0 * kPi);
  out[i] = vol * g;
}

// Each thread produces JT consecutive outputs j of one (o, i), so every input
// value it streams is used JT times.
constexpr int JT = 8;
__global__ void k_axis_apply(const double* __restrict__ in, double* __restrict__ out,
                             const double* __restrict__ mat, int64_t outer, int M, int J,
                             int64_t inner, int64_t total) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int JB = (J + JT - 1) / JT;
  const int64_t i = t % inner;
  const int64_t rest = t / inner;
  const int jb = (int)(rest % JB);
  const int64_t o = rest / JB;
  const int j0 = jb * JT;
  double acc[JT];
#pragma unroll
  for (int u = 0; u < JT; ++u) acc[u] = 0.0;
  const double* src = in + o * (int64_t)M * inner + i;
  for (int m = 0; m < M; ++m) {
    const double x = src[(int64_t)m * inner];
    const double* row = mat + (int64_t)m * J + j0;
#pragma unroll
    for (int u = 0; u < JT; ++u)
      if (j0 + u < J) acc[u] = fma(row[u], x, acc[u]);
  }
  double* dst = out + o * (int64_t)J * inner + i;
#pragma unroll
  for (int u = 0; u < JT; ++u)
    if (j0 + u < J) dst[(int64_t)(j0 + u) * inner] = acc[u];
}

template <typename T>
__global__ void k_scale_convert(const double* __restrict__ in, T* __restrict__ out, int64_t count,
                                double scale) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = (T)(in[i] * scale);
}

inline unsigned blocks_for(int64_t total, int bs) { return (unsigned)((total + bs - 1) / bs); }

}  // namespace

hipError_t launch_ghat(double* out, int dim, const int64_t* ext, const double* dk, double L,
                       hipStream_t s) {
  const int64_t e2 = dim == 3 ? ext[2] : 1;
  const int64_t total = ext[0] * ext[1] * e2;
  hipLaunchKernelGGL(k_ghat, dim3(blocks_for(total, 256)), dim3(256), 0, s, out, dim, ext[0],
                     ext[1], e2, dk[0], dk[1], dim == 3 ? dk[2] : 0.0, L, total);
  return hipGetLastError();
}

hipError_t launch_he_kernel(double* out, int dim, const int64_t* n, const double* h, double origin,
                            hipStream_t s) {
  const int64_t n2 = dim == 3 ? n[2] : 1;
  const int64_t total = n[0] * n[1] * n2;
  hipLaunchKernelGGL(k_he, dim3(blocks_for(total, 256)), dim3(256), 0, s, out, dim, n[0], n[1], n2,
                     h[0], h[1], dim == 3 ? h[2] : 0.0, total, origin);
  return hipGetLastError();
}

hipError_t launch_axis_apply(const double* in, double* out, const double* mat, int64_t outer,
                             int M, int J, int64_t inner, hipStream_t s) {
  const int64_t total = outer * ((J + JT - 1) / JT) * inner;
  hipLaunchKernelGGL(k_axis_apply, dim3(blocks_for(total, 256)), dim3(256), 0, s, in, out, mat,
                     outer, M, J, inner, total);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_convert(const double* in, T* out, int64_t count, double scale,
                                hipStream_t s) {
  hipLaunchKernelGGL(k_scale_convert<T>, dim3(blocks_for(count, 256)), dim3(256), 0, s, in, out,
                     count, scale);
  return hipGetLastError();
}

template hipError_t launch_scale_convert<float>(const double*, float*, int64_t, double, hipStream_t);
template hipError_t launch_scale_convert<double>(const double*, double*, int64_t, double, hipStream_t);

}  // namespace vgf
