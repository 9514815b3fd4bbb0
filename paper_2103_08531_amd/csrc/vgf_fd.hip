// vgf_fd.hip -- the finite-difference field of the comparison figures
// (Sec. III.A, "Finite Diff"): E = -D phi with second-order differences,
// centred at interior points and one-sided on the two end planes of each
// axis, and its transpose for the adjoint. Elementwise and HBM-bound: one
// thread per grid point, neighbours along the contiguous axis share cache
// lines, the strided neighbours come through L2.
#include "vgf_internal.hpp"

namespace vgf {

namespace {

// (D phi)[i] * 2h along one axis: centred inside, one-sided at i = 0, N-1
template <typename T>
__device__ __forceinline__ T d_row(const T* __restrict__ f, int64_t base, int64_t st, int i, int N) {
  if (i == 0) return T(-3) * f[base] + T(4) * f[base + st] - f[base + 2 * st];
  if (i == N - 1) return T(3) * f[base] - T(4) * f[base - st] + f[base - 2 * st];
  return f[base + st] - f[base - st];
}

// (D^T y)[j] * 2h along one axis: the transpose of d_row, gathered by column
template <typename T>
__device__ __forceinline__ T dt_col(const T* __restrict__ y, int64_t base, int64_t st, int j, int N) {
  T t = T(0);
  if (j - 1 >= 1 && j - 1 <= N - 2) t += y[base - st];  // row j-1: +1 at column j
  if (j + 1 >= 1 && j + 1 <= N - 2) t -= y[base + st];  // row j+1: -1 at column j
  const int64_t row0 = base - (int64_t)j * st, rowl = base + (int64_t)(N - 1 - j) * st;
  if (j == 0) t += T(-3) * y[row0];
  if (j == 1) t += T(4) * y[row0];
  if (j == 2) t += T(-1) * y[row0];
  if (j == N - 1) t += T(3) * y[rowl];
  if (j == N - 2) t += T(-4) * y[rowl];
  if (j == N - 3) t += y[rowl];
  return t;
}

template <typename T>
__device__ __forceinline__ void fd_field_at(const T* __restrict__ phi, T* __restrict__ E, const FdGeom& g,
                                            int64_t i) {
  int64_t rem = i;
  int idx[3];
  for (int a = g.dim - 1; a >= 0; --a) {
    idx[a] = (int)(rem % g.n[a]);
    rem /= g.n[a];
  }
  for (int a = 0; a < g.dim; ++a)
    E[a * g.total + i] = -d_row(phi, i, g.stride[a], idx[a], g.n[a]) * (T)g.inv2h[a];
}

template <typename T>
__global__ void k_fd_field(const T* __restrict__ phi, T* __restrict__ E, FdGeom g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.total) return;
  fd_field_at(phi, E, g, i);
}

// entry blockIdx.y of a batch group
template <typename T>
__global__ void k_fd_field_entries(const T* const* __restrict__ phi_tab, T* const* __restrict__ E_tab, FdGeom g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.total) return;
  fd_field_at(phi_tab[blockIdx.y], E_tab[blockIdx.y], g, i);
}

template <typename T>
__global__ void k_fd_adjoint(const T* __restrict__ g_phi, const T* __restrict__ g_E, T* __restrict__ out,
                             FdGeom g) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.total) return;
  int64_t rem = i;
  int idx[3];
  for (int a = g.dim - 1; a >= 0; --a) {
    idx[a] = (int)(rem % g.n[a]);
    rem /= g.n[a];
  }
  T acc = g_phi ? g_phi[i] : T(0);
  for (int a = 0; a < g.dim; ++a)
    acc -= dt_col(g_E + a * g.total, i, g.stride[a], idx[a], g.n[a]) * (T)g.inv2h[a];
  out[i] = acc;
}

}  // namespace

template <typename T>
hipError_t launch_fd_field(const T* phi, T* E, const FdGeom& g, hipStream_t s) {
  if (g.total == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((g.total + 255) / 256);
  hipLaunchKernelGGL(k_fd_field<T>, dim3(blocks), dim3(256), 0, s, phi, E, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fd_field_entries(const T* const* phi_tab, T* const* E_tab, int nentry, const FdGeom& g,
                                   hipStream_t s) {
  if (g.total == 0 || nentry == 0) return hipSuccess;
  if (nentry < 0 || nentry > 65535) return hipErrorInvalidValue;
  const unsigned blocks = (unsigned)((g.total + 255) / 256);
  hipLaunchKernelGGL(k_fd_field_entries<T>, dim3(blocks, (unsigned)nentry), dim3(256), 0, s, phi_tab, E_tab, g);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fd_adjoint(const T* g_phi, const T* g_E, T* out, const FdGeom& g, hipStream_t s) {
  if (g.total == 0) return hipSuccess;
  const unsigned blocks = (unsigned)((g.total + 255) / 256);
  hipLaunchKernelGGL(k_fd_adjoint<T>, dim3(blocks), dim3(256), 0, s, g_phi, g_E, out, g);
  return hipGetLastError();
}

template hipError_t launch_fd_field<float>(const float*, float*, const FdGeom&, hipStream_t);
template hipError_t launch_fd_field<double>(const double*, double*, const FdGeom&, hipStream_t);
template hipError_t launch_fd_field_entries<float>(const float* const*, float* const*, int, const FdGeom&,
                                                   hipStream_t);
template hipError_t launch_fd_field_entries<double>(const double* const*, double* const*, int, const FdGeom&,
                                                    hipStream_t);
template hipError_t launch_fd_adjoint<float>(const float*, const float*, float*, const FdGeom&, hipStream_t);
template hipError_t launch_fd_adjoint<double>(const double*, const double*, double*, const FdGeom&,
                                              hipStream_t);

}  // namespace vgf
