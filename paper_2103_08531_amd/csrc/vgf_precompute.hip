// vgf_precompute.hip -- plan-time kernels, all in FP64.
//
// VGF (Sec. II of the paper): the closed-form spectrum of the kernel
// truncated at radius L (Eq. 7 in 2D, Eq. 8 in 3D) is sampled on the
// non-negative octant of the 4N-oversampled frequency grid; its inverse DFT
// restricted to offsets |n_a| < N_a is the numerical Green's function. Both
// that restricted inverse DFT and the 2N DFT of the resulting even kernel are
// separable cosine transforms of real even data, applied one axis at a time
// as FP64 matrix-core GEMMs (k_gemm_f64) with cosine tables built on the host.
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

// The axis transforms are dense contractions, out[o][j][i] = sum_m
// mat[m][j] in[o][m][i], so they run as FP64 GEMMs on the matrix cores:
// C[b][r][c] = sum_k A[b][r][k] B[b][k][c] with arbitrary element strides.
// A workgroup of four wavefronts owns a 64 x 64 tile of C (32 x 32 per
// wavefront, four 16 x 16 MFMA blocks) and walks k in slabs of 32 through
// LDS; each thread loads its share of the next slab into registers while the
// wavefronts multiply the current one. v_mfma_f64_16x16x4f64 lane layout:
// lane l holds A[l%16][l/16], B[l/16][l%16] and D[4v + l/16][l%16]
// (v = 0..3). The products are accumulated in increasing k, four at a time.
typedef double d4 __attribute__((ext_vector_type(4)));
struct GemmF64 {
  const double* A;
  const double* B;
  double* C;
  int64_t a_b, a_r, a_k;
  int64_t b_b, b_k, b_c;
  int64_t c_b, c_r, c_c;
  int64_t R, Cn;
  int K;
};
constexpr int GT = 64;               // rows and columns of C per workgroup
constexpr int GK = 32;               // k per LDS slab
constexpr int GE = GT * GK / 256;    // elements of each operand per thread and slab

__global__ __launch_bounds__(256) void k_gemm_f64(GemmF64 g) {
  __shared__ double As[GK][GT + 1];  // [k][row]
  __shared__ double Bs[GK][GT + 1];  // [k][column]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int64_t r0 = (int64_t)blockIdx.y * GT, c0 = (int64_t)blockIdx.x * GT;
  const double* __restrict__ A = g.A + (int64_t)blockIdx.z * g.a_b;
  const double* __restrict__ B = g.B + (int64_t)blockIdx.z * g.b_b;
  const bool a_kfast = g.a_k == 1;  // A contiguous along k (else along rows)
  // element e = tid + 256 i of a slab: A at (row, k) = (e / GK, e % GK) when
  // A is contiguous along k, else (e % GT, e / GT); B at (e / GT, e % GT)
  double ra[GE], rb[GE];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int i = 0; i < GE; ++i) {
      const int e = tid + 256 * i;
      const int rr = a_kfast ? e / GK : e % GT, kk = a_kfast ? e % GK : e / GT;
      const int64_t r = r0 + rr;
      const int k = k0 + kk;
      ra[i] = (r < g.R && k < g.K) ? A[r * g.a_r + (int64_t)k * g.a_k] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < GE; ++i) {
      const int e = tid + 256 * i;
      const int64_t c = c0 + e % GT;
      const int k = k0 + e / GT;
      rb[i] = (c < g.Cn && k < g.K) ? B[(int64_t)k * g.b_k + c * g.b_c] : 0.0;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < GE; ++i) {
      const int e = tid + 256 * i;
      const int rr = a_kfast ? e / GK : e % GT, kk = a_kfast ? e % GK : e / GT;
      As[kk][rr] = ra[i];
      Bs[e / GT][e % GT] = rb[i];
    }
  };
  d4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  fetch(0);
  stash();
  __syncthreads();
  for (int k0 = 0; k0 < g.K; k0 += GK) {
    const bool more = k0 + GK < g.K;
    if (more) fetch(k0 + GK);  // in flight during this slab's products
#pragma unroll
    for (int ks = 0; ks < GK; ks += 4) {
      const int kk = ks + lane / 16;
      double av[2], bv[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) av[i] = As[kk][wr * 32 + i * 16 + lane % 16];
#pragma unroll
      for (int j = 0; j < 2; ++j) bv[j] = Bs[kk][wc * 32 + j * 16 + lane % 16];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();  // every wavefront is done with this slab
    if (more) {
      stash();
      __syncthreads();
    }
  }
  double* __restrict__ C = g.C + (int64_t)blockIdx.z * g.c_b;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = r0 + wr * 32 + i * 16 + 4 * v + lane / 16;
        const int64_t c = c0 + wc * 32 + j * 16 + lane % 16;
        if (r < g.R && c < g.Cn) C[r * g.c_r + c * g.c_c] = acc[i][j][v];
      }
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

// out[o][j][i] = sum_m mat[m][j] in[o][m][i]: per o a GEMM with rows j and
// columns i when the axis has an inner extent, else one GEMM with rows o and
// columns j.
hipError_t launch_axis_apply(const double* in, double* out, const double* mat, int64_t outer,
                             int M, int J, int64_t inner, hipStream_t s) {
  GemmF64 g{};
  g.K = M;
  if (inner > 1) {
    g.A = mat;  // A[j][m] = mat[m][j]
    g.a_b = 0; g.a_r = 1; g.a_k = J;
    g.B = in;   // B[m][i]
    g.b_b = (int64_t)M * inner; g.b_k = inner; g.b_c = 1;
    g.C = out;  // C[j][i]
    g.c_b = (int64_t)J * inner; g.c_r = inner; g.c_c = 1;
    g.R = J;
    g.Cn = inner;
  } else {
    g.A = in;   // A[o][m]
    g.a_b = 0; g.a_r = M; g.a_k = 1;
    g.B = mat;  // B[m][j]
    g.b_b = 0; g.b_k = J; g.b_c = 1;
    g.C = out;  // C[o][j]
    g.c_b = 0; g.c_r = J; g.c_c = 1;
    g.R = outer;
    g.Cn = J;
    outer = 1;
  }
  const int64_t gx = (g.Cn + GT - 1) / GT, gy = (g.R + GT - 1) / GT;
  if (gx > 0x7fffffff || gy > 65535 || outer > 65535) return hipErrorInvalidValue;
  if (gx == 0 || gy == 0 || outer == 0) return hipSuccess;
  hipLaunchKernelGGL(k_gemm_f64, dim3((unsigned)gx, (unsigned)gy, (unsigned)outer), dim3(256), 0, s, g);
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
