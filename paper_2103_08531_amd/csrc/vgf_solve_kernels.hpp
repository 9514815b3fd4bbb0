// vgf_solve_kernels.hpp -- the per-solve passes of the zero-padded 2N FFT
// convolution (Eq. 3 of the paper, used by both HE and VGF) with the
// spectral field (multiplication by -i k before the inverse FFT, Sec. III.A):
//
//   r2c      pruned real-to-complex transform along the last (contiguous)
//            axis: N reals per line -> N+1 complex (the zero half of the
//            padded line is never read).
//   c2c      strided complex transform along a middle axis (3D axis 1), with
//            pruned input (forward) or pruned output (inverse).
//   fused    along axis 0: pruned forward transform, multiplication by the
//            real kernel spectrum (phi) and by -i k_a times it (E_a), and one
//            pruned inverse transform per requested field, all in one pass
//            (the forward spectrum never leaves registers).
//   fused_adj  the adjoint of `fused`: several pruned forward transforms,
//            accumulated with the conjugate multipliers, one inverse.
//   c2r      inverse complex-to-real transform along the last axis, keeping
//            the first N outputs of the 2N line.
// Pairs of real lines travel as one complex line (re, im) through r2c/c2r.
#pragma once
#include "vgf_fft.hpp"
#include "vgf_internal.hpp"

namespace vgf {

// Tile shape for length P: NL lines (contiguous columns) per workgroup, 16
// complex values per thread, LDS tile <= 64 KiB.
template <typename T, int P> struct Tile {
  static constexpr int CB = (int)sizeof(cplx<T>);
  static constexpr int pick_nl() {
    int nl = sizeof(T) == 4 ? 16 : 8;
    while (nl > 1 && P * nl * CB > 65536) nl /= 2;
    return nl;
  }
  static constexpr int NL = pick_nl();
  static constexpr int EPT = 16;
  static constexpr int NQ = (P + EPT - 1) / EPT;  // threads per line
  static constexpr int NT = NL * NQ;
  static_assert(NT <= 1024, "workgroup too large");
  static_assert(n_stages(P) >= 2, "transform needs at least two stages");
};

// ---------------------------------------------------------------------------
// r2c: lines of N = P/2 reals (contiguous) -> lines of N+1 complex
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ __launch_bounds__((Tile<T, P>::NT)) void k_r2c(const T* __restrict__ in,
                                                       cplx<T>* __restrict__ out, int64_t nlines,
                                                       const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TL = Tile<T, P>;
  constexpr int NL = TL::NL, NT = TL::NT, LP = NL + 1, N = P / 2, H = N + 1;
  constexpr int NSTG = n_stages(P);
  __shared__ C lds[P * LP];
  const int tid = threadIdx.x, l = tid % NL, q = tid / NL;
  const int64_t line0 = (int64_t)blockIdx.x * (2 * NL);

  for (int idx = tid; idx < 2 * NL * N; idx += NT) {
    const int ll = idx / N, pos = idx - ll * N;
    const int64_t line = line0 + ll;
    const T val = line < nlines ? in[line * N + pos] : T(0);
    reinterpret_cast<T*>(&lds[pos * LP + (ll >> 1)])[ll & 1] = val;
  }
  __syncthreads();

  using S0 = Stage<T, P, NT, NL, LP, -1, 0>;
  typename S0::Regs g0;
  S0::template load_first<true>(g0, q, [&](int pos) { return lds[pos * LP + l]; });
  S0::butterflies(g0, q);
  __syncthreads();
  S0::lds_out(g0, lds, l, q);
  __syncthreads();
  using SL = Stage<T, P, NT, NL, LP, -1, NSTG - 1>;
  typename SL::Regs gl;
  middle_and_last<T, P, NT, NL, LP, -1>(gl, lds, tw, l, q);
  __syncthreads();
  SL::lds_out(gl, lds, l, q);
  __syncthreads();

  // Z = X + iY  ->  X[k] = (Z[k] + conj Z[P-k]) / 2,  Y[k] = -i (Z[k] - conj Z[P-k]) / 2
  for (int idx = tid; idx < 2 * NL * H; idx += NT) {
    const int ll = idx / H, k = idx - ll * H;
    const int64_t line = line0 + ll;
    if (line >= nlines) continue;
    const int c = ll >> 1;
    const C z = lds[k * LP + c];
    const C zm = lds[((P - k) % P) * LP + c];
    C o;
    if ((ll & 1) == 0) o = C{T(0.5) * (z.x + zm.x), T(0.5) * (z.y - zm.y)};
    else o = C{T(0.5) * (z.y + zm.y), T(0.5) * (zm.x - z.x)};
    out[line * H + k] = o;
  }
}

// ---------------------------------------------------------------------------
// c2r: lines of N+1 complex (Hermitian half) -> first N reals of the 2N line
// blockIdx.y selects the field (in/out field strides).
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ __launch_bounds__((Tile<T, P>::NT)) void k_c2r(const cplx<T>* __restrict__ in,
                                                       T* __restrict__ out, int64_t nlines,
                                                       int64_t in_fs, int64_t out_fs,
                                                       const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TL = Tile<T, P>;
  constexpr int NL = TL::NL, NT = TL::NT, LP = NL + 1, N = P / 2, H = N + 1;
  constexpr int NSTG = n_stages(P);
  __shared__ C lds[P * LP];
  const int tid = threadIdx.x, l = tid % NL, q = tid / NL;
  const int64_t line0 = (int64_t)blockIdx.x * (2 * NL);
  in += blockIdx.y * in_fs;
  out += blockIdx.y * out_fs;

  // Z[k] = X[k] + i Y[k], Z[P-k] = conj X[k] + i conj Y[k]; the imaginary
  // parts of X, Y at k = 0 and k = N are dropped (real by symmetry).
  for (int idx = tid; idx < NL * H; idx += NT) {
    const int c = idx / H, k = idx - c * H;
    const int64_t la = line0 + 2 * c, lb = la + 1;
    const C X = la < nlines ? in[la * H + k] : C{T(0), T(0)};
    const C Y = lb < nlines ? in[lb * H + k] : C{T(0), T(0)};
    if (k == 0 || k == N) {
      lds[k * LP + c] = C{X.x, Y.x};
    } else {
      lds[k * LP + c] = C{X.x - Y.y, X.y + Y.x};
      lds[(P - k) * LP + c] = C{X.x + Y.y, Y.x - X.y};
    }
  }
  __syncthreads();

  using S0 = Stage<T, P, NT, NL, LP, 1, 0>;
  typename S0::Regs g0;
  S0::template load_first<false>(g0, q, [&](int pos) { return lds[pos * LP + l]; });
  S0::butterflies(g0, q);
  __syncthreads();
  S0::lds_out(g0, lds, l, q);
  __syncthreads();
  using SL = Stage<T, P, NT, NL, LP, 1, NSTG - 1>;
  typename SL::Regs gl;
  middle_and_last<T, P, NT, NL, LP, 1>(gl, lds, tw, l, q);
  __syncthreads();
  SL::template store_last<true>(gl, q, [&](int pos, C v) { lds[pos * LP + l] = v; });
  __syncthreads();

  for (int idx = tid; idx < 2 * NL * N; idx += NT) {
    const int ll = idx / N, pos = idx - ll * N;
    const int64_t line = line0 + ll;
    if (line >= nlines) continue;
    const C z = lds[pos * LP + (ll >> 1)];
    out[line * N + pos] = (ll & 1) ? z.y : z.x;
  }
}

// ---------------------------------------------------------------------------
// c2c along a strided axis. Columns (contiguous) are the lines; element `pos`
// of column `col` in batch b, field f is at
//   base + f*fs + b*bs + pos*ls + col.
// grid = (ceil(ncols/NL), nbatch, nfields)
// ---------------------------------------------------------------------------
template <typename T, int P, int SIGN, bool PRUNE_IN, bool PRUNE_OUT>
__global__ __launch_bounds__((Tile<T, P>::NT)) void k_c2c(const cplx<T>* __restrict__ in,
                                                       cplx<T>* __restrict__ out, StridedArgs sa,
                                                       const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TL = Tile<T, P>;
  constexpr int NL = TL::NL, NT = TL::NT, LP = NL;
  constexpr int NSTG = n_stages(P);
  __shared__ C lds[P * LP];
  const int tid = threadIdx.x, l = tid % NL, q = tid / NL;
  const int64_t col = (int64_t)blockIdx.x * NL + l;
  const bool valid = col < sa.ncols;
  const C* src = in + blockIdx.z * sa.fs_in + blockIdx.y * sa.bs_in + col;
  C* dst = out + blockIdx.z * sa.fs_out + blockIdx.y * sa.bs_out + col;

  using S0 = Stage<T, P, NT, NL, LP, SIGN, 0>;
  typename S0::Regs g0;
  S0::template load_first<PRUNE_IN>(g0, q, [&](int pos) {
    return valid ? src[pos * sa.ls_in] : C{T(0), T(0)};
  });
  S0::butterflies(g0, q);
  S0::lds_out(g0, lds, l, q);
  __syncthreads();
  using SL = Stage<T, P, NT, NL, LP, SIGN, NSTG - 1>;
  typename SL::Regs gl;
  middle_and_last<T, P, NT, NL, LP, SIGN>(gl, lds, tw, l, q);
  SL::template store_last<PRUNE_OUT>(gl, q, [&](int pos, C v) {
    if (valid) dst[pos * sa.ls_out] = v;
  });
}

// signed frequency of index k on a length-P axis (P = 2N), with the Nyquist
// index N mapped to 0 (its derivative factor is zero).
__device__ __forceinline__ int signed_freq_zn(int k, int N) {
  return k < N ? k : (k == N ? 0 : k - 2 * N);
}

// Column coordinates of the axis-0 lines: in 3D column c of the [P1][H2]
// plane is (k1, k2); in 2D it is k1 in [0, H1).
template <typename T> struct ColCoord {
  int f1, s1, k2, s2;  // folded / signed indices of the inner axes
  __device__ __forceinline__ ColCoord(const FusedGeom<T>& g, int64_t col) {
    if (g.dim == 3) {
      const int k1 = (int)(col / g.h_last);
      k2 = (int)(col - (int64_t)k1 * g.h_last);
      f1 = k1 <= g.n1 ? k1 : 2 * g.n1 - k1;
      s1 = signed_freq_zn(k1, g.n1);
      s2 = k2 < g.n2 ? k2 : 0;
    } else {
      const int k1 = (int)col;
      f1 = k1;
      s1 = k1 < g.n1 ? k1 : 0;
      k2 = 0;
      s2 = 0;
    }
  }
  __device__ __forceinline__ int64_t spec_index(const FusedGeom<T>& g, int k0) const {
    const int f0 = k0 <= g.n0 ? k0 : 2 * g.n0 - k0;
    if (g.dim == 3) return ((int64_t)f0 * (g.n1 + 1) + f1) * (g.n2 + 1) + k2;
    return (int64_t)f0 * (g.n1 + 1) + f1;
  }
  // wavenumber of axis a (0..dim-1) at row k0
  __device__ __forceinline__ T wavenumber(const FusedGeom<T>& g, int axis, int k0) const {
    if (axis == 0) return g.ks0 * (T)signed_freq_zn(k0, g.n0);
    if (axis == 1) return g.ks1 * (T)s1;
    return g.ks2 * (T)s2;
  }
};

// ---------------------------------------------------------------------------
// fused axis-0 pass: forward (pruned in) -> per field: multiply, inverse
// (pruned out). in: [N0][ncols], out field f: out + f*out_fs, [N0][ncols].
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ __launch_bounds__((Tile<T, P>::NT)) void k_fused(const cplx<T>* __restrict__ in,
                                                         cplx<T>* __restrict__ out,
                                                         FusedGeom<T> g,
                                                         const T* __restrict__ spec,
                                                         const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TL = Tile<T, P>;
  constexpr int NL = TL::NL, NT = TL::NT, LP = NL;
  constexpr int NSTG = n_stages(P);
  __shared__ C lds[P * LP];
  const int tid = threadIdx.x, l = tid % NL, q = tid / NL;
  const int64_t col = (int64_t)blockIdx.x * NL + l;
  const bool valid = col < g.ncols;
  const C* src = in + col;

  using S0 = Stage<T, P, NT, NL, LP, -1, 0>;
  typename S0::Regs g0;
  S0::template load_first<true>(g0, q, [&](int pos) {
    return valid ? src[pos * g.ncols] : C{T(0), T(0)};
  });
  S0::butterflies(g0, q);
  S0::lds_out(g0, lds, l, q);
  __syncthreads();
  using SL = Stage<T, P, NT, NL, LP, -1, NSTG - 1>;
  typename SL::Regs rh;  // forward spectrum, natural order positions j + r*NB
  middle_and_last<T, P, NT, NL, LP, -1>(rh, lds, tw, l, q);

  using IS0 = Stage<T, P, NT, NL, LP, 1, 0>;
  using ISL = Stage<T, P, NT, NL, LP, 1, NSTG - 1>;
  static_assert(IS0::R == SL::R && IS0::NTASK == SL::NTASK, "register hand-off");

  const ColCoord<T> cc(g, valid ? col : 0);
  T sv[SL::NTASK][SL::R];
#pragma unroll
  for (int t = 0; t < SL::NTASK; ++t) {
    if (!SL::active(t, q)) continue;
    const int j = q + t * SL::NQ;
#pragma unroll
    for (int r = 0; r < SL::R; ++r) sv[t][r] = valid ? spec[cc.spec_index(g, SL::in_pos(j, r))] : T(0);
  }

  for (int fi = 0; fi < g.nf; ++fi) {
    const int code = g.fields[fi];
    typename IS0::Regs v;
#pragma unroll
    for (int t = 0; t < SL::NTASK; ++t) {
      if (!SL::active(t, q)) continue;
      const int j = q + t * SL::NQ;
#pragma unroll
      for (int r = 0; r < SL::R; ++r) {
        const C x = rh.v[t][r];
        const T s = sv[t][r];
        if (code == 0) {
          v.v[t][r] = C{x.x * s, x.y * s};
        } else {  // -i k s x
          const T gk = cc.wavenumber(g, code - 1, SL::in_pos(j, r)) * s;
          v.v[t][r] = C{gk * x.y, -gk * x.x};
        }
      }
    }
    IS0::butterflies(v, q);
    __syncthreads();
    IS0::lds_out(v, lds, l, q);
    __syncthreads();
    typename ISL::Regs o;
    middle_and_last<T, P, NT, NL, LP, 1>(o, lds, tw, l, q);
    C* dst = out + fi * g.out_fs + col;
    ISL::template store_last<true>(o, q, [&](int pos, C val) {
      if (valid) dst[pos * g.ncols] = val;
    });
  }
}

// ---------------------------------------------------------------------------
// adjoint of the fused pass: in field f: in + f*in_fs ([N0][ncols] each);
// acc = sum_f conj(m_f) * FFT(in_f); out = pruned inverse of acc.
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ __launch_bounds__((Tile<T, P>::NT)) void k_fused_adj(const cplx<T>* __restrict__ in,
                                                             cplx<T>* __restrict__ out,
                                                             FusedGeom<T> g,
                                                             const T* __restrict__ spec,
                                                             const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TL = Tile<T, P>;
  constexpr int NL = TL::NL, NT = TL::NT, LP = NL;
  constexpr int NSTG = n_stages(P);
  __shared__ C lds[P * LP];
  const int tid = threadIdx.x, l = tid % NL, q = tid / NL;
  const int64_t col = (int64_t)blockIdx.x * NL + l;
  const bool valid = col < g.ncols;

  using S0 = Stage<T, P, NT, NL, LP, -1, 0>;
  using SL = Stage<T, P, NT, NL, LP, -1, NSTG - 1>;
  using IS0 = Stage<T, P, NT, NL, LP, 1, 0>;
  using ISL = Stage<T, P, NT, NL, LP, 1, NSTG - 1>;
  static_assert(IS0::R == SL::R && IS0::NTASK == SL::NTASK, "register hand-off");

  const ColCoord<T> cc(g, valid ? col : 0);
  T sv[SL::NTASK][SL::R];
  typename IS0::Regs acc;
#pragma unroll
  for (int t = 0; t < SL::NTASK; ++t) {
    const int j = q + t * SL::NQ;
#pragma unroll
    for (int r = 0; r < SL::R; ++r) {
      acc.v[t][r] = C{T(0), T(0)};
      sv[t][r] = (SL::active(t, q) && valid) ? spec[cc.spec_index(g, SL::in_pos(j, r))] : T(0);
    }
  }

  for (int fi = 0; fi < g.nf; ++fi) {
    const int code = g.fields[fi];
    const C* src = in + fi * g.in_fs + col;
    typename S0::Regs g0;
    S0::template load_first<true>(g0, q, [&](int pos) {
      return valid ? src[pos * g.ncols] : C{T(0), T(0)};
    });
    S0::butterflies(g0, q);
    __syncthreads();
    S0::lds_out(g0, lds, l, q);
    __syncthreads();
    typename SL::Regs rh;
    middle_and_last<T, P, NT, NL, LP, -1>(rh, lds, tw, l, q);
#pragma unroll
    for (int t = 0; t < SL::NTASK; ++t) {
      if (!SL::active(t, q)) continue;
      const int j = q + t * SL::NQ;
#pragma unroll
      for (int r = 0; r < SL::R; ++r) {
        const C x = rh.v[t][r];
        const T s = sv[t][r];
        if (code == 0) {
          acc.v[t][r].x += x.x * s;
          acc.v[t][r].y += x.y * s;
        } else {  // conj(-i k s) = +i k s
          const T gk = cc.wavenumber(g, code - 1, SL::in_pos(j, r)) * s;
          acc.v[t][r].x -= gk * x.y;
          acc.v[t][r].y += gk * x.x;
        }
      }
    }
  }
  IS0::butterflies(acc, q);
  __syncthreads();
  IS0::lds_out(acc, lds, l, q);
  __syncthreads();
  typename ISL::Regs o;
  middle_and_last<T, P, NT, NL, LP, 1>(o, lds, tw, l, q);
  C* dst = out + col;
  ISL::template store_last<true>(o, q, [&](int pos, C val) {
    if (valid) dst[pos * g.ncols] = val;
  });
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define VGF_FOR_EACH_P(X) \
  X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(768) X(1024)

template <typename T, int P>
hipError_t launch_r2c_p(const T* in, cplx<T>* out, int64_t nlines, const cplx<T>* tw, hipStream_t s) {
  using TL = Tile<T, P>;
  const int64_t blocks = (nlines + 2 * TL::NL - 1) / (2 * TL::NL);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL((k_r2c<T, P>), dim3((unsigned)blocks), dim3(TL::NT), 0, s, in, out, nlines, tw);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t launch_c2r_p(const cplx<T>* in, T* out, int64_t nlines, int nf, int64_t in_fs,
                        int64_t out_fs, const cplx<T>* tw, hipStream_t s) {
  using TL = Tile<T, P>;
  const int64_t blocks = (nlines + 2 * TL::NL - 1) / (2 * TL::NL);
  if (blocks == 0 || nf == 0) return hipSuccess;
  hipLaunchKernelGGL((k_c2r<T, P>), dim3((unsigned)blocks, nf), dim3(TL::NT), 0, s, in, out, nlines,
                     in_fs, out_fs, tw);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t launch_c2c_p(int sign, const cplx<T>* in, cplx<T>* out, const StridedArgs& sa,
                        const cplx<T>* tw, hipStream_t s) {
  using TL = Tile<T, P>;
  const int64_t bx = (sa.ncols + TL::NL - 1) / TL::NL;
  if (bx == 0 || sa.nbatch == 0 || sa.nfields == 0) return hipSuccess;
  dim3 grid((unsigned)bx, (unsigned)sa.nbatch, (unsigned)sa.nfields);
  if (sign < 0)
    hipLaunchKernelGGL((k_c2c<T, P, -1, true, false>), grid, dim3(TL::NT), 0, s, in, out, sa, tw);
  else
    hipLaunchKernelGGL((k_c2c<T, P, 1, false, true>), grid, dim3(TL::NT), 0, s, in, out, sa, tw);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t launch_fused_p(bool adjoint, const cplx<T>* in, cplx<T>* out, const FusedGeom<T>& g,
                          const T* spec, const cplx<T>* tw, hipStream_t s) {
  using TL = Tile<T, P>;
  const int64_t bx = (g.ncols + TL::NL - 1) / TL::NL;
  if (bx == 0) return hipSuccess;
  if (adjoint)
    hipLaunchKernelGGL((k_fused_adj<T, P>), dim3((unsigned)bx), dim3(TL::NT), 0, s, in, out, g, spec, tw);
  else
    hipLaunchKernelGGL((k_fused<T, P>), dim3((unsigned)bx), dim3(TL::NT), 0, s, in, out, g, spec, tw);
  return hipGetLastError();
}

#define VGF_DEFINE_DISPATCH(T)                                                                   \
  template <>                                                                                    \
  hipError_t launch_r2c<T>(int P, const T* in, cplx<T>* out, int64_t nlines, const cplx<T>* tw,  \
                           hipStream_t s) {                                                      \
    switch (P) {                                                                                 \
      VGF_FOR_EACH_P(VGF_CASE_R2C)                                                               \
      default: return hipErrorInvalidValue;                                                      \
    }                                                                                            \
  }                                                                                              \
  template <>                                                                                    \
  hipError_t launch_c2r<T>(int P, const cplx<T>* in, T* out, int64_t nlines, int nf,             \
                           int64_t in_fs, int64_t out_fs, const cplx<T>* tw, hipStream_t s) {    \
    switch (P) {                                                                                 \
      VGF_FOR_EACH_P(VGF_CASE_C2R)                                                               \
      default: return hipErrorInvalidValue;                                                      \
    }                                                                                            \
  }                                                                                              \
  template <>                                                                                    \
  hipError_t launch_c2c<T>(int P, int sign, const cplx<T>* in, cplx<T>* out,                     \
                           const StridedArgs& sa, const cplx<T>* tw, hipStream_t s) {            \
    switch (P) {                                                                                 \
      VGF_FOR_EACH_P(VGF_CASE_C2C)                                                               \
      default: return hipErrorInvalidValue;                                                      \
    }                                                                                            \
  }                                                                                              \
  template <>                                                                                    \
  hipError_t launch_fused<T>(int P, bool adjoint, const cplx<T>* in, cplx<T>* out,               \
                             const FusedGeom<T>& g, const T* spec, const cplx<T>* tw,            \
                             hipStream_t s) {                                                    \
    switch (P) {                                                                                 \
      VGF_FOR_EACH_P(VGF_CASE_FUSED)                                                             \
      default: return hipErrorInvalidValue;                                                      \
    }                                                                                            \
  }

#define VGF_CASE_R2C(PP) case PP: return launch_r2c_p<VGF_T, PP>(in, out, nlines, tw, s);
#define VGF_CASE_C2R(PP) case PP: return launch_c2r_p<VGF_T, PP>(in, out, nlines, nf, in_fs, out_fs, tw, s);
#define VGF_CASE_C2C(PP) case PP: return launch_c2c_p<VGF_T, PP>(sign, in, out, sa, tw, s);
#define VGF_CASE_FUSED(PP) case PP: return launch_fused_p<VGF_T, PP>(adjoint, in, out, g, spec, tw, s);

}  // namespace vgf
