// vgf_solve_kernels.hpp -- the per-solve passes of the zero-padded 2N FFT
// convolution (Eq. 3 of the paper, shared by HE and VGF) with the field by
// Fourier differentiation (multiplication by -i k before the inverse FFT,
// Sec. III.A).
//
// The factor -i k_a of E_a only involves axis a, so it commutes with the
// transforms along the other axes. Each pass therefore applies the
// derivative of its own axis: the axis-0 pass produces the spectra of phi and
// of E_0 only, the axis-1 inverse produces E_1 from phi's spectrum, and the
// final complex-to-real pass produces E_2 (3D) from phi's spectrum. Forward
// passes of the adjoint do the mirror image: they sum their inputs after
// multiplying by +i k of their own axis.
//
//   k_r2c      pruned real-to-complex transforms along the last (contiguous)
//              axis: N reals per line -> N+1 complex (the zero half of the
//              padded line is never read); sums up to two inputs.
//   k_c2c_fwd  strided forward transform along a middle axis (3D axis 1),
//              pruned input; sums up to two inputs.
//   k_fused    along axis 0: pruned forward transform, multiplication by the
//              real kernel spectrum (phi) and by -i k_0 times it (E_0), and a
//              pruned inverse per output; the forward spectrum never leaves
//              registers.
//   k_fused_adj  the adjoint of k_fused.
//   k_c2c_inv  strided inverse transform along a middle axis, pruned output;
//              up to two outputs from one input.
//   k_c2r      inverse complex-to-real transform along the last axis keeping
//              the first N outputs of the 2N line; up to two outputs.
// Pairs of real lines travel as one complex line (re, im) through r2c/c2r.
// FFT twiddles are staged in LDS once per workgroup.
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

// signed frequency of index k on a length-2N axis, Nyquist index N -> 0
__device__ __forceinline__ int signed_freq_zn(int k, int N) {
  return k < N ? k : (k == N ? 0 : k - 2 * N);
}

// x * (code == 0 ? 1 : code * i * k)
template <typename C, typename T>
__device__ __forceinline__ C deriv(C x, int code, T k) {
  if (code == 0) return x;
  if (code < 0) return C{k * x.y, -k * x.x};
  return C{-k * x.y, k * x.x};
}

template <typename C, int P, int NT>
__device__ __forceinline__ void stage_twiddles(C* twl, const C* __restrict__ tw, int tid) {
  for (int i = tid; i < P; i += NT) twl[i] = tw[i];
}

// ---------------------------------------------------------------------------
// k_r2c: out = sum_t m_t(k) R2C(in_t), lines of N = P/2 reals -> N+1 complex
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ __launch_bounds__((Tile<T, P>::NT)) void k_r2c(R2CArgs<T> a,
                                                         const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TL = Tile<T, P>;
  constexpr int NL = TL::NL, NT = TL::NT, LP = NL + 1, N = P / 2, H = N + 1;
  constexpr int NSTG = n_stages(P);
  constexpr int NSLOT = (2 * NL * H + NT - 1) / NT;
  __shared__ C lds[P * LP];
  __shared__ C twl[P];
  const int tid = threadIdx.x, l = tid % NL, q = tid / NL;
  const int64_t line0 = (int64_t)blockIdx.x * (2 * NL);
  stage_twiddles<C, P, NT>(twl, tw, tid);

  C acc[NSLOT];
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) acc[s] = C{T(0), T(0)};

  for (int term = 0; term < a.d.n; ++term) {
    const T* __restrict__ in = a.in[term];
    const int code = a.d.code[term];
    if (term > 0) __syncthreads();
    for (int idx = tid; idx < 2 * NL * N; idx += NT) {
      const int ll = idx / N, pos = idx - ll * N;
      const int64_t line = line0 + ll;
      const T val = line < a.nlines ? in[line * N + pos] : T(0);
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
    middle_and_last<T, P, NT, NL, LP, -1>(gl, lds, twl, l, q);
    __syncthreads();
    SL::lds_out(gl, lds, l, q);
    __syncthreads();
    // Z = X + iY  ->  X[k] = (Z[k] + conj Z[P-k]) / 2,  Y[k] = -i (Z[k] - conj Z[P-k]) / 2
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
      const int idx = tid + s * NT;
      if (idx >= 2 * NL * H) continue;
      const int ll = idx / H, k = idx - ll * H;
      const int c = ll >> 1;
      const C z = lds[k * LP + c];
      const C zm = lds[((P - k) % P) * LP + c];
      C o;
      if ((ll & 1) == 0) o = C{T(0.5) * (z.x + zm.x), T(0.5) * (z.y - zm.y)};
      else o = C{T(0.5) * (z.y + zm.y), T(0.5) * (zm.x - z.x)};
      o = deriv(o, code, a.d.ks * (T)signed_freq_zn(k, N));
      acc[s].x += o.x;
      acc[s].y += o.y;
    }
  }
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int idx = tid + s * NT;
    if (idx >= 2 * NL * H) continue;
    const int ll = idx / H, k = idx - ll * H;
    const int64_t line = line0 + ll;
    if (line < a.nlines) a.out[line * H + k] = acc[s];
  }
}

// ---------------------------------------------------------------------------
// k_c2r: out_o = first N reals of C2R(m_o(k) in), lines of N+1 complex
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ __launch_bounds__((Tile<T, P>::NT)) void k_c2r(C2RArgs<T> a,
                                                         const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TL = Tile<T, P>;
  constexpr int NL = TL::NL, NT = TL::NT, LP = NL + 1, N = P / 2, H = N + 1;
  constexpr int NSTG = n_stages(P);
  constexpr int NSLOT = (NL * H + NT - 1) / NT;
  __shared__ C lds[P * LP];
  __shared__ C twl[P];
  const int tid = threadIdx.x, l = tid % NL, q = tid / NL;
  const int64_t line0 = (int64_t)blockIdx.x * (2 * NL);
  stage_twiddles<C, P, NT>(twl, tw, tid);

  // this thread's (line pair, k) slots of the input
  C xs[NSLOT], ys[NSLOT];
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int idx = tid + s * NT;
    xs[s] = ys[s] = C{T(0), T(0)};
    if (idx >= NL * H) continue;
    const int c = idx / H, k = idx - c * H;
    const int64_t la = line0 + 2 * c, lb = la + 1;
    if (la < a.nlines) xs[s] = a.in[la * H + k];
    if (lb < a.nlines) ys[s] = a.in[lb * H + k];
  }

  for (int o = 0; o < a.d.n; ++o) {
    const int code = a.d.code[o];
    T* __restrict__ out = a.out[o];
    if (o > 0) __syncthreads();
    // Z[k] = X[k] + i Y[k], Z[P-k] = conj X[k] + i conj Y[k]; the imaginary
    // parts of X, Y at k = 0 and k = N are dropped (real by symmetry).
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
      const int idx = tid + s * NT;
      if (idx >= NL * H) continue;
      const int c = idx / H, k = idx - c * H;
      const T kk = a.d.ks * (T)signed_freq_zn(k, N);
      const C X = deriv(xs[s], code, kk), Y = deriv(ys[s], code, kk);
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
    middle_and_last<T, P, NT, NL, LP, 1>(gl, lds, twl, l, q);
    __syncthreads();
    SL::template store_last<true>(gl, q, [&](int pos, C v) { lds[pos * LP + l] = v; });
    __syncthreads();
    for (int idx = tid; idx < 2 * NL * N; idx += NT) {
      const int ll = idx / N, pos = idx - ll * N;
      const int64_t line = line0 + ll;
      if (line >= a.nlines) continue;
      const C z = lds[pos * LP + (ll >> 1)];
      out[line * N + pos] = (ll & 1) ? z.y : z.x;
    }
  }
}

// ---------------------------------------------------------------------------
// k_c2c_fwd: out = sum_t m_t(pos) FFT(in_t) along a strided axis, pruned input
// grid = (ceil(ncols/NL), nbatch)
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ __launch_bounds__((Tile<T, P>::NT)) void k_c2c_fwd(C2CFwdArgs<T> a,
                                                             const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TL = Tile<T, P>;
  constexpr int NL = TL::NL, NT = TL::NT, LP = NL, N = P / 2;
  constexpr int NSTG = n_stages(P);
  __shared__ C lds[P * LP];
  __shared__ C twl[P];
  const int tid = threadIdx.x, l = tid % NL, q = tid / NL;
  const int64_t col = (int64_t)blockIdx.x * NL + l;
  const bool valid = col < a.g.ncols;
  stage_twiddles<C, P, NT>(twl, tw, tid);
  using S0 = Stage<T, P, NT, NL, LP, -1, 0>;
  using SL = Stage<T, P, NT, NL, LP, -1, NSTG - 1>;
  typename SL::Regs acc;

  for (int term = 0; term < a.d.n; ++term) {
    const C* src = a.in[term] + blockIdx.y * a.g.bs_in + col;
    const int code = a.d.code[term];
    if (term > 0) __syncthreads();
    typename S0::Regs g0;
    S0::template load_first<true>(g0, q, [&](int pos) {
      return valid ? src[pos * a.g.ls_in] : C{T(0), T(0)};
    });
    S0::butterflies(g0, q);
    S0::lds_out(g0, lds, l, q);
    __syncthreads();
    typename SL::Regs gl;
    middle_and_last<T, P, NT, NL, LP, -1>(gl, lds, twl, l, q);
#pragma unroll
    for (int t = 0; t < SL::NTASK; ++t) {
      if (!SL::active(t, q)) continue;
      const int j = q + t * SL::NQ;
#pragma unroll
      for (int r = 0; r < SL::R; ++r) {
        const C v = deriv(gl.v[t][r], code, a.d.ks * (T)signed_freq_zn(SL::out_pos(j, r), N));
        if (term == 0) acc.v[t][r] = v;
        else { acc.v[t][r].x += v.x; acc.v[t][r].y += v.y; }
      }
    }
  }
  C* dst = a.out + blockIdx.y * a.g.bs_out + col;
  SL::template store_last<false>(acc, q, [&](int pos, C v) {
    if (valid) dst[pos * a.g.ls_out] = v;
  });
}

// ---------------------------------------------------------------------------
// k_c2c_inv: out_o = first P/2 of IFFT(m_o(pos) in) along a strided axis
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ __launch_bounds__((Tile<T, P>::NT)) void k_c2c_inv(C2CInvArgs<T> a,
                                                             const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TL = Tile<T, P>;
  constexpr int NL = TL::NL, NT = TL::NT, LP = NL, N = P / 2;
  constexpr int NSTG = n_stages(P);
  __shared__ C lds[P * LP];
  __shared__ C twl[P];
  const int tid = threadIdx.x, l = tid % NL, q = tid / NL;
  const int64_t col = (int64_t)blockIdx.x * NL + l;
  const bool valid = col < a.g.ncols;
  stage_twiddles<C, P, NT>(twl, tw, tid);
  using S0 = Stage<T, P, NT, NL, LP, 1, 0>;
  using SL = Stage<T, P, NT, NL, LP, 1, NSTG - 1>;
  const C* src = a.in + blockIdx.y * a.g.bs_in + col;
  typename S0::Regs gin;
  S0::template load_first<false>(gin, q, [&](int pos) {
    return valid ? src[pos * a.g.ls_in] : C{T(0), T(0)};
  });

  for (int o = 0; o < a.d.n; ++o) {
    const int code = a.d.code[o];
    if (o > 0) __syncthreads();
    typename S0::Regs g0;
#pragma unroll
    for (int t = 0; t < S0::NTASK; ++t) {
      if (!S0::active(t, q)) continue;
      const int j = q + t * S0::NQ;
#pragma unroll
      for (int r = 0; r < S0::R; ++r)
        g0.v[t][r] = deriv(gin.v[t][r], code, a.d.ks * (T)signed_freq_zn(S0::in_pos(j, r), N));
    }
    S0::butterflies(g0, q);
    S0::lds_out(g0, lds, l, q);
    __syncthreads();
    typename SL::Regs gl;
    middle_and_last<T, P, NT, NL, LP, 1>(gl, lds, twl, l, q);
    C* dst = a.out[o] + blockIdx.y * a.g.bs_out + col;
    SL::template store_last<true>(gl, q, [&](int pos, C v) {
      if (valid) dst[pos * a.g.ls_out] = v;
    });
  }
}

// Column coordinates of the axis-0 lines: in 3D column c of the [P1][H2]
// plane is (k1, k2); in 2D it is k1 in [0, H1).
template <typename T> struct ColCoord {
  int f1, k2;  // folded axis-1 index, axis-2 index
  __device__ __forceinline__ ColCoord(const FusedGeom<T>& g, int64_t col) {
    if (g.dim == 3) {
      const int k1 = (int)(col / g.h_last);
      k2 = (int)(col - (int64_t)k1 * g.h_last);
      f1 = k1 <= g.n1 ? k1 : 2 * g.n1 - k1;
    } else {
      f1 = (int)col;
      k2 = 0;
    }
  }
  __device__ __forceinline__ int64_t spec_index(const FusedGeom<T>& g, int k0) const {
    const int f0 = k0 <= g.n0 ? k0 : 2 * g.n0 - k0;
    if (g.dim == 3) return ((int64_t)f0 * (g.n1 + 1) + f1) * (g.n2 + 1) + k2;
    return (int64_t)f0 * (g.n1 + 1) + f1;
  }
};

// ---------------------------------------------------------------------------
// k_fused: forward (pruned in) -> per output field: multiply, inverse
// (pruned out). in: [N0][ncols]; output f at out + f*out_fs, [N0][ncols].
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
  __shared__ C twl[P];
  const int tid = threadIdx.x, l = tid % NL, q = tid / NL;
  const int64_t col = (int64_t)blockIdx.x * NL + l;
  const bool valid = col < g.ncols;
  const C* src = in + col;
  stage_twiddles<C, P, NT>(twl, tw, tid);

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
  middle_and_last<T, P, NT, NL, LP, -1>(rh, lds, twl, l, q);

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
        const C m = C{x.x * s, x.y * s};
        v.v[t][r] = code == 0 ? m
                              : deriv(m, -1, g.ks0 * (T)signed_freq_zn(SL::in_pos(j, r), g.n0));
      }
    }
    IS0::butterflies(v, q);
    __syncthreads();
    IS0::lds_out(v, lds, l, q);
    __syncthreads();
    typename ISL::Regs o;
    middle_and_last<T, P, NT, NL, LP, 1>(o, lds, twl, l, q);
    C* dst = out + fi * g.out_fs + col;
    ISL::template store_last<true>(o, q, [&](int pos, C val) {
      if (valid) dst[pos * g.ncols] = val;
    });
  }
}

// ---------------------------------------------------------------------------
// k_fused_adj: acc = sum_f conj(m_f) * FFT(in_f); out = pruned inverse of acc
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
  __shared__ C twl[P];
  const int tid = threadIdx.x, l = tid % NL, q = tid / NL;
  const int64_t col = (int64_t)blockIdx.x * NL + l;
  const bool valid = col < g.ncols;
  stage_twiddles<C, P, NT>(twl, tw, tid);

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
    middle_and_last<T, P, NT, NL, LP, -1>(rh, lds, twl, l, q);
#pragma unroll
    for (int t = 0; t < SL::NTASK; ++t) {
      if (!SL::active(t, q)) continue;
      const int j = q + t * SL::NQ;
#pragma unroll
      for (int r = 0; r < SL::R; ++r) {
        const C x = rh.v[t][r];
        const T s = sv[t][r];
        C m = C{x.x * s, x.y * s};
        if (code != 0) m = deriv(m, 1, g.ks0 * (T)signed_freq_zn(SL::in_pos(j, r), g.n0));
        acc.v[t][r].x += m.x;
        acc.v[t][r].y += m.y;
      }
    }
  }
  IS0::butterflies(acc, q);
  __syncthreads();
  IS0::lds_out(acc, lds, l, q);
  __syncthreads();
  typename ISL::Regs o;
  middle_and_last<T, P, NT, NL, LP, 1>(o, lds, twl, l, q);
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
hipError_t launch_r2c_p(const R2CArgs<T>& a, const cplx<T>* tw, hipStream_t s) {
  using TL = Tile<T, P>;
  const int64_t blocks = (a.nlines + 2 * TL::NL - 1) / (2 * TL::NL);
  if (blocks == 0 || a.d.n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_r2c<T, P>), dim3((unsigned)blocks), dim3(TL::NT), 0, s, a, tw);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t launch_c2r_p(const C2RArgs<T>& a, const cplx<T>* tw, hipStream_t s) {
  using TL = Tile<T, P>;
  const int64_t blocks = (a.nlines + 2 * TL::NL - 1) / (2 * TL::NL);
  if (blocks == 0 || a.d.n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_c2r<T, P>), dim3((unsigned)blocks), dim3(TL::NT), 0, s, a, tw);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t launch_c2c_fwd_p(const C2CFwdArgs<T>& a, const cplx<T>* tw, hipStream_t s) {
  using TL = Tile<T, P>;
  const int64_t bx = (a.g.ncols + TL::NL - 1) / TL::NL;
  if (bx == 0 || a.g.nbatch == 0 || a.d.n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_c2c_fwd<T, P>), dim3((unsigned)bx, (unsigned)a.g.nbatch), dim3(TL::NT), 0,
                     s, a, tw);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t launch_c2c_inv_p(const C2CInvArgs<T>& a, const cplx<T>* tw, hipStream_t s) {
  using TL = Tile<T, P>;
  const int64_t bx = (a.g.ncols + TL::NL - 1) / TL::NL;
  if (bx == 0 || a.g.nbatch == 0 || a.d.n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_c2c_inv<T, P>), dim3((unsigned)bx, (unsigned)a.g.nbatch), dim3(TL::NT), 0,
                     s, a, tw);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t launch_fused_p(bool adjoint, const cplx<T>* in, cplx<T>* out, const FusedGeom<T>& g,
                          const T* spec, const cplx<T>* tw, hipStream_t s) {
  using TL = Tile<T, P>;
  const int64_t bx = (g.ncols + TL::NL - 1) / TL::NL;
  if (bx == 0 || g.nf == 0) return hipSuccess;
  if (adjoint)
    hipLaunchKernelGGL((k_fused_adj<T, P>), dim3((unsigned)bx), dim3(TL::NT), 0, s, in, out, g, spec, tw);
  else
    hipLaunchKernelGGL((k_fused<T, P>), dim3((unsigned)bx), dim3(TL::NT), 0, s, in, out, g, spec, tw);
  return hipGetLastError();
}

#define VGF_CASE_R2C(PP) case PP: return launch_r2c_p<VGF_T, PP>(a, tw, s);
#define VGF_CASE_C2R(PP) case PP: return launch_c2r_p<VGF_T, PP>(a, tw, s);
#define VGF_CASE_C2CF(PP) case PP: return launch_c2c_fwd_p<VGF_T, PP>(a, tw, s);
#define VGF_CASE_C2CI(PP) case PP: return launch_c2c_inv_p<VGF_T, PP>(a, tw, s);
#define VGF_CASE_FUSED(PP) case PP: return launch_fused_p<VGF_T, PP>(adjoint, in, out, g, spec, tw, s);

#define VGF_DEFINE_DISPATCH(T)                                                                  \
  template <>                                                                                   \
  hipError_t launch_r2c<T>(int P, const R2CArgs<T>& a, const cplx<T>* tw, hipStream_t s) {      \
    switch (P) { VGF_FOR_EACH_P(VGF_CASE_R2C) default: return hipErrorInvalidValue; }           \
  }                                                                                             \
  template <>                                                                                   \
  hipError_t launch_c2r<T>(int P, const C2RArgs<T>& a, const cplx<T>* tw, hipStream_t s) {      \
    switch (P) { VGF_FOR_EACH_P(VGF_CASE_C2R) default: return hipErrorInvalidValue; }           \
  }                                                                                             \
  template <>                                                                                   \
  hipError_t launch_c2c_fwd<T>(int P, const C2CFwdArgs<T>& a, const cplx<T>* tw,               \
                               hipStream_t s) {                                                 \
    switch (P) { VGF_FOR_EACH_P(VGF_CASE_C2CF) default: return hipErrorInvalidValue; }          \
  }                                                                                             \
  template <>                                                                                   \
  hipError_t launch_c2c_inv<T>(int P, const C2CInvArgs<T>& a, const cplx<T>* tw,               \
                               hipStream_t s) {                                                 \
    switch (P) { VGF_FOR_EACH_P(VGF_CASE_C2CI) default: return hipErrorInvalidValue; }          \
  }                                                                                             \
  template <>                                                                                   \
  hipError_t launch_fused<T>(int P, bool adjoint, const cplx<T>* in, cplx<T>* out,              \
                             const FusedGeom<T>& g, const T* spec, const cplx<T>* tw,           \
                             hipStream_t s) {                                                   \
    switch (P) { VGF_FOR_EACH_P(VGF_CASE_FUSED) default: return hipErrorInvalidValue; }         \
  }

}  // namespace vgf
