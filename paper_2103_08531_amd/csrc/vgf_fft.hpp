// vgf_fft.hpp -- device-side building blocks of the batched FFTs used by the
// solve path (gfx950, wave64).
//
// A workgroup transforms NL lines of length P at once. The lines are the
// columns of an LDS tile laid out [position][line] with row pitch LP, so the
// NL lines of a tile are contiguous in both HBM (adjacent columns of the
// array) and LDS, and a wavefront touches consecutive addresses in both.
// Thread tid owns line l = tid % NL and the butterflies j = q, q + NQ, ...
// (q = tid / NL, NQ = NT / NL) of every stage.
//
// The transform is a Stockham autosort FFT: stage s with radix R and
// Ns = product of the earlier radices reads positions j + r*P/R, multiplies
// input r by w^(r*(j mod Ns)*P/(Ns*R)) (w = exp(-+2 pi i / P)), does an
// R-point DFT and writes positions (j div Ns)*Ns*R + (j mod Ns) + r*Ns.
// Results come out in natural order. Radices are 8, 4, 2 and 3.
//
// Zero padding to 2N (Eq. 3 of the paper pads rho to twice the box) is never
// materialised: the forward transforms see only the first P/2 inputs, and
// the first stage (radix R even, Ns = 1) skips its inputs r >= R/2, which are
// exactly the positions >= P/2. Symmetrically, the inverse transforms keep
// only the first P/2 outputs, and their last stage (Ns = P/R) stores only
// outputs r < R/2.
#pragma once
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "vgf_internal.hpp"
#include "vgf_lds_pads.hpp"

namespace vgf {

// Every floating-point operation of the transforms is written out: products
// that should be fused use fmaT, all others are plain operations, and the
// solve kernels are compiled without contraction (-ffp-contract=off). The
// rounding of each result is then fixed by the source, so every launch shape
// (tile schedule, batch grouping) that runs the same per-line code gives the
// same bits, whatever registers the compiler assigns in each instantiation.
__host__ __device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__host__ __device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename C> __host__ __device__ __forceinline__ C c_add(C a, C b) { return C{a.x + b.x, a.y + b.y}; }
template <typename C> __host__ __device__ __forceinline__ C c_sub(C a, C b) { return C{a.x - b.x, a.y - b.y}; }
// a * b: one product and one fused multiply-add per component
template <typename C> __host__ __device__ __forceinline__ C c_mul(C a, C b) {
  return C{fmaT(a.x, b.x, -(a.y * b.y)), fmaT(a.x, b.y, a.y * b.x)};
}
// a * conj(b)
template <typename C> __host__ __device__ __forceinline__ C c_mulc(C a, C b) {
  return C{fmaT(a.x, b.x, a.y * b.y), fmaT(a.y, b.x, -(a.x * b.y))};
}
// b + s * a for a real s (two fused multiply-adds)
template <typename C, typename T> __host__ __device__ __forceinline__ C c_fma(T s, C a, C b) {
  return C{fmaT(s, a.x, b.x), fmaT(s, a.y, b.y)};
}
// multiply by S*i  (S = -1: -i, S = +1: +i)
template <int S, typename C> __host__ __device__ __forceinline__ C c_muli(C a) {
  if constexpr (S < 0) return C{a.y, -a.x};
  else return C{-a.y, a.x};
}
// b + S i s a for a real s: S i s a = (-S s a.y, S s a.x)
template <int S, typename C, typename T> __host__ __device__ __forceinline__ C c_fmai(T s, C a, C b) {
  if constexpr (S < 0) return C{fmaT(s, a.y, b.x), fmaT(-s, a.x, b.y)};
  else return C{fmaT(-s, a.y, b.x), fmaT(s, a.x, b.y)};
}

// ---------------------------------------------------------------------------
// radix plan (compile time). P = 2^a 3^b. Forward order: the power-of-two
// stages (8s, then the 4s or the 2), then the 3s; the inverse uses the
// reverse order, so the last forward stage and the first inverse stage have
// the same radix and the same butterfly-to-thread map. Where 2^a = 8^q * 2
// (a = 3q + 1, q >= 1) and b >= 1, the 2 and one 3 form a radix-6 stage
// (8^q, 6, 3^(b-1)) instead of 8^(q-1), 4, 4, 3^b: one stage and one LDS
// exchange fewer. Only where the radix-6 stage's P/6 butterflies fill the
// 64 lanes of a wavefront evenly (P/6 <= 64 or a multiple of 64: P = 48,
// 144, 384, 1152); at 432 and 1296 its second round of butterflies would
// leave most lanes idle (measured slower in FP64 at 216^3).
// ---------------------------------------------------------------------------
constexpr int pow2_of(int P) { int a = 0; while (P % 2 == 0) { P /= 2; ++a; } return a; }
constexpr int pow3_of(int P) { while (P % 2 == 0) P /= 2; int b = 0; while (P % 3 == 0) { P /= 3; ++b; } return b; }
constexpr bool fft_len_ok(int P) {
  int p = P;
  while (p % 2 == 0) p /= 2;
  while (p % 3 == 0) p /= 3;
  return p == 1 && pow2_of(P) >= 1;
}
constexpr bool radix6_plan(int P) {
  return pow2_of(P) % 3 == 1 && pow2_of(P) >= 4 && pow3_of(P) >= 1 && (P / 6 <= 64 || (P / 6) % 64 == 0);
}
constexpr int n_pow2_stages(int P) { return radix6_plan(P) ? pow2_of(P) / 3 : (pow2_of(P) + 2) / 3; }
constexpr int n_stages(int P) { return n_pow2_stages(P) + pow3_of(P); }
constexpr int fwd_radix(int P, int s) {
  const int a = pow2_of(P), q = a / 3, r = a % 3, s2 = n_pow2_stages(P);
  if (radix6_plan(P)) return s < q ? 8 : (s == q ? 6 : 3);
  if (s >= s2) return 3;
  if (r == 0) return 8;
  if (r == 2) return (s < q) ? 8 : 4;
  if (q == 0) return 2;
  return (s < q - 1) ? 8 : 4;
}
template <int SIGN> constexpr int radix_at(int P, int s) {
  return SIGN < 0 ? fwd_radix(P, s) : fwd_radix(P, n_stages(P) - 1 - s);
}
template <int SIGN> constexpr int ns_at(int P, int s) {
  int ns = 1;
  for (int i = 0; i < s; ++i) ns *= radix_at<SIGN>(P, i);
  return ns;
}
// forward and inverse run the same radix sequence (one twiddle table serves
// both directions)
template <int P> constexpr bool radix_palindrome() {
  for (int s = 0; s < n_stages(P); ++s)
    if (fwd_radix(P, s) != fwd_radix(P, n_stages(P) - 1 - s)) return false;
  return true;
}

// ---------------------------------------------------------------------------
// R-point DFTs in registers, y_k = sum_j x_j exp(S 2 pi i jk / R)
// ---------------------------------------------------------------------------
template <typename T> struct K {
  static constexpr T r12 = T(0.70710678118654752440084436210484903928);  // 1/sqrt(2)
  static constexpr T s3 = T(0.86602540378443864676372317075293618347);   // sqrt(3)/2
};

template <int S, typename C> __host__ __device__ __forceinline__ void dft4(C& a0, C& a1, C& a2, C& a3) {
  C t0 = c_add(a0, a2), t1 = c_sub(a0, a2);
  C t2 = c_add(a1, a3), t3 = c_muli<S>(c_sub(a1, a3));
  a0 = c_add(t0, t2);
  a2 = c_sub(t0, t2);
  a1 = c_add(t1, t3);
  a3 = c_sub(t1, t3);
}

// dft4 with a2 = a3 = 0 (the zero half of a padded input; adding a zero
// explicitly would not be folded away, since x + 0 is not x for x = -0)
template <int S, typename C> __host__ __device__ __forceinline__ void dft4_half(C& a0, C& a1, C& a2, C& a3) {
  const C b0 = a0, b1 = a1, t3 = c_muli<S>(a1);
  a0 = c_add(b0, b1);
  a2 = c_sub(b0, b1);
  a1 = c_add(b0, t3);
  a3 = c_sub(b0, t3);
}

// The last level of a radix-8 DIT butterfly: v_k = e_k + W^k o_k and
// v_{k+4} = e_k - W^k o_k with W = exp(S 2 pi i / 8) = (1 + S i)/sqrt2 and
// o_k = c o'_k. W o = c/sqrt2 (o.x - S o.y, o.y + S o.x) and
// W^3 o = -c/sqrt2 (o.x + S o.y, o.y - S o.x): the sums are formed first and
// the scale enters the fused multiply-adds.
template <int S, typename C, typename T>
__host__ __device__ __forceinline__ void dft8_combine(C* v, C e0, C e1, C e2, C e3, C o0, C o1, C o2, C o3, T c) {
  const T q = c * K<T>::r12;
  const C p1 = S < 0 ? C{o1.x + o1.y, o1.y - o1.x} : C{o1.x - o1.y, o1.y + o1.x};
  const C p3 = S < 0 ? C{o3.x - o3.y, o3.y + o3.x} : C{o3.x + o3.y, o3.y - o3.x};
  v[0] = c_fma(c, o0, e0);
  v[4] = c_fma(-c, o0, e0);
  v[2] = c_fmai<S>(c, o2, e2);
  v[6] = c_fmai<S>(-c, o2, e2);
  v[1] = c_fma(q, p1, e1);
  v[5] = c_fma(-q, p1, e1);
  v[3] = c_fma(-q, p3, e3);
  v[7] = c_fma(q, p3, e3);
}

template <int S, bool HALF, typename C> __host__ __device__ __forceinline__ void dft8_impl(C* v) {
  using T = decltype(v[0].x);
  // even / odd 4-point DFTs
  C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  if constexpr (HALF) {
    dft4_half<S>(e0, e1, e2, e3);
    dft4_half<S>(o0, o1, o2, o3);
  } else {
    dft4<S>(e0, e1, e2, e3);
    dft4<S>(o0, o1, o2, o3);
  }
  // W^0 and W^2 need no product: o0 and S i o2 are added as they are
  const T q = K<T>::r12;
  const C p1 = S < 0 ? C{o1.x + o1.y, o1.y - o1.x} : C{o1.x - o1.y, o1.y + o1.x};
  const C p3 = S < 0 ? C{o3.x - o3.y, o3.y + o3.x} : C{o3.x + o3.y, o3.y - o3.x};
  const C t2 = c_muli<S>(o2);
  v[0] = c_add(e0, o0);
  v[4] = c_sub(e0, o0);
  v[2] = c_add(e2, t2);
  v[6] = c_sub(e2, t2);
  v[1] = c_fma(q, p1, e1);
  v[5] = c_fma(-q, p1, e1);
  v[3] = c_fma(-q, p3, e3);
  v[7] = c_fma(q, p3, e3);
}

template <int S, typename C> __host__ __device__ __forceinline__ void dft3_impl(C* v) {
  using T = decltype(v[0].x);
  const C a0 = v[0], a1 = v[1], a2 = v[2];
  const C s = c_add(a1, a2), d = c_sub(a1, a2);
  const C m = c_fma(T(-0.5), s, a0);  // a0 - s/2
  v[0] = c_add(a0, s);
  v[1] = c_fmai<S>(K<T>::s3, d, m);   // m + S i (sqrt3/2) d
  v[2] = c_fmai<S>(-K<T>::s3, d, m);
}

// 6-point DFT as two 3-point DFTs of the even and odd inputs, combined with
// W = exp(S 2 pi i / 6) = 1/2 + S i sqrt(3)/2 and W^2 = -1/2 + S i sqrt(3)/2
// (W^3 = -1): v_k = e_k + W^k o_k, v_{k+3} = e_k - W^k o_k.
template <int S, typename C> __host__ __device__ __forceinline__ void dft6_impl(C* v) {
  using T = decltype(v[0].x);
  C e[3] = {v[0], v[2], v[4]};
  C o[3] = {v[1], v[3], v[5]};
  dft3_impl<S>(e);
  dft3_impl<S>(o);
  const T h = T(0.5);
  const C w1 = c_fmai<S>(K<T>::s3, o[1], C{h * o[1].x, h * o[1].y});    // W o_1
  const C w2 = c_fmai<S>(K<T>::s3, o[2], C{-h * o[2].x, -h * o[2].y});  // W^2 o_2
  v[0] = c_add(e[0], o[0]);
  v[3] = c_sub(e[0], o[0]);
  v[1] = c_add(e[1], w1);
  v[4] = c_sub(e[1], w1);
  v[2] = c_add(e[2], w2);
  v[5] = c_sub(e[2], w2);
}

// run: full R-point DFT; run_half: the same with inputs R/2 .. R-1 zero
// (never read)
template <int R, int S, typename C> struct Dft;
template <int S, typename C> struct Dft<2, S, C> {
  __host__ __device__ __forceinline__ static void run(C* v) { C a = v[0], b = v[1]; v[0] = c_add(a, b); v[1] = c_sub(a, b); }
  __host__ __device__ __forceinline__ static void run_half(C* v) { v[1] = v[0]; }
};
template <int S, typename C> struct Dft<3, S, C> {
  __host__ __device__ __forceinline__ static void run(C* v) { dft3_impl<S>(v); }
};
template <int S, typename C> struct Dft<4, S, C> {
  __host__ __device__ __forceinline__ static void run(C* v) { dft4<S>(v[0], v[1], v[2], v[3]); }
  __host__ __device__ __forceinline__ static void run_half(C* v) { dft4_half<S>(v[0], v[1], v[2], v[3]); }
};
template <int S, typename C> struct Dft<6, S, C> {
  __host__ __device__ __forceinline__ static void run(C* v) { dft6_impl<S>(v); }
};
template <int S, typename C> struct Dft<8, S, C> {
  __host__ __device__ __forceinline__ static void run(C* v) { dft8_impl<S, false>(v); }
  __host__ __device__ __forceinline__ static void run_half(C* v) { dft8_impl<S, true>(v); }
};

// ---------------------------------------------------------------------------
// Twiddled radix-8 and radix-4 butterflies with the twiddles in scaled form.
// Input r of a butterfly is multiplied by w_r = cos(th_r) + S i sin(th_r),
// th_r = 2 pi r m / (Ns R) for butterfly m = j mod Ns. Writing
// w_r = c_r (1 + S i t_r), c_r = cos th_r, t_r = tan th_r, the rotation
// u_r = a_r (1 + S i t_r) costs two fused multiply-adds, and the scale c_r is
// carried into the sums of the DFT, where it rides on fused multiply-adds
// that are needed anyway: x2 + x6 = c2 (u2 + (c6/c2) u6), and so on. Only
// the input with th = pi m / Ns (r = R/2), whose cosine vanishes at
// m = Ns/2, keeps the full complex product. The cosines that are divided by
// are nonzero for Ns not divisible by 3 (the stages that use this form).
// Slots of a radix-8 butterfly (7 complex values, the table space of the
// R-1 plain twiddles): (t1, t2), (t3, t5), (t6, t7), w4, (c6/c2, c5/c1),
// (c7/c3, c3/c1), (c2, c1). Radix 4: (t1, t3), w2, (c3/c1, c1). A plain
// twiddle w is stored with the forward sign (cos th, -sin th) and conjugated
// for S > 0; the tangents are those of the angle th itself (th >= 0).
// ---------------------------------------------------------------------------
template <int S, typename C, typename T>
__host__ __device__ __forceinline__ C rot_tan(C a, T t) {  // a (1 + S i t)
  if constexpr (S < 0) return C{fmaT(t, a.y, a.x), fmaT(-t, a.x, a.y)};
  else return C{fmaT(-t, a.y, a.x), fmaT(t, a.x, a.y)};
}
template <int S, typename C> __host__ __device__ __forceinline__ C twiddle_mul(C a, C w) {
  if constexpr (S < 0) return c_mul(a, w);
  else return c_mulc(a, w);
}

template <int S, typename C> __host__ __device__ __forceinline__ void dft8_tw(C* v, const C* w) {
  using T = decltype(v[0].x);
  const T t1 = w[0].x, t2 = w[0].y, t3 = w[1].x, t5 = w[1].y, t6 = w[2].x, t7 = w[2].y;
  const T r62 = w[4].x, r51 = w[4].y, r73 = w[5].x, r31 = w[5].y, c2 = w[6].x, c1 = w[6].y;
  const C u1 = rot_tan<S>(v[1], t1), u2 = rot_tan<S>(v[2], t2), u3 = rot_tan<S>(v[3], t3);
  const C u5 = rot_tan<S>(v[5], t5), u6 = rot_tan<S>(v[6], t6), u7 = rot_tan<S>(v[7], t7);
  const C x4 = twiddle_mul<S>(v[4], w[3]);
  // even half: DFT4 of (a0, c2 u2, x4, c2 (c6/c2) u6)
  const C g0 = c_add(v[0], x4), g1 = c_sub(v[0], x4);
  const C s26 = c_fma(r62, u6, u2), d26 = c_fma(-r62, u6, u2);
  const C e0 = c_fma(c2, s26, g0), e2 = c_fma(-c2, s26, g0);
  const C e1 = c_fmai<S>(c2, d26, g1), e3 = c_fmai<S>(-c2, d26, g1);
  // odd half: DFT4 of (c1 u1, c3 u3, c5 u5, c7 u7) = c1 (o0', o1', o2', o3')
  const C s15 = c_fma(r51, u5, u1), d15 = c_fma(-r51, u5, u1);
  const C s37 = c_fma(r73, u7, u3), d37 = c_fma(-r73, u7, u3);
  const C o0 = c_fma(r31, s37, s15), o2 = c_fma(-r31, s37, s15);
  const C o1 = c_fmai<S>(r31, d37, d15), o3 = c_fmai<S>(-r31, d37, d15);
  dft8_combine<S>(v, e0, e1, e2, e3, o0, o1, o2, o3, c1);
}

template <int S, typename C> __host__ __device__ __forceinline__ void dft4_tw(C* v, const C* w) {
  using T = decltype(v[0].x);
  const T t1 = w[0].x, t3 = w[0].y, r31 = w[2].x, c1 = w[2].y;
  const C u1 = rot_tan<S>(v[1], t1), u3 = rot_tan<S>(v[3], t3);
  const C x2 = twiddle_mul<S>(v[2], w[1]);
  const C g0 = c_add(v[0], x2), g1 = c_sub(v[0], x2);
  const C s13 = c_fma(r31, u3, u1), d13 = c_fma(-r31, u3, u1);
  v[0] = c_fma(c1, s13, g0);
  v[2] = c_fma(-c1, s13, g0);
  v[1] = c_fmai<S>(c1, d13, g1);
  v[3] = c_fmai<S>(-c1, d13, g1);
}

// Stages whose twiddles are stored in the scaled form above.
constexpr bool stage_scaled(int R, int NS) { return NS > 1 && (R == 8 || R == 4) && NS % 3 != 0; }

// ---------------------------------------------------------------------------
// one Stockham stage of a workgroup-wide batched transform
// ---------------------------------------------------------------------------
// LDS layouts of a tile of NL lines: 0 = [position][line] with row pitch LP
// (strided axes: adjacent lines are adjacent columns in HBM); 1 = [line][position]
// with one pad slot every 8 positions and line pitch LP (contiguous axes,
// one wavefront per line group; the pad keeps radix-8 scatters free of bank
// conflicts); 2 = [line][position] of a 512-point line held by one wavefront
// (three radix-8 stages, one butterfly per lane), with a layout of its own for
// each of the two exchanges (see Stage::in_index); 3 = [line][position] with a
// pad of its own per exchange, p + k (p >> s), from the table lds_pad (the
// pad of layout 1 where the table keeps it).
template <int LAYOUT, int LP>
__device__ __forceinline__ int lds_index(int pos, int l) {
  static_assert(LAYOUT == 0 || LAYOUT == 1, "layouts 2 and 3 are addressed per exchange");
  if constexpr (LAYOUT == 0) return pos * LP + l;
  else return l * LP + pos + (pos >> 3);
}
template <int P> constexpr int line_pitch() { return P + P / 8; }

template <typename T, int P, int NT, int NL, int LP, int SIGN, int S, int LAYOUT = 0>
struct Stage {
  using C = cplx<T>;
  static constexpr int R = radix_at<SIGN>(P, S);
  static constexpr int NS = ns_at<SIGN>(P, S);
  static constexpr int NB = P / R;  // butterflies per line
  static constexpr int NQ = NT / NL;
  static constexpr int NTASK = (NB + NQ - 1) / NQ;
  static constexpr bool EXACT = (NB % NQ) == 0;
  static constexpr bool LAST = (S == n_stages(P) - 1);
  static constexpr bool SCALED = stage_scaled(R, NS);
  static_assert(NT % NL == 0, "threads must cover whole lines");

  struct Regs { C v[NTASK][R]; };
  // the twiddle slots of the thread's butterflies (R - 1 per butterfly)
  struct Tw { C w[NTASK][R - 1]; };

  __device__ __forceinline__ static bool active(int t, int q) { return EXACT || (q + t * NQ) < NB; }
  __device__ __forceinline__ static int in_pos(int j, int r) { return j + r * NB; }
  __device__ __forceinline__ static int out_pos(int j, int r) { return (j / NS) * NS * R + (j % NS) + r * NS; }

  // first stage (Ns = 1, no twiddles); ld(j, r) returns the input at
  // position j + r*NB (r is a compile-time constant at every call).
  // PRUNE: inputs at positions >= P/2 are zero and are not read.
  template <bool PRUNE, class Load>
  __device__ __forceinline__ static void load_first(Regs& g, int q, Load&& ld) {
    static_assert(S == 0, "load_first is the first stage");
    static_assert(!PRUNE || R % 2 == 0, "pruned inputs need an even first radix");
#pragma unroll
    for (int t = 0; t < NTASK; ++t) {
      if (!active(t, q)) continue;
      const int j = q + t * NQ;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (PRUNE && r >= R / 2) g.v[t][r] = C{T(0), T(0)};
        else g.v[t][r] = ld(j, r);
      }
    }
  }

  // R-point DFTs of the first stage (no twiddles). HALF: the first stage of
  // a pruned load (inputs r >= R/2 are zero)
  template <bool HALF = false> __device__ __forceinline__ static void butterflies(Regs& g, int q) {
    static_assert(NS == 1, "a stage with twiddles uses tw_butterflies");
#pragma unroll
    for (int t = 0; t < NTASK; ++t) {
      if (!active(t, q)) continue;
      if constexpr (HALF) Dft<R, SIGN, C>::run_half(g.v[t]);
      else Dft<R, SIGN, C>::run(g.v[t]);
    }
  }

  // This stage's twiddle slots from a stage-major table (LDS or global
  // memory): slot k of butterfly j at (NS - R_0) + k*NS + (j mod NS), so the
  // R-1 slots of one butterfly are read from one base with immediate offsets.
  __device__ __forceinline__ static void load_tw(Tw& tw, const C* tab, int q) {
    static_assert(NS > 1, "the first stage has no twiddles");
#pragma unroll
    for (int t = 0; t < NTASK; ++t) {
      if (!active(t, q)) continue;
      const int j = q + t * NQ;
      const C* tb = tab + (NS - radix_at<SIGN>(P, 0)) + (j % NS);
#pragma unroll
      for (int k = 0; k < R - 1; ++k) tw.w[t][k] = tb[k * NS];
    }
  }

  // twiddles and R-point DFTs of a stage with NS > 1
  __device__ __forceinline__ static void tw_butterflies(Regs& g, const Tw& tw, int q) {
#pragma unroll
    for (int t = 0; t < NTASK; ++t) {
      if (!active(t, q)) continue;
      if constexpr (SCALED && R == 8) {
        dft8_tw<SIGN>(g.v[t], tw.w[t]);
      } else if constexpr (SCALED && R == 4) {
        dft4_tw<SIGN>(g.v[t], tw.w[t]);
      } else {
#pragma unroll
        for (int r = 1; r < R; ++r) g.v[t][r] = twiddle_mul<SIGN>(g.v[t][r], tw.w[t][r - 1]);
        Dft<R, SIGN, C>::run(g.v[t]);
      }
    }
  }

  // LDS index of in_pos(j, r) / out_pos(j, r) of line l, written as a
  // per-(j, l) base plus r times a compile-time step wherever the layout
  // allows it, so one address serves all R accesses (immediate offsets).
  //
  // Layout 2: position p = 64 a2 + 8 a1 + a0 sits at
  //   exchange 0 (stage 0 -> 1): 72 a2 + 18 (a1 >> 1) + (a1 & 1) + 2 a0,
  //   exchange 1 (stage 1 -> 2): 72 a2 + 8 a1 + a0.
  // LDS resolves bank conflicts of 8-byte writes over each half-wavefront
  // (32 lanes, 32 slots of 8 bytes) and of 8-byte reads over each quarter
  // (16 lanes, 16 slots). Stage 0 writes (a2, a1) = lane digits and a0 = r,
  // stage 1 writes a2 = lane >> 3, a0 = lane & 7 and a1 = r, and both reads
  // take a2 = r and (a1, a0) = lane digits: every access of the three
  // patterns then touches distinct slots, while layout 1 serves the reads in
  // two passes.
  // layout 1 addressing (also layout 3 where its table keeps that pad)
  __device__ __forceinline__ static int in_index1(int j, int r, int l) {
    if constexpr (NB % 8 == 0) return l * LP + j + (j >> 3) + r * (NB + NB / 8);
    else return lds_index<1, LP>(in_pos(j, r), l);
  }
  __device__ __forceinline__ static int out_index1(int j, int r, int l) {
    if constexpr (NS % 8 == 0 || (NS == 1 && 8 % R == 0)) {
      const int u = (j / NS) * NS * R + (j % NS);
      return l * LP + u + (u >> 3) + r * (NS == 1 ? 1 : NS + NS / 8);
    } else {
      return lds_index<1, LP>(out_pos(j, r), l);
    }
  }
  // layout 3: the pad of exchange S - 1 (reads) or S (writes); the table
  // holds only pads under which every access is a per-lane base plus r times
  // a constant
  static constexpr LdsPad pad_in() { return lds_pad(P, SIGN, S - 1, NQ); }
  static constexpr LdsPad pad_out() { return lds_pad(P, SIGN, S, NQ); }
  static constexpr bool pad1(LdsPad p) { return p.k == 1 && p.s == 3; }

  __device__ __forceinline__ static int in_index(int j, int r, int l) {
    if constexpr (LAYOUT == 3) {
      constexpr LdsPad pd = pad_in();
      if constexpr (pad1(pd)) {
        return in_index1(j, r, l);
      } else {
        constexpr int step = NB + pd.k * (NB >> pd.s);
        return l * LP + j + pd.k * (j >> pd.s) + r * step;
      }
    } else if constexpr (LAYOUT == 2) {
      static_assert(P == 512 && R == 8 && NQ == 64 && NTASK == 1 && S >= 1, "layout 2: 512-point lines");
      if constexpr (S == 1) return l * LP + 18 * (j >> 4) + ((j >> 3) & 1) + 2 * (j & 7) + 72 * r;
      else return l * LP + j + 72 * r;
    } else if constexpr (LAYOUT == 1 && NB % 8 == 0) {
      return l * LP + j + (j >> 3) + r * (NB + NB / 8);
    } else {
      return lds_index<LAYOUT, LP>(in_pos(j, r), l);
    }
  }
  __device__ __forceinline__ static int out_index(int j, int r, int l) {
    if constexpr (LAYOUT == 3) {
      constexpr LdsPad pd = pad_out();
      if constexpr (pad1(pd)) {
        return out_index1(j, r, l);
      } else {
        constexpr int step = NS + pd.k * (NS >> pd.s);
        const int u = (j / NS) * NS * R + (j % NS);
        return l * LP + u + pd.k * (u >> pd.s) + r * step;
      }
    } else if constexpr (LAYOUT == 2) {
      static_assert(P == 512 && R == 8 && NQ == 64 && NTASK == 1 && S <= 1, "layout 2: 512-point lines");
      if constexpr (S == 0) return l * LP + 72 * (j >> 3) + 18 * ((j & 7) >> 1) + (j & 1) + 2 * r;
      else return l * LP + 72 * (j >> 3) + (j & 7) + 8 * r;
    } else if constexpr (LAYOUT == 1 && (NS % 8 == 0 || (NS == 1 && 8 % R == 0))) {
      const int u = (j / NS) * NS * R + (j % NS);
      return l * LP + u + (u >> 3) + r * (NS == 1 ? 1 : NS + NS / 8);
    } else {
      return lds_index<LAYOUT, LP>(out_pos(j, r), l);
    }
  }

  // read this stage's inputs from the LDS tile
  __device__ __forceinline__ static void lds_in(Regs& g, const C* lds, int l, int q) {
#pragma unroll
    for (int t = 0; t < NTASK; ++t) {
      if (!active(t, q)) continue;
      const int j = q + t * NQ;
#pragma unroll
      for (int r = 0; r < R; ++r) g.v[t][r] = lds[in_index(j, r, l)];
    }
  }

  __device__ __forceinline__ static void lds_out(const Regs& g, C* lds, int l, int q) {
#pragma unroll
    for (int t = 0; t < NTASK; ++t) {
      if (!active(t, q)) continue;
      const int j = q + t * NQ;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[out_index(j, r, l)] = g.v[t][r];
    }
  }

  // last stage outputs (Ns = P/R, so positions are j + r*NB); st(j, r, value)
  // with r a compile-time constant. PRUNE: only positions < P/2 are stored.
  template <bool PRUNE, class Store>
  __device__ __forceinline__ static void store_last(const Regs& g, int q, Store&& st) {
    static_assert(LAST, "store_last is the last stage");
    static_assert(!PRUNE || R % 2 == 0, "pruned outputs need an even last radix");
#pragma unroll
    for (int t = 0; t < NTASK; ++t) {
      if (!active(t, q)) continue;
      const int j = q + t * NQ;
#pragma unroll
      for (int r = 0; r < R; ++r) {
        if (PRUNE && r >= R / 2) continue;
        st(j, r, g.v[t][r]);
      }
    }
  }
};

#ifndef VGF_MINW_DIV
#define VGF_MINW_DIV 2
#endif

// Waves per SIMD that the LDS footprint of a workgroup allows (160 KiB of
// LDS per CU, 4 SIMDs): the register budget is tied to this occupancy so the
// compiler does not trade it away for registers.
constexpr int lds_waves_per_simd(int lds_bytes, int threads) {
  int wg = lds_bytes > 0 ? (160 * 1024) / lds_bytes : 8;
  if (wg > 8) wg = 8;
  if (wg < 1) wg = 1;
  int w = wg * ((threads + 63) / 64) / 4 / VGF_MINW_DIV;
  if (w < 1) w = 1;
  if (w > 8) w = 8;
  return w;
}

template <int B, int E> struct StaticFor {
  template <class F> __device__ __forceinline__ static void run(F&& f) {
    if constexpr (B < E) {
      f(std::integral_constant<int, B>{});
      StaticFor<B + 1, E>::run(f);
    }
  }
};

// Ordering of LDS accesses among the lanes of one wavefront (the lines of a
// wave-local tile are touched by that wave only).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool WAVE> __device__ __forceinline__ void tile_sync() {
  if constexpr (WAVE) wave_sync();
  else __syncthreads();
}

// Runs stages [1, n_stages - 1) of a transform through the LDS tile. On entry
// stage 0's outputs are in LDS (and a barrier has been passed); on exit the
// last stage's twiddled-and-transformed results are in `last`. WAVE: the
// tile belongs to one wavefront, which orders its own LDS accesses.
template <typename T, int P, int NT, int NL, int LP, int SIGN, int LAYOUT = 0, bool WAVE = false>
__device__ __forceinline__ void middle_and_last(
    typename Stage<T, P, NT, NL, LP, SIGN, n_stages(P) - 1, LAYOUT>::Regs& last, cplx<T>* lds,
    const cplx<T>* tw, int l, int q) {
  constexpr int NSTG = n_stages(P);
  StaticFor<1, NSTG - 1>::run([&](auto sI) {
    constexpr int s = decltype(sI)::value;
    using St = Stage<T, P, NT, NL, LP, SIGN, s, LAYOUT>;
    typename St::Regs g;
    typename St::Tw w;
    St::lds_in(g, lds, l, q);
    St::load_tw(w, tw, q);
    St::tw_butterflies(g, w, q);
    tile_sync<WAVE>();
    St::lds_out(g, lds, l, q);
    tile_sync<WAVE>();
  });
  using SL = Stage<T, P, NT, NL, LP, SIGN, NSTG - 1, LAYOUT>;
  typename SL::Tw w;
  SL::lds_in(last, lds, l, q);
  SL::load_tw(w, tw, q);
  SL::tw_butterflies(last, w, q);
}

// middle_and_last with the last stage's twiddle slots supplied by the caller
// (held in registers across the lines a wavefront walks).
template <typename T, int P, int NT, int NL, int LP, int SIGN, int LAYOUT = 0, bool WAVE = false>
__device__ __forceinline__ void middle_and_last_tw(
    typename Stage<T, P, NT, NL, LP, SIGN, n_stages(P) - 1, LAYOUT>::Regs& last, cplx<T>* lds,
    const cplx<T>* tw, const typename Stage<T, P, NT, NL, LP, SIGN, n_stages(P) - 1, LAYOUT>::Tw& wl, int l,
    int q) {
  constexpr int NSTG = n_stages(P);
  StaticFor<1, NSTG - 1>::run([&](auto sI) {
    constexpr int s = decltype(sI)::value;
    using St = Stage<T, P, NT, NL, LP, SIGN, s, LAYOUT>;
    typename St::Regs g;
    typename St::Tw w;
    St::lds_in(g, lds, l, q);
    St::load_tw(w, tw, q);
    St::tw_butterflies(g, w, q);
    tile_sync<WAVE>();
    St::lds_out(g, lds, l, q);
    tile_sync<WAVE>();
  });
  using SL = Stage<T, P, NT, NL, LP, SIGN, NSTG - 1, LAYOUT>;
  SL::lds_in(last, lds, l, q);
  SL::tw_butterflies(last, wl, q);
}

// Ping-pong variant for kernels that run one workgroup per CU anyway: LDS
// phases alternate between two tiles, so each stage boundary needs a single
// barrier (between the writes and the reads of one phase); a tile is written
// again only two phases after it was read, with a barrier in between.
template <typename C, int TILE> struct PingPong {
  C* base;  // 2 * TILE elements
  int off;  // 0 or TILE
  __device__ __forceinline__ C* now() const { return base + off; }
  __device__ __forceinline__ void flip() { off = TILE - off; }
};

// Stage 0 (already butterflied, in registers) -> LDS -> remaining stages; the
// last stage's results end in `last`. Uses one barrier per LDS phase.
template <typename T, int P, int NT, int NL, int LP, int SIGN>
__device__ __forceinline__ void transform_pp(
    const typename Stage<T, P, NT, NL, LP, SIGN, 0>::Regs& g0,
    typename Stage<T, P, NT, NL, LP, SIGN, n_stages(P) - 1>::Regs& last, PingPong<cplx<T>, P * LP>& pp,
    const cplx<T>* tw, int l, int q) {
  constexpr int NSTG = n_stages(P);
  using S0 = Stage<T, P, NT, NL, LP, SIGN, 0>;
  S0::lds_out(g0, pp.now(), l, q);
  __syncthreads();
  StaticFor<1, NSTG - 1>::run([&](auto sI) {
    constexpr int s = decltype(sI)::value;
    using St = Stage<T, P, NT, NL, LP, SIGN, s>;
    typename St::Regs g;
    typename St::Tw w;
    St::lds_in(g, pp.now(), l, q);
    St::load_tw(w, tw, q);
    St::tw_butterflies(g, w, q);
    pp.flip();
    St::lds_out(g, pp.now(), l, q);
    __syncthreads();
  });
  using SL = Stage<T, P, NT, NL, LP, SIGN, NSTG - 1>;
  typename SL::Tw w;
  SL::lds_in(last, pp.now(), l, q);
  SL::load_tw(w, tw, q);
  SL::tw_butterflies(last, w, q);
  pp.flip();
}

}  // namespace vgf
