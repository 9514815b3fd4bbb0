// vgf_solve_kernels.hpp -- the per-solve passes of the zero-padded 2N FFT
// convolution (Eq. 3 of the paper, shared by HE and VGF) with the field by
// Fourier differentiation (multiplication by -i k before the inverse FFT,
// Sec. III.A).
//
// The factor -i k_a of E_a only involves axis a, so it commutes with the
// transforms along the other axes. Each pass therefore applies the
// derivative of its own axis, and the number of arrays grows only as the
// passes that derive a field from phi's spectrum are reached. Forward passes
// of the adjoint do the mirror image: they sum their inputs after
// multiplying by +i k of their own axis.
//
// Default layout (multiply pass along the contiguous last axis):
//   k_r2c_s    pruned real-to-complex transforms along axis 0 (strided), two
//              adjacent real columns as one complex column.
//   k_c2c_fwd  strided forward transform along axis 1 (3D), pruned input;
//              sums up to two inputs.
//   k_fused_c  one wavefront per last-axis line: pruned forward transform,
//              multiplication by the real kernel spectrum (phi) and by -i k
//              of the last axis (E_last), a pruned inverse per output.
//   k_c2c_inv  strided inverse along axis 1, pruned output: phi and E_1 from
//              phi's spectrum (held in registers between the two), E_last
//              from its own spectrum, in one launch.
//   k_c2r_s    complex-to-real along axis 0 keeping the first N outputs: phi
//              and E_0 from phi's spectrum, the other fields from theirs.
// Axis-0 layout (and gradient-kernel fields): k_r2c / k_c2r along the last
// axis (a wavefront per pair of real lines), k_fused / k_fused_grad along
// axis 0 (strided), and the same axis-1 kernels.
// FFT twiddles are staged in LDS once per workgroup. Large solves use
// non-temporal loads and stores in the middle passes (load_nt / store_nt).
#pragma once
#include "vgf_fft.hpp"
#include "vgf_internal.hpp"

// Complex values per thread in the Stockham kernels: 8 (one radix-8
// butterfly per stage) measured fastest at 256^3 in both precisions.
#ifndef VGF_EPT
#define VGF_EPT 8
#endif

namespace vgf {

// Loads and stores with the non-temporal hint. The solve passes read and
// write each array once; when the arrays are much larger than the caches
// (the plan decides per solve from the input bytes), the hint keeps those
// lines from displacing cached data that is still reused (measured faster at
// 256^3; small grids, whose arrays stay cached between passes, are faster
// with plain accesses).
__device__ __forceinline__ float2 load_nt(const float2* p) {
  typedef float V __attribute__((ext_vector_type(2)));
  const V w = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  return make_float2(w.x, w.y);
}
__device__ __forceinline__ double2 load_nt(const double2* p) {
  typedef double V __attribute__((ext_vector_type(2)));
  const V w = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  return make_double2(w.x, w.y);
}
__device__ __forceinline__ void store_nt(float2* p, float2 v) {
  typedef float V __attribute__((ext_vector_type(2)));
  const V w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<V*>(p));
}
__device__ __forceinline__ void store_nt(double2* p, double2 v) {
  typedef double V __attribute__((ext_vector_type(2)));
  const V w = {v.x, v.y};
  __builtin_nontemporal_store(w, reinterpret_cast<V*>(p));
}

// The two complex values of a pair of adjacent real columns, adjacent in
// memory (16-byte aligned in FP32): one 16-byte access per lane in FP32, so
// every load or store instruction of a wavefront covers whole cache lines.
__device__ __forceinline__ void load_pair(const float2* p, float2& a, float2& b) {
  const float4 v = *reinterpret_cast<const float4*>(p);
  a = make_float2(v.x, v.y);
  b = make_float2(v.z, v.w);
}
__device__ __forceinline__ void load_pair(const double2* p, double2& a, double2& b) {
  a = p[0];
  b = p[1];
}
__device__ __forceinline__ void load_pair_nt(const float2* p, float2& a, float2& b) {
  typedef float V __attribute__((ext_vector_type(4)));
  const V w = __builtin_nontemporal_load(reinterpret_cast<const V*>(p));
  a = make_float2(w.x, w.y);
  b = make_float2(w.z, w.w);
}
__device__ __forceinline__ void load_pair_nt(const double2* p, double2& a, double2& b) {
  a = load_nt(p);
  b = load_nt(p + 1);
}
__device__ __forceinline__ void store_pair(float2* p, float2 a, float2 b) {
  *reinterpret_cast<float4*>(p) = make_float4(a.x, a.y, b.x, b.y);
}
__device__ __forceinline__ void store_pair(double2* p, double2 a, double2 b) {
  p[0] = a;
  p[1] = b;
}

// Tile shape for length P: NL lines (contiguous columns) per workgroup, 16
// complex values per thread, LDS tile <= 64 KiB.
template <typename T, int P, int NL_FORCE = 0> struct Tile {
  static constexpr int CB = (int)sizeof(cplx<T>);
  static constexpr int pick_nl() {
    if (NL_FORCE > 0) return NL_FORCE;
    int nl = sizeof(T) == 4 ? 16 : 8;
    while (nl > 1 && P * nl * CB > 65536) nl /= 2;
    return nl;
  }
  static constexpr int NL = pick_nl();
  static constexpr int EPT = VGF_EPT;
  static constexpr int NQ = (P + EPT - 1) / EPT;  // threads per line
  static constexpr int NT = NL * NQ;
  static_assert(NT <= 1024, "workgroup too large");
  static_assert(n_stages(P) >= 2, "transform needs at least two stages");
  // LDS of the strided kernels (tile + twiddles) and of r2c/c2r (padded tile)
  static constexpr int MINW = lds_waves_per_simd((P * NL + P) * CB, NT);
  static constexpr int MINW_T = lds_waves_per_simd((P * (NL + 1) + P) * CB, NT);
  static constexpr int MINW_PP = lds_waves_per_simd((2 * P * NL + P) * CB, NT);
};

// Tile schedules of the strided passes: variant 0 uses the default tile
// width (one 128-byte row segment per position), variant 1 half of it (more,
// smaller workgroups: less padding waste on narrow planes, more workgroups
// per CU). Every column is transformed with the same arithmetic in both, so
// the choice never changes a result bit.
constexpr int kTileVariants = kTileVariantsHost;
template <typename T, int P> constexpr int strided_nl() {
  static_assert(VGF_EPT == 8, "strided_tile_width assumes 8 values per thread");
  return strided_tile_width(P, (int)sizeof(T));
}
// The half-width schedule: half of the default width, or, for FP64 lengths
// 576 to 1024 whose default tile is wider than 64 KiB of LDS allows, half of
// that narrower width, so grids with few columns (2D 512^2: 38 against 41 us)
// keep small tiles and many workgroups. The 2D lengths above 1024 measured
// faster with plain halving (2D 768^2 and 1024^2: 56 and 100 us against 58
// and 106 us).
template <typename T, int P> constexpr int strided_nl_half() {
  constexpr int w = (strided_nl<T, P>() > Tile<T, P>::NL && P <= 1024) ? Tile<T, P>::NL : strided_nl<T, P>();
  return w > 1 ? w / 2 : 1;
}
template <typename T, int P, int V>
struct TileV : Tile<T, P, (V == 0 ? strided_nl<T, P>() : strided_nl_half<T, P>())> {};
// the axis-0 layout's tiles (two LDS buffers in its multiply pass) keep the
// 64 KiB rule of Tile
template <typename T, int P, int V>
struct TileV64 : Tile<T, P, (V == 0 ? 0 : (Tile<T, P>::NL > 1 ? Tile<T, P>::NL / 2 : 1))> {};

// Block -> column tile of the strided passes. Half-width tiles (V = 1) split
// each 128-byte row segment between two workgroups; workgroups are dealt to
// the 8 XCDs round-robin, so the two halves go to blocks 8 apart (same XCD,
// consecutive dispatch rounds) and the second half is read from that XCD's
// L2. A bijection on [0, nb).
template <int V> __device__ __forceinline__ int64_t tile_of_block(int64_t b, int64_t nb) {
  if constexpr (V == 0) {
    return b;
  } else {
    const int64_t full = nb & ~(int64_t)15;
    if (b >= full) return b;
    const int64_t x = b & 7, k = b >> 3;
    return ((((k >> 1) << 3) + x) << 1) + (k & 1);
  }
}

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
// acc + deriv(x, code, k), the product fused into the sum
template <typename C, typename T>
__device__ __forceinline__ C deriv_add(C acc, C x, int code, T k) {
  if (code == 0) return C{acc.x + x.x, acc.y + x.y};
  if (code < 0) return C{fmaT(k, x.y, acc.x), fmaT(-k, x.x, acc.y)};
  return C{fmaT(-k, x.y, acc.x), fmaT(k, x.x, acc.y)};
}

// Twiddles of the stages of one direction in LDS, stage-major (see
// Stage::load_tw): the plan keeps, per axis, the table of the forward radix
// order at tw[0, P) and that of the inverse order at tw[P, 2P) (the same
// values when the order is a palindrome), each P - R_0 entries long; a
// workgroup copies the one it needs.
template <typename C, int P, int NT, int SIGN>
__device__ __forceinline__ void stage_twiddles(C* twl, const C* __restrict__ tw, int tid) {
  constexpr int R0 = radix_at<SIGN>(P, 0);
  const C* __restrict__ src = tw + (SIGN < 0 ? 0 : P);
  for (int e = tid; e < P - R0; e += NT) twl[e] = src[e];
}
// LDS entries for the twiddles of a kernel that runs both directions, the
// forward table first; the inverse table (tw_inverse) is a second one only
// where the radix sequences differ.
template <int P> constexpr int tw_both_size() { return radix_palindrome<P>() ? P : 2 * P; }
template <typename C, int P, int NT>
__device__ __forceinline__ void stage_twiddles_both(C* twl, const C* __restrict__ tw, int tid) {
  stage_twiddles<C, P, NT, -1>(twl, tw, tid);
  if constexpr (!radix_palindrome<P>()) stage_twiddles<C, P, NT, 1>(twl + P, tw, tid);
}
template <int P, typename C> __device__ __forceinline__ C* tw_inverse(C* twl) {
  if constexpr (radix_palindrome<P>()) return twl;
  else return twl + P;
}

// ---------------------------------------------------------------------------
// Contiguous-axis passes (r2c / c2r): each wavefront owns whole line pairs.
// NQ lanes share one pair (two real lines packed as one complex line), lanes
// run along the line, so HBM accesses are contiguous per lane group and every
// FFT exchange stays inside the wavefront (LDS tile per wave, wave-level
// ordering only). Twiddles are staged once per workgroup.
// ---------------------------------------------------------------------------
// Lanes per line: P / 8 rounded up to a power of two (at most 64). Lengths
// with a factor 3 then leave some lanes idle in their radix-8 stages rather
// than give each lane a second, mostly inactive set of butterflies: the
// 192-point multiply pass (32 lanes per line instead of 16) needs 116
// instead of 197 VGPRs and takes 23 instead of 27 us at 96^3.
template <int P> constexpr int wave_nq() {
  int nq = 1;
  while (nq * 8 < P && nq * 2 <= 64) nq *= 2;
  return nq;
}
#ifndef VGF_FC_MINW32
#define VGF_FC_MINW32 1
#endif
#ifndef VGF_FC_MINW64
#define VGF_FC_MINW64 1
#endif
#ifndef VGF_FC_GPW
#define VGF_FC_GPW 4
#endif
// line order of the forward multiply pass: 1 = the wavefronts of a workgroup
// take neighbouring lines and step by WPB, 0 = each wavefront walks its own
// gpw consecutive lines (same results either way)
#ifndef VGF_FC_WALK
#define VGF_FC_WALK 1
#endif
// multiply pass of P >= 512 through k_fused_c1 (1) or k_fused_c (0)
#ifndef VGF_FC1
#define VGF_FC1 1
#endif
// k_fused_c1 exchanges 512-point lines through LDS layout 2 (1) or 1 (0)
#ifndef VGF_LAY2
#define VGF_LAY2 1
#endif
// the multiply passes exchange other lengths through the per-exchange pads of
// layout 3 (1) or the pad of layout 1 (0)
#ifndef VGF_LAY3
#define VGF_LAY3 1
#endif
constexpr int kPadLayout = VGF_LAY3 ? 3 : 1;
constexpr int64_t kFusedCMinBlocks = 2048;
// V = 1 (the multiply pass's second lane schedule): half the lanes per line,
// twice the lines per wavefront and twice the butterflies per lane, where the
// four wavefronts' tiles then still fit 64 KiB of LDS (else as V = 0); the
// per-line arithmetic is the same.
template <typename T, int P> constexpr bool half_lanes_fit() {
  return wave_nq<P>() > 1 && 4 * (128 / wave_nq<P>()) * line_pitch<P>() * (int)sizeof(cplx<T>) <= 65536;
}
// Wavefronts per workgroup of the contiguous passes: four, fewer where
// their line tiles and the twiddle tables would not fit the 160 KiB of LDS
// (FP64 lines of 2048 points).
template <typename T, int P, int LPW> constexpr int tilew_wpb() {
  int w = 4;
  while (w > 1 && (w * LPW * line_pitch<P>() + tw_both_size<P>()) * (int)sizeof(cplx<T>) > 160 * 1024) w /= 2;
  return w;
}
template <typename T, int P, int V = 0> struct TileW {
  static constexpr int NQ = (V == 1 && half_lanes_fit<T, P>()) ? wave_nq<P>() / 2 : wave_nq<P>();  // lanes per line (pair)
  static constexpr int LPW = 64 / NQ;      // lines (line pairs) per wavefront
  static constexpr int WPB = tilew_wpb<T, P, LPW>();  // wavefronts per workgroup
  static constexpr int NT = 64 * WPB;
  static constexpr int LP = line_pitch<P>();
  static constexpr int PAIRS = LPW * WPB;  // line pairs per workgroup
  // minimum waves per SIMD asked of the register allocator by k_fused_c
  static constexpr int MINW_FC = sizeof(T) == 4 ? VGF_FC_MINW32 : VGF_FC_MINW64;
  static_assert(n_stages(P) >= 2, "transform needs at least two stages");
};

// Entry and entry-local line of global line la of a multi-entry launch
// (lpe lines per entry; lpe <= 0 means a single entry).
struct EntryLine {
  int64_t e, line;
  __device__ __forceinline__ EntryLine(int64_t la, int64_t lpe, int64_t nlines) {
    if (lpe <= 0 || lpe >= nlines) {
      e = 0;
      line = la;
    } else {
      e = la / lpe;
      line = la - e * lpe;
    }
  }
};

// ---------------------------------------------------------------------------
// k_r2c: out = sum_t m_t(k) R2C(in_t), lines of N = P/2 reals -> N+1 complex
// ---------------------------------------------------------------------------
template <typename T, int P, int NTERM>
__global__ __launch_bounds__((TileW<T, P>::NT)) void k_r2c(R2CArgs<T> a,
                                                          const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TW = TileW<T, P>;
  constexpr int NQ = TW::NQ, LPW = TW::LPW, LP = TW::LP, N = P / 2, H = N + 1;
  constexpr int NSTG = n_stages(P);
  constexpr int NSLOT = (H + NQ - 1) / NQ;
  using S0 = Stage<T, P, 64, LPW, LP, -1, 0, 1>;
  using SL = Stage<T, P, 64, LPW, LP, -1, NSTG - 1, 1>;
  __shared__ C tiles[TW::WPB * LPW * LP];
  __shared__ C twl[P];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l = lane / NQ, q = lane % NQ;
  C* tile = tiles + w * LPW * LP;
  const int64_t pair = ((int64_t)blockIdx.x * TW::WPB + w) * LPW + l;
  const int64_t la = 2 * pair, lb = la + 1;
  const bool va = la < a.nlines, vb = lb < a.nlines;
  const EntryLine el(va ? la : 0, a.lpe, a.nlines);
  stage_twiddles<C, P, TW::NT, -1>(twl, tw, tid);
  __syncthreads();

  C acc_a[NSLOT], acc_b[NSLOT];
#pragma unroll
  for (int term = 0; term < NTERM; ++term) {
    const T* __restrict__ base = a.in_tab[term] ? a.in_tab[term][el.e] + a.in_off[term] : a.in[term];
    const T* __restrict__ xa = base + el.line * N;
    const T* __restrict__ xb = base + (vb ? el.line + 1 : el.line) * N;
    const int code = a.d.code[term];
    typename S0::Regs g0;
    S0::template load_first<true>(g0, q, [&](int j, int r) {
      const int pos = S0::in_pos(j, r);
      return C{va ? xa[pos] : T(0), vb ? xb[pos] : T(0)};
    });
    S0::template butterflies<true>(g0, q);
    wave_sync();
    S0::lds_out(g0, tile, l, q);
    wave_sync();
    typename SL::Regs gl;
    middle_and_last<T, P, 64, LPW, LP, -1, 1, true>(gl, tile, twl, l, q);
    wave_sync();
    SL::lds_out(gl, tile, l, q);
    wave_sync();
    // Z = X + iY  ->  X[k] = (Z[k] + conj Z[P-k]) / 2,  Y[k] = -i (Z[k] - conj Z[P-k]) / 2
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
      const int k = q + NQ * s;
      if (k >= H) continue;
      const C z = tile[lds_index<1, LP>(k, l)];
      const C zm = tile[lds_index<1, LP>((P - k) % P, l)];
      const C xk = C{T(0.5) * (z.x + zm.x), T(0.5) * (z.y - zm.y)};
      const C yk = C{T(0.5) * (z.y + zm.y), T(0.5) * (zm.x - z.x)};
      const T kk = a.d.ks * (T)(k < N ? k : 0);
      if (term == 0) {
        acc_a[s] = deriv(xk, code, kk);
        acc_b[s] = deriv(yk, code, kk);
      } else {
        acc_a[s] = deriv_add(acc_a[s], xk, code, kk);
        acc_b[s] = deriv_add(acc_b[s], yk, code, kk);
      }
    }
  }
  C* __restrict__ out = a.out + el.e * a.out_es + el.line * a.hs;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int k = q + NQ * s;
    if (k >= H) continue;
    if (va) out[k] = acc_a[s];
    if (vb) out[a.hs + k] = acc_b[s];
  }
}

// ---------------------------------------------------------------------------
// k_c2r: out_o = first N reals of C2R(m_o(k) in), lines of N+1 complex
// ---------------------------------------------------------------------------
template <typename T, int P, int NOUT>
__global__ __launch_bounds__((TileW<T, P>::NT)) void k_c2r(C2RArgs<T> a,
                                                          const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TW = TileW<T, P>;
  constexpr int NQ = TW::NQ, LPW = TW::LPW, LP = TW::LP, N = P / 2, H = N + 1;
  constexpr int NSTG = n_stages(P);
  constexpr int NSLOT = (H + NQ - 1) / NQ;
  using S0 = Stage<T, P, 64, LPW, LP, 1, 0, 1>;
  using SL = Stage<T, P, 64, LPW, LP, 1, NSTG - 1, 1>;
  __shared__ C tiles[TW::WPB * LPW * LP];
  __shared__ C twl[P];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l = lane / NQ, q = lane % NQ;
  C* tile = tiles + w * LPW * LP;
  const int64_t pair = ((int64_t)blockIdx.x * TW::WPB + w) * LPW + l;
  const int64_t la = 2 * pair, lb = la + 1;
  const bool va = la < a.nlines, vb = lb < a.nlines;
  const EntryLine el(va ? la : 0, a.lpe, a.nlines);
  const C* __restrict__ in = a.in + el.e * a.in_es + el.line * a.hs;

  // this lane's k-slots of the two half-spectra
  C xs[NSLOT], ys[NSLOT];
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int k = q + NQ * s;
    xs[s] = ys[s] = C{T(0), T(0)};
    if (k >= H) continue;
    if (va) xs[s] = in[k];
    if (vb) ys[s] = in[a.hs + k];
  }
  stage_twiddles<C, P, TW::NT, 1>(twl, tw, tid);
  __syncthreads();

#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    const int code = a.d.code[o];
    // Z[k] = X[k] + i Y[k], Z[P-k] = conj X[k] + i conj Y[k]; the imaginary
    // parts of X, Y at k = 0 and k = N are dropped (real by symmetry).
    wave_sync();
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
      const int k = q + NQ * s;
      if (k >= H) continue;
      C X = xs[s], Y = ys[s];
      if (code != 0) {
        const T kk = a.d.ks * (T)(k < N ? k : 0);
        X = deriv(X, code, kk);
        Y = deriv(Y, code, kk);
      }
      if (k == 0 || k == N) {
        tile[lds_index<1, LP>(k, l)] = C{X.x, Y.x};
      } else {
        tile[lds_index<1, LP>(k, l)] = C{X.x - Y.y, X.y + Y.x};
        tile[lds_index<1, LP>(P - k, l)] = C{X.x + Y.y, Y.x - X.y};
      }
    }
    wave_sync();
    typename S0::Regs g0;
    S0::template load_first<false>(g0, q, [&](int j, int r) { return tile[lds_index<1, LP>(S0::in_pos(j, r), l)]; });
    S0::butterflies(g0, q);
    wave_sync();
    S0::lds_out(g0, tile, l, q);
    wave_sync();
    typename SL::Regs gl;
    middle_and_last<T, P, 64, LPW, LP, 1, 1, true>(gl, tile, twl, l, q);
    T* __restrict__ base = a.out_tab[o] ? a.out_tab[o][el.e] + a.out_off[o] : a.out[o];
    T* __restrict__ oa = base + el.line * N;
    T* __restrict__ ob = oa + N;
    SL::template store_last<true>(gl, q, [&](int j, int r, C v) {
      const int pos = SL::out_pos(j, r);
      if (va) oa[pos] = v.x;
      if (vb) ob[pos] = v.y;
    });
  }
}

// ---------------------------------------------------------------------------
// Addressing of the strided passes. Every array the solve path touches holds
// fewer than 2^31 elements, so element offsets are 32-bit and added to a
// workgroup-uniform base. Element (row, col) is at base + col + row*ls; a
// stage's rows are j + r*NB with r a compile-time constant, so the per-r
// part r*NB*ls is uniform. Lanes past the last column load the last column
// (in bounds, never stored).
// ---------------------------------------------------------------------------
struct ColIO {
  uint32_t col;   // clamped column
  uint32_t ls;    // row stride (elements)
  bool valid;
  ColIO() = default;
  __device__ __forceinline__ ColIO(int64_t c, int64_t ncols, int64_t ls_) {
    valid = c < ncols;
    col = (uint32_t)(valid ? c : ncols - 1);
    ls = (uint32_t)ls_;
  }
  // offset of row j + r*NB
  template <int NB>
  __device__ __forceinline__ uint32_t off(int j, int r) const {
    return col + (uint32_t)j * ls + (uint32_t)(r * NB) * ls;
  }
};

// wavenumber factor of position j + r*NB on a length-P axis (P = 2N), with
// the Nyquist position N -> 0. For an even radix the rows j + r*NB cross N
// exactly at r = R/2 (and equal it only for j = 0), which r, a compile-time
// constant at every call, decides; odd radices compare at run time.
template <typename T, int R, int NB>
__device__ __forceinline__ T axis_k(T ks, int j, int r) {
  constexpr int P = R * NB, N = P / 2;
  if constexpr (R % 2 == 0) {
    T k = ks * (T)(j + r * NB - (r >= R / 2 ? P : 0));
    if (r == R / 2 && j == 0) k = T(0);
    return k;
  } else {
    const int pos = j + r * NB;
    return ks * (T)(pos < N ? pos : (pos == N ? 0 : pos - P));
  }
}

// ---------------------------------------------------------------------------
// k_c2c_fwd: out = sum_t m_t(pos) FFT(in_t) along a strided axis, pruned input
// grid = (ceil(ncols/NL), nbatch)
// ---------------------------------------------------------------------------
template <typename T, int P, int NTERM, int V>
__global__ __launch_bounds__((TileV<T, P, V>::NT), (TileV<T, P, V>::MINW)) void k_c2c_fwd(C2CFwdArgs<T> a,
                                                                     const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TL = TileV<T, P, V>;
  constexpr int NL = TL::NL, NT = TL::NT, LP = NL;
  constexpr int NSTG = n_stages(P);
  __shared__ C lds[P * LP];
  __shared__ C twl[P];
  const int tid = threadIdx.x, l = tid % NL, q = tid / NL;
  stage_twiddles<C, P, NT, -1>(twl, tw, tid);
  using S0 = Stage<T, P, NT, NL, LP, -1, 0>;
  using SL = Stage<T, P, NT, NL, LP, -1, NSTG - 1>;
  const ColIO ci(tile_of_block<V>(blockIdx.x, gridDim.x) * NL + l, a.g.ncols, a.g.ls_in);
  const ColIO co(tile_of_block<V>(blockIdx.x, gridDim.x) * NL + l, a.g.ncols, a.g.ls_out);
  typename SL::Regs acc;

  const int e = (int)blockIdx.y / a.g.nbatch, bb = (int)blockIdx.y - e * a.g.nbatch;
#pragma unroll
  for (int term = 0; term < NTERM; ++term) {
    const C* __restrict__ src = a.in[term] + e * a.g.es_in + bb * a.g.bs_in;
    const int code = a.d.code[term];
    if (term > 0) __syncthreads();
    typename S0::Regs g0;
    S0::template load_first<true>(g0, q, [&](int j, int r) { return src[ci.off<S0::NB>(j, r)]; });
    S0::template butterflies<true>(g0, q);
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
        const T kk = code != 0 ? axis_k<T, SL::R, SL::NB>(a.d.ks, j, r) : T(0);
        if (term == 0) acc.v[t][r] = deriv(gl.v[t][r], code, kk);
        else acc.v[t][r] = deriv_add(acc.v[t][r], gl.v[t][r], code, kk);
      }
    }
  }
  if (!co.valid) return;
  C* __restrict__ dst = a.out + e * a.g.es_out + bb * a.g.bs_out;
  if (a.g.nt_store)
    SL::template store_last<false>(acc, q, [&](int j, int r, C v) { store_nt(&dst[co.off<SL::NB>(j, r)], v); });
  else
    SL::template store_last<false>(acc, q, [&](int j, int r, C v) { dst[co.off<SL::NB>(j, r)] = v; });
}

// ---------------------------------------------------------------------------
// k_c2c_inv: out_o = first P/2 of IFFT(m_o(pos) in) along a strided axis
// ---------------------------------------------------------------------------
template <typename T, int P, int NOUT, int V>
__global__ __launch_bounds__((TileV<T, P, V>::NT), (TileV<T, P, V>::MINW)) void k_c2c_inv(C2CInvArgs<T> a,
                                                                     const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TL = TileV<T, P, V>;
  constexpr int NL = TL::NL, NT = TL::NT, LP = NL;
  constexpr int NSTG = n_stages(P);
  __shared__ C lds[P * LP];
  __shared__ C twl[P];
  const int tid = threadIdx.x, l0 = tid % NL, q0 = tid / NL;
  using S0 = Stage<T, P, NT, NL, LP, 1, 0>;
  using SL = Stage<T, P, NT, NL, LP, 1, NSTG - 1>;
  ColIO ci(tile_of_block<V>(blockIdx.x, gridDim.x) * NL + l0, a.g.ncols, a.g.ls_in);
  const ColIO co(tile_of_block<V>(blockIdx.x, gridDim.x) * NL + l0, a.g.ncols, a.g.ls_out);
  if (a.g.in_tile) {
    // tiled input: the column's block of P rows of B elements
    const uint32_t sh = (uint32_t)a.g.in_tile, c = ci.col;
    ci.col = ((c >> sh) * (uint32_t)P << sh) + (c & ((1u << sh) - 1u));
    ci.ls = 1u << sh;
  }
  const int e = (int)blockIdx.y / a.g.nbatch, bb = (int)blockIdx.y - e * a.g.nbatch;
  const C* __restrict__ src = a.in + e * a.g.es_in + bb * a.g.bs_in;
  // NOUT = 3: outputs 0 and 1 from `in` (factors d), output 2 from in2
  // without a factor, in the same launch
  const C* __restrict__ src2 = NOUT == 3 ? a.in2 + e * a.g.es_in + bb * a.g.bs_in : src;
  typename S0::Regs gin;
  if (a.g.nt_load)
    S0::template load_first<false>(gin, q0, [&](int j, int r) { return load_nt(&src[ci.off<S0::NB>(j, r)]); });
  else
    S0::template load_first<false>(gin, q0, [&](int j, int r) { return src[ci.off<S0::NB>(j, r)]; });
  stage_twiddles<C, P, NT, 1>(twl, tw, tid);

#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    const int code = o < 2 ? a.d.code[o] : 0;
    // this output's copies of the thread's line and position: addresses are
    // recomputed per output instead of held through every transform
    int l = l0, q = q0;
    if (o > 0) asm volatile("" : "+v"(l), "+v"(q));
    if (o > 0) __syncthreads();  // the previous output's LDS reads are done
    if (o == 2) {
      // output 2 reads its own input here, not at the start (the laundered
      // offset keeps the compiler from hoisting the loads): output 1 reuses
      // the column held in registers, which the per-output copies of l and q
      // leave room for
      uint32_t z = 0;
      asm volatile("" : "+s"(z));
      if (a.g.nt_load)
        S0::template load_first<false>(gin, q, [&](int j, int r) { return load_nt(&src2[ci.off<S0::NB>(j, r) + z]); });
      else
        S0::template load_first<false>(gin, q, [&](int j, int r) { return src2[ci.off<S0::NB>(j, r) + z]; });
    }
    typename S0::Regs g0;
    if (code == 0) {
      g0 = gin;
    } else {
#pragma unroll
      for (int t = 0; t < S0::NTASK; ++t) {
        if (!S0::active(t, q)) continue;
        int j = q + t * S0::NQ;
        asm volatile("" : "+v"(j));  // wavenumbers computed here, not held from the start
#pragma unroll
        for (int r = 0; r < S0::R; ++r)
          g0.v[t][r] = deriv(gin.v[t][r], code, axis_k<T, S0::R, S0::NB>(a.d.ks, j, r));
      }
    }
    S0::butterflies(g0, q);
    S0::lds_out(g0, lds, l, q);
    __syncthreads();
    typename SL::Regs gl;
    middle_and_last<T, P, NT, NL, LP, 1>(gl, lds, twl, l, q);
    if (co.valid) {
      C* __restrict__ dst = (o < 2 ? a.out[o] : a.out2) + e * a.g.es_out + bb * a.g.bs_out;
      if (a.g.nt_store)
        SL::template store_last<true>(gl, q, [&](int j, int r, C v) { store_nt(&dst[co.off<SL::NB>(j, r)], v); });
      else
        SL::template store_last<true>(gl, q, [&](int j, int r, C v) { dst[co.off<SL::NB>(j, r)] = v; });
    }
  }
}

// Tile of the fused axis-0 pass (two LDS tiles, more registers).
template <typename T, int P, int V> struct TileF : TileV64<T, P, V> {
  // inverse fields as two straight-line copies (measured faster in FP64;
  // in FP32 at 1024 threads the copies exceed 128 VGPRs and spill)
  static constexpr bool SPLIT_FIELDS = sizeof(T) == 8;
};

// Kernel-spectrum addressing for the axis-0 lines: column c of the inner
// plane (3D: (k1, k2) of [P1][H2]; 2D: k1 of [H1]) reads the octant at
// [f0][f1][k2] with f_a = min(k_a, 2N_a - k_a). Row j + r*NB folds for
// r >= R/2 (compile time), so the index is a per-lane base plus a uniform
// per-r term.
// Columns of the axis-0 pass: the last axis is stored at a padded stride
// hs >= h_last, so a column is valid only if its last-axis index is below
// h_last; other lanes compute on in-bounds padding and store nothing.
template <typename T> struct FusedCol {
  ColIO io;
  uint32_t colpart;  // octant offset of (f1, k2) (3D) or f1 (2D)
  FusedCol() = default;
  __device__ __forceinline__ FusedCol(const FusedGeom<T>& g, int64_t c) : io(c, g.ncols, g.ncols) {
    const int64_t cc = io.col;
    if (g.dim == 3) {
      const int k1 = (int)(cc / g.hs);
      int k2 = (int)(cc - (int64_t)k1 * g.hs);
      if (k2 >= g.h_last) {
        io.valid = false;
        k2 = g.h_last - 1;
      }
      const int f1 = k1 <= g.n1 ? k1 : 2 * g.n1 - k1;
      colpart = (uint32_t)(f1 * (g.n2 + 1) + k2);
    } else {
      int k1 = (int)cc;
      if (k1 >= g.h_last) {
        io.valid = false;
        k1 = g.h_last - 1;
      }
      colpart = (uint32_t)k1;
    }
  }
};

template <typename T> struct SpecIdx {
  uint32_t lo, hi, plane;  // lo = colpart + j*plane, hi = colpart + (P0 - j)*plane
  __device__ __forceinline__ SpecIdx(const FusedGeom<T>& g, uint32_t colpart, int j) {
    plane = g.dim == 3 ? (uint32_t)((g.n1 + 1) * (g.n2 + 1)) : (uint32_t)(g.n1 + 1);
    lo = colpart + (uint32_t)j * plane;
    hi = colpart + (uint32_t)(2 * g.n0 - j) * plane;
  }
  template <int R, int NB>
  __device__ __forceinline__ uint32_t at(int j, int r) const {
    if constexpr (R % 2 == 0) {
      return r < R / 2 ? lo + (uint32_t)(r * NB) * plane : hi - (uint32_t)(r * NB) * plane;
    } else {  // odd radix: the fold point N falls inside a stripe of rows
      constexpr int N = R * NB / 2;
      return j + r * NB <= N ? lo + (uint32_t)(r * NB) * plane : hi - (uint32_t)(r * NB) * plane;
    }
  }
};

// ---------------------------------------------------------------------------
// k_fused: forward (pruned in) -> per output field: multiply, inverse
// (pruned out). in: [N0][ncols]; output f at out + f*out_fs, [N0][ncols].
// Persistent: workgroup b takes tiles b, b + gridDim.x, ... and issues the
// next tile's loads (column data and kernel-spectrum values) before the
// barrier-separated transforms of the current tile, so HBM traffic overlaps
// the FFT arithmetic of the same CU.
// ---------------------------------------------------------------------------
template <typename T, int P, int V>
__global__ __launch_bounds__((TileF<T, P, V>::NT), (TileF<T, P, V>::MINW_PP)) void k_fused(const cplx<T>* __restrict__ in,
                                                           cplx<T>* __restrict__ out,
                                                           FusedGeom<T> g,
                                                           const T* __restrict__ spec,
                                                           const cplx<T>* __restrict__ tw,
                                                           int ntiles) {
  using C = cplx<T>;
  using TL = TileF<T, P, V>;
  constexpr int NL = TL::NL, NT = TL::NT, LP = NL;
  constexpr int NSTG = n_stages(P);
  using S0 = Stage<T, P, NT, NL, LP, -1, 0>;
  using SL = Stage<T, P, NT, NL, LP, -1, NSTG - 1>;
  using IS0 = Stage<T, P, NT, NL, LP, 1, 0>;
  using ISL = Stage<T, P, NT, NL, LP, 1, NSTG - 1>;
  static_assert(IS0::R == SL::R && IS0::NTASK == SL::NTASK, "register hand-off");
  __shared__ C lds[2 * P * LP];
  __shared__ C twl[tw_both_size<P>()];
  PingPong<C, P * LP> pp;
  pp.base = lds;
  pp.off = 0;
  const int tid = threadIdx.x, l = tid % NL, q = tid / NL;
  // Tile order. Workgroups are dealt round-robin over the 8 XCDs (separate
  // L2s), so XCD x = b % 8 walks its own contiguous chunk of tiles. In 3D the
  // rows k1 of the [P1][hs] plane are visited as 0, N1, 1, P1-1, 2, P1-2, ...:
  // rows k1 and P1-k1 read the same kernel-spectrum octant rows, and
  // neighbouring tiles share 128-byte lines of it, so both reuses land in the
  // same L2 shortly after the first touch.
  // ntiles tiles per entry; the launch covers ntiles * nentry (entry-major).
  const int total = ntiles * g.nentry;
  const bool pairs = g.dim == 3 && g.hs % NL == 0;
  const int tiles_per_row = pairs ? g.hs / NL : ntiles;
  const int nrows = ntiles / tiles_per_row;
  const bool xcd = (gridDim.x % 8) == 0 && gridDim.x >= 8;
  const int per_xcd = xcd ? (int)gridDim.x / 8 : (int)gridDim.x;
  const int chunk = xcd ? (total + 7) / 8 : total;
  const int chunk0 = xcd ? (int)(blockIdx.x % 8) * chunk : 0;
  const int chunk1 = chunk0 + chunk < total ? chunk0 + chunk : total;
  int u = chunk0 + (xcd ? (int)blockIdx.x / 8 : (int)blockIdx.x);
  if (u >= chunk1) return;
  // position u in the visiting order as (entry ue, tile-in-entry ut); both
  // advance by per_xcd per step without a division
  int ue = u / ntiles, ut = u - ue * ntiles;
  const int step_e = per_xcd / ntiles, step_t = per_xcd - step_e * ntiles;
  auto advance = [&]() {
    u += per_xcd;
    ue += step_e;
    ut += step_t;
    if (ut >= ntiles) {
      ut -= ntiles;
      ++ue;
    }
  };
  // tile index of the tile-in-entry position tt (mirrored k1 rows adjacent)
  auto tile_of = [&](int tt) -> int {
    if (!pairs) return tt;
    const int row = tt / tiles_per_row, blk = tt - row * tiles_per_row;
    int k1;
    if (row == 0) k1 = 0;
    else if (row == 1) k1 = nrows / 2;
    else {
      const int m = (row - 2) / 2 + 1;
      k1 = (row % 2 == 0) ? m : nrows - m;
    }
    return k1 * tiles_per_row + blk;
  };
  stage_twiddles_both<C, P, NT>(twl, tw, tid);

  // loads of one tile: the stage-0 inputs and the kernel spectrum at this
  // thread's forward-output rows (natural order j + r*NB)
  auto load_tile = [&](const FusedCol<T>& fc, int e, typename S0::Regs& g0, T (&sv)[SL::NTASK][SL::R]) {
    const ColIO& cio = fc.io;
    const C* __restrict__ src = in + e * g.in_es;
    S0::template load_first<true>(g0, q, [&](int j, int r) { return src[cio.off<S0::NB>(j, r)]; });
#pragma unroll
    for (int t = 0; t < SL::NTASK; ++t) {
      if (!SL::active(t, q)) continue;
      const int j = q + t * SL::NQ;
      const SpecIdx<T> si(g, fc.colpart, j);
#pragma unroll
      for (int r = 0; r < SL::R; ++r) sv[t][r] = spec[si.template at<SL::R, SL::NB>(j, r)];
    }
  };

  FusedCol<T> fcn(g, (int64_t)tile_of(ut) * NL + l);
  int ent = ue;
  typename S0::Regs g0n;
  T svn[SL::NTASK][SL::R];
  load_tile(fcn, ent, g0n, svn);

  for (;;) {
    const FusedCol<T> fc = fcn;
    const int e = ent;
    typename S0::Regs g0 = g0n;
    T sv[SL::NTASK][SL::R];
#pragma unroll
    for (int t = 0; t < SL::NTASK; ++t)
#pragma unroll
      for (int r = 0; r < SL::R; ++r) sv[t][r] = svn[t][r];
    advance();
    const bool more = u < chunk1;
    if (more) {
      fcn = FusedCol<T>(g, (int64_t)tile_of(ut) * NL + l);
      ent = ue;
      load_tile(fcn, ent, g0n, svn);
    }

    S0::template butterflies<true>(g0, q);
    typename SL::Regs rh;  // forward spectrum times the kernel spectrum
    transform_pp<T, P, NT, NL, LP, -1>(g0, rh, pp, twl, l, q);
#pragma unroll
    for (int t = 0; t < SL::NTASK; ++t)
#pragma unroll
      for (int r = 0; r < SL::R; ++r) {
        rh.v[t][r].x *= sv[t][r];
        rh.v[t][r].y *= sv[t][r];
      }

    // inverse of one output field (fi = 0: phi's spectrum, 1: E_0's), stored
    auto inverse_store = [&](typename IS0::Regs& v, int fi) {
      IS0::butterflies(v, q);
      typename ISL::Regs o;
      transform_pp<T, P, NT, NL, LP, 1>(v, o, pp, tw_inverse<P>(twl), l, q);
      if (fc.io.valid) {
        C* __restrict__ dst = out + e * g.out_es + fi * g.out_fs;
        ISL::template store_last<true>(o, q, [&](int j, int r, C val) { dst[fc.io.template off<ISL::NB>(j, r)] = val; });
      }
    };
    // field 0 always (phi's spectrum, also the source of E_1 and E_2 later);
    // field 1 (-i k_0 times it) when E is requested.
    auto field_input = [&](typename IS0::Regs& v, bool d0) {
      if (!d0) {
#pragma unroll
        for (int t = 0; t < SL::NTASK; ++t)
#pragma unroll
          for (int r = 0; r < SL::R; ++r) v.v[t][r] = rh.v[t][r];
      } else {
#pragma unroll
        for (int t = 0; t < SL::NTASK; ++t) {
          if (!SL::active(t, q)) continue;
          const int j = q + t * SL::NQ;
#pragma unroll
          for (int r = 0; r < SL::R; ++r)
            v.v[t][r] = deriv(rh.v[t][r], -1, axis_k<T, SL::R, SL::NB>(g.ks0, j, r));
        }
      }
    };
    if constexpr (TL::SPLIT_FIELDS) {
      // two straight-line copies: no per-element selection between factors
      {
        typename IS0::Regs v;
        field_input(v, false);
        inverse_store(v, 0);
      }
      if (g.nf > 1) {
        typename IS0::Regs v;
        field_input(v, true);
        inverse_store(v, 1);
      }
    } else {
      // one copy in a loop (fits the register budget of the wider tiles)
      for (int fi = 0; fi < g.nf; ++fi) {
        typename IS0::Regs v;
        field_input(v, g.fields[fi] != 0);
        inverse_store(v, fi);
      }
    }
    if (!more) break;
  }
}

// ---------------------------------------------------------------------------
// k_fused_adj: acc = sum_f conj(m_f) * FFT(in_f); out = pruned inverse of acc
// ---------------------------------------------------------------------------
template <typename T, int P>
__global__ __launch_bounds__((Tile<T, P>::NT), (Tile<T, P>::MINW)) void k_fused_adj(const cplx<T>* __restrict__ in,
                                                               cplx<T>* __restrict__ out,
                                                               FusedGeom<T> g,
                                                               const T* __restrict__ spec,
                                                               const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TL = Tile<T, P>;
  constexpr int NL = TL::NL, NT = TL::NT, LP = NL;
  constexpr int NSTG = n_stages(P);
  __shared__ C lds[P * LP];
  __shared__ C twl[tw_both_size<P>()];
  const int tid = threadIdx.x, l = tid % NL, q = tid / NL;
  const FusedCol<T> fc(g, (int64_t)blockIdx.x * NL + l);
  const ColIO& cio = fc.io;
  stage_twiddles_both<C, P, NT>(twl, tw, tid);

  using S0 = Stage<T, P, NT, NL, LP, -1, 0>;
  using SL = Stage<T, P, NT, NL, LP, -1, NSTG - 1>;
  using IS0 = Stage<T, P, NT, NL, LP, 1, 0>;
  using ISL = Stage<T, P, NT, NL, LP, 1, NSTG - 1>;
  static_assert(IS0::R == SL::R && IS0::NTASK == SL::NTASK, "register hand-off");

  typename IS0::Regs acc;
#pragma unroll
  for (int t = 0; t < SL::NTASK; ++t)
#pragma unroll
    for (int r = 0; r < SL::R; ++r) acc.v[t][r] = C{T(0), T(0)};

  for (int fi = 0; fi < g.nf; ++fi) {
    const int code = g.fields[fi];
    const C* __restrict__ src = in + fi * g.in_fs;
    typename S0::Regs g0;
    S0::template load_first<true>(g0, q, [&](int j, int r) { return src[cio.off<S0::NB>(j, r)]; });
    S0::template butterflies<true>(g0, q);
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
        const T kk = code != 0 ? axis_k<T, SL::R, SL::NB>(g.ks0, j, r) : T(0);
        acc.v[t][r] = deriv_add(acc.v[t][r], rh.v[t][r], code != 0 ? 1 : 0, kk);
      }
    }
  }
  // the kernel spectrum is real: apply it once to the sum
#pragma unroll
  for (int t = 0; t < SL::NTASK; ++t) {
    if (!SL::active(t, q)) continue;
    const int j = q + t * SL::NQ;
    const SpecIdx<T> si(g, fc.colpart, j);
#pragma unroll
    for (int r = 0; r < SL::R; ++r) {
      const T sv = spec[si.template at<SL::R, SL::NB>(j, r)];
      acc.v[t][r].x *= sv;
      acc.v[t][r].y *= sv;
    }
  }
  IS0::butterflies(acc, q);
  __syncthreads();
  IS0::lds_out(acc, lds, l, q);
  __syncthreads();
  typename ISL::Regs o;
  middle_and_last<T, P, NT, NL, LP, 1>(o, lds, tw_inverse<P>(twl), l, q);
  if (cio.valid)
    ISL::template store_last<true>(o, q, [&](int j, int r, C val) { out[cio.off<ISL::NB>(j, r)] = val; });
}

// ---------------------------------------------------------------------------
// Gradient-kernel fields (E_a = w_a * rho with w_a the restricted inverse 4N
// transform of -i k_a Ghat). The 2N spectrum of the odd kernel w_a is
// -i T_a with T_a real, odd in the axis-a frequency and even in the others;
// the octants hold T_a for frequency indices in [0, N]. Field 0 multiplies
// by the kernel spectrum, field 1 + a by -i s_a T_a, s_a = -1 where the
// axis-a index exceeds N_a (axis 0: the row of the line; axis 1 in 3D: the
// column's k1; the last axis is a half spectrum). One tile per workgroup;
// the forward launch covers the entries of a batch group along blockIdx.y.
// ---------------------------------------------------------------------------
template <typename T, int R, int NB>
__device__ __forceinline__ bool row_above_nyquist(int j, int r) {
  if constexpr (R % 2 == 0) {
    return r >= R / 2;  // row N itself has T_0 = 0, either sign is right
  } else {
    constexpr int N = R * NB / 2;
    return j + r * NB > N;
  }
}

template <typename T, typename SL, typename RegsOut, typename RegsIn>
__device__ __forceinline__ void grad_multiply(RegsOut& v, const RegsIn& x, const FusedGeom<T>& g, const GradSpec<T>& sp,
                                              uint32_t colpart, bool neg1, int field, int sgn, int q) {
#pragma unroll
  for (int t = 0; t < SL::NTASK; ++t) {
    if (!SL::active(t, q)) continue;
    const int j = q + t * SL::NQ;
    const SpecIdx<T> si(g, colpart, j);
    const T* __restrict__ sa = sp.s[field];
#pragma unroll
    for (int r = 0; r < SL::R; ++r) {
      T val = sa[si.template at<SL::R, SL::NB>(j, r)];
      if (field == 0) {
        v.v[t][r] = {x.v[t][r].x * val, x.v[t][r].y * val};
      } else {
        const bool neg = field == 1 ? row_above_nyquist<T, SL::R, SL::NB>(j, r) : (field == 2 && g.dim == 3 && neg1);
        if (neg) val = -val;
        v.v[t][r] = deriv(x.v[t][r], sgn, val);
      }
    }
  }
}

// Both gradient-field kernels ask for full occupancy in FP32 (64 VGPRs: the
// allocator then spills 16 bytes per lane, measured 22% faster than one
// 1024-thread workgroup per CU); FP64 fits two workgroups without it.
template <typename T, int P> constexpr int grad_minw() { return Tile<T, P>::MINW * (sizeof(T) == 4 ? 2 : 1); }

template <typename T, int P>
__global__ __launch_bounds__((Tile<T, P>::NT), (grad_minw<T, P>())) void k_fused_grad(const cplx<T>* __restrict__ in,
                                                                cplx<T>* __restrict__ out,
                                                                FusedGeom<T> g, GradSpec<T> sp,
                                                                const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TL = Tile<T, P>;
  constexpr int NL = TL::NL, NT = TL::NT, LP = NL;
  constexpr int NSTG = n_stages(P);
  __shared__ C lds[P * LP];
  __shared__ C twl[tw_both_size<P>()];
  const int tid = threadIdx.x, l = tid % NL, q = tid / NL;
  const FusedCol<T> fc(g, (int64_t)blockIdx.x * NL + l);
  const ColIO& cio = fc.io;
  const bool neg1 = g.dim == 3 && (int)(cio.col / (uint32_t)g.hs) > g.n1;
  const int e = (int)blockIdx.y;  // entry
  const C* __restrict__ src = in + e * g.in_es;
  stage_twiddles_both<C, P, NT>(twl, tw, tid);
  using S0 = Stage<T, P, NT, NL, LP, -1, 0>;
  using SL = Stage<T, P, NT, NL, LP, -1, NSTG - 1>;
  using IS0 = Stage<T, P, NT, NL, LP, 1, 0>;
  using ISL = Stage<T, P, NT, NL, LP, 1, NSTG - 1>;
  static_assert(IS0::R == SL::R && IS0::NTASK == SL::NTASK, "register hand-off");

  typename S0::Regs g0;
  S0::template load_first<true>(g0, q, [&](int j, int r) { return src[cio.off<S0::NB>(j, r)]; });
  S0::template butterflies<true>(g0, q);
  S0::lds_out(g0, lds, l, q);
  __syncthreads();
  typename SL::Regs rh;
  middle_and_last<T, P, NT, NL, LP, -1>(rh, lds, twl, l, q);
  for (int fi = 0; fi < g.nf; ++fi) {
    // this field's copies of the thread's line and position: the LDS and
    // twiddle addresses are recomputed per field instead of held through
    // every transform
    int lf = l, qf = q;
    asm volatile("" : "+v"(lf), "+v"(qf));
    typename IS0::Regs v;
    grad_multiply<T, SL>(v, rh, g, sp, fc.colpart, neg1, g.fields[fi], -1, qf);
    IS0::butterflies(v, qf);
    __syncthreads();
    IS0::lds_out(v, lds, lf, qf);
    __syncthreads();
    typename ISL::Regs o;
    middle_and_last<T, P, NT, NL, LP, 1>(o, lds, tw_inverse<P>(twl), lf, qf);
    if (cio.valid) {
      C* __restrict__ dst = out + e * g.out_es + fi * g.out_fs;
      ISL::template store_last<true>(o, qf, [&](int j, int r, C val) { dst[cio.off<ISL::NB>(j, r)] = val; });
    }
  }
}

// adjoint: acc = sum_f conj(m_f) FFT(in_f), out = pruned inverse of acc
template <typename T, int P>
__global__ __launch_bounds__((Tile<T, P>::NT), (grad_minw<T, P>())) void k_fused_grad_adj(
    const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out, FusedGeom<T> g, GradSpec<T> sp,
    const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TL = Tile<T, P>;
  constexpr int NL = TL::NL, NT = TL::NT, LP = NL;
  constexpr int NSTG = n_stages(P);
  __shared__ C lds[P * LP];
  __shared__ C twl[tw_both_size<P>()];
  const int tid = threadIdx.x, l = tid % NL, q = tid / NL;
  const FusedCol<T> fc(g, (int64_t)blockIdx.x * NL + l);
  const ColIO& cio = fc.io;
  const bool neg1 = g.dim == 3 && (int)(cio.col / (uint32_t)g.hs) > g.n1;
  stage_twiddles_both<C, P, NT>(twl, tw, tid);
  using S0 = Stage<T, P, NT, NL, LP, -1, 0>;
  using SL = Stage<T, P, NT, NL, LP, -1, NSTG - 1>;
  using IS0 = Stage<T, P, NT, NL, LP, 1, 0>;
  using ISL = Stage<T, P, NT, NL, LP, 1, NSTG - 1>;
  static_assert(IS0::R == SL::R && IS0::NTASK == SL::NTASK, "register hand-off");

  typename IS0::Regs acc;
#pragma unroll
  for (int t = 0; t < SL::NTASK; ++t)
#pragma unroll
    for (int r = 0; r < SL::R; ++r) acc.v[t][r] = C{T(0), T(0)};
  for (int fi = 0; fi < g.nf; ++fi) {
    // this field's copies of the thread's line and position (as in k_fused_grad)
    int lf = l, qf = q;
    asm volatile("" : "+v"(lf), "+v"(qf));
    const C* __restrict__ src = in + fi * g.in_fs;
    typename S0::Regs g0;
    S0::template load_first<true>(g0, qf, [&](int j, int r) { return src[cio.off<S0::NB>(j, r)]; });
    S0::template butterflies<true>(g0, qf);
    __syncthreads();
    S0::lds_out(g0, lds, lf, qf);
    __syncthreads();
    typename SL::Regs rh;
    middle_and_last<T, P, NT, NL, LP, -1>(rh, lds, twl, lf, qf);
    typename IS0::Regs m;
    grad_multiply<T, SL>(m, rh, g, sp, fc.colpart, neg1, g.fields[fi], 1, qf);
#pragma unroll
    for (int t = 0; t < SL::NTASK; ++t) {
      if (!SL::active(t, qf)) continue;
#pragma unroll
      for (int r = 0; r < SL::R; ++r) {
        acc.v[t][r].x += m.v[t][r].x;
        acc.v[t][r].y += m.v[t][r].y;
      }
    }
  }
  IS0::butterflies(acc, q);
  __syncthreads();
  IS0::lds_out(acc, lds, l, q);
  __syncthreads();
  typename ISL::Regs o;
  middle_and_last<T, P, NT, NL, LP, 1>(o, lds, tw_inverse<P>(twl), l, q);
  if (cio.valid)
    ISL::template store_last<true>(o, q, [&](int j, int r, C val) { out[cio.off<ISL::NB>(j, r)] = val; });
}

// ---------------------------------------------------------------------------
// Layout with the multiply along the contiguous axis. The real-to-complex
// transform runs along axis 0 over strided columns (k_r2c_s), the complex
// passes follow, the multiply-and-inverse pass runs along the contiguous
// last axis with one wavefront per line group (k_fused_c), and the final
// complex-to-real transform is again along axis 0 (k_c2r_s).
//
// Axis-0 real transforms: two adjacent real columns travel as one complex
// column z = x_a + i x_b; after the transform
//   X_a[k] = (Z[k] + conj Z[P-k]) / 2,  X_b[k] = -i (Z[k] - conj Z[P-k]) / 2,
// exchanged through the LDS tile; the inverse builds Z from X_a, X_b the same
// way. A workgroup covers NL column pairs (one 128-byte row segment of the
// real array); blockIdx.y is the entry.
// ---------------------------------------------------------------------------
template <typename T, int P, int NTERM, int V>
__global__ __launch_bounds__((TileV<T, P, V>::NT), (TileV<T, P, V>::MINW)) void k_r2c_s(R2CSArgs<T> a,
                                                                   const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TL = TileV<T, P, V>;
  constexpr int NL = TL::NL, NT = TL::NT, LP = NL, N = P / 2, H = N + 1;
  constexpr int NSTG = n_stages(P);
  constexpr int NQ = NT / NL;
  constexpr int NSLOT = (H + NQ - 1) / NQ;
  using S0 = Stage<T, P, NT, NL, LP, -1, 0>;
  using SL = Stage<T, P, NT, NL, LP, -1, NSTG - 1>;
  __shared__ C lds[P * LP];
  __shared__ C twl[P];
  const int tid = threadIdx.x, l = tid % NL, q = tid / NL;
  const int e = (int)blockIdx.y;
  const int64_t npairs = a.ncols / 2;
  const ColIO ci(tile_of_block<V>(blockIdx.x, gridDim.x) * NL + l, npairs, npairs);
  stage_twiddles<C, P, NT, -1>(twl, tw, tid);

  C acc_a[NSLOT], acc_b[NSLOT];
#pragma unroll
  for (int term = 0; term < NTERM; ++term) {
    const T* base = a.in_tab[term] ? a.in_tab[term][e] + a.in_off[term] : a.in[term];
    const C* __restrict__ src = reinterpret_cast<const C*>(base);
    const int code = a.d.code[term];
    if (term > 0) __syncthreads();  // the previous term's reads of the tile are done
    typename S0::Regs g0;
    if (a.nt_load)
      S0::template load_first<true>(g0, q, [&](int j, int r) { return load_nt(&src[ci.off<S0::NB>(j, r)]); });
    else
      S0::template load_first<true>(g0, q, [&](int j, int r) { return src[ci.off<S0::NB>(j, r)]; });
    S0::template butterflies<true>(g0, q);
    S0::lds_out(g0, lds, l, q);
    __syncthreads();
    typename SL::Regs gl;
    middle_and_last<T, P, NT, NL, LP, -1>(gl, lds, twl, l, q);
    __syncthreads();
    SL::lds_out(gl, lds, l, q);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
      const int k = q + NQ * s;
      if (k >= H) continue;
      const C z = lds[lds_index<0, LP>(k, l)];
      const C zm = lds[lds_index<0, LP>((P - k) % P, l)];
      const C xa = C{T(0.5) * (z.x + zm.x), T(0.5) * (z.y - zm.y)};
      const C xb = C{T(0.5) * (z.y + zm.y), T(0.5) * (zm.x - z.x)};
      const T kk = a.d.ks * (T)(k < N ? k : 0);
      if (term == 0) {
        acc_a[s] = deriv(xa, code, kk);
        acc_b[s] = deriv(xb, code, kk);
      } else {
        acc_a[s] = deriv_add(acc_a[s], xa, code, kk);
        acc_b[s] = deriv_add(acc_b[s], xb, code, kk);
      }
    }
  }
  if (!ci.valid) return;
  C* __restrict__ out = a.out + e * a.out_es + 2 * (int64_t)ci.col;
#pragma unroll
  for (int s = 0; s < NSLOT; ++s) {
    const int k = q + NQ * s;
    if (k >= H) continue;
    store_pair(out + k * a.ncols, acc_a[s], acc_b[s]);
  }
}

template <typename T, int P, int NOUT, int V>
__global__ __launch_bounds__((TileV<T, P, V>::NT), (TileV<T, P, V>::MINW)) void k_c2r_s(C2RSArgs<T> a,
                                                                   const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using TL = TileV<T, P, V>;
  constexpr int NL = TL::NL, NT = TL::NT, LP = NL, N = P / 2, H = N + 1;
  constexpr int NSTG = n_stages(P);
  constexpr int NQ = NT / NL;
  constexpr int NSLOT = (H + NQ - 1) / NQ;
  using S0 = Stage<T, P, NT, NL, LP, 1, 0>;
  using SL = Stage<T, P, NT, NL, LP, 1, NSTG - 1>;
  __shared__ C lds[P * LP];
  __shared__ C twl[P];
  const int tid = threadIdx.x, l0 = tid % NL, q0 = tid / NL;
  const int e = (int)blockIdx.y;
  const int64_t npairs = a.ncols / 2;
  const ColIO ci(tile_of_block<V>(blockIdx.x, gridDim.x) * NL + l0, npairs, npairs);
  const C* __restrict__ in = a.in + e * a.in_es + 2 * (int64_t)ci.col;
  // FP64 holds the columns of `in` through the outputs taken from it
  // (measured faster); in FP32 holding them takes more registers than two
  // workgroups per CU allow, and reading them again from cache is faster
  constexpr bool HOLD = sizeof(T) == 8;
  C xs[NSLOT], ys[NSLOT];
  auto load = [&](const C* __restrict__ src, bool nt) {
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
      const int k = q0 + NQ * s;
      xs[s] = ys[s] = C{T(0), T(0)};
      if (k >= H) continue;
      if (nt) load_pair_nt(src + k * a.ncols, xs[s], ys[s]);
      else load_pair(src + k * a.ncols, xs[s], ys[s]);
    }
  };
  load(in, false);
  stage_twiddles<C, P, NT, 1>(twl, tw, tid);

#pragma unroll
  for (int o = 0; o < NOUT; ++o) {
    const bool own = o < a.d.n;  // from `in` with its factor, else from in_x
    const int code = own ? a.d.code[o] : 0;
    if (o > 0 && !(HOLD && own)) {
      // read the columns (again, from cache, for an output of `in`) here
      // rather than hold them in registers through the previous output's
      // transform
      uint32_t z = 0;
      asm volatile("" : "+s"(z));
      load((own ? in : a.in_x[o - a.d.n] + e * a.in_es + 2 * (int64_t)ci.col) + z, !own && a.nt_x);
    }
    __syncthreads();  // twiddles staged / the previous output's reads are done
    // this output's copies of the thread's line and position: the compiler
    // then recomputes the LDS addresses per output instead of holding one
    // set in registers through every transform
    int l = l0, q = q0;
    if (o > 0) asm volatile("" : "+v"(l), "+v"(q));
    // Z[k] = X[k] + i Y[k], Z[P-k] = conj X[k] + i conj Y[k]; the imaginary
    // parts of X, Y at k = 0 and k = N are dropped (real by symmetry)
#pragma unroll
    for (int s = 0; s < NSLOT; ++s) {
      const int k = q + NQ * s;
      if (k >= H) continue;
      C X = xs[s], Y = ys[s];
      if (code != 0) {
        const T kk = a.d.ks * (T)(k < N ? k : 0);
        X = deriv(X, code, kk);
        Y = deriv(Y, code, kk);
      }
      if (k == 0 || k == N) {
        lds[lds_index<0, LP>(k, l)] = C{X.x, Y.x};
      } else {
        lds[lds_index<0, LP>(k, l)] = C{X.x - Y.y, X.y + Y.x};
        lds[lds_index<0, LP>(P - k, l)] = C{X.x + Y.y, Y.x - X.y};
      }
    }
    __syncthreads();
    typename S0::Regs g0;
    S0::template load_first<false>(g0, q, [&](int j, int r) { return lds[lds_index<0, LP>(S0::in_pos(j, r), l)]; });
    S0::butterflies(g0, q);
    __syncthreads();
    S0::lds_out(g0, lds, l, q);
    __syncthreads();
    typename SL::Regs gl;
    middle_and_last<T, P, NT, NL, LP, 1>(gl, lds, twl, l, q);
    if (ci.valid) {
      T* base = a.out_tab[o] ? a.out_tab[o][e] + a.out_off[o] : a.out[o];
      C* __restrict__ dst = reinterpret_cast<C*>(base);
      SL::template store_last<true>(gl, q, [&](int j, int r, C v) { dst[ci.off<SL::NB>(j, r)] = v; });
    }
  }
}

// Position of a line of the multiply pass, walked without divisions: entry
// e and (k0, k1) with entry-local line k0 * p1 + k1 (3D: k0 is the axis-0
// row, k1 the axis-1 wavenumber index; 2D: one row block, k1 = the line).
struct LineWalk {
  int e, k0, k1;
  int p1, h0;
  __device__ __forceinline__ void advance(int by) {
    k1 += by;
    while (k1 >= p1) {
      k1 -= p1;
      if (++k0 == h0) {
        k0 = 0;
        ++e;
      }
    }
  }
};

// Address of position j + r NB of a line written in the tiled layout
// (FusedCGeom::ytile = sh, bs = p1 << sh): a uniform base per r plus a 32-bit
// per-lane offset, which the stores take as scalar base and vector offset
// without 64-bit address arithmetic per store.
template <int NB, typename C>
__device__ __forceinline__ C* tiled_ptr(C* d, int j, int r, int sh, int bs) {
  C* dr = d + (int64_t)r * (int64_t)((NB >> sh) * bs);
  // byte offset as a 32-bit value (every tiled plane is below 4 GiB)
  const uint32_t lo = (uint32_t)((j >> sh) * bs + (j & ((1 << sh) - 1))) * (uint32_t)sizeof(C);
  return reinterpret_cast<C*>(reinterpret_cast<char*>(dr) + lo);
}

// Multiply-and-inverse pass along the contiguous last axis: each wavefront
// walks gpw groups of LPW lines (VGF_FC_WALK sets their order; lanes along
// the line, every exchange inside the wavefront). Line (k0, k1) of length n_last is
// transformed forward (pruned input), multiplied by the kernel-spectrum
// octant row (k0, fold(k1)) at fold(k_last), and inverted (pruned output) as
// phi's spectrum and, when requested, as -i k_last times it (E_last). The
// walk over several groups shares the twiddle staging and the index set-up
// among them and needs no per-line division.
template <typename T, int P, int V>
__global__ __launch_bounds__((TileW<T, P, V>::NT), (TileW<T, P, V>::MINW_FC)) void k_fused_c(
    const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out, FusedCGeom<T> g, const T* __restrict__ spec,
    const cplx<T>* __restrict__ tw, int gpw) {
  using C = cplx<T>;
  using TW = TileW<T, P, V>;
  constexpr int NQ = TW::NQ, LPW = TW::LPW, LP = TW::LP, N = P / 2;
  constexpr int NSTG = n_stages(P);
  // exchanges through the per-exchange pads of layout 3
  using S0 = Stage<T, P, 64, LPW, LP, -1, 0, kPadLayout>;
  using SL = Stage<T, P, 64, LPW, LP, -1, NSTG - 1, kPadLayout>;
  using IS0 = Stage<T, P, 64, LPW, LP, 1, 0, kPadLayout>;
  using ISL = Stage<T, P, 64, LPW, LP, 1, NSTG - 1, kPadLayout>;
  static_assert(IS0::R == SL::R && IS0::NTASK == SL::NTASK, "register hand-off");
  __shared__ C tiles[TW::WPB * LPW * LP];
  __shared__ C twl[tw_both_size<P>()];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l = lane / NQ, q = lane % NQ;
  C* tile = tiles + w * LPW * LP;
  // VGF_FC_WALK: the workgroup's WPB wavefronts take consecutive line groups
  // and step by WPB groups (neighbouring lines read and written together);
  // else each wavefront walks its own gpw consecutive groups
  constexpr int STEP = VGF_FC_WALK ? TW::WPB : 1;
  int64_t line = (VGF_FC_WALK ? (int64_t)blockIdx.x * TW::WPB * gpw + w : ((int64_t)blockIdx.x * TW::WPB + w) * gpw) *
                     LPW + l;
  LineWalk wk;
  wk.p1 = g.dim == 3 ? 2 * g.n1 : (int)g.lpe;
  wk.h0 = g.dim == 3 ? g.n0 + 1 : 1;
  {
    const EntryLine el(line < g.nlines ? line : 0, g.lpe, g.nlines);
    wk.e = (int)el.e;
    wk.k0 = (int)el.line / wk.p1;
    wk.k1 = (int)el.line - wk.k0 * wk.p1;
  }
  stage_twiddles_both<C, P, TW::NT>(twl, tw, tid);
  __syncthreads();

  // this lane's kernel-spectrum values of the line at the walk position
  constexpr int NV = SL::NTASK * SL::R;
  T sv[NV];
  auto load_spec = [&](bool ok) {
    const int row = !ok ? 0
                        : g.dim == 3 ? wk.k0 * (g.n1 + 1) + (wk.k1 <= g.n1 ? wk.k1 : wk.p1 - wk.k1)
                                     : wk.k1;
    const T* __restrict__ srow = spec + (int64_t)row * (N + 1);
#pragma unroll
    for (int t = 0; t < SL::NTASK; ++t) {
      if (!SL::active(t, q)) continue;
      const int j = q + t * SL::NQ;
#pragma unroll
      for (int r = 0; r < SL::R; ++r) {
        const int p = j + r * SL::NB;
        sv[t * SL::R + r] = srow[p <= N ? p : P - p];
      }
    }
  };
  typename S0::Regs x;
  auto load_input = [&](bool ok) {
    const C* __restrict__ src = ok ? in + wk.e * g.in_es + ((int64_t)wk.k0 * wk.p1 + wk.k1) * N : in;
    if (g.nt)
      S0::template load_first<true>(x, q, [&](int j, int r) { return load_nt(&src[S0::in_pos(j, r)]); });
    else
      S0::template load_first<true>(x, q, [&](int j, int r) { return src[S0::in_pos(j, r)]; });
  };
  bool valid = line < g.nlines;
  for (int it = 0; it < gpw; ++it) {
    load_spec(valid);
    load_input(valid);
    const bool store = valid;
    // plain rows: line (k0, k1) at (k0 p1 + k1) N; tiled: its B-element
    // pieces at k0 p1 N + k1 B + (x >> log2 B) p1 B
    C* __restrict__ dst = !store ? out
                          : out + wk.e * g.out_es +
                                (g.ytile ? (int64_t)wk.k0 * wk.p1 * N + ((int64_t)wk.k1 << g.ytile)
                                         : ((int64_t)wk.k0 * wk.p1 + wk.k1) * N);
    S0::template butterflies<true>(x, q);
    wave_sync();  // the previous line's reads of the tile are done
    S0::lds_out(x, tile, l, q);
    line += STEP * LPW;
    wk.advance(STEP * LPW);
    valid = line < g.nlines;
    wave_sync();
    typename SL::Regs rh;  // forward spectrum, then times the kernel spectrum
    middle_and_last<T, P, 64, LPW, LP, -1, kPadLayout, true>(rh, tile, twl, l, q);
#pragma unroll
    for (int t = 0; t < SL::NTASK; ++t) {
      if (!SL::active(t, q)) continue;
#pragma unroll
      for (int r = 0; r < SL::R; ++r) {
        rh.v[t][r].x *= sv[t * SL::R + r];
        rh.v[t][r].y *= sv[t * SL::R + r];
      }
    }
    for (int fi = 0; fi < g.nf; ++fi) {
      typename IS0::Regs v;
#pragma unroll
      for (int t = 0; t < SL::NTASK; ++t) {
        if (!SL::active(t, q)) continue;
        int j = q + t * SL::NQ;
        // FP64: recompute the wavenumbers per line rather than hold them in
        // registers across the loop (the compiler would hoist them)
        if constexpr (sizeof(T) == 8) asm volatile("" : "+v"(j));
#pragma unroll
        for (int r = 0; r < SL::R; ++r)
          v.v[t][r] = fi == 0 ? rh.v[t][r] : deriv(rh.v[t][r], -1, axis_k<T, SL::R, SL::NB>(g.ks, j, r));
      }
      IS0::butterflies(v, q);
      wave_sync();  // the previous transform's reads of the tile are done
      IS0::lds_out(v, tile, l, q);
      wave_sync();
      typename ISL::Regs o;
      middle_and_last<T, P, 64, LPW, LP, 1, kPadLayout, true>(o, tile, tw_inverse<P>(twl), l, q);
      if (store) {
        C* __restrict__ d = dst + fi * g.fs;
        if (g.ytile) {
          // position j + r NB: block (j >> sh) + r (NB >> sh), offset j mod B
          const int sh = g.ytile, bs = wk.p1 << sh;
          if (g.nt)
            ISL::template store_last<true>(o, q, [&](int j, int r, C val) {
              store_nt(tiled_ptr<ISL::NB>(d, j, r, sh, bs), val);
            });
          else
            ISL::template store_last<true>(o, q, [&](int j, int r, C val) {
              *tiled_ptr<ISL::NB>(d, j, r, sh, bs) = val;
            });
        } else if (g.nt) {
          ISL::template store_last<true>(o, q, [&](int j, int r, C val) { store_nt(&d[j + r * ISL::NB], val); });
        } else {
          ISL::template store_last<true>(o, q, [&](int j, int r, C val) { d[j + r * ISL::NB] = val; });
        }
      }
    }
  }
}

// The multiply pass for lines of P >= 512, one line per wavefront (all 64
// lanes along it). The line a wavefront works on is the same for all its
// lanes, so the walk and every line base address live in scalar registers
// and each lane keeps fixed per-lane offsets; the number of output fields is
// a template parameter (straight-line code for phi and E_last); and the
// twiddle slots of the last stage of each direction, the same for every
// line, are loaded once and held in registers. Same arithmetic per line as
// k_fused_c.
template <typename T, int P, int NF>
__global__ __launch_bounds__((TileW<T, P>::NT), (TileW<T, P>::MINW_FC)) void k_fused_c1(
    const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out, FusedCGeom<T> g, const T* __restrict__ spec,
    const cplx<T>* __restrict__ tw, int gpw) {
  using C = cplx<T>;
  using TW = TileW<T, P>;
  static_assert(TW::LPW == 1 && TW::NQ == 64, "one line per wavefront");
  constexpr int LP = TW::LP, N = P / 2;
  constexpr int NSTG = n_stages(P);
  // 512-point lines exchange through the bank-conflict-free layout 2, the
  // other lengths through the per-exchange pads of layout 3
  constexpr int LAY = (VGF_LAY2 && P == 512) ? 2 : kPadLayout;
  using S0 = Stage<T, P, 64, 1, LP, -1, 0, LAY>;
  using SL = Stage<T, P, 64, 1, LP, -1, NSTG - 1, LAY>;
  using IS0 = Stage<T, P, 64, 1, LP, 1, 0, LAY>;
  using ISL = Stage<T, P, 64, 1, LP, 1, NSTG - 1, LAY>;
  static_assert(IS0::R == SL::R && IS0::NTASK == SL::NTASK, "register hand-off");
  __shared__ C tiles[TW::WPB * LP];
  __shared__ C twl[tw_both_size<P>()];
  const int tid = threadIdx.x, q = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  C* tile = tiles + w * LP;
  // VGF_FC_WALK: consecutive lines to the WPB wavefronts, then steps of WPB
  // lines; else each wavefront walks its own gpw consecutive lines
  constexpr int STEP = VGF_FC_WALK ? TW::WPB : 1;
  int64_t line = VGF_FC_WALK ? (int64_t)blockIdx.x * TW::WPB * gpw + w : ((int64_t)blockIdx.x * TW::WPB + w) * gpw;
  LineWalk wk;
  wk.p1 = g.dim == 3 ? 2 * g.n1 : (int)g.lpe;
  wk.h0 = g.dim == 3 ? g.n0 + 1 : 1;
  {
    const EntryLine el(line < g.nlines ? line : 0, g.lpe, g.nlines);
    wk.e = (int)el.e;
    wk.k0 = (int)el.line / wk.p1;
    wk.k1 = (int)el.line - wk.k0 * wk.p1;
  }
  stage_twiddles_both<C, P, TW::NT>(twl, tw, tid);
  __syncthreads();
  // the last stages' twiddle slots stay in registers when they are few
  // (one butterfly per lane); otherwise they are read from LDS per line
  constexpr bool TWREG = SL::NTASK * (SL::R - 1) <= 8 && ISL::NTASK * (ISL::R - 1) <= 8;
  typename SL::Tw twf;
  typename ISL::Tw twi;
  if constexpr (TWREG) {
    SL::load_tw(twf, twl, q);
    ISL::load_tw(twi, tw_inverse<P>(twl), q);
  }

  for (int it = 0; it < gpw && line < g.nlines; ++it, line += STEP) {
    const int64_t lofs = ((int64_t)wk.k0 * wk.p1 + wk.k1) * N;
    const int row = g.dim == 3 ? wk.k0 * (g.n1 + 1) + (wk.k1 <= g.n1 ? wk.k1 : wk.p1 - wk.k1) : wk.k1;
    const T* __restrict__ srow = spec + (int64_t)row * (N + 1);
    const C* __restrict__ src = in + wk.e * g.in_es + lofs;
    // plain rows, or the tiled layout: the line's B-element pieces at
    // k0 p1 N + k1 B + (x >> log2 B) p1 B
    C* __restrict__ dst = out + wk.e * g.out_es +
                          (g.ytile ? (int64_t)wk.k0 * wk.p1 * N + ((int64_t)wk.k1 << g.ytile) : lofs);
    const int ybs = wk.p1 << g.ytile;
    wk.advance(STEP);
    typename S0::Regs x;
    if (g.nt)
      S0::template load_first<true>(x, q, [&](int j, int r) { return load_nt(&src[S0::in_pos(j, r)]); });
    else
      S0::template load_first<true>(x, q, [&](int j, int r) { return src[S0::in_pos(j, r)]; });
    T sv[SL::NTASK][SL::R];
#pragma unroll
    for (int t = 0; t < SL::NTASK; ++t) {
      if (!SL::active(t, q)) continue;
      const int j = q + t * SL::NQ;
#pragma unroll
      for (int r = 0; r < SL::R; ++r) {
        const int p = j + r * SL::NB;
        sv[t][r] = srow[p <= N ? p : P - p];
      }
    }
    S0::template butterflies<true>(x, q);
    wave_sync();  // the previous line's reads of the tile are done
    S0::lds_out(x, tile, 0, q);
    wave_sync();
    typename SL::Regs rh;  // forward spectrum, then times the kernel spectrum
    if constexpr (TWREG) middle_and_last_tw<T, P, 64, 1, LP, -1, LAY, true>(rh, tile, twl, twf, 0, q);
    else middle_and_last<T, P, 64, 1, LP, -1, LAY, true>(rh, tile, twl, 0, q);
#pragma unroll
    for (int t = 0; t < SL::NTASK; ++t) {
      if (!SL::active(t, q)) continue;
#pragma unroll
      for (int r = 0; r < SL::R; ++r) {
        rh.v[t][r].x *= sv[t][r];
        rh.v[t][r].y *= sv[t][r];
      }
    }
    StaticFor<0, NF>::run([&](auto fI) {
      constexpr int fi = decltype(fI)::value;
      typename IS0::Regs v;
#pragma unroll
      for (int t = 0; t < SL::NTASK; ++t) {
        if (!SL::active(t, q)) continue;
        const int j = q + t * SL::NQ;
#pragma unroll
        for (int r = 0; r < SL::R; ++r)
          v.v[t][r] = fi == 0 ? rh.v[t][r] : deriv(rh.v[t][r], -1, axis_k<T, SL::R, SL::NB>(g.ks, j, r));
      }
      IS0::butterflies(v, q);
      wave_sync();  // the previous transform's reads of the tile are done
      IS0::lds_out(v, tile, 0, q);
      wave_sync();
      typename ISL::Regs o;
      if constexpr (TWREG) middle_and_last_tw<T, P, 64, 1, LP, 1, LAY, true>(o, tile, tw_inverse<P>(twl), twi, 0, q);
      else middle_and_last<T, P, 64, 1, LP, 1, LAY, true>(o, tile, tw_inverse<P>(twl), 0, q);
      C* __restrict__ d = dst + fi * g.fs;
      if (g.ytile) {
        // position j + r NB: block (j >> sh) + r (NB >> sh), offset j mod B
        const int sh = g.ytile;
        if (g.nt)
          ISL::template store_last<true>(o, q, [&](int j, int r, C val) {
            store_nt(tiled_ptr<ISL::NB>(d, j, r, sh, ybs), val);
          });
        else
          ISL::template store_last<true>(o, q, [&](int j, int r, C val) {
            *tiled_ptr<ISL::NB>(d, j, r, sh, ybs) = val;
          });
      } else if (g.nt) {
        ISL::template store_last<true>(o, q, [&](int j, int r, C val) { store_nt(&d[j + r * ISL::NB], val); });
      } else {
        ISL::template store_last<true>(o, q, [&](int j, int r, C val) { d[j + r * ISL::NB] = val; });
      }
    });
  }
}

// adjoint: acc = sum_f conj(m_f) FFT(in_f) (m_f = 1 or -i k_last), times the
// real kernel spectrum, inverted with pruned output; the same line walk as
// the forward pass
template <typename T, int P, int V>
__global__ __launch_bounds__((TileW<T, P, V>::NT), (TileW<T, P, V>::MINW_FC)) void k_fused_c_adj(
    const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out, FusedCGeom<T> g, const T* __restrict__ spec,
    const cplx<T>* __restrict__ tw, int gpw) {
  using C = cplx<T>;
  using TW = TileW<T, P, V>;
  constexpr int NQ = TW::NQ, LPW = TW::LPW, LP = TW::LP, N = P / 2;
  constexpr int NSTG = n_stages(P);
  // one 512-point line per wavefront: the bank-conflict-free layout 2;
  // otherwise the per-exchange pads of layout 3
  constexpr int LAY = (VGF_LAY2 && P == 512 && LPW == 1 && NQ == 64) ? 2 : kPadLayout;
  using S0 = Stage<T, P, 64, LPW, LP, -1, 0, LAY>;
  using SL = Stage<T, P, 64, LPW, LP, -1, NSTG - 1, LAY>;
  using IS0 = Stage<T, P, 64, LPW, LP, 1, 0, LAY>;
  using ISL = Stage<T, P, 64, LPW, LP, 1, NSTG - 1, LAY>;
  static_assert(IS0::R == SL::R && IS0::NTASK == SL::NTASK, "register hand-off");
  __shared__ C tiles[TW::WPB * LPW * LP];
  __shared__ C twl[tw_both_size<P>()];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l = lane / NQ, q = lane % NQ;
  C* tile = tiles + w * LPW * LP;
  // line order as in k_fused_c (VGF_FC_WALK)
  constexpr int STEP = VGF_FC_WALK ? TW::WPB : 1;
  int64_t line = (VGF_FC_WALK ? (int64_t)blockIdx.x * TW::WPB * gpw + w : ((int64_t)blockIdx.x * TW::WPB + w) * gpw) *
                     LPW + l;
  LineWalk wk;
  wk.p1 = g.dim == 3 ? 2 * g.n1 : (int)g.lpe;
  wk.h0 = g.dim == 3 ? g.n0 + 1 : 1;
  {
    const EntryLine el(line < g.nlines ? line : 0, g.lpe, g.nlines);
    wk.e = (int)el.e;
    wk.k0 = (int)el.line / wk.p1;
    wk.k1 = (int)el.line - wk.k0 * wk.p1;
  }
  stage_twiddles_both<C, P, TW::NT>(twl, tw, tid);
  __syncthreads();

  bool valid = line < g.nlines;
  for (int it = 0; it < gpw; ++it) {
    const int64_t lofs = ((int64_t)wk.k0 * wk.p1 + wk.k1) * N;
    const int row = !valid ? 0
                           : g.dim == 3 ? wk.k0 * (g.n1 + 1) + (wk.k1 <= g.n1 ? wk.k1 : wk.p1 - wk.k1)
                                        : wk.k1;
    const T* __restrict__ srow = spec + (int64_t)row * (N + 1);
    typename IS0::Regs acc;
#pragma unroll
    for (int t = 0; t < SL::NTASK; ++t)
#pragma unroll
      for (int r = 0; r < SL::R; ++r) acc.v[t][r] = C{T(0), T(0)};
    for (int fi = 0; fi < g.nf; ++fi) {
      const C* __restrict__ src = valid ? in + wk.e * g.in_es + fi * g.fs + lofs : in;
      typename S0::Regs g0;
      S0::template load_first<true>(g0, q, [&](int j, int r) { return src[S0::in_pos(j, r)]; });
      S0::template butterflies<true>(g0, q);
      wave_sync();  // the previous transform's reads of the tile are done
      S0::lds_out(g0, tile, l, q);
      wave_sync();
      typename SL::Regs rh;
      middle_and_last<T, P, 64, LPW, LP, -1, LAY, true>(rh, tile, twl, l, q);
      const bool d = g.fields[fi] != 0;
#pragma unroll
      for (int t = 0; t < SL::NTASK; ++t) {
        if (!SL::active(t, q)) continue;
        int j = q + t * SL::NQ;
        if constexpr (sizeof(T) == 8) asm volatile("" : "+v"(j));
#pragma unroll
        for (int r = 0; r < SL::R; ++r) {
          const T kk = d ? axis_k<T, SL::R, SL::NB>(g.ks, j, r) : T(0);
          acc.v[t][r] = deriv_add(acc.v[t][r], rh.v[t][r], d ? 1 : 0, kk);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < SL::NTASK; ++t) {
      if (!SL::active(t, q)) continue;
      const int j = q + t * SL::NQ;
#pragma unroll
      for (int r = 0; r < SL::R; ++r) {
        const int p = j + r * SL::NB;
        const T sv = srow[p <= N ? p : P - p];
        acc.v[t][r].x *= sv;
        acc.v[t][r].y *= sv;
      }
    }
    IS0::butterflies(acc, q);
    wave_sync();
    IS0::lds_out(acc, tile, l, q);
    wave_sync();
    typename ISL::Regs o;
    middle_and_last<T, P, 64, LPW, LP, 1, LAY, true>(o, tile, tw_inverse<P>(twl), l, q);
    if (valid) {
      if (g.ytile) {
        // the axis-1 inverse's tile order (as in k_fused_c)
        const int sh = g.ytile, bs = wk.p1 << sh;
        C* __restrict__ dst = out + wk.e * g.out_es + (int64_t)wk.k0 * wk.p1 * N + ((int64_t)wk.k1 << sh);
        ISL::template store_last<true>(o, q, [&](int j, int r, C val) {
          *tiled_ptr<ISL::NB>(dst, j, r, sh, bs) = val;
        });
      } else {
        C* __restrict__ dst = out + wk.e * g.out_es + lofs;
        ISL::template store_last<true>(o, q, [&](int j, int r, C val) { dst[j + r * ISL::NB] = val; });
      }
    }
    line += STEP * LPW;
    wk.advance(STEP * LPW);
    valid = line < g.nlines;
  }
}

// ---------------------------------------------------------------------------
// gradient-kernel fields with the multiply pass along the contiguous axis
// ---------------------------------------------------------------------------
// Multiplier of field f (0: the kernel spectrum, 1 + a: -i T_a) at position p
// of line (k0, k1): the octant value of the field's spectrum, negated for a
// gradient field where its own axis index is mirrored (axis 1 in 3D: k1 > n1;
// the last axis: p > N; axis 0 holds only its non-negative half).
template <typename T, int P>
__device__ __forceinline__ T grad_value(const T* __restrict__ srow, int f, int last_field, bool neg1, int p) {
  constexpr int N = P / 2;
  const T v = srow[p <= N ? p : P - p];
  const bool neg = (f == last_field && p > N) || (f == 2 && last_field == 3 && neg1);
  return neg ? -v : v;
}

// Forward: each line (k0, k1) of X2 (X1 in 2D) is transformed (pruned input)
// and, for each requested field, multiplied by that field's spectrum and
// inverted (pruned output) into out + fi * fs. The line walk and tiles are
// those of k_fused_c (one schedule).
template <typename T, int P>
__global__ __launch_bounds__((TileW<T, P>::NT), (TileW<T, P>::MINW_FC)) void k_fused_cg(
    const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out, FusedCGeom<T> g, GradSpec<T> sp,
    const cplx<T>* __restrict__ tw, int gpw) {
  using C = cplx<T>;
  using TW = TileW<T, P>;
  constexpr int NQ = TW::NQ, LPW = TW::LPW, LP = TW::LP, N = P / 2;
  constexpr int NSTG = n_stages(P);
  // one 512-point line per wavefront: the bank-conflict-free layout 2;
  // otherwise the per-exchange pads of layout 3
  constexpr int LAY = (VGF_LAY2 && P == 512 && LPW == 1 && NQ == 64) ? 2 : kPadLayout;
  using S0 = Stage<T, P, 64, LPW, LP, -1, 0, LAY>;
  using SL = Stage<T, P, 64, LPW, LP, -1, NSTG - 1, LAY>;
  using IS0 = Stage<T, P, 64, LPW, LP, 1, 0, LAY>;
  using ISL = Stage<T, P, 64, LPW, LP, 1, NSTG - 1, LAY>;
  static_assert(IS0::R == SL::R && IS0::NTASK == SL::NTASK, "register hand-off");
  __shared__ C tiles[TW::WPB * LPW * LP];
  __shared__ C twl[tw_both_size<P>()];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l = lane / NQ, q = lane % NQ;
  C* tile = tiles + w * LPW * LP;
  // line order as in k_fused_c (VGF_FC_WALK)
  constexpr int STEP = VGF_FC_WALK ? TW::WPB : 1;
  int64_t line = (VGF_FC_WALK ? (int64_t)blockIdx.x * TW::WPB * gpw + w : ((int64_t)blockIdx.x * TW::WPB + w) * gpw) *
                     LPW + l;
  LineWalk wk;
  wk.p1 = g.dim == 3 ? 2 * g.n1 : (int)g.lpe;
  wk.h0 = g.dim == 3 ? g.n0 + 1 : 1;
  {
    const EntryLine el(line < g.nlines ? line : 0, g.lpe, g.nlines);
    wk.e = (int)el.e;
    wk.k0 = (int)el.line / wk.p1;
    wk.k1 = (int)el.line - wk.k0 * wk.p1;
  }
  stage_twiddles_both<C, P, TW::NT>(twl, tw, tid);
  __syncthreads();
  const int last_field = g.dim;  // 1 + the last axis
  for (int it = 0; it < gpw; ++it) {
    const bool valid = line < g.nlines;
    const int64_t lofs = ((int64_t)wk.k0 * wk.p1 + wk.k1) * N;
    const bool neg1 = g.dim == 3 && wk.k1 > g.n1;
    const int row = !valid ? 0
                           : g.dim == 3 ? wk.k0 * (g.n1 + 1) + (wk.k1 <= g.n1 ? wk.k1 : wk.p1 - wk.k1)
                                        : wk.k1;
    const int64_t e = wk.e;
    const C* __restrict__ src = valid ? in + e * g.in_es + lofs : in;
    typename S0::Regs x;
    if (g.nt)
      S0::template load_first<true>(x, q, [&](int j, int r) { return load_nt(&src[S0::in_pos(j, r)]); });
    else
      S0::template load_first<true>(x, q, [&](int j, int r) { return src[S0::in_pos(j, r)]; });
    S0::template butterflies<true>(x, q);
    wave_sync();  // the previous line's reads of the tile are done
    S0::lds_out(x, tile, l, q);
    wave_sync();
    typename SL::Regs rh;  // the line's spectrum
    middle_and_last<T, P, 64, LPW, LP, -1, LAY, true>(rh, tile, twl, l, q);
    for (int fi = 0; fi < g.nf; ++fi) {
      const int f = g.fields[fi];
      const T* __restrict__ srow = sp.s[f] + (int64_t)row * (N + 1);
      typename IS0::Regs v;
#pragma unroll
      for (int t = 0; t < SL::NTASK; ++t) {
        if (!SL::active(t, q)) continue;
        const int j = q + t * SL::NQ;
#pragma unroll
        for (int r = 0; r < SL::R; ++r) {
          const T m = grad_value<T, P>(srow, f, last_field, neg1, j + r * SL::NB);
          v.v[t][r] = f == 0 ? C{rh.v[t][r].x * m, rh.v[t][r].y * m} : deriv(rh.v[t][r], -1, m);
        }
      }
      IS0::butterflies(v, q);
      wave_sync();  // the previous transform's reads of the tile are done
      IS0::lds_out(v, tile, l, q);
      wave_sync();
      typename ISL::Regs o;
      middle_and_last<T, P, 64, LPW, LP, 1, LAY, true>(o, tile, tw_inverse<P>(twl), l, q);
      if (valid && g.ytile) {
        // the axis-1 inverse's tile order (as in k_fused_c)
        const int sh = g.ytile, bs = wk.p1 << sh;
        C* __restrict__ d = out + e * g.out_es + fi * g.fs + (int64_t)wk.k0 * wk.p1 * N + ((int64_t)wk.k1 << sh);
        if (g.nt)
          ISL::template store_last<true>(o, q, [&](int j, int r, C val) {
            store_nt(tiled_ptr<ISL::NB>(d, j, r, sh, bs), val);
          });
        else
          ISL::template store_last<true>(o, q, [&](int j, int r, C val) {
            *tiled_ptr<ISL::NB>(d, j, r, sh, bs) = val;
          });
      } else if (valid) {
        C* __restrict__ d = out + e * g.out_es + fi * g.fs + lofs;
        if (g.nt)
          ISL::template store_last<true>(o, q, [&](int j, int r, C val) { store_nt(&d[j + r * ISL::NB], val); });
        else
          ISL::template store_last<true>(o, q, [&](int j, int r, C val) { d[j + r * ISL::NB] = val; });
      }
    }
    line += STEP * LPW;
    wk.advance(STEP * LPW);
  }
}

// Adjoint: acc = sum_f conj(m_f) FFT(in_f) with the multipliers of
// k_fused_cg (+i T_a for the fields), inverted once (pruned output).
template <typename T, int P>
__global__ __launch_bounds__((TileW<T, P>::NT), (TileW<T, P>::MINW_FC)) void k_fused_cg_adj(
    const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out, FusedCGeom<T> g, GradSpec<T> sp,
    const cplx<T>* __restrict__ tw, int gpw) {
  using C = cplx<T>;
  using TW = TileW<T, P>;
  constexpr int NQ = TW::NQ, LPW = TW::LPW, LP = TW::LP, N = P / 2;
  constexpr int NSTG = n_stages(P);
  // one 512-point line per wavefront: the bank-conflict-free layout 2;
  // otherwise the per-exchange pads of layout 3
  constexpr int LAY = (VGF_LAY2 && P == 512 && LPW == 1 && NQ == 64) ? 2 : kPadLayout;
  using S0 = Stage<T, P, 64, LPW, LP, -1, 0, LAY>;
  using SL = Stage<T, P, 64, LPW, LP, -1, NSTG - 1, LAY>;
  using IS0 = Stage<T, P, 64, LPW, LP, 1, 0, LAY>;
  using ISL = Stage<T, P, 64, LPW, LP, 1, NSTG - 1, LAY>;
  static_assert(IS0::R == SL::R && IS0::NTASK == SL::NTASK, "register hand-off");
  __shared__ C tiles[TW::WPB * LPW * LP];
  __shared__ C twl[tw_both_size<P>()];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l = lane / NQ, q = lane % NQ;
  C* tile = tiles + w * LPW * LP;
  int64_t line = ((int64_t)blockIdx.x * TW::WPB + w) * gpw * LPW + l;
  LineWalk wk;
  wk.p1 = g.dim == 3 ? 2 * g.n1 : (int)g.lpe;
  wk.h0 = g.dim == 3 ? g.n0 + 1 : 1;
  {
    const EntryLine el(line < g.nlines ? line : 0, g.lpe, g.nlines);
    wk.e = (int)el.e;
    wk.k0 = (int)el.line / wk.p1;
    wk.k1 = (int)el.line - wk.k0 * wk.p1;
  }
  stage_twiddles_both<C, P, TW::NT>(twl, tw, tid);
  __syncthreads();
  const int last_field = g.dim;
  for (int it = 0; it < gpw; ++it) {
    const bool valid = line < g.nlines;
    const int64_t lofs = ((int64_t)wk.k0 * wk.p1 + wk.k1) * N;
    const bool neg1 = g.dim == 3 && wk.k1 > g.n1;
    const int row = !valid ? 0
                           : g.dim == 3 ? wk.k0 * (g.n1 + 1) + (wk.k1 <= g.n1 ? wk.k1 : wk.p1 - wk.k1)
                                        : wk.k1;
    const int64_t e = wk.e;
    typename IS0::Regs acc;
#pragma unroll
    for (int t = 0; t < SL::NTASK; ++t)
#pragma unroll
      for (int r = 0; r < SL::R; ++r) acc.v[t][r] = C{T(0), T(0)};
    for (int fi = 0; fi < g.nf; ++fi) {
      const int f = g.fields[fi];
      const C* __restrict__ src = valid ? in + e * g.in_es + fi * g.fs + lofs : in;
      typename S0::Regs g0;
      S0::template load_first<true>(g0, q, [&](int j, int r) { return src[S0::in_pos(j, r)]; });
      S0::template butterflies<true>(g0, q);
      wave_sync();  // the previous transform's reads of the tile are done
      S0::lds_out(g0, tile, l, q);
      wave_sync();
      typename SL::Regs rh;
      middle_and_last<T, P, 64, LPW, LP, -1, LAY, true>(rh, tile, twl, l, q);
      const T* __restrict__ srow = sp.s[f] + (int64_t)row * (N + 1);
#pragma unroll
      for (int t = 0; t < SL::NTASK; ++t) {
        if (!SL::active(t, q)) continue;
        const int j = q + t * SL::NQ;
#pragma unroll
        for (int r = 0; r < SL::R; ++r) {
          const T m = grad_value<T, P>(srow, f, last_field, neg1, j + r * SL::NB);
          if (f == 0) {
            acc.v[t][r].x = fmaT(rh.v[t][r].x, m, acc.v[t][r].x);
            acc.v[t][r].y = fmaT(rh.v[t][r].y, m, acc.v[t][r].y);
          } else {
            acc.v[t][r] = deriv_add(acc.v[t][r], rh.v[t][r], 1, m);
          }
        }
      }
    }
    IS0::butterflies(acc, q);
    wave_sync();
    IS0::lds_out(acc, tile, l, q);
    wave_sync();
    typename ISL::Regs o;
    middle_and_last<T, P, 64, LPW, LP, 1, LAY, true>(o, tile, tw_inverse<P>(twl), l, q);
    if (valid) {
      C* __restrict__ dst = out + e * g.out_es + lofs;
      ISL::template store_last<true>(o, q, [&](int j, int r, C val) { dst[j + r * ISL::NB] = val; });
    }
    line += LPW;
    wk.advance(LPW);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <typename T, int P>
hipError_t launch_r2c_p(const R2CArgs<T>& a, const cplx<T>* tw, hipStream_t s) {
  using TW = TileW<T, P>;
  const int64_t pairs = (a.nlines + 1) / 2;
  const int64_t blocks = (pairs + TW::PAIRS - 1) / TW::PAIRS;
  if (blocks == 0 || a.d.n == 0) return hipSuccess;
  if (a.d.n == 2)
    hipLaunchKernelGGL((k_r2c<T, P, 2>), dim3((unsigned)blocks), dim3(TW::NT), 0, s, a, tw);
  else
    hipLaunchKernelGGL((k_r2c<T, P, 1>), dim3((unsigned)blocks), dim3(TW::NT), 0, s, a, tw);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t launch_c2r_p(const C2RArgs<T>& a, const cplx<T>* tw, hipStream_t s) {
  using TW = TileW<T, P>;
  const int64_t pairs = (a.nlines + 1) / 2;
  const int64_t blocks = (pairs + TW::PAIRS - 1) / TW::PAIRS;
  if (blocks == 0 || a.d.n == 0) return hipSuccess;
  if (a.d.n == 2)
    hipLaunchKernelGGL((k_c2r<T, P, 2>), dim3((unsigned)blocks), dim3(TW::NT), 0, s, a, tw);
  else
    hipLaunchKernelGGL((k_c2r<T, P, 1>), dim3((unsigned)blocks), dim3(TW::NT), 0, s, a, tw);
  return hipGetLastError();
}

template <typename T, int P, int V>
hipError_t launch_c2c_fwd_v(const C2CFwdArgs<T>& a, const cplx<T>* tw, hipStream_t s) {
  using TL = TileV<T, P, V>;
  const int64_t bx = (a.g.ncols + TL::NL - 1) / TL::NL;
  const int64_t by = (int64_t)a.g.nbatch * a.g.nentry;
  if (bx == 0 || by == 0 || a.d.n == 0) return hipSuccess;
  if (by > 65535) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)bx, (unsigned)by);
  if (a.d.n == 2)
    hipLaunchKernelGGL((k_c2c_fwd<T, P, 2, V>), grid, dim3(TL::NT), 0, s, a, tw);
  else
    hipLaunchKernelGGL((k_c2c_fwd<T, P, 1, V>), grid, dim3(TL::NT), 0, s, a, tw);
  return hipGetLastError();
}

template <typename T, int P, int V>
hipError_t launch_c2c_inv_v(const C2CInvArgs<T>& a, const cplx<T>* tw, hipStream_t s) {
  using TL = TileV<T, P, V>;
  const int64_t bx = (a.g.ncols + TL::NL - 1) / TL::NL;
  const int64_t by = (int64_t)a.g.nbatch * a.g.nentry;
  if (bx == 0 || by == 0 || a.d.n == 0) return hipSuccess;
  if (by > 65535) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)bx, (unsigned)by);
  if (a.in2 != nullptr && (a.d.n != 2 || a.out2 == nullptr)) return hipErrorInvalidValue;
  if (a.in2 != nullptr)
    hipLaunchKernelGGL((k_c2c_inv<T, P, 3, V>), grid, dim3(TL::NT), 0, s, a, tw);
  else if (a.d.n == 2)
    hipLaunchKernelGGL((k_c2c_inv<T, P, 2, V>), grid, dim3(TL::NT), 0, s, a, tw);
  else
    hipLaunchKernelGGL((k_c2c_inv<T, P, 1, V>), grid, dim3(TL::NT), 0, s, a, tw);
  return hipGetLastError();
}

template <typename T, int P, int V>
hipError_t launch_fused_v(const cplx<T>* in, cplx<T>* out, const FusedGeom<T>& g, const T* spec,
                          const cplx<T>* tw, hipStream_t s) {
  using TL = TileF<T, P, V>;
  const int64_t bx = (g.ncols + TL::NL - 1) / TL::NL;
  if (bx == 0) return hipSuccess;
  // one persistent workgroup per resident slot of the current device
  constexpr int kMaxDevices = 64;
  static int slots_of[kMaxDevices] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  int slots = __atomic_load_n(&slots_of[dev], __ATOMIC_RELAXED);
  if (slots == 0) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)k_fused<T, P, V>, TL::NT, 0) !=
            hipSuccess)
      return hipGetLastError();
    slots = cus * (per_cu > 0 ? per_cu : 1);
    __atomic_store_n(&slots_of[dev], slots, __ATOMIC_RELAXED);
  }
  const int64_t total = bx * g.nentry;
  if (total > INT32_MAX) return hipErrorInvalidConfiguration;
  const int grid = (int)(total < slots ? total : slots);
  hipLaunchKernelGGL((k_fused<T, P, V>), dim3((unsigned)grid), dim3(TL::NT), 0, s, in, out, g, spec, tw,
                     (int)bx);
  return hipGetLastError();
}

// Default tile of the strided passes on grids with few columns (2D grids,
// thin 3D grids): where the full-width tiles would give fewer workgroups
// than the chip has CUs, the default schedule takes the half-width tiles,
// for lengths of 256 points or more and for the long FP64 lengths whose
// full-width tile exceeds 64 KiB of LDS. Shorter columns stay at full
// width (32^3 FP64: 24 against 27 us). Every column gets the same
// arithmetic either way, so no result bit changes.
constexpr int64_t kStridedFewBlocks = 256;
template <typename T, int P> inline int strided_variant(int variant, int64_t cols, int64_t batches) {
  if (variant != 0 || (P < 256 && strided_nl<T, P>() <= Tile<T, P>::NL)) return variant;
  const int64_t wgs = (cols + TileV<T, P, 0>::NL - 1) / TileV<T, P, 0>::NL * batches;
  return wgs < kStridedFewBlocks ? 1 : 0;
}

template <typename T, int P>
hipError_t launch_c2c_fwd_p(int variant, const C2CFwdArgs<T>& a, const cplx<T>* tw, hipStream_t s) {
  variant = strided_variant<T, P>(variant, a.g.ncols, (int64_t)a.g.nbatch * a.g.nentry);
  return variant == 1 ? launch_c2c_fwd_v<T, P, 1>(a, tw, s) : launch_c2c_fwd_v<T, P, 0>(a, tw, s);
}

template <typename T, int P>
hipError_t launch_c2c_inv_p(int variant, const C2CInvArgs<T>& a, const cplx<T>* tw, hipStream_t s) {
  variant = strided_variant<T, P>(variant, a.g.ncols, (int64_t)a.g.nbatch * a.g.nentry);
  return variant == 1 ? launch_c2c_inv_v<T, P, 1>(a, tw, s) : launch_c2c_inv_v<T, P, 0>(a, tw, s);
}

template <typename T, int P>
hipError_t launch_fused_p(int variant, bool adjoint, const cplx<T>* in, cplx<T>* out, const FusedGeom<T>& g,
                          const T* spec, const cplx<T>* tw, hipStream_t s) {
  if (g.nf == 0 || g.nentry == 0) return hipSuccess;
  // forward outputs are field 0 (times the kernel spectrum), then optionally
  // field 1 (times -i k_0 and the kernel spectrum), in this order
  if (!adjoint && (g.fields[0] != 0 || (g.nf > 1 && g.fields[1] != 1) || g.nf > 2))
    return hipErrorInvalidValue;
  if (adjoint) {
    if (g.nentry != 1) return hipErrorInvalidValue;  // the adjoint runs one entry per launch
    using TL = Tile<T, P>;
    const int64_t bx = (g.ncols + TL::NL - 1) / TL::NL;
    if (bx == 0) return hipSuccess;
    hipLaunchKernelGGL((k_fused_adj<T, P>), dim3((unsigned)bx), dim3(TL::NT), 0, s, in, out, g, spec, tw);
    return hipGetLastError();
  }
  return variant == 1 ? launch_fused_v<T, P, 1>(in, out, g, spec, tw, s)
                      : launch_fused_v<T, P, 0>(in, out, g, spec, tw, s);
}

template <typename T, int P>
hipError_t launch_fused_grad_p(bool adjoint, const cplx<T>* in, cplx<T>* out, const FusedGeom<T>& g,
                               const GradSpec<T>& sp, const cplx<T>* tw, hipStream_t s) {
  using TL = Tile<T, P>;
  if (g.nf == 0 || g.nentry == 0) return hipSuccess;
  if (g.nf > 4 || g.nentry < 0 || g.nentry > 65535) return hipErrorInvalidValue;
  if (adjoint && g.nentry != 1) return hipErrorInvalidValue;  // the adjoint runs one entry per launch
  const int64_t bx = (g.ncols + TL::NL - 1) / TL::NL;
  if (bx == 0) return hipSuccess;
  if (adjoint)
    hipLaunchKernelGGL((k_fused_grad_adj<T, P>), dim3((unsigned)bx), dim3(TL::NT), 0, s, in, out, g, sp, tw);
  else
    hipLaunchKernelGGL((k_fused_grad<T, P>), dim3((unsigned)bx, (unsigned)g.nentry), dim3(TL::NT), 0, s, in,
                       out, g, sp, tw);
  return hipGetLastError();
}

template <typename T, int P, int V>
hipError_t launch_r2c_s_v(const R2CSArgs<T>& a, const cplx<T>* tw, hipStream_t s) {
  using TL = TileV<T, P, V>;
  if (a.ncols % 2 != 0) return hipErrorInvalidValue;
  const int64_t bx = (a.ncols / 2 + TL::NL - 1) / TL::NL;
  if (bx == 0 || a.nentry == 0 || a.d.n == 0) return hipSuccess;
  if (a.nentry > 65535) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)bx, (unsigned)a.nentry);
  if (a.d.n == 2)
    hipLaunchKernelGGL((k_r2c_s<T, P, 2, V>), grid, dim3(TL::NT), 0, s, a, tw);
  else
    hipLaunchKernelGGL((k_r2c_s<T, P, 1, V>), grid, dim3(TL::NT), 0, s, a, tw);
  return hipGetLastError();
}

template <typename T, int P, int V>
hipError_t launch_c2r_s_v(const C2RSArgs<T>& a, const cplx<T>* tw, hipStream_t s) {
  using TL = TileV<T, P, V>;
  if (a.ncols % 2 != 0) return hipErrorInvalidValue;
  const int64_t bx = (a.ncols / 2 + TL::NL - 1) / TL::NL;
  if (bx == 0 || a.nentry == 0 || a.d.n == 0) return hipSuccess;
  if (a.nentry > 65535) return hipErrorInvalidConfiguration;
  const dim3 grid((unsigned)bx, (unsigned)a.nentry);
  if (a.d.n < 1 || a.d.n > 2 || a.nx < 0 || a.nx > 3 || a.d.n + a.nx > 4) return hipErrorInvalidValue;
  switch (a.d.n + a.nx) {
    case 1: hipLaunchKernelGGL((k_c2r_s<T, P, 1, V>), grid, dim3(TL::NT), 0, s, a, tw); break;
    case 2: hipLaunchKernelGGL((k_c2r_s<T, P, 2, V>), grid, dim3(TL::NT), 0, s, a, tw); break;
    case 3: hipLaunchKernelGGL((k_c2r_s<T, P, 3, V>), grid, dim3(TL::NT), 0, s, a, tw); break;
    default: hipLaunchKernelGGL((k_c2r_s<T, P, 4, V>), grid, dim3(TL::NT), 0, s, a, tw); break;
  }
  return hipGetLastError();
}

template <typename T, int P>
hipError_t launch_r2c_s_p(int variant, const R2CSArgs<T>& a, const cplx<T>* tw, hipStream_t s) {
  variant = strided_variant<T, P>(variant, a.ncols / 2, a.nentry);
  return variant == 1 ? launch_r2c_s_v<T, P, 1>(a, tw, s) : launch_r2c_s_v<T, P, 0>(a, tw, s);
}

template <typename T, int P>
hipError_t launch_c2r_s_p(int variant, const C2RSArgs<T>& a, const cplx<T>* tw, hipStream_t s) {
  variant = strided_variant<T, P>(variant, a.ncols / 2, a.nentry);
  return variant == 1 ? launch_c2r_s_v<T, P, 1>(a, tw, s) : launch_c2r_s_v<T, P, 0>(a, tw, s);
}

// Multiply pass along the contiguous axis. schedule bit 0: lanes per line
// (TileW variant), bit 1: lines each wavefront walks (VGF_FC_GPW, or 16).
template <typename T, int P, int V>
hipError_t launch_fused_c_v(int schedule, bool adjoint, const cplx<T>* in, cplx<T>* out, const FusedCGeom<T>& g,
                            const T* spec, const cplx<T>* tw, hipStream_t s) {
  using TW = TileW<T, P, V>;
  // line groups per wavefront: the schedule's walk length, shortened where
  // the grid would drop below kFusedCMinBlocks workgroups
  const int64_t groups = (g.nlines + TW::LPW - 1) / TW::LPW;
  int gpw = (schedule & 2) ? 16 : VGF_FC_GPW;
  while (gpw > 1 && (groups + (int64_t)TW::WPB * gpw - 1) / ((int64_t)TW::WPB * gpw) < kFusedCMinBlocks) gpw /= 2;
  const int64_t blocks = (groups + (int64_t)TW::WPB * gpw - 1) / ((int64_t)TW::WPB * gpw);
  if (adjoint)
    hipLaunchKernelGGL((k_fused_c_adj<T, P, V>), dim3((unsigned)blocks), dim3(TW::NT), 0, s, in, out, g, spec, tw, gpw);
  else if constexpr (TW::LPW == 1 && VGF_FC1)
    if (g.nf == 2)
      hipLaunchKernelGGL((k_fused_c1<T, P, 2>), dim3((unsigned)blocks), dim3(TW::NT), 0, s, in, out, g, spec, tw, gpw);
    else
      hipLaunchKernelGGL((k_fused_c1<T, P, 1>), dim3((unsigned)blocks), dim3(TW::NT), 0, s, in, out, g, spec, tw, gpw);
  else
    hipLaunchKernelGGL((k_fused_c<T, P, V>), dim3((unsigned)blocks), dim3(TW::NT), 0, s, in, out, g, spec, tw, gpw);
  return hipGetLastError();
}

// Gradient-kernel multiply pass along the contiguous axis (one schedule).
template <typename T, int P>
hipError_t launch_fused_cg_p(bool adjoint, const cplx<T>* in, cplx<T>* out, const FusedCGeom<T>& g,
                             const GradSpec<T>& sp, const cplx<T>* tw, hipStream_t s) {
  using TW = TileW<T, P>;
  if (g.nf == 0 || g.nlines == 0) return hipSuccess;
  if (g.nf < 0 || g.nf > 4 || (g.lpe > 0 && g.nlines % g.lpe != 0)) return hipErrorInvalidValue;
  for (int i = 0; i < g.nf; ++i)
    if (g.fields[i] < 0 || g.fields[i] > g.dim || !sp.s[g.fields[i]]) return hipErrorInvalidValue;
  const int64_t groups = (g.nlines + TW::LPW - 1) / TW::LPW;
  int gpw = VGF_FC_GPW;
  while (gpw > 1 && (groups + (int64_t)TW::WPB * gpw - 1) / ((int64_t)TW::WPB * gpw) < kFusedCMinBlocks) gpw /= 2;
  const int64_t blocks = (groups + (int64_t)TW::WPB * gpw - 1) / ((int64_t)TW::WPB * gpw);
  if (adjoint)
    hipLaunchKernelGGL((k_fused_cg_adj<T, P>), dim3((unsigned)blocks), dim3(TW::NT), 0, s, in, out, g, sp, tw, gpw);
  else
    hipLaunchKernelGGL((k_fused_cg<T, P>), dim3((unsigned)blocks), dim3(TW::NT), 0, s, in, out, g, sp, tw, gpw);
  return hipGetLastError();
}

template <typename T, int P>
hipError_t launch_fused_c_p(int schedule, bool adjoint, const cplx<T>* in, cplx<T>* out, const FusedCGeom<T>& g,
                            const T* spec, const cplx<T>* tw, hipStream_t s) {
  if (g.nf == 0 || g.nlines == 0) return hipSuccess;
  if (g.nf > 2 || (g.lpe > 0 && g.nlines % g.lpe != 0) || schedule < 0 || schedule > 3) return hipErrorInvalidValue;
  return (schedule & 1) ? launch_fused_c_v<T, P, 1>(schedule, adjoint, in, out, g, spec, tw, s)
                        : launch_fused_c_v<T, P, 0>(schedule, adjoint, in, out, g, spec, tw, s);
}

// The per-length launchers of one precision VGF_T: declared extern in the
// dispatch unit (vgf_solve_f32.hip / vgf_solve_f64.hip) and instantiated in
// the unit of the length's group (vgf_solve_f32_g1.hip, ...), so the lengths
// compile in parallel.
#define VGF_LAUNCHERS_P(PFX, PP)                                                                           \
  PFX hipError_t launch_r2c_p<VGF_T, PP>(const R2CArgs<VGF_T>&, const cplx<VGF_T>*, hipStream_t);         \
  PFX hipError_t launch_c2r_p<VGF_T, PP>(const C2RArgs<VGF_T>&, const cplx<VGF_T>*, hipStream_t);         \
  PFX hipError_t launch_c2c_fwd_p<VGF_T, PP>(int, const C2CFwdArgs<VGF_T>&, const cplx<VGF_T>*, hipStream_t); \
  PFX hipError_t launch_c2c_inv_p<VGF_T, PP>(int, const C2CInvArgs<VGF_T>&, const cplx<VGF_T>*, hipStream_t); \
  PFX hipError_t launch_fused_p<VGF_T, PP>(int, bool, const cplx<VGF_T>*, cplx<VGF_T>*, const FusedGeom<VGF_T>&, \
                                           const VGF_T*, const cplx<VGF_T>*, hipStream_t);                 \
  PFX hipError_t launch_fused_grad_p<VGF_T, PP>(bool, const cplx<VGF_T>*, cplx<VGF_T>*,                     \
                                                const FusedGeom<VGF_T>&, const GradSpec<VGF_T>&,           \
                                                const cplx<VGF_T>*, hipStream_t);                          \
  PFX hipError_t launch_r2c_s_p<VGF_T, PP>(int, const R2CSArgs<VGF_T>&, const cplx<VGF_T>*, hipStream_t); \
  PFX hipError_t launch_c2r_s_p<VGF_T, PP>(int, const C2RSArgs<VGF_T>&, const cplx<VGF_T>*, hipStream_t); \
  PFX hipError_t launch_fused_c_p<VGF_T, PP>(int, bool, const cplx<VGF_T>*, cplx<VGF_T>*, const FusedCGeom<VGF_T>&, \
                                             const VGF_T*, const cplx<VGF_T>*, hipStream_t);               \
  PFX hipError_t launch_fused_cg_p<VGF_T, PP>(bool, const cplx<VGF_T>*, cplx<VGF_T>*, const FusedCGeom<VGF_T>&, \
                                              const GradSpec<VGF_T>&, const cplx<VGF_T>*, hipStream_t);
#define VGF_EXTERN_P(PP) VGF_LAUNCHERS_P(extern template, PP)
#define VGF_INSTANTIATE_P(PP) VGF_LAUNCHERS_P(template, PP)
// the launchers of the longer 2D lengths (VGF_FOR_EACH_P_WIDE)
#define VGF_LAUNCHERS_P_WIDE(PFX, PP)                                                                      \
  PFX hipError_t launch_r2c_s_p<VGF_T, PP>(int, const R2CSArgs<VGF_T>&, const cplx<VGF_T>*, hipStream_t); \
  PFX hipError_t launch_c2r_s_p<VGF_T, PP>(int, const C2RSArgs<VGF_T>&, const cplx<VGF_T>*, hipStream_t); \
  PFX hipError_t launch_fused_c_p<VGF_T, PP>(int, bool, const cplx<VGF_T>*, cplx<VGF_T>*, const FusedCGeom<VGF_T>&, \
                                             const VGF_T*, const cplx<VGF_T>*, hipStream_t);               \
  PFX hipError_t launch_fused_cg_p<VGF_T, PP>(bool, const cplx<VGF_T>*, cplx<VGF_T>*, const FusedCGeom<VGF_T>&, \
                                              const GradSpec<VGF_T>&, const cplx<VGF_T>*, hipStream_t);
#define VGF_EXTERN_P_WIDE(PP) VGF_LAUNCHERS_P_WIDE(extern template, PP)
#define VGF_INSTANTIATE_P_WIDE(PP) VGF_LAUNCHERS_P_WIDE(template, PP)

#define VGF_CASE_R2CS(PP) case PP: return launch_r2c_s_p<VGF_T, PP>(variant, a, tw, s);
#define VGF_CASE_C2RS(PP) case PP: return launch_c2r_s_p<VGF_T, PP>(variant, a, tw, s);
#define VGF_CASE_FC(PP) case PP: return launch_fused_c_p<VGF_T, PP>(schedule, adjoint, in, out, g, spec, tw, s);
#define VGF_CASE_FCG(PP) case PP: return launch_fused_cg_p<VGF_T, PP>(adjoint, in, out, g, sp, tw, s);
#define VGF_CASE_R2C(PP) case PP: return launch_r2c_p<VGF_T, PP>(a, tw, s);
#define VGF_CASE_FGRAD(PP) case PP: return launch_fused_grad_p<VGF_T, PP>(adjoint, in, out, g, sp, tw, s);
#define VGF_CASE_C2R(PP) case PP: return launch_c2r_p<VGF_T, PP>(a, tw, s);
#define VGF_CASE_C2CF(PP) case PP: return launch_c2c_fwd_p<VGF_T, PP>(variant, a, tw, s);
#define VGF_CASE_C2CI(PP) case PP: return launch_c2c_inv_p<VGF_T, PP>(variant, a, tw, s);
#define VGF_CASE_FUSED(PP) case PP: return launch_fused_p<VGF_T, PP>(variant, adjoint, in, out, g, spec, tw, s);

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
  hipError_t launch_c2c_fwd<T>(int P, int variant, const C2CFwdArgs<T>& a, const cplx<T>* tw,  \
                               hipStream_t s) {                                                 \
    switch (P) { VGF_FOR_EACH_P(VGF_CASE_C2CF) default: return hipErrorInvalidValue; }          \
  }                                                                                             \
  template <>                                                                                   \
  hipError_t launch_c2c_inv<T>(int P, int variant, const C2CInvArgs<T>& a, const cplx<T>* tw,  \
                               hipStream_t s) {                                                 \
    switch (P) { VGF_FOR_EACH_P(VGF_CASE_C2CI) default: return hipErrorInvalidValue; }          \
  }                                                                                             \
  template <>                                                                                   \
  hipError_t launch_fused<T>(int P, int variant, bool adjoint, const cplx<T>* in, cplx<T>* out, \
                             const FusedGeom<T>& g, const T* spec, const cplx<T>* tw,           \
                             hipStream_t s) {                                                   \
    switch (P) { VGF_FOR_EACH_P(VGF_CASE_FUSED) default: return hipErrorInvalidValue; }         \
  }                                                                                             \
  template <>                                                                                   \
  hipError_t launch_r2c_s<T>(int P, int variant, const R2CSArgs<T>& a, const cplx<T>* tw,      \
                             hipStream_t s) {                                                   \
    switch (P) { VGF_FOR_EACH_P(VGF_CASE_R2CS) VGF_FOR_EACH_P_WIDE(VGF_CASE_R2CS) default: return hipErrorInvalidValue; }          \
  }                                                                                             \
  template <>                                                                                   \
  hipError_t launch_c2r_s<T>(int P, int variant, const C2RSArgs<T>& a, const cplx<T>* tw,      \
                             hipStream_t s) {                                                   \
    switch (P) { VGF_FOR_EACH_P(VGF_CASE_C2RS) VGF_FOR_EACH_P_WIDE(VGF_CASE_C2RS) default: return hipErrorInvalidValue; }          \
  }                                                                                             \
  template <>                                                                                   \
  hipError_t launch_fused_c<T>(int P, int schedule, bool adjoint, const cplx<T>* in, cplx<T>* out,            \
                               const FusedCGeom<T>& g, const T* spec, const cplx<T>* tw,        \
                               hipStream_t s) {                                                 \
    switch (P) { VGF_FOR_EACH_P(VGF_CASE_FC) VGF_FOR_EACH_P_WIDE(VGF_CASE_FC) default: return hipErrorInvalidValue; }            \
  }                                                                                             \
  template <>                                                                                   \
  hipError_t launch_fused_cg<T>(int P, bool adjoint, const cplx<T>* in, cplx<T>* out,           \
                                const FusedCGeom<T>& g, const GradSpec<T>& sp,                  \
                                const cplx<T>* tw, hipStream_t s) {                             \
    switch (P) { VGF_FOR_EACH_P(VGF_CASE_FCG) VGF_FOR_EACH_P_WIDE(VGF_CASE_FCG) default: return hipErrorInvalidValue; }           \
  }                                                                                             \
  template <>                                                                                   \
  hipError_t launch_fused_grad<T>(int P, bool adjoint, const cplx<T>* in, cplx<T>* out,         \
                                  const FusedGeom<T>& g, const GradSpec<T>& sp,                 \
                                  const cplx<T>* tw, hipStream_t s) {                           \
    switch (P) { VGF_FOR_EACH_P(VGF_CASE_FGRAD) default: return hipErrorInvalidValue; }         \
  }

}  // namespace vgf
