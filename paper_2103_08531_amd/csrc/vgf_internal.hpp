// vgf_internal.hpp -- declarations shared by the host runtime and the kernel
// translation units of libvgf (not part of the public C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace vgf {

template <typename T> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };
template <typename T> using cplx = typename cplx_of<T>::type;

// FFT lengths P = 2N the library instantiates: every P = 2^a 3^b with a >= 2
// (N = P/2 even) from 16 to 1024, i.e. N = 2^a 3^b, a >= 1, 8 <= N <= 512.
// The kernels of each length are compiled in one of four groups.
#define VGF_P_GROUP1(X) X(16) X(24) X(32) X(36) X(48) X(64) X(72)
#define VGF_P_GROUP2(X) X(96) X(108) X(128) X(144) X(192) X(216)
#define VGF_P_GROUP3(X) X(256) X(288) X(324) X(384) X(432)
#define VGF_P_GROUP4(X) X(512) X(576) X(648) X(768) X(864) X(972) X(1024)
#define VGF_FOR_EACH_P(X) VGF_P_GROUP1(X) VGF_P_GROUP2(X) VGF_P_GROUP3(X) VGF_P_GROUP4(X)

inline bool supported_fft_len(int64_t P) {
#define VGF_CASE_LEN(PP) case PP:
  switch (P) {
    VGF_FOR_EACH_P(VGF_CASE_LEN)
    return true;
    default:
      return false;
  }
#undef VGF_CASE_LEN
}

// Longer lengths, P = 2^a 3^b from 1152 to 2048 (N = 576 .. 1024), for the
// passes of 2D grids in the default layout only: the axis-0 R2C and C2R and
// the multiply pass along the contiguous axis. Two more compile groups.
#define VGF_P_GROUP5(X) X(1152) X(1296) X(1536)
#define VGF_P_GROUP6(X) X(1728) X(1944) X(2048)
#define VGF_FOR_EACH_P_WIDE(X) VGF_P_GROUP5(X) VGF_P_GROUP6(X)

inline bool supported_fft_len_wide(int64_t P) {
#define VGF_CASE_LEN(PP) case PP:
  switch (P) {
    VGF_FOR_EACH_P_WIDE(VGF_CASE_LEN)
    return true;
    default:
      return false;
  }
#undef VGF_CASE_LEN
}

// Geometry of a batch of lines along a strided axis: element pos of
// column col (contiguous), batch b of entry e is at
// base + e*es + b*bs + pos*ls + col. The launch covers nbatch x nentry
// batches (entries: independent right-hand sides of one plan whose
// workspaces sit es elements apart).
struct StridedGeom {
  int64_t ncols;
  int64_t ls_in, ls_out;
  int64_t bs_in, bs_out;
  int nbatch;
  int nentry = 1;
  int64_t es_in = 0, es_out = 0;
  // non-temporal loads of the input / stores of the outputs (large arrays)
  bool nt_load = false, nt_store = false;
  // inverse passes: log2 of the block width B of a tiled input (0: rows of
  // ls_in elements). Tiled, column c of transform row k sits at
  // (c >> log2 B) * P * B + k * B + (c mod B): the B columns of a workgroup's
  // tile are one contiguous block of P rows.
  int in_tile = 0;
};

// Spectral derivative factors along the transformed axis. A forward pass
// sums up to two inputs, each multiplied after its transform; an inverse
// pass expands one input into up to two outputs, each multiplied before its
// transform. code 0: factor 1; -1: factor -i k; +1: factor +i k, where
// k = ks * s and s is the signed frequency of the position on the 2N axis
// (the Nyquist index gets s = 0).
template <typename T> struct Deriv {
  int n;
  int code[2];
  T ks;
};

// Contiguous-axis passes. nlines = lines of all entries; entry e owns lines
// [e*lpe, (e+1)*lpe) (lpe even, so a line pair never straddles entries).
// A user array of entry e is in[t] (one entry) or in_tab[t][e] + in_off[t]
// (device table of per-entry base pointers, several entries); workspace
// arrays of entry e sit e*es elements from the first.
template <typename T> struct R2CArgs {
  const T* in[2];
  cplx<T>* out;    // lines of N+1 values at stride hs
  int64_t nlines;
  int64_t hs;
  Deriv<T> d;
  int64_t lpe = 0;
  const T* const* in_tab[2] = {nullptr, nullptr};
  int64_t in_off[2] = {0, 0};
  int64_t out_es = 0;
};

template <typename T> struct C2RArgs {
  const cplx<T>* in;  // lines of N+1 values at stride hs
  T* out[2];
  int64_t nlines;
  int64_t hs;
  Deriv<T> d;
  int64_t lpe = 0;
  T* const* out_tab[2] = {nullptr, nullptr};
  int64_t out_off[2] = {0, 0};
  int64_t in_es = 0;
};

template <typename T> struct C2CFwdArgs {
  const cplx<T>* in[2];
  cplx<T>* out;
  StridedGeom g;
  Deriv<T> d;
};

template <typename T> struct C2CInvArgs {
  const cplx<T>* in;
  cplx<T>* out[2];
  StridedGeom g;
  Deriv<T> d;
  // optional (with d.n == 2): a second input of the same layout, transformed
  // without a factor into out2 by the same launch
  const cplx<T>* in2 = nullptr;
  cplx<T>* out2 = nullptr;
};

// Geometry of the axis-0 (outermost) fused pass. Forward: one input, outputs
// fields[f] in {0: times the kernel spectrum, 1: times -i k_0 and the kernel
// spectrum}, at out + f*out_fs; fields must be {0} or {0, 1}. Adjoint: inputs
// fields[f] at in + f*in_fs, summed with the conjugate factors, one output.
template <typename T> struct FusedGeom {
  int64_t ncols;     // columns of the inner plane: P1*hs (3D) or hs (2D)
  int64_t out_fs;
  int64_t in_fs;
  int dim;
  int n0, n1, n2;    // points per axis (n2 unused in 2D)
  int h_last;        // N_last + 1 (valid values along the last axis)
  int hs;            // padded stride of the last axis (>= h_last)
  T ks0;             // 2 pi / (P_0 h_0)
  int nf;
  int fields[4];
  int nentry = 1;    // entries (right-hand sides) of the launch
  int64_t in_es = 0, out_es = 0;  // element strides between entries
};

template <typename T>
hipError_t launch_r2c(int P, const R2CArgs<T>& a, const cplx<T>* tw, hipStream_t s);
template <typename T>
hipError_t launch_c2r(int P, const C2RArgs<T>& a, const cplx<T>* tw, hipStream_t s);
// Number of tile-schedule variants of the strided passes (see TileV).
constexpr int kTileVariantsHost = 2;

// Largest LDS tile (bytes) of the default layout's strided passes; their
// default tile is one 128-byte row segment wide wherever that fits in this
// and in 1024 threads (8 values per thread), else narrower.
#ifndef VGF_STRIDED_LDS
#define VGF_STRIDED_LDS 131072
#endif
constexpr int strided_tile_width(int P, int value_bytes) {
  int nl = 128 / (2 * value_bytes);
  const int nq = (P + 7) / 8;
  while (nl > 1 && (P * nl * 2 * value_bytes > VGF_STRIDED_LDS || nl * nq > 1024)) nl /= 2;
  return nl;
}
// The strided passes take a tile-schedule variant (0 or 1, see TileV):
// every variant computes identical results; only the launch shape differs.
template <typename T>
hipError_t launch_c2c_fwd(int P, int variant, const C2CFwdArgs<T>& a, const cplx<T>* tw, hipStream_t s);
template <typename T>
hipError_t launch_c2c_inv(int P, int variant, const C2CInvArgs<T>& a, const cplx<T>* tw, hipStream_t s);
template <typename T>
hipError_t launch_fused(int P, int variant, bool adjoint, const cplx<T>* in, cplx<T>* out,
                        const FusedGeom<T>& g, const T* spec, const cplx<T>* tw, hipStream_t s);

// ---- solve layout with the multiply pass along the contiguous axis ----
// Axis-0 transforms of real data: two adjacent real columns travel as one
// complex column. Real input / output arrays are [N0][ncols] (ncols even);
// the half spectrum is [N0 + 1][ncols] complex. Entry e (blockIdx.y) uses the
// pointer tables when given, else the direct pointers; workspace arrays of
// entry e sit e * es elements from the first.
template <typename T> struct R2CSArgs {
  const T* in[2];
  const T* const* in_tab[2];
  int64_t in_off[2];
  cplx<T>* out;
  int64_t out_es;
  int64_t ncols;  // real columns per row
  int nentry;
  Deriv<T> d;     // per input term: factor applied after its transform
  bool nt_load = false;  // non-temporal loads of the inputs (large arrays)
};
template <typename T> struct C2RSArgs {
  const cplx<T>* in;
  int64_t in_es;
  T* out[4];
  T* const* out_tab[4];
  int64_t out_off[4];
  int64_t ncols;
  int nentry;
  Deriv<T> d;     // outputs 0 .. d.n-1 from `in`, each with its factor
  // outputs d.n .. d.n+nx-1 from in_x[0 .. nx), without a factor, in the
  // same launch (inputs laid out like `in`)
  const cplx<T>* in_x[3];
  int nx;
  // non-temporal loads of the in_x inputs (read once; keeps `in`, which the
  // second output of `in` reads again, in the caches)
  bool nt_x = false;
};
// Lines along the contiguous last axis (length n_last in, 2 n_last transformed)
// of the arrays [H0][P1][n_last] (3D) or [H0][n_last] (2D), H0 = n0 + 1; line
// (k0, k1) multiplies by the kernel-spectrum octant row (k0, fold(k1)).
template <typename T> struct FusedCGeom {
  int dim;
  int n0, n1, n_last;
  int64_t lpe;        // lines per entry: H0 * P1 (3D) or H0 (2D)
  int64_t nlines;     // lines of all entries
  int64_t in_es, out_es;
  int64_t fs;         // field stride (elements): output fields (forward), input fields (adjoint)
  T ks;               // 2 pi / (P_last h_last)
  int nf;             // forward: 1 (phi) or 2 (phi, E_last); adjoint: inputs
  int fields[4];      // adjoint: per input 0 or 1 (+i k_last); gradient kernels: 0 .. dim
                      // (the multipliers of GradSpec), up to four fields
  bool nt = false;    // forward: non-temporal loads and stores (large arrays)
  // 3D (forward and adjoint): log2 of the block width B of the tiled output
  // layout read by the axis-1 inverse (StridedGeom::in_tile), 0 for plain rows. Tiled,
  // output x_last of line (k0, k1) sits at
  // k0 P1 n_last + (x_last >> log2 B) P1 B + k1 B + (x_last mod B);
  // n_last and the last inverse stage's butterfly count are multiples of B.
  int ytile = 0;
};
template <typename T>
hipError_t launch_r2c_s(int P, int variant, const R2CSArgs<T>& a, const cplx<T>* tw, hipStream_t s);
template <typename T>
hipError_t launch_c2r_s(int P, int variant, const C2RSArgs<T>& a, const cplx<T>* tw, hipStream_t s);
// schedule (0..3) of the multiply pass: bit 0 halves the lanes per line,
// bit 1 lengthens each wavefront's walk over lines; results do not depend on it
template <typename T>
hipError_t launch_fused_c(int P, int schedule, bool adjoint, const cplx<T>* in, cplx<T>* out,
                          const FusedCGeom<T>& g, const T* spec, const cplx<T>* tw, hipStream_t s);

// Spectra of the gradient-kernel fields: s[0] the kernel spectrum octant,
// s[1 + a] the octant of T_a (the 2N spectrum of the odd gradient kernel of
// axis a is -i T_a), all in plan precision, divided by prod_a P_a. A fused
// launch in this mode takes fields f in {0, 1, .., dim}: 0 multiplies by
// s[0], 1 + a by -i T_a (the adjoint by the conjugates).
template <typename T> struct GradSpec {
  const T* s[4];
};
template <typename T>
hipError_t launch_fused_grad(int P, bool adjoint, const cplx<T>* in, cplx<T>* out, const FusedGeom<T>& g,
                             const GradSpec<T>& sp, const cplx<T>* tw, hipStream_t s);
// The same multipliers in the multiply pass along the contiguous axis
// (FusedCGeom lines; forward: g.nf outputs at out + i * fs for the fields
// g.fields[i]; adjoint: g.nf inputs at in + i * fs summed into one output).
template <typename T>
hipError_t launch_fused_cg(int P, bool adjoint, const cplx<T>* in, cplx<T>* out, const FusedCGeom<T>& g,
                           const GradSpec<T>& sp, const cplx<T>* tw, hipStream_t s);

// ---- finite-difference field (second order; centred inside, one-sided at
// the two end planes of each axis) ----
struct FdGeom {
  int dim;
  int n[3];
  int64_t stride[3];  // element stride of each axis
  int64_t total;
  double inv2h[3];    // 1 / (2 h_a)
};
// E[a] = -(D_a phi), E planar [dim][total]
template <typename T>
hipError_t launch_fd_field(const T* phi, T* E, const FdGeom& g, hipStream_t s);
// the same for the nentry entries of a batch group (blockIdx.y): phi of
// entry e is phi_tab[e], its field E_tab[e] (device pointer tables)
template <typename T>
hipError_t launch_fd_field_entries(const T* const* phi_tab, T* const* E_tab, int nentry, const FdGeom& g,
                                   hipStream_t s);
// out = g_phi - sum_a D_a^T g_E[a]  (g_phi may be null: zero)
template <typename T>
hipError_t launch_fd_adjoint(const T* g_phi, const T* g_E, T* out, const FdGeom& g, hipStream_t s);

// ---- batched solves ----
// Up to kMax device pointers, written to dst[0, n) by one small launch.
struct PtrChunk {
  static constexpr int kMax = 64;
  int n;
  void* p[kMax];
};
hipError_t launch_set_pointers(void** dst, const PtrChunk& c, hipStream_t s);

// ---- plan-time precompute (FP64) ----
// F{G^L}(|k_m|) on m in [0, ext_0) x [0, ext_1) (x [0, ext_2)),
// k_{m,a} = m_a * dk_a.
hipError_t launch_ghat(double* out, int dim, const int64_t* ext, const double* dk, double L,
                       hipStream_t s);
// HE kernel octant: vol * G(|n h|), origin value `origin`.
hipError_t launch_he_kernel(double* out, int dim, const int64_t* n, const double* h, double origin,
                            hipStream_t s);
// out[o][j][i] = sum_{m < M} mat[m*J + j] * in[(o*M + m)*inner + i]
hipError_t launch_axis_apply(const double* in, double* out, const double* mat, int64_t outer,
                             int M, int J, int64_t inner, hipStream_t s);
// out[i] = (T)(in[i] * scale)
template <typename T>
hipError_t launch_scale_convert(const double* in, T* out, int64_t count, double scale,
                                hipStream_t s);

}  // namespace vgf
