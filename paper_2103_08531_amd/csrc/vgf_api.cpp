// vgf_api.cpp -- host runtime behind the C ABI in include/vgf.h.
//
// A plan fixes the grid, the method (VGF or HE), the precision and the
// requested outputs. Plan creation runs the one-time FP64 precompute on the
// GPU (Sec. II of the paper: the windowed-kernel spectrum on the
// 4N-oversampled grid, its inverse DFT restricted to the 2N solve grid, and
// that kernel's 2N spectrum), then keeps only what solves need: the real,
// even kernel spectrum on its non-negative octant, pre-divided by the inverse
// FFT normalisation prod_a(2 N_a) and rounded once to the plan precision.
//
// Solve data flow, default layout (3D; axis 2 contiguous, P_a = 2 N_a,
// H0 = N_0 + 1):
//   rho [N0][N1][N2]  --r2c axis 0-->  X1 [H0][N1][N2]
//   X1                --c2c axis 1-->  X2 [H0][P1][N2]
//   X2  --axis 2 (fwd, x kernel, inv of phi and -i k_2 phi)-->  Y [H0][P1][N2] x2
//   Y                 --c2c^-1 axis 1--> Z: phi, E_1 (from phi), E_2 [H0][N1][N2]
//   Z                 --c2r axis 0-->  phi / E_a [N0][N1][N2]
// The axis-0 layout (gradient-kernel plans, VGF_LAYOUT_AXIS0) swaps the
// roles of axes 0 and 2: r2c/c2r along axis 2 (H = N_2 + 1 padded to Hs),
// the multiply pass along axis 0. 2D skips the middle-axis passes. All
// passes are asynchronous on the caller's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "vgf.h"
#include "vgf_fft.hpp"
#include "vgf_internal.hpp"

using vgf::cplx;

struct vgf_plan_s {
  int dim = 0;
  int64_t n[3] = {1, 1, 1};
  double h[3] = {1, 1, 1};
  int64_t P[3] = {1, 1, 1};
  int64_t H = 1;   // N_last + 1: values of a half-spectrum line
  int64_t Hs = 1;  // H padded to 128 bytes: row stride of the workspace arrays
  vgf_method method = VGF_METHOD_VGF;
  vgf_precision prec = VGF_F64;
  double L = 0.0;
  unsigned outputs = 0;
  int nf_max = 0;

  // device memory
  void* spec = nullptr;          // octant prod(n_a+1), plan type, scaled by 1/prod(P)
  double* w64 = nullptr;         // restricted kernel octant prod(n_a), FP64
  double* spec64 = nullptr;      // unscaled spectrum octant, FP64
  void* tw[3] = {nullptr, nullptr, nullptr};  // per-axis twiddles exp(-2 pi i e / P_a)
  void* ws = nullptr;            // solve workspace
  size_t off_x1 = 0, off_x2 = 0, off_y = 0, off_z = 0;
  size_t ws_bytes = 0;           // solve workspace (a multiple of 256 bytes)
  int schedule[5] = {0, 0, 0, 0, 0};  // tile variant per pass (VGF_PASS_* order)
  bool fd = false;               // E by finite differences of phi (VGF_FIELD_CENTERED)
  bool gradk = false;            // E by gradient kernels (VGF_FIELD_GRADIENT_KERNEL)
  bool contig = false;           // multiply pass along the contiguous axis (else along axis 0)
  double* wgrad64 = nullptr;     // [dim][prod(n)] gradient-kernel octants, FP64
  double* specg64 = nullptr;     // [dim][prod(n+1)] their spectra T_a, FP64, unscaled
  void* specg = nullptr;         // [dim][prod(n+1)] plan type, scaled by 1/prod(P)
  size_t off_phi = 0;            // real phi array in the workspace (fd only)
  int64_t stream_min = 0;        // input bytes per launch from which solves stream (stream_min_env)
  bool tile_y = true;            // 3D default layout: tiled hand-off to the axis-1 inverse (tile_y_env)
  size_t bytes = 0;
  hipError_t last_err = hipSuccess;

  // per-pass timing (vgf_plan_profile_begin / _end)
  bool profiling = false;
  int prof_cap = 0, prof_used = 0, prof_nlaunch = 0;
  std::vector<hipEvent_t> prof_events;  // prof_cap x kMaxMarks
  std::vector<int> prof_tags;           // pass of each launch, prof_cap x kMaxMarks
};

// Workspace of the allocation-free solve (vgf_solve_noalloc): a file-scope
// device array, so every device the library runs on holds its own copy until
// the process ends. In host code this name only stands for the symbol; the
// device address comes from hipGetSymbolAddress, once per device
// (scratch_address), and is what kernels and copies receive. Every pass of a
// solve writes what the next one reads, so nothing in it has to start at
// zero; it keeps the last call's contents.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr long double kPiL = 3.14159265358979323846264338327950288L;

constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on the current device, looked up on the first
// call per device (plan creation does it, so a later solve only reads it).
hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// n points along an axis: every even n = 2^a 3^b from 8 to 512; 2D plans in
// the default layout also take 576 .. 1024 (the longer lengths are built for
// their passes only)
bool size_supported(int64_t n, bool wide) {
  return n >= 8 && (vgf::supported_fft_len(2 * n) || (wide && vgf::supported_fft_len_wide(2 * n)));
}

double he_origin(int dim, const double* h, vgf_method m);

int64_t prod(const int64_t* v, int d) {
  int64_t p = 1;
  for (int a = 0; a < d; ++a) p *= v[a];
  return p;
}

// cos / sin of 2 pi t / n, argument reduced exactly in integers and the
// function evaluated in long double, then rounded once.
void cis(int64_t t, int64_t n, long double* c, long double* s) {
  t %= n;
  if (t < 0) t += n;
  const long double ang = 2.0L * kPiL * (long double)t / (long double)n;
  *c = cosl(ang);
  *s = sinl(ang);
}

// cis(t, n) for every residue t mod n, evaluated once (the cosine tables of
// the precompute index it with products m * j)
struct CisTable {
  std::vector<long double> c, s;
  int64_t n;
  explicit CisTable(int64_t n_) : c((size_t)n_), s((size_t)n_), n(n_) {
    for (int64_t t = 0; t < n; ++t) cis(t, n, &c[(size_t)t], &s[(size_t)t]);
  }
  void at(int64_t t, long double* cc, long double* ss) const {
    t %= n;
    if (t < 0) t += n;
    *cc = c[(size_t)t];
    *ss = s[(size_t)t];
  }
};

// Stage-major twiddle tables of one axis of length P, the forward radix
// order at [0, P) and the inverse order at [P, 2P) (equal when the order is
// a palindrome). Stage s (Ns > 1, radix R) keeps the R - 1 slots of
// butterfly m < Ns at (Ns - R_0) + k Ns + m. A plain slot k holds
// w_r = cos th_r - i sin th_r, th_r = 2 pi r m / (Ns R), r = k + 1 (the
// forward sign; the inverse conjugates). Stages in scaled form
// (vgf::stage_scaled: radix 8 and 4 with 3 not dividing Ns) hold tangents,
// cosine ratios and cosines (slot layout at vgf::dft8_tw / vgf::dft4_tw).
// Every value is evaluated in long double from exactly reduced angles and
// rounded once. Returns false if a divisor would vanish (it cannot for the
// stages that use the scaled form).
template <typename T> bool make_stage_twiddles(int P, std::vector<cplx<T>>& out) {
  out.assign((size_t)2 * P, cplx<T>{T(0), T(0)});
  auto put = [&](size_t i, long double x, long double y) {
    out[i].x = (T)x;
    out[i].y = (T)y;
  };
  for (int dir = 0; dir < 2; ++dir) {
    const int nst = vgf::n_stages(P);
    auto radix = [&](int st) { return dir == 0 ? vgf::fwd_radix(P, st) : vgf::fwd_radix(P, nst - 1 - st); };
    const int R0 = radix(0);
    const size_t base = (size_t)dir * P;
    int ns = R0;
    for (int st = 1; st < nst; ++st) {
      const int R = radix(st);
      for (int m = 0; m < ns; ++m) {
        auto at = [&](int k) { return base + (size_t)(ns - R0) + (size_t)k * ns + (size_t)m; };
        long double c[8], sn[8];
        for (int r = 0; r < R; ++r) cis((int64_t)r * m, (int64_t)ns * R, &c[r], &sn[r]);
        if (vgf::stage_scaled(R, ns)) {
          const int nz[] = {1, 2, 3, 5, 6, 7};
          for (int r : nz)
            if (r < R && r != R / 2 && c[r] == 0.0L) return false;
          if (R == 8) {
            put(at(0), sn[1] / c[1], sn[2] / c[2]);
            put(at(1), sn[3] / c[3], sn[5] / c[5]);
            put(at(2), sn[6] / c[6], sn[7] / c[7]);
            put(at(3), c[4], -sn[4]);
            put(at(4), c[6] / c[2], c[5] / c[1]);
            put(at(5), c[7] / c[3], c[3] / c[1]);
            put(at(6), c[2], c[1]);
          } else {
            put(at(0), sn[1] / c[1], sn[3] / c[3]);
            put(at(1), c[2], -sn[2]);
            put(at(2), c[3] / c[1], c[1]);
          }
        } else {
          for (int r = 1; r < R; ++r) put(at(r - 1), c[r], -sn[r]);
        }
      }
      ns *= R;
    }
  }
  return true;
}

// Input bytes (rho of all entries of a launch) from which the forward solve
// uses non-temporal loads and stores in its middle passes: the arrays are
// then several times the caches. Read once per plan.
int64_t stream_min_env() {
  constexpr int64_t kDefault = (int64_t)32 << 20;
  const char* e = std::getenv("VGF_STREAM_MIN_BYTES");
  if (!e || !*e) return kDefault;
  char* end = nullptr;
  const long long v = std::strtoll(e, &end, 10);
  if (end == e) return kDefault;  // not a number
  return v < 0 ? 0 : (int64_t)v;
}

// VGF_TILED_Y=0 keeps the multiply pass's output in plain rows (the tiled
// hand-off to the axis-1 inverse is the default). Read once per plan.
bool tile_y_env() {
  const char* e = std::getenv("VGF_TILED_Y");
  return !(e && e[0] == '0' && e[1] == 0);
}

// log2 of the block width B of the tiled hand-off from the multiply pass to
// the axis-1 inverse (3D, default layout), 0 where it is not used. B is the
// inverse's default tile width (strided_tile_width), so each of its
// workgroups reads one contiguous block; n_last and the butterfly count of
// the last inverse stage along the last axis must be multiples of B.
template <typename T> int y_tile_log2(vgf_plan p) {
  if (!p->tile_y || p->dim != 3) return 0;
  const int64_t P1 = p->P[1], P2 = p->P[2], N2 = p->n[2];
  const int b = vgf::strided_tile_width((int)P1, (int)sizeof(T));
  const int64_t nb_last = P2 / vgf::fwd_radix((int)P2, 0);
  if (b < 2 || N2 % b != 0 || nb_last % b != 0) return 0;
  int sh = 0;
  while ((1 << sh) < b) ++sh;
  return sh;
}

size_t max_workspace_env() {
  const char* e = std::getenv("VGF_MAX_WORKSPACE");
  if (!e || !*e) return (size_t)-1;
  char* end = nullptr;
  unsigned long long v = std::strtoull(e, &end, 10);
  return (size_t)v;
}

struct DevFree {
  void operator()(void* p) const {
    if (p) (void)hipFree(p);
  }
};

void release(vgf_plan p) {
  if (!p) return;
  DevFree f;
  f(p->spec);
  f(p->w64);
  f(p->spec64);
  f(p->wgrad64);
  f(p->specg64);
  f(p->specg);
  for (int a = 0; a < 3; ++a) f(p->tw[a]);
  f(p->ws);
  for (hipEvent_t ev : p->prof_events) (void)hipEventDestroy(ev);
  delete p;
}

// Uploads an FP64 table and applies it along one axis:
// out[o][j][i] = sum_m mat[m*J + j] in[o][m][i]. Waits for the stream so
// the host table can be reused for the next axis.
hipError_t apply_axis(const std::vector<double>& host_mat, double* dmat, const double* in,
                      double* out, int64_t outer, int M, int J, int64_t inner, hipStream_t s) {
  hipError_t e = hipMemcpyAsync(dmat, host_mat.data(), sizeof(double) * host_mat.size(),
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = vgf::launch_axis_apply(in, out, dmat, outer, M, J, inner, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e;
}

// The one-time FP64 precompute. Fills p->w64 (kernel octant), p->spec64
// (spectrum octant) and p->spec (plan-precision scaled copy); temporaries
// are freed before returning.
vgf_status precompute(vgf_plan p, hipStream_t s) {
  const int d = p->dim;
  double *bufA = nullptr, *bufB = nullptr, *mat = nullptr;
  std::vector<double> host_mat;
  int64_t cur[3] = {1, 1, 1}, ext[3] = {1, 1, 1}, oct = 1, gsz = 1, maxmat = 0;
  double dk[3] = {0, 0, 0}, pp = 1.0;
  hipError_t err = hipSuccess;

  for (int a = 0; a < d; ++a) {
    ext[a] = 2 * p->n[a] + 1;
    oct *= p->n[a] + 1;
    pp *= (double)p->P[a];
    maxmat = std::max<int64_t>(maxmat, std::max(ext[a] * p->n[a], p->n[a] * (p->n[a] + 1)));
  }
  gsz = p->method == VGF_METHOD_VGF ? prod(ext, d) : oct;
  do {
    if ((err = hipMalloc(&bufA, sizeof(double) * (size_t)gsz)) != hipSuccess) break;
    if ((err = hipMalloc(&bufB, sizeof(double) * (size_t)gsz)) != hipSuccess) break;
    if ((err = hipMalloc(&mat, sizeof(double) * (size_t)maxmat)) != hipSuccess) break;

    // (i) spectrum samples on m in [0, 2N]^d of the 4N grid, k = 2 pi m / (4 N h)
    for (int a = 0; a < d; ++a)
      dk[a] = (double)(2.0L * kPiL / (4.0L * (long double)p->n[a] * (long double)p->h[a]));
    // (ii) inverse DFT over the 4N grid restricted to n_a in [0, N_a), one
    // axis at a time. Even axes:
    //  out[j] = (4N)^{-1} (f(0) + 2 sum_{0<m<2N} f(m) cos(2 pi m j / 4N) + f(2N) cos(pi j));
    // the odd axis of a gradient kernel (-i k_a times the spectrum; pairing
    // m with -m leaves a sine, the m = 0 and m = -2N terms vanish):
    //  out[j] = (4N)^{-1} 2 sum_{0<m<2N} k_m f(m) sin(2 pi m j / 4N).
    auto restricted = [&](double* target, int odd_axis) -> hipError_t {
      hipError_t e = vgf::launch_ghat(bufA, d, ext, dk, p->L, s);
      for (int a = 0; a < d; ++a) cur[a] = ext[a];
      double *src = bufA, *dst = bufB;
      for (int a = 0; a < d && e == hipSuccess; ++a) {
        const int64_t N = p->n[a], M4 = 4 * p->n[a], Mi = ext[a];
        host_mat.assign((size_t)(Mi * N), 0.0);
        const CisTable ct(M4);
        for (int64_t m = 0; m < Mi; ++m)
          for (int64_t j = 0; j < N; ++j) {
            long double c, sn;
            ct.at(m * j, &c, &sn);
            if (a == odd_axis) {
              const long double km = 2.0L * kPiL * (long double)m / ((long double)M4 * (long double)p->h[a]);
              host_mat[(size_t)(m * N + j)] =
                  (m == 0 || m == 2 * N) ? 0.0 : (double)(2.0L * km * sn / (long double)M4);
            } else {
              const long double wgt = (m == 0 || m == 2 * N) ? 1.0L : 2.0L;
              host_mat[(size_t)(m * N + j)] = (double)(wgt * c / (long double)M4);
            }
          }
        int64_t outer = 1, inner = 1;
        for (int b = 0; b < a; ++b) outer *= cur[b];
        for (int b = a + 1; b < d; ++b) inner *= cur[b];
        double* tgt = (a == d - 1) ? target : dst;
        e = apply_axis(host_mat, mat, src, tgt, outer, (int)Mi, (int)N, inner, s);
        cur[a] = N;
        std::swap(src, dst);
      }
      return e;
    };
    // (iii) spectrum of the 2N-periodic kernel (zero where |n_a| = N_a), on
    // k in [0, N]: even axes S[k] = w[0] + 2 sum_{0<n<N} w[n] cos(2 pi n k / 2N);
    // the odd axis of a gradient kernel gives -i T with
    // T[k] = 2 sum_{0<n<N} w[n] sin(2 pi n k / 2N).
    auto spectrum = [&](const double* from, double* target, int odd_axis) -> hipError_t {
      hipError_t e = hipSuccess;
      for (int a = 0; a < d; ++a) cur[a] = p->n[a];
      double* tmp[2] = {bufA, bufB};
      for (int a = 0; a < d && e == hipSuccess; ++a) {
        const int64_t N = p->n[a], P2 = 2 * p->n[a];
        host_mat.assign((size_t)(N * (N + 1)), 0.0);
        const CisTable ct(P2);
        for (int64_t m = 0; m < N; ++m)
          for (int64_t k = 0; k <= N; ++k) {
            long double c, sn;
            ct.at(m * k, &c, &sn);
            host_mat[(size_t)(m * (N + 1) + k)] =
                a == odd_axis ? (m == 0 ? 0.0 : (double)(2.0L * sn)) : (double)((m == 0 ? 1.0L : 2.0L) * c);
          }
        int64_t outer = 1, inner = 1;
        for (int b = 0; b < a; ++b) outer *= cur[b];
        for (int b = a + 1; b < d; ++b) inner *= cur[b];
        double* tgt = (a == d - 1) ? target : tmp[a % 2];
        e = apply_axis(host_mat, mat, from, tgt, outer, (int)N, (int)(N + 1), inner, s);
        cur[a] = N + 1;
        from = tgt;
      }
      return e;
    };

    if (p->method == VGF_METHOD_VGF) {
      if ((err = restricted(p->w64, -1)) != hipSuccess) break;
    } else {
      if ((err = vgf::launch_he_kernel(p->w64, d, p->n, p->h, he_origin(d, p->h, p->method), s)) !=
          hipSuccess)
        break;
    }
    if ((err = spectrum(p->w64, p->spec64, -1)) != hipSuccess) break;
    if (p->gradk) {
      const int64_t vol = prod(p->n, d);
      for (int ax = 0; ax < d && err == hipSuccess; ++ax) {
        if ((err = restricted(p->wgrad64 + ax * vol, ax)) != hipSuccess) break;
        if ((err = spectrum(p->wgrad64 + ax * vol, p->specg64 + ax * oct, ax)) != hipSuccess) break;
        if (p->prec == VGF_F32)
          err = vgf::launch_scale_convert<float>(p->specg64 + ax * oct, (float*)p->specg + ax * oct, oct,
                                                 1.0 / pp, s);
        else
          err = vgf::launch_scale_convert<double>(p->specg64 + ax * oct, (double*)p->specg + ax * oct, oct,
                                                  1.0 / pp, s);
      }
      if (err != hipSuccess) break;
    }

    // plan-precision copy, divided by the inverse FFT normalisation
    if (p->prec == VGF_F32)
      err = vgf::launch_scale_convert<float>(p->spec64, (float*)p->spec, oct, 1.0 / pp, s);
    else
      err = vgf::launch_scale_convert<double>(p->spec64, (double*)p->spec, oct, 1.0 / pp, s);
    if (err != hipSuccess) break;
    err = hipStreamSynchronize(s);
  } while (false);

  (void)hipStreamSynchronize(s);
  (void)hipFree(bufA);
  (void)hipFree(bufB);
  (void)hipFree(mat);
  if (err == hipSuccess) return VGF_OK;
  p->last_err = err;
  return err == hipErrorOutOfMemory ? VGF_ERR_OUT_OF_MEMORY : VGF_ERR_HIP;
}

vgf_status hip_status(vgf_plan p, hipError_t e) {
  if (e == hipSuccess) return VGF_OK;
  p->last_err = e;
  return VGF_ERR_HIP;
}

constexpr int kMaxLaunches = 16;           // per solve, as reported by profiling
constexpr int kMaxMarks = kMaxLaunches + 1;  // an event at the start and after every launch
constexpr int vgf_tile_variants() { return vgf::kTileVariantsHost; }

// Records an event at the start of a solve and after each of its launches,
// tagged with the launch's pass: into the plan's profiling slots when the
// plan is profiling, or into caller-given arrays (tuning).
struct Marks {
  vgf_plan p;
  hipStream_t s;
  hipEvent_t* ev = nullptr;
  int* tags = nullptr;
  bool own = false;  // plan profiling slot
  int n = 0;
  Marks(vgf_plan p_, hipStream_t s_, bool on, hipEvent_t* given, int* given_tags) : p(p_), s(s_) {
    if (given) {
      ev = given;
      tags = given_tags;
    } else if (on && p->profiling && p->prof_used < p->prof_cap) {
      ev = &p->prof_events[(size_t)p->prof_used * kMaxMarks];
      tags = &p->prof_tags[(size_t)p->prof_used * kMaxMarks];
      ++p->prof_used;
      own = true;
    }
    if (ev) {
      (void)hipEventRecord(ev[0], s);
      n = 1;
    }
  }
  void mark(int pass) {
    if (ev && n < kMaxMarks) {
      tags[n - 1] = pass;
      (void)hipEventRecord(ev[n++], s);
    }
  }
  ~Marks() {
    if (own) p->prof_nlaunch = n - 1;
  }
};

// Origin weight w[0] of the Hockney-Eastwood kernels (w[n] = vol G(|n h|)
// elsewhere; Sec. I and the legends of the comparison figures, Sec. III.A):
//   HE         the singular factor (1/r, -ln r) replaced by 1: vol * G0;
//   HE_NEARBY  vol * G(r0), r0 = half the smallest spacing;
//   HE_CELLAVG the integral of G over the cell prod_a [-h_a/2, h_a/2], in
//              closed form: with (a, b, c) the half-widths and d the corner
//              distance, 8 x the corner-box integral of 1/r,
//                ab ln((c+d)/|(a,b)|) + bc ln((a+d)/|(b,c)|) + ca ln((b+d)/|(c,a)|)
//                - a^2/2 atan(bc/(ad)) - b^2/2 atan(ca/(bd)) - c^2/2 atan(ab/(cd)),
//              over 4 pi (3D); in 2D -4/(2 pi) x the corner integral of ln r,
//                (ab ln(a^2+b^2) - 3ab + a^2 atan(b/a) + b^2 atan(a/b)) / 2.
double he_origin(int dim, const double* h, vgf_method m) {
  long double vol = 1.0L, hmin = h[0];
  for (int a = 0; a < dim; ++a) {
    vol *= (long double)h[a];
    hmin = std::min(hmin, (long double)h[a]);
  }
  if (m == VGF_METHOD_HE_NEARBY) {
    const long double r0 = 0.5L * hmin;
    return (double)(vol * (dim == 3 ? 1.0L / (4.0L * kPiL * r0) : -logl(r0) / (2.0L * kPiL)));
  }
  if (m == VGF_METHOD_HE_CELLAVG) {
    if (dim == 3) {
      const long double a = 0.5L * h[0], b = 0.5L * h[1], c = 0.5L * h[2];
      const long double dd = sqrtl(a * a + b * b + c * c);
      const long double I = a * b * logl((c + dd) / sqrtl(a * a + b * b)) +
                            b * c * logl((a + dd) / sqrtl(b * b + c * c)) +
                            c * a * logl((b + dd) / sqrtl(c * c + a * a)) -
                            0.5L * a * a * atanl(b * c / (a * dd)) - 0.5L * b * b * atanl(c * a / (b * dd)) -
                            0.5L * c * c * atanl(a * b / (c * dd));
      return (double)(8.0L * I / (4.0L * kPiL));
    }
    const long double a = 0.5L * h[0], b = 0.5L * h[1];
    const long double J = 0.5L * (a * b * logl(a * a + b * b) - 3.0L * a * b + a * a * atanl(b / a) +
                                  b * b * atanl(a / b));
    return (double)(-4.0L * J / (2.0L * kPiL));
  }
  return (double)(vol * (dim == 3 ? 1.0L / (4.0L * kPiL) : 1.0L / (2.0L * kPiL)));
}

// 2 pi / (P_a h_a): wavenumber of one frequency step along axis a
double wavenumber_step(vgf_plan p, int a) {
  return (double)(2.0L * kPiL / ((long double)p->P[a] * (long double)p->h[a]));
}

template <typename T> struct Bufs {
  cplx<T>* x1;
  cplx<T>* x2;
  cplx<T>* y;
  cplx<T>* z;
};

template <typename T> Bufs<T> bufs(vgf_plan p) {
  char* base = (char*)p->ws;
  return Bufs<T>{(cplx<T>*)(base + p->off_x1), (cplx<T>*)(base + p->off_x2),
                 (cplx<T>*)(base + p->off_y), (cplx<T>*)(base + p->off_z)};
}

template <typename T> vgf::FusedGeom<T> fused_geom(vgf_plan p) {
  vgf::FusedGeom<T> g{};
  const int d = p->dim;
  g.dim = d;
  g.n0 = (int)p->n[0];
  g.n1 = (int)p->n[1];
  g.n2 = d == 3 ? (int)p->n[2] : 0;
  g.h_last = (int)p->H;
  g.hs = (int)p->Hs;
  g.ncols = d == 3 ? p->P[1] * p->Hs : p->Hs;
  g.ks0 = (T)wavenumber_step(p, 0);
  return g;
}

template <typename T> vgf::Deriv<T> deriv1(vgf_plan p, int axis, int code) {
  vgf::Deriv<T> d{};
  d.n = 1;
  d.code[0] = code;
  d.ks = (T)wavenumber_step(p, axis);
  return d;
}

template <typename T> vgf::Deriv<T> deriv2(vgf_plan p, int axis, int code0, int code1) {
  vgf::Deriv<T> d = deriv1<T>(p, axis, code0);
  d.n = 2;
  d.code[1] = code1;
  return d;
}

#define VGF_RUN(expr)                                  \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_status(p, e_);    \
  } while (0)

// a launch of pass `pass` inside a solve: run, check, mark its end
#define VGF_LAUNCH(pass, expr)                         \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return hip_status(p, e_);    \
    mk.mark(pass);                                     \
  } while (0)

// The arrays of the entries (right-hand sides of one plan) that one launch
// of each pass covers. One entry: direct pointers and the plan workspace.
// Several: device tables of per-entry base pointers (rho, phi, E) and
// workspaces es elements apart.
template <typename T> struct Entries {
  int count = 1;
  char* ws = nullptr;
  int64_t es = 0;  // cplx<T> elements between the workspaces of two entries
  const T* rho = nullptr;
  T* phi = nullptr;
  T* E = nullptr;
  const T* const* rho_tab = nullptr;
  T* const* phi_tab = nullptr;
  T* const* E_tab = nullptr;
  bool want_phi = false, want_E = false;
};

// output o of a c2r launch: phi (field < 0) or E_field
template <typename T>
void c2r_out(vgf::C2RArgs<T>& ca, int o, const Entries<T>& en, int field, int64_t vol) {
  if (!en.phi_tab && !en.E_tab) {
    ca.out[o] = field < 0 ? en.phi : en.E + field * vol;
  } else {
    ca.out[o] = nullptr;
    ca.out_tab[o] = field < 0 ? en.phi_tab : en.E_tab;
    ca.out_off[o] = field < 0 ? 0 : field * vol;
  }
}

// Forward solve. Each pass applies the derivative factor of its own axis:
// the axis-0 pass yields the spectra of phi (Yp) and E_0 (Y0); the last
// two axes derive E_1 and E_2 from phi's spectrum as they invert.
// pass ids (also the order of plan->schedule)
enum { kPassR2C = 0, kPassC2CF = 1, kPassFused = 2, kPassC2CI = 3, kPassC2R = 4, kPasses = 5 };

// Tile variant of a pass's launch under a schedule value: bit 0 selects the
// variant of the pass's first launch, bit 1 that of its later launches (the
// passes that launch more than once start with the launch that forms two
// outputs from phi's spectrum).
inline int launch_variant(const int* sched, int pass, int idx) { return (sched[pass] >> (idx > 0 ? 1 : 0)) & 1; }
constexpr int kScheduleValues = 4;

template <typename T>
vgf::GradSpec<T> grad_spec(vgf_plan p) {
  vgf::GradSpec<T> sp{};
  int64_t oct = 1;
  for (int a = 0; a < p->dim; ++a) oct *= p->n[a] + 1;
  sp.s[0] = (const T*)p->spec;
  for (int a = 0; a < p->dim; ++a) sp.s[1 + a] = (const T*)p->specg + a * oct;
  return sp;
}

// Forward solve with gradient kernels: no derivative factors after the
// axis-0 pass, which multiplies each requested field by its own spectrum;
// every field is then inverted on its own. Each launch covers all entries.
template <typename T>
vgf_status enqueue_solve_grad(vgf_plan p, const Entries<T>& en, hipStream_t s, bool marks, const int* sched,
                              hipEvent_t* mark_events, int* mark_tags) {
  const int d = p->dim;
  const int64_t N0 = p->n[0], N1 = p->n[1], H = p->H, Hs = p->Hs;
  const int64_t vol = prod(p->n, d);
  char* base = en.ws;
  Bufs<T> b{(cplx<T>*)(base + p->off_x1), (cplx<T>*)(base + p->off_x2), (cplx<T>*)(base + p->off_y),
            (cplx<T>*)(base + p->off_z)};
  auto tw = [&](int a) { return (const cplx<T>*)p->tw[a]; };
  vgf::FusedGeom<T> g = fused_geom<T>(p);
  g.nf = 0;
  if (en.want_phi) g.fields[g.nf++] = 0;
  if (en.want_E)
    for (int a = 0; a < d; ++a) g.fields[g.nf++] = 1 + a;
  g.nentry = en.count;
  g.in_es = g.out_es = en.es;
  Marks mk(p, s, marks, mark_events, mark_tags);
  const int64_t lpe = d == 3 ? N0 * N1 : N0;  // contiguous lines per entry
  vgf::R2CArgs<T> ra{};
  ra.nlines = lpe * en.count;
  ra.lpe = lpe;
  ra.hs = Hs;
  ra.out = b.x1;
  ra.out_es = en.es;
  ra.d = deriv1<T>(p, d - 1, 0);
  if (en.rho_tab) ra.in_tab[0] = en.rho_tab;
  else ra.in[0] = en.rho;
  VGF_LAUNCH(kPassR2C, vgf::launch_r2c<T>((int)p->P[d - 1], ra, tw(d - 1), s));
  const cplx<T>* fused_in = b.x1;
  if (d == 3) {
    const int64_t P1 = p->P[1];
    vgf::StridedGeom fg{H, Hs, Hs, N1 * Hs, P1 * Hs, (int)N0};
    fg.nentry = en.count;
    fg.es_in = fg.es_out = en.es;
    vgf::C2CFwdArgs<T> fa{{b.x1, nullptr}, b.x2, fg, deriv1<T>(p, 1, 0)};
    VGF_LAUNCH(kPassC2CF, vgf::launch_c2c_fwd<T>((int)P1, launch_variant(sched, kPassC2CF, 0), fa, tw(1), s));
    fused_in = b.x2;
    g.out_fs = N0 * P1 * Hs;
  } else {
    g.out_fs = N0 * Hs;
  }
  VGF_LAUNCH(kPassFused, vgf::launch_fused_grad<T>((int)p->P[0], false, fused_in, b.y, g, grad_spec<T>(p), tw(0), s));
  const cplx<T>* lastin = b.y;
  int64_t last_fs = g.out_fs;
  if (d == 3) {
    const int64_t P1 = p->P[1], zfs = N0 * N1 * Hs;
    vgf::StridedGeom ig{H, Hs, Hs, P1 * Hs, N1 * Hs, (int)N0};
    ig.nentry = en.count;
    ig.es_in = ig.es_out = en.es;
    for (int f = 0; f < g.nf; ++f) {
      vgf::C2CInvArgs<T> ia{b.y + f * g.out_fs, {b.z + f * zfs, nullptr}, ig, deriv1<T>(p, 1, 0)};
      VGF_LAUNCH(kPassC2CI, vgf::launch_c2c_inv<T>((int)P1, launch_variant(sched, kPassC2CI, f), ia, tw(1), s));
    }
    lastin = b.z;
    last_fs = zfs;
  }
  for (int f = 0; f < g.nf; ++f) {
    vgf::C2RArgs<T> ca{};
    ca.in = lastin + f * last_fs;
    ca.in_es = en.es;
    ca.nlines = lpe * en.count;
    ca.lpe = lpe;
    ca.hs = Hs;
    ca.d = deriv1<T>(p, d - 1, 0);
    c2r_out(ca, 0, en, g.fields[f] - 1, vol);
    VGF_LAUNCH(kPassC2R, vgf::launch_c2r<T>((int)p->P[d - 1], ca, tw(d - 1), s));
  }
  return VGF_OK;
}

// output o of an axis-0 complex-to-real launch: phi (field < 0) or E_field
template <typename T>
void c2r_s_out(vgf::C2RSArgs<T>& ca, int o, const Entries<T>& en, int field, int64_t vol) {
  if (!en.phi_tab && !en.E_tab) {
    ca.out[o] = field < 0 ? en.phi : en.E + field * vol;
  } else {
    ca.out[o] = nullptr;
    ca.out_tab[o] = field < 0 ? en.phi_tab : en.E_tab;
    ca.out_off[o] = field < 0 ? 0 : field * vol;
  }
}

// Forward solve with the multiply pass along the contiguous last axis:
//   rho [N0][..]  --r2c axis 0-->  X1 [N0+1][N1]([N2])
//   (3D) X1       --c2c axis 1-->  X2 [N0+1][P1][N2]
//   X2 (X1 in 2D) --axis-last pass: forward, x kernel, phi and -i k_last phi, inverse-->  Y
//   (3D) Y        --c2c^-1 axis 1-->  Z: phi, E_1 (from phi), E_2
//   Z (Y in 2D)   --c2r axis 0-->  phi, E_0 (from phi), and the other fields
// Each pass again applies the derivative of its own axis.
template <typename T>
vgf_status enqueue_solve_c(vgf_plan p, const Entries<T>& en, hipStream_t s, bool marks, const int* sched,
                           hipEvent_t* mark_events, int* mark_tags) {
  const int d = p->dim;
  const int64_t N0 = p->n[0], N1 = p->n[1], H0 = N0 + 1, NL = p->n[d - 1];
  const int64_t vol = prod(p->n, d);
  const bool want_phi = en.want_phi, want_E = en.want_E;
  char* base = en.ws;
  Bufs<T> b{(cplx<T>*)(base + p->off_x1), (cplx<T>*)(base + p->off_x2), (cplx<T>*)(base + p->off_y),
            (cplx<T>*)(base + p->off_z)};
  auto tw = [&](int a) { return (const cplx<T>*)p->tw[a]; };
  Marks mk(p, s, marks, mark_events, mark_tags);
  // large arrays: non-temporal input loads of the axis-0 R2C, stores of the
  // axis-1 forward, loads and stores of the multiply pass and of the axis-1
  // inverse (the combination measured fastest; the axis-0 C2R, whose FP32
  // form reads phi's spectrum twice, stays plain)
  const bool nt = vol * en.count * (int64_t)sizeof(T) >= p->stream_min;
  vgf::R2CSArgs<T> ra{};
  if (en.rho_tab) ra.in_tab[0] = en.rho_tab;
  else ra.in[0] = en.rho;
  ra.out = b.x1;
  ra.out_es = en.es;
  ra.ncols = vol / N0;
  ra.nentry = en.count;
  ra.d = deriv1<T>(p, 0, 0);
  ra.nt_load = nt;
  VGF_LAUNCH(kPassR2C, vgf::launch_r2c_s<T>((int)p->P[0], launch_variant(sched, kPassR2C, 0), ra, tw(0), s));
  const cplx<T>* fin = b.x1;
  vgf::FusedCGeom<T> g{};
  g.dim = d;
  g.n0 = (int)N0;
  g.n1 = (int)N1;
  g.n_last = (int)NL;
  g.lpe = d == 3 ? H0 * p->P[1] : H0;
  g.nlines = g.lpe * en.count;
  g.in_es = g.out_es = en.es;
  g.fs = g.lpe * NL;
  g.ks = (T)wavenumber_step(p, d - 1);
  g.nf = want_E ? 2 : 1;
  g.nt = nt;
  g.ytile = y_tile_log2<T>(p);
  if (d == 3) {
    const int64_t P1 = p->P[1], N2 = NL;
    vgf::StridedGeom fg{N2, N2, N2, N1 * N2, P1 * N2, (int)H0};
    fg.nentry = en.count;
    fg.es_in = fg.es_out = en.es;
    fg.nt_store = nt;
    vgf::C2CFwdArgs<T> fa{{b.x1, nullptr}, b.x2, fg, deriv1<T>(p, 1, 0)};
    VGF_LAUNCH(kPassC2CF, vgf::launch_c2c_fwd<T>((int)P1, launch_variant(sched, kPassC2CF, 0), fa, tw(1), s));
    fin = b.x2;
  }
  VGF_LAUNCH(kPassFused, vgf::launch_fused_c<T>((int)p->P[d - 1], sched[kPassFused], false, fin, b.y, g,
                                                (const T*)p->spec, tw(d - 1), s));
  // axis-0 inputs: phi's spectrum, and the spectra of E_1 (3D) and E_last
  const cplx<T>* zphi = b.y;
  const cplx<T>* zf[2] = {nullptr, nullptr};  // E_1, E_2 (3D) or E_1 (2D)
  int64_t zes = g.fs;
  if (d == 3) {
    const int64_t P1 = p->P[1], N2 = NL, zfs = H0 * N1 * N2;
    vgf::StridedGeom ig{N2, N2, N2, P1 * N2, N1 * N2, (int)H0};
    ig.nentry = en.count;
    ig.es_in = ig.es_out = en.es;
    ig.nt_load = ig.nt_store = nt;
    ig.in_tile = g.ytile;  // the multiply pass wrote this launch's tile order
    // one launch: phi and E_1 from phi's spectrum, E_2 from its own
    vgf::C2CInvArgs<T> ia{b.y, {b.z, b.z + zfs}, ig, want_E ? deriv2<T>(p, 1, 0, -1) : deriv1<T>(p, 1, 0)};
    if (want_E) {
      ia.in2 = b.y + g.fs;
      ia.out2 = b.z + 2 * zfs;
    }
    VGF_LAUNCH(kPassC2CI, vgf::launch_c2c_inv<T>((int)P1, launch_variant(sched, kPassC2CI, 0), ia, tw(1), s));
    zphi = b.z;
    zf[0] = b.z + zfs;
    zf[1] = b.z + 2 * zfs;
    zes = zfs;
  } else {
    zf[0] = b.y + g.fs;
  }
  (void)zes;
  // one launch: phi and E_0 (or E_0 alone) from phi's spectrum, then the
  // other fields from their own spectra
  vgf::C2RSArgs<T> ca{};
  ca.in = zphi;
  ca.in_es = en.es;
  ca.ncols = vol / N0;
  ca.nentry = en.count;
  // FP32 reads phi's spectrum a second time for E_0: non-temporal loads of
  // the once-read inputs keep those columns in the caches (C2R 157 -> 152 us
  // at 256^3); FP64 holds them in registers, and the hint only slowed it
  ca.nt_x = nt && sizeof(T) == 4;
  if (want_phi && want_E) {
    ca.d = deriv2<T>(p, 0, 0, -1);
    c2r_s_out(ca, 0, en, -1, vol);
    c2r_s_out(ca, 1, en, 0, vol);
  } else {
    ca.d = deriv1<T>(p, 0, want_phi ? 0 : -1);
    c2r_s_out(ca, 0, en, want_phi ? -1 : 0, vol);
  }
  if (want_E) {
    for (int a = 1; a < d; ++a) {
      ca.in_x[ca.nx] = zf[a - 1];
      c2r_s_out(ca, ca.d.n + ca.nx, en, a, vol);
      ++ca.nx;
    }
  }
  VGF_LAUNCH(kPassC2R, vgf::launch_c2r_s<T>((int)p->P[0], launch_variant(sched, kPassC2R, 0), ca, tw(0), s));
  return VGF_OK;
}

// Multiply-pass geometry of the default layout (lines along the contiguous
// last axis of X2 in 3D, X1 in 2D).
template <typename T>
vgf::FusedCGeom<T> fused_c_geom(vgf_plan p, int count, int64_t es, bool nt) {
  const int d = p->dim;
  const int64_t N0 = p->n[0], H0 = N0 + 1, NL = p->n[d - 1];
  vgf::FusedCGeom<T> g{};
  g.dim = d;
  g.n0 = (int)N0;
  g.n1 = (int)p->n[1];
  g.n_last = (int)NL;
  g.lpe = d == 3 ? H0 * p->P[1] : H0;
  g.nlines = g.lpe * count;
  g.in_es = g.out_es = es;
  g.fs = g.lpe * NL;
  g.ks = (T)wavenumber_step(p, d - 1);
  g.nt = nt;
  return g;
}

// Forward solve with gradient kernels in the default layout: the axis-0 R2C
// and the axis-1 forward as for Fourier fields, then the multiply pass along
// the contiguous axis gives every requested field its own spectrum (phi: the
// kernel spectrum, E_a: -i T_a) and inverts each, and every field is then
// inverted on its own along axis 1 and axis 0 (no derivative factors).
template <typename T>
vgf_status enqueue_solve_cg(vgf_plan p, const Entries<T>& en, hipStream_t s, bool marks, const int* sched,
                            hipEvent_t* mark_events, int* mark_tags) {
  const int d = p->dim;
  const int64_t N0 = p->n[0], N1 = p->n[1], H0 = N0 + 1, NL = p->n[d - 1];
  const int64_t vol = prod(p->n, d);
  char* base = en.ws;
  Bufs<T> b{(cplx<T>*)(base + p->off_x1), (cplx<T>*)(base + p->off_x2), (cplx<T>*)(base + p->off_y),
            (cplx<T>*)(base + p->off_z)};
  auto tw = [&](int a) { return (const cplx<T>*)p->tw[a]; };
  Marks mk(p, s, marks, mark_events, mark_tags);
  const bool nt = vol * en.count * (int64_t)sizeof(T) >= p->stream_min;
  vgf::R2CSArgs<T> ra{};
  if (en.rho_tab) ra.in_tab[0] = en.rho_tab;
  else ra.in[0] = en.rho;
  ra.out = b.x1;
  ra.out_es = en.es;
  ra.ncols = vol / N0;
  ra.nentry = en.count;
  ra.d = deriv1<T>(p, 0, 0);
  ra.nt_load = nt;
  VGF_LAUNCH(kPassR2C, vgf::launch_r2c_s<T>((int)p->P[0], launch_variant(sched, kPassR2C, 0), ra, tw(0), s));
  const cplx<T>* fin = b.x1;
  vgf::FusedCGeom<T> g = fused_c_geom<T>(p, en.count, en.es, nt);
  g.ytile = y_tile_log2<T>(p);
  g.nf = 0;
  if (en.want_phi) g.fields[g.nf++] = 0;
  if (en.want_E)
    for (int a = 0; a < d; ++a) g.fields[g.nf++] = 1 + a;
  if (d == 3) {
    const int64_t P1 = p->P[1], N2 = NL;
    vgf::StridedGeom fg{N2, N2, N2, N1 * N2, P1 * N2, (int)H0};
    fg.nentry = en.count;
    fg.es_in = fg.es_out = en.es;
    fg.nt_store = nt;
    vgf::C2CFwdArgs<T> fa{{b.x1, nullptr}, b.x2, fg, deriv1<T>(p, 1, 0)};
    VGF_LAUNCH(kPassC2CF, vgf::launch_c2c_fwd<T>((int)P1, launch_variant(sched, kPassC2CF, 0), fa, tw(1), s));
    fin = b.x2;
  }
  VGF_LAUNCH(kPassFused, vgf::launch_fused_cg<T>((int)p->P[d - 1], false, fin, b.y, g, grad_spec<T>(p),
                                                 tw(d - 1), s));
  // spectra along axis 0 of the fields, one array each
  const cplx<T>* zin = b.y;
  int64_t zfs = g.fs;
  if (d == 3) {
    const int64_t P1 = p->P[1], N2 = NL;
    zfs = H0 * N1 * N2;
    vgf::StridedGeom ig{N2, N2, N2, P1 * N2, N1 * N2, (int)H0};
    ig.nentry = en.count;
    ig.es_in = ig.es_out = en.es;
    ig.nt_load = ig.nt_store = nt;
    ig.in_tile = g.ytile;  // the multiply pass wrote the inverse's tile order
    for (int f = 0; f < g.nf; ++f) {
      vgf::C2CInvArgs<T> ia{b.y + f * g.fs, {b.z + f * zfs, nullptr}, ig, deriv1<T>(p, 1, 0)};
      VGF_LAUNCH(kPassC2CI, vgf::launch_c2c_inv<T>((int)P1, launch_variant(sched, kPassC2CI, f), ia, tw(1), s));
    }
    zin = b.z;
  }
  // one axis-0 launch: the first field from its own spectrum (no factor),
  // the others as extra inputs
  vgf::C2RSArgs<T> ca{};
  ca.in = zin;
  ca.in_es = en.es;
  ca.ncols = vol / N0;
  ca.nentry = en.count;
  ca.d = deriv1<T>(p, 0, 0);
  c2r_s_out(ca, 0, en, g.fields[0] - 1, vol);
  for (int f = 1; f < g.nf; ++f) {
    ca.in_x[ca.nx] = zin + f * zfs;
    c2r_s_out(ca, 1 + ca.nx, en, g.fields[f] - 1, vol);
    ++ca.nx;
  }
  VGF_LAUNCH(kPassC2R, vgf::launch_c2r_s<T>((int)p->P[0], launch_variant(sched, kPassC2R, 0), ca, tw(0), s));
  return VGF_OK;
}

template <typename T>
vgf_status enqueue_solve(vgf_plan p, const Entries<T>& en, hipStream_t s, bool marks,
                         const int* sched, hipEvent_t* mark_events = nullptr, int* mark_tags = nullptr) {
  if (p->gradk && p->contig) return enqueue_solve_cg<T>(p, en, s, marks, sched, mark_events, mark_tags);
  if (p->gradk) return enqueue_solve_grad<T>(p, en, s, marks, sched, mark_events, mark_tags);
  if (p->contig) return enqueue_solve_c<T>(p, en, s, marks, sched, mark_events, mark_tags);
  const int d = p->dim;
  const int64_t N0 = p->n[0], N1 = p->n[1], H = p->H, Hs = p->Hs;
  const int64_t vol = prod(p->n, d);
  const bool want_phi = en.want_phi, want_E = en.want_E;
  char* base = en.ws;
  Bufs<T> b{(cplx<T>*)(base + p->off_x1), (cplx<T>*)(base + p->off_x2), (cplx<T>*)(base + p->off_y),
            (cplx<T>*)(base + p->off_z)};
  const T* spec = (const T*)p->spec;
  auto tw = [&](int a) { return (const cplx<T>*)p->tw[a]; };
  vgf::FusedGeom<T> g = fused_geom<T>(p);
  g.nf = 0;
  g.fields[g.nf++] = 0;
  if (want_E) g.fields[g.nf++] = 1;
  g.nentry = en.count;
  g.in_es = g.out_es = en.es;
  Marks mk(p, s, marks, mark_events, mark_tags);
  const int64_t lpe = d == 3 ? N0 * N1 : N0;  // contiguous lines per entry
  vgf::R2CArgs<T> ra{};
  ra.nlines = lpe * en.count;
  ra.lpe = lpe;
  ra.hs = Hs;
  ra.out = b.x1;
  ra.out_es = en.es;
  ra.d = deriv1<T>(p, d - 1, 0);
  if (en.rho_tab) ra.in_tab[0] = en.rho_tab;
  else ra.in[0] = en.rho;
  // c2r launches: one complex input, up to two outputs
  auto c2r = [&](const cplx<T>* in, int f0, int code0, int f1, int code1) -> hipError_t {
    vgf::C2RArgs<T> ca{};
    ca.in = in;
    ca.in_es = en.es;
    ca.nlines = lpe * en.count;
    ca.lpe = lpe;
    ca.hs = Hs;
    ca.d = f1 == -2 ? deriv1<T>(p, d - 1, code0) : deriv2<T>(p, d - 1, code0, code1);
    c2r_out(ca, 0, en, f0, vol);
    if (f1 != -2) c2r_out(ca, 1, en, f1, vol);
    return vgf::launch_c2r<T>((int)p->P[d - 1], ca, tw(d - 1), s);
  };
  if (d == 3) {
    const int64_t P1 = p->P[1];
    const int64_t yfs = N0 * P1 * Hs, zfs = N0 * N1 * Hs;
    g.out_fs = yfs;
    VGF_LAUNCH(kPassR2C, vgf::launch_r2c<T>((int)p->P[2], ra, tw(2), s));
    vgf::StridedGeom fg{H, Hs, Hs, N1 * Hs, P1 * Hs, (int)N0};
    fg.nentry = en.count;
    fg.es_in = fg.es_out = en.es;
    vgf::C2CFwdArgs<T> fa{{b.x1, nullptr}, b.x2, fg, deriv1<T>(p, 1, 0)};
    VGF_LAUNCH(kPassC2CF, vgf::launch_c2c_fwd<T>((int)P1, launch_variant(sched, kPassC2CF, 0), fa, tw(1), s));
    VGF_LAUNCH(kPassFused, vgf::launch_fused<T>((int)p->P[0], launch_variant(sched, kPassFused, 0), false, b.x2, b.y, g, spec, tw(0), s));
    // Yp -> Zp (phi, and E_2 later) and Z1 = -i k_1 Zp; Y0 -> Z0
    vgf::StridedGeom ig{H, Hs, Hs, P1 * Hs, N1 * Hs, (int)N0};
    ig.nentry = en.count;
    ig.es_in = ig.es_out = en.es;
    cplx<T>* zp = b.z;
    cplx<T>* z1 = b.z + zfs;
    cplx<T>* z0 = b.z + 2 * zfs;
    // one launch: phi and E_1 from phi's spectrum, E_0 from its own
    vgf::C2CInvArgs<T> ia{b.y, {zp, z1}, ig, want_E ? deriv2<T>(p, 1, 0, -1) : deriv1<T>(p, 1, 0)};
    if (want_E) {
      ia.in2 = b.y + yfs;
      ia.out2 = z0;
    }
    VGF_LAUNCH(kPassC2CI, vgf::launch_c2c_inv<T>((int)P1, launch_variant(sched, kPassC2CI, 0), ia, tw(1), s));
    if (want_phi && want_E) VGF_LAUNCH(kPassC2R, c2r(zp, -1, 0, 2, -1));
    else if (want_phi) VGF_LAUNCH(kPassC2R, c2r(zp, -1, 0, -2, 0));
    else VGF_LAUNCH(kPassC2R, c2r(zp, 2, -1, -2, 0));
    if (want_E) {
      VGF_LAUNCH(kPassC2R, c2r(z1, 1, 0, -2, 0));
      VGF_LAUNCH(kPassC2R, c2r(z0, 0, 0, -2, 0));
    }
  } else {
    const int64_t yfs = N0 * Hs;
    g.out_fs = yfs;
    VGF_LAUNCH(kPassR2C, vgf::launch_r2c<T>((int)p->P[1], ra, tw(1), s));
    VGF_LAUNCH(kPassFused, vgf::launch_fused<T>((int)p->P[0], launch_variant(sched, kPassFused, 0), false, b.x1, b.y, g, spec, tw(0), s));
    if (want_phi && want_E) VGF_LAUNCH(kPassC2R, c2r(b.y, -1, 0, 1, -1));
    else if (want_phi) VGF_LAUNCH(kPassC2R, c2r(b.y, -1, 0, -2, 0));
    else VGF_LAUNCH(kPassC2R, c2r(b.y, 1, -1, -2, 0));
    if (want_E) VGF_LAUNCH(kPassC2R, c2r(b.y + yfs, 0, 0, -2, 0));
  }
  return VGF_OK;
}

// ---------------------------------------------------------------------------
// Autotuning of the schedules. Four candidate schedules (every strided pass
// at tile width v & 1, the contiguous multiply pass at value v) run two
// warm-up enqueues each, then the candidates run interleaved `reps` times;
// HIP events at the pass boundaries give each pass's time, each pass takes
// its fastest repetition per value and keeps the default unless another
// value is more than 2% faster. The choice is cached per process for the
// grid, precision, outputs, field mode and number of entries per launch.
// ---------------------------------------------------------------------------
struct TuneKey {
  int prec, dim, outs, count;
  int64_t n[3];
  bool operator<(const TuneKey& o) const {
    if (prec != o.prec) return prec < o.prec;
    if (dim != o.dim) return dim < o.dim;
    if (outs != o.outs) return outs < o.outs;
    if (count != o.count) return count < o.count;
    for (int a = 0; a < 3; ++a)
      if (n[a] != o.n[a]) return n[a] < o.n[a];
    return false;
  }
};

std::mutex g_tune_mu;
std::map<TuneKey, std::array<int, kPasses>> g_tune_cache;

// passes with schedule variants: the strided ones of the plan's layout (tile
// width) and, in the default layout, the multiply pass along the contiguous
// axis (lanes per line and walk length)
bool pass_tunable(vgf_plan p, int pass) {
  if (p->gradk && p->contig)
    return pass == kPassR2C || pass == kPassC2R || (p->dim == 3 && (pass == kPassC2CF || pass == kPassC2CI));
  if (p->gradk) return p->dim == 3 && (pass == kPassC2CF || pass == kPassC2CI);
  if (p->contig)
    return pass == kPassR2C || pass == kPassC2R || pass == kPassFused ||
           (p->dim == 3 && (pass == kPassC2CF || pass == kPassC2CI));
  return pass == kPassFused || (p->dim == 3 && (pass == kPassC2CF || pass == kPassC2CI));
}
// the contiguous multiply pass takes its schedule value (0..3) whole; the
// strided passes hold one tile-width bit per launch class
bool pass_whole_value(vgf_plan p, int pass) { return p->contig && pass == kPassFused; }

// run(sched, events) enqueues one solve (or one group of entries) with the
// given schedule, recording the pass boundaries into events when non-null.
template <class Run>
vgf_status tune_schedule(vgf_plan p, int reps, hipStream_t s, Run run, int* best, hipError_t* herr) {
  // candidate v (0..3) sets every strided pass to tile width v & 1 (both
  // launch classes) and the contiguous multiply pass to schedule value v
  constexpr int NC = 4;
  static_assert(vgf_tile_variants() == 2, "schedule values hold one bit per launch class");
  std::vector<hipEvent_t> ev((size_t)reps * NC * kMaxMarks, nullptr);
  std::vector<int> tags((size_t)reps * NC * kMaxMarks, -1);
  hipError_t e = hipSuccess;
  for (size_t i = 0; i < ev.size() && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
  int sched[NC][kPasses];
  for (int v = 0; v < NC; ++v)
    for (int k = 0; k < kPasses; ++k)
      sched[v][k] = !pass_tunable(p, k) ? 0 : pass_whole_value(p, k) ? v : (v & 1) * 3;
  vgf_status st = VGF_OK;
  // warm-up of every candidate, then the candidates interleaved rep by rep
  // so that clock ramps bias none of them; each timed solve follows an
  // untimed one of the same candidate, so that it sees the caches a run of
  // that schedule leaves (a pass's time depends on what ran before it)
  for (int w = 0; w < 2 && st == VGF_OK && e == hipSuccess; ++w)
    for (int v = 0; v < NC && st == VGF_OK; ++v) st = run(sched[v], nullptr, nullptr);
  for (int r = 0; r < reps && st == VGF_OK && e == hipSuccess; ++r)
    for (int v = 0; v < NC && st == VGF_OK; ++v) {
      const size_t o = ((size_t)r * NC + v) * kMaxMarks;
      st = run(sched[v], nullptr, nullptr);
      if (st == VGF_OK) st = run(sched[v], &ev[o], &tags[o]);
    }
  // fastest repetition of each pass's first launch (class 0) and of its
  // later launches together (class 1) under each candidate
  double t[NC][kPasses][2];
  bool later[kPasses] = {};
  for (int v = 0; v < NC; ++v)
    for (int k = 0; k < kPasses; ++k) t[v][k][0] = t[v][k][1] = 1e30;
  if (st == VGF_OK && e == hipSuccess) e = hipStreamSynchronize(s);
  for (int r = 0; r < reps && st == VGF_OK && e == hipSuccess; ++r)
    for (int v = 0; v < NC && e == hipSuccess; ++v) {
      const size_t o = ((size_t)r * NC + v) * kMaxMarks;
      double pass_ms[kPasses][2] = {};
      int seen[kPasses] = {};
      for (int i = 0; i + 1 < kMaxMarks && tags[o + i] >= 0 && e == hipSuccess; ++i) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, ev[o + i], ev[o + i + 1]);
        const int k = tags[o + i], c = seen[k]++ > 0 ? 1 : 0;
        pass_ms[k][c] += ms;
        if (c) later[k] = true;
      }
      for (int k = 0; k < kPasses; ++k)
        for (int c = 0; c < 2; ++c) t[v][k][c] = std::min(t[v][k][c], pass_ms[k][c]);
    }
  // per pass (and launch class), keep the default unless another value is
  // faster by more than 2%; a strided pass without later launches gives them
  // its first launch's width (the adjoint may launch it more than once)
  bool changed = false;
  for (int k = 0; k < kPasses; ++k) {
    best[k] = 0;
    if (!pass_tunable(p, k)) continue;
    if (pass_whole_value(p, k)) {
      int b = 0;
      for (int v = 1; v < NC; ++v)
        if (t[v][k][0] < 0.98 * t[b][k][0]) b = v;
      best[k] = b;
    } else {
      int b[2] = {0, 0};
      for (int c = 0; c < 2; ++c) {
        const double w0 = std::min(t[0][k][c], t[2][k][c]), w1 = std::min(t[1][k][c], t[3][k][c]);
        if (w1 < 0.98 * w0) b[c] = 1;
      }
      if (!later[k]) b[1] = b[0];
      best[k] = b[0] | (b[1] << 1);
    }
    changed = changed || best[k] != 0;
  }
  // a pass's time also depends on the passes before it (caches, tails), so
  // the mixed schedule must beat the default on the whole solve by 1%
  if (changed && st == VGF_OK && e == hipSuccess) {
    const int* cand[2] = {sched[0], best};
    double total[2] = {1e30, 1e30};
    for (int r = 0; r < reps && st == VGF_OK && e == hipSuccess; ++r)
      for (int c = 0; c < 2 && st == VGF_OK; ++c) {
        const size_t o = ((size_t)r * NC + c) * kMaxMarks;
        for (int i = 0; i < kMaxMarks; ++i) tags[o + i] = -1;
        st = run(cand[c], nullptr, nullptr);
        if (st == VGF_OK) st = run(cand[c], &ev[o], &tags[o]);
      }
    if (st == VGF_OK && e == hipSuccess) e = hipStreamSynchronize(s);
    for (int r = 0; r < reps && st == VGF_OK && e == hipSuccess; ++r)
      for (int c = 0; c < 2 && e == hipSuccess; ++c) {
        const size_t o = ((size_t)r * NC + c) * kMaxMarks;
        int last = 0;
        while (last + 1 < kMaxMarks && tags[o + last] >= 0) ++last;
        float ms = 0.f;
        if (last > 0) e = hipEventElapsedTime(&ms, ev[o], ev[o + last]);
        total[c] = std::min(total[c], (double)ms);
      }
    if (st == VGF_OK && e == hipSuccess && !(total[1] < 0.99 * total[0]))
      for (int k = 0; k < kPasses; ++k) best[k] = 0;
  }
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (st != VGF_OK) return st;
  if (e != hipSuccess) {
    *herr = e;
    return VGF_ERR_HIP;
  }
  return VGF_OK;
}

template <class Run>
vgf_status tune_cached(vgf_plan p, bool want_phi, bool want_E, int count, int reps, hipStream_t s, Run run,
                       int* sched_out, hipError_t* herr) {
  // the pass structure depends on the outputs and on the field mode
  // and on whether the solve streams (non-temporal accesses)
  const int64_t in_bytes = prod(p->n, p->dim) * count * (p->prec == VGF_F32 ? 4 : 8);
  const int outs = (want_phi ? 1 : 0) | (want_E ? 2 : 0) | (p->fd ? 4 : 0) | (p->gradk ? 8 : 0) |
                   (p->contig ? 16 : 0) | (in_bytes >= p->stream_min ? 32 : 0);
  TuneKey key{(int)p->prec, p->dim, outs, count, {p->n[0], p->n[1], p->dim == 3 ? p->n[2] : 0}};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune_cache.find(key);
    if (it != g_tune_cache.end()) {
      for (int k = 0; k < kPasses; ++k) sched_out[k] = it->second[k];
      return VGF_OK;
    }
  }
  int best[kPasses];
  vgf_status st = tune_schedule(p, reps, s, run, best, herr);
  if (st != VGF_OK) return st;
  std::array<int, kPasses> a{};
  for (int k = 0; k < kPasses; ++k) a[k] = sched_out[k] = best[k];
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_cache[key] = a;
  return VGF_OK;
}

vgf::FdGeom fd_geom(vgf_plan p) {
  vgf::FdGeom g{};
  g.dim = p->dim;
  g.total = prod(p->n, p->dim);
  int64_t st = 1;
  for (int a = p->dim - 1; a >= 0; --a) {
    g.n[a] = (int)p->n[a];
    g.stride[a] = st;
    st *= p->n[a];
    g.inv2h[a] = 0.5 / p->h[a];
  }
  return g;
}

// One solve on workspace ws (the plan's own, or the static scratch of
// vgf_solve_noalloc), laid out as the plan's offsets describe.
template <typename T>
vgf_status solve_t(vgf_plan p, const T* rho, T* phi, T* E, hipStream_t s, char* ws) {
  Entries<T> en;
  en.ws = ws;
  en.rho = rho;
  en.phi = phi;
  en.E = E;
  en.want_phi = phi != nullptr;
  en.want_E = E != nullptr;
  if (!(p->fd && E)) return enqueue_solve<T>(p, en, s, true, p->schedule);
  // E = -D phi: phi (the caller's, or the workspace's), then the differences
  T* ph = phi ? phi : (T*)(ws + p->off_phi);
  en.phi = ph;
  en.E = nullptr;
  en.want_phi = true;
  en.want_E = false;
  vgf_status st = enqueue_solve<T>(p, en, s, true, p->schedule);
  if (st != VGF_OK) return st;
  return hip_status(p, vgf::launch_fd_field<T>(ph, E, fd_geom(p), s));
}

// Adjoint: the mirror image of solve_t. Forward passes sum their inputs
// after multiplying by +i k of their own axis (the conjugate of -i k), the
// axis-0 pass multiplies by the (real) kernel spectrum and +i k_0, and the
// inverse passes are plain.
// Adjoint with gradient kernels: every cotangent is transformed on its own,
// the axis-0 pass sums them with the conjugate multipliers (+i T_a for the
// fields), and the sum is inverted once.
template <typename T>
vgf_status adjoint_grad_t(vgf_plan p, const T* g_phi, const T* g_E, T* g_rho, hipStream_t s) {
  const int d = p->dim;
  const int64_t N0 = p->n[0], N1 = p->n[1], H = p->H, Hs = p->Hs;
  const int64_t vol = prod(p->n, d);
  Bufs<T> b = bufs<T>(p);
  auto tw = [&](int a) { return (const cplx<T>*)p->tw[a]; };
  vgf::FusedGeom<T> g = fused_geom<T>(p);
  const T* srcs[4];
  g.nf = 0;
  if (g_phi) {
    srcs[g.nf] = g_phi;
    g.fields[g.nf++] = 0;
  }
  if (g_E)
    for (int a = 0; a < d; ++a) {
      srcs[g.nf] = g_E + a * vol;
      g.fields[g.nf++] = 1 + a;
    }
  const int64_t lpe = d == 3 ? N0 * N1 : N0;
  if (d == 3) {
    const int64_t P1 = p->P[1], yfs = N0 * P1 * Hs, zfs = N0 * N1 * Hs;
    const vgf::StridedGeom fg{H, Hs, Hs, N1 * Hs, P1 * Hs, (int)N0};
    for (int f = 0; f < g.nf; ++f) {
      vgf::R2CArgs<T> ra{{srcs[f], nullptr}, b.z + f * zfs, lpe, Hs, deriv1<T>(p, 2, 0)};
      ra.lpe = lpe;
      VGF_RUN(vgf::launch_r2c<T>((int)p->P[2], ra, tw(2), s));
      vgf::C2CFwdArgs<T> fa{{b.z + f * zfs, nullptr}, b.y + f * yfs, fg, deriv1<T>(p, 1, 0)};
      VGF_RUN(vgf::launch_c2c_fwd<T>((int)P1, launch_variant(p->schedule, kPassC2CF, f), fa, tw(1), s));
    }
    g.in_fs = yfs;
    VGF_RUN(vgf::launch_fused_grad<T>((int)p->P[0], true, b.y, b.x2, g, grad_spec<T>(p), tw(0), s));
    const vgf::StridedGeom ig{H, Hs, Hs, P1 * Hs, N1 * Hs, (int)N0};
    vgf::C2CInvArgs<T> ia{b.x2, {b.x1, nullptr}, ig, deriv1<T>(p, 1, 0)};
    VGF_RUN(vgf::launch_c2c_inv<T>((int)P1, launch_variant(p->schedule, kPassC2CI, 0), ia, tw(1), s));
  } else {
    const int64_t yfs = N0 * Hs;
    for (int f = 0; f < g.nf; ++f) {
      vgf::R2CArgs<T> ra{{srcs[f], nullptr}, b.y + f * yfs, lpe, Hs, deriv1<T>(p, 1, 0)};
      ra.lpe = lpe;
      VGF_RUN(vgf::launch_r2c<T>((int)p->P[1], ra, tw(1), s));
    }
    g.in_fs = yfs;
    VGF_RUN(vgf::launch_fused_grad<T>((int)p->P[0], true, b.y, b.x1, g, grad_spec<T>(p), tw(0), s));
  }
  vgf::C2RArgs<T> ca{b.x1, {g_rho, nullptr}, lpe, Hs, deriv1<T>(p, d - 1, 0)};
  ca.lpe = lpe;
  VGF_RUN(vgf::launch_c2r<T>((int)p->P[d - 1], ca, tw(d - 1), s));
  return VGF_OK;
}

// Adjoint with gradient kernels in the default layout: every cotangent goes
// through the axis-0 R2C and the axis-1 forward on its own; the multiply
// pass sums their line transforms with the conjugate multipliers (+i T_a for
// the fields) and inverts the sum once, followed by one axis-1 inverse and
// one axis-0 C2R.
template <typename T>
vgf_status adjoint_cg_t(vgf_plan p, const T* g_phi, const T* g_E, T* g_rho, hipStream_t s) {
  const int d = p->dim;
  const int64_t N0 = p->n[0], N1 = p->n[1], H0 = N0 + 1, NL = p->n[d - 1];
  const int64_t vol = prod(p->n, d);
  Bufs<T> b = bufs<T>(p);
  auto tw = [&](int a) { return (const cplx<T>*)p->tw[a]; };
  const bool nt = vol * (int64_t)sizeof(T) >= p->stream_min;
  vgf::FusedCGeom<T> g = fused_c_geom<T>(p, 1, 0, false);
  const T* srcs[4];
  g.nf = 0;
  if (g_phi) {
    srcs[g.nf] = g_phi;
    g.fields[g.nf++] = 0;
  }
  if (g_E)
    for (int a = 0; a < d; ++a) {
      srcs[g.nf] = g_E + a * vol;
      g.fields[g.nf++] = 1 + a;
    }
  // the line transforms' inputs: [field][lines] at stride fs in Y
  for (int f = 0; f < g.nf; ++f) {
    vgf::R2CSArgs<T> ra{};
    ra.in[0] = srcs[f];
    ra.out = d == 3 ? b.x1 : b.y + f * g.fs;
    ra.ncols = vol / N0;
    ra.nentry = 1;
    ra.d = deriv1<T>(p, 0, 0);
    ra.nt_load = nt;
    VGF_RUN(vgf::launch_r2c_s<T>((int)p->P[0], launch_variant(p->schedule, kPassR2C, 0), ra, tw(0), s));
    if (d == 3) {
      const int64_t P1 = p->P[1], N2 = NL;
      const vgf::StridedGeom fg{N2, N2, N2, N1 * N2, P1 * N2, (int)H0};
      vgf::C2CFwdArgs<T> fa{{b.x1, nullptr}, b.y + f * g.fs, fg, deriv1<T>(p, 1, 0)};
      VGF_RUN(vgf::launch_c2c_fwd<T>((int)P1, launch_variant(p->schedule, kPassC2CF, 0), fa, tw(1), s));
    }
  }
  cplx<T>* acc = d == 3 ? b.x2 : b.x1;
  VGF_RUN(vgf::launch_fused_cg<T>((int)p->P[d - 1], true, b.y, acc, g, grad_spec<T>(p), tw(d - 1), s));
  const cplx<T>* zin = acc;
  if (d == 3) {
    const int64_t P1 = p->P[1], N2 = NL;
    const vgf::StridedGeom ig{N2, N2, N2, P1 * N2, N1 * N2, (int)H0};
    vgf::C2CInvArgs<T> ia{acc, {b.z, nullptr}, ig, deriv1<T>(p, 1, 0)};
    VGF_RUN(vgf::launch_c2c_inv<T>((int)P1, launch_variant(p->schedule, kPassC2CI, 0), ia, tw(1), s));
    zin = b.z;
  }
  vgf::C2RSArgs<T> ca{};
  ca.in = zin;
  ca.ncols = vol / N0;
  ca.nentry = 1;
  ca.d = deriv1<T>(p, 0, 0);
  ca.out[0] = g_rho;
  VGF_RUN(vgf::launch_c2r_s<T>((int)p->P[0], launch_variant(p->schedule, kPassC2R, 0), ca, tw(0), s));
  return VGF_OK;
}

// Adjoint in the contiguous-multiply layout: the mirror image of
// enqueue_solve_c (forward passes sum their inputs with +i k of their axis).
// The cotangents of the entries one adjoint launch covers: direct pointers
// (one entry, the plan workspace) or device tables of per-entry pointers
// with workspaces es elements apart (a batch group).
template <typename T> struct AdjEntries {
  int count = 1;
  char* ws = nullptr;
  int64_t es = 0;
  const T* g_phi = nullptr;
  const T* g_E = nullptr;
  T* g_rho = nullptr;
  const T* const* g_phi_tab = nullptr;
  const T* const* g_E_tab = nullptr;
  T* const* g_rho_tab = nullptr;
  bool has_phi = false, has_E = false;
};

template <typename T>
vgf_status adjoint_c_entries(vgf_plan p, const AdjEntries<T>& en, const int* sched, hipStream_t s) {
  const int d = p->dim;
  const int64_t N0 = p->n[0], N1 = p->n[1], H0 = N0 + 1, NL = p->n[d - 1];
  const int64_t vol = prod(p->n, d);
  char* base = en.ws;
  Bufs<T> b{(cplx<T>*)(base + p->off_x1), (cplx<T>*)(base + p->off_x2), (cplx<T>*)(base + p->off_y),
            (cplx<T>*)(base + p->off_z)};
  auto tw = [&](int a) { return (const cplx<T>*)p->tw[a]; };
  const int64_t lpe = d == 3 ? H0 * p->P[1] : H0;
  const int64_t fs = lpe * NL;             // field stride of Y
  const int64_t zfs = H0 * N1 * (d == 3 ? NL : 1);  // field stride of Z (3D)
  // axis 0: A = R2C(g_phi) + i k_0 R2C(g_E0); the other fields plain.
  // Input term: g_phi (field < 0) or field `field` of g_E.
  int nr2c = 0;  // launches of the r2c kernel so far
  auto r2c = [&](cplx<T>* out, int f0, int code0, int f1, int code1, bool t0, bool t1) -> hipError_t {
    vgf::R2CSArgs<T> ra{};
    ra.out = out;
    ra.out_es = en.es;
    ra.ncols = vol / N0;
    ra.nentry = en.count;
    ra.d.ks = (T)wavenumber_step(p, 0);
    ra.d.n = 0;
    auto term = [&](int f, int code) {
      const int t = ra.d.n++;
      ra.d.code[t] = code;
      if (en.count == 1 && !en.g_phi_tab && !en.g_E_tab) {
        ra.in[t] = f < 0 ? en.g_phi : en.g_E + f * vol;
      } else {
        ra.in_tab[t] = f < 0 ? en.g_phi_tab : en.g_E_tab;
        ra.in_off[t] = f < 0 ? 0 : f * vol;
      }
    };
    if (t0) term(f0, code0);
    if (t1) term(f1, code1);
    return vgf::launch_r2c_s<T>((int)p->P[0], launch_variant(sched, kPassR2C, nr2c++), ra, tw(0), s);
  };
  vgf::FusedCGeom<T> g{};
  g.dim = d;
  g.n0 = (int)N0;
  g.n1 = (int)N1;
  g.n_last = (int)NL;
  g.lpe = lpe;
  g.nlines = lpe * en.count;
  g.in_es = g.out_es = en.es;
  g.fs = fs;
  g.ks = (T)wavenumber_step(p, d - 1);
  g.nf = 0;
  if (d == 3) {
    const int64_t P1 = p->P[1], N2 = NL;
    cplx<T>* za = b.z;
    cplx<T>* zb1 = b.z + zfs;
    cplx<T>* zb2 = b.z + 2 * zfs;
    VGF_RUN(r2c(za, -1, 0, 0, 1, en.has_phi, en.has_E));
    if (en.has_E) {
      VGF_RUN(r2c(zb1, 1, 0, 0, 0, true, false));
      VGF_RUN(r2c(zb2, 2, 0, 0, 0, true, false));
    }
    vgf::StridedGeom fg{N2, N2, N2, N1 * N2, P1 * N2, (int)H0};
    fg.nentry = en.count;
    fg.es_in = fg.es_out = en.es;
    vgf::C2CFwdArgs<T> fa{{za, zb1}, b.y, fg, en.has_E ? deriv2<T>(p, 1, 0, 1) : deriv1<T>(p, 1, 0)};
    VGF_RUN(vgf::launch_c2c_fwd<T>((int)P1, launch_variant(sched, kPassC2CF, 0), fa, tw(1), s));
    g.fields[g.nf++] = 0;
    if (en.has_E) {
      vgf::C2CFwdArgs<T> f2{{zb2, nullptr}, b.y + fs, fg, deriv1<T>(p, 1, 0)};
      VGF_RUN(vgf::launch_c2c_fwd<T>((int)P1, launch_variant(sched, kPassC2CF, 1), f2, tw(1), s));
      g.fields[g.nf++] = 1;
    }
    // the multiply pass writes X2 in the axis-1 inverse's tile order
    g.ytile = y_tile_log2<T>(p);
    VGF_RUN(vgf::launch_fused_c<T>((int)p->P[2], sched[kPassFused], true, b.y, b.x2, g, (const T*)p->spec, tw(2), s));
    vgf::StridedGeom ig{N2, N2, N2, P1 * N2, N1 * N2, (int)H0};
    ig.nentry = en.count;
    ig.es_in = ig.es_out = en.es;
    ig.in_tile = g.ytile;
    vgf::C2CInvArgs<T> ia{b.x2, {b.x1, nullptr}, ig, deriv1<T>(p, 1, 0)};
    VGF_RUN(vgf::launch_c2c_inv<T>((int)P1, launch_variant(sched, kPassC2CI, 0), ia, tw(1), s));
  } else {
    VGF_RUN(r2c(b.y, -1, 0, 0, 1, en.has_phi, en.has_E));
    g.fields[g.nf++] = 0;
    if (en.has_E) {
      VGF_RUN(r2c(b.y + fs, 1, 0, 0, 0, true, false));
      g.fields[g.nf++] = 1;
    }
    VGF_RUN(vgf::launch_fused_c<T>((int)p->P[1], sched[kPassFused], true, b.y, b.x1, g, (const T*)p->spec, tw(1), s));
  }
  vgf::C2RSArgs<T> ca{};
  ca.in = b.x1;
  ca.in_es = en.es;
  if (en.g_rho_tab) ca.out_tab[0] = en.g_rho_tab;
  else ca.out[0] = en.g_rho;
  ca.ncols = vol / N0;
  ca.nentry = en.count;
  ca.d = deriv1<T>(p, 0, 0);
  VGF_RUN(vgf::launch_c2r_s<T>((int)p->P[0], launch_variant(sched, kPassC2R, 0), ca, tw(0), s));
  return VGF_OK;
}

template <typename T>
vgf_status adjoint_c_t(vgf_plan p, const T* g_phi, const T* g_E, T* g_rho, hipStream_t s) {
  AdjEntries<T> en;
  en.ws = (char*)p->ws;
  en.g_phi = g_phi;
  en.g_E = g_E;
  en.g_rho = g_rho;
  en.has_phi = g_phi != nullptr;
  en.has_E = g_E != nullptr;
  return adjoint_c_entries<T>(p, en, p->schedule, s);
}

template <typename T>
vgf_status adjoint_t(vgf_plan p, const T* g_phi, const T* g_E, T* g_rho, hipStream_t s) {
  if (p->gradk && p->contig) return adjoint_cg_t<T>(p, g_phi, g_E, g_rho, s);
  if (p->gradk) return adjoint_grad_t<T>(p, g_phi, g_E, g_rho, s);
  if (p->contig) return adjoint_c_t<T>(p, g_phi, g_E, g_rho, s);
  const int d = p->dim;
  const int64_t N0 = p->n[0], N1 = p->n[1], H = p->H, Hs = p->Hs;
  const int64_t vol = prod(p->n, d);
  Bufs<T> b = bufs<T>(p);
  const T* spec = (const T*)p->spec;
  auto tw = [&](int a) { return (const cplx<T>*)p->tw[a]; };
  vgf::FusedGeom<T> g = fused_geom<T>(p);
  g.nf = 0;
  g.fields[g.nf++] = 0;
  if (g_E) g.fields[g.nf++] = 1;
  const int last = d - 1;
  // A = R2C(g_phi) + i k_last R2C(g_E[last])
  vgf::R2CArgs<T> ra{};
  ra.nlines = d == 3 ? N0 * N1 : N0;
  ra.hs = Hs;
  ra.d.ks = (T)wavenumber_step(p, last);
  ra.d.n = 0;
  if (g_phi) { ra.in[ra.d.n] = g_phi; ra.d.code[ra.d.n++] = 0; }
  if (g_E) { ra.in[ra.d.n] = g_E + last * vol; ra.d.code[ra.d.n++] = 1; }
  if (d == 3) {
    const int64_t P1 = p->P[1];
    const int64_t yfs = N0 * P1 * Hs, zfs = N0 * N1 * Hs;
    cplx<T>* za = b.z;
    cplx<T>* zb1 = b.z + zfs;
    cplx<T>* zb0 = b.z + 2 * zfs;
    ra.out = za;
    VGF_RUN(vgf::launch_r2c<T>((int)p->P[2], ra, tw(2), s));
    if (g_E) {
      vgf::R2CArgs<T> r1{{g_E + vol, nullptr}, zb1, N0 * N1, Hs, deriv1<T>(p, 2, 0)};
      VGF_RUN(vgf::launch_r2c<T>((int)p->P[2], r1, tw(2), s));
      vgf::R2CArgs<T> r0{{g_E, nullptr}, zb0, N0 * N1, Hs, deriv1<T>(p, 2, 0)};
      VGF_RUN(vgf::launch_r2c<T>((int)p->P[2], r0, tw(2), s));
    }
    const vgf::StridedGeom fg{H, Hs, Hs, N1 * Hs, P1 * Hs, (int)N0};
    vgf::C2CFwdArgs<T> fa{{za, zb1}, b.y, fg, g_E ? deriv2<T>(p, 1, 0, 1) : deriv1<T>(p, 1, 0)};
    VGF_RUN(vgf::launch_c2c_fwd<T>((int)P1, launch_variant(p->schedule, kPassC2CF, 0), fa, tw(1), s));
    if (g_E) {
      vgf::C2CFwdArgs<T> f0{{zb0, nullptr}, b.y + yfs, fg, deriv1<T>(p, 1, 0)};
      VGF_RUN(vgf::launch_c2c_fwd<T>((int)P1, launch_variant(p->schedule, kPassC2CF, 1), f0, tw(1), s));
    }
    g.in_fs = yfs;
    VGF_RUN(vgf::launch_fused<T>((int)p->P[0], 0, true, b.y, b.x2, g, spec, tw(0), s));
    const vgf::StridedGeom ig{H, Hs, Hs, P1 * Hs, N1 * Hs, (int)N0};
    vgf::C2CInvArgs<T> ia{b.x2, {b.x1, nullptr}, ig, deriv1<T>(p, 1, 0)};
    VGF_RUN(vgf::launch_c2c_inv<T>((int)P1, launch_variant(p->schedule, kPassC2CI, 0), ia, tw(1), s));
    vgf::C2RArgs<T> ca{b.x1, {g_rho, nullptr}, N0 * N1, Hs, deriv1<T>(p, 2, 0)};
    VGF_RUN(vgf::launch_c2r<T>((int)p->P[2], ca, tw(2), s));
  } else {
    const int64_t yfs = N0 * Hs;
    ra.out = b.y;
    VGF_RUN(vgf::launch_r2c<T>((int)p->P[1], ra, tw(1), s));
    if (g_E) {
      vgf::R2CArgs<T> r0{{g_E, nullptr}, b.y + yfs, N0, Hs, deriv1<T>(p, 1, 0)};
      VGF_RUN(vgf::launch_r2c<T>((int)p->P[1], r0, tw(1), s));
    }
    g.in_fs = yfs;
    VGF_RUN(vgf::launch_fused<T>((int)p->P[0], 0, true, b.y, b.x1, g, spec, tw(0), s));
    vgf::C2RArgs<T> ca{b.x1, {g_rho, nullptr}, N0, Hs, deriv1<T>(p, 1, 0)};
    VGF_RUN(vgf::launch_c2r<T>((int)p->P[1], ca, tw(1), s));
  }
  return VGF_OK;
}

vgf_status check_solve_args(vgf_plan p, const void* rho, const void* phi, const void* E) {
  if (!p || !rho) return VGF_ERR_INVALID_ARG;
  if (!phi && !E) return VGF_ERR_INVALID_ARG;
  if (phi && !(p->outputs & VGF_OUT_PHI)) return VGF_ERR_NOT_REQUESTED;
  if (E && !(p->outputs & VGF_OUT_E)) return VGF_ERR_NOT_REQUESTED;
  return VGF_OK;
}

}  // namespace

extern "C" {

const char* vgf_status_string(vgf_status st) {
  switch (st) {
    case VGF_OK: return "ok";
    case VGF_ERR_INVALID_ARG: return "invalid argument";
    case VGF_ERR_UNSUPPORTED_SIZE: return "unsupported grid size";
    case VGF_ERR_L_WINDOW: return "truncation radius L outside the admissible window";
    case VGF_ERR_OUT_OF_MEMORY: return "out of device memory (or above VGF_MAX_WORKSPACE)";
    case VGF_ERR_HIP: return "HIP runtime error";
    case VGF_ERR_NOT_REQUESTED: return "output not requested at plan creation";
    case VGF_ERR_SCRATCH_LIMIT:
      return "solve workspace larger than the 64 MiB static scratch of vgf_solve_noalloc";
  }
  return "unknown status";
}

vgf_status vgf_plan_create(vgf_plan* out, int dim, const int64_t* n, const double* h,
                           vgf_method method, vgf_precision prec, double L, unsigned outputs,
                           hipStream_t stream) {
  if (!out) return VGF_ERR_INVALID_ARG;
  *out = nullptr;
  if ((dim != 2 && dim != 3) || !n || !h) return VGF_ERR_INVALID_ARG;
  if (method != VGF_METHOD_VGF && method != VGF_METHOD_HE && method != VGF_METHOD_HE_NEARBY &&
      method != VGF_METHOD_HE_CELLAVG)
    return VGF_ERR_INVALID_ARG;
  if (prec != VGF_F64 && prec != VGF_F32) return VGF_ERR_INVALID_ARG;
  if ((outputs &
       ~(unsigned)(VGF_OUT_PHI | VGF_OUT_E | VGF_FIELD_CENTERED | VGF_FIELD_GRADIENT_KERNEL | VGF_LAYOUT_AXIS0)) ||
      !(outputs & (VGF_OUT_PHI | VGF_OUT_E)))
    return VGF_ERR_INVALID_ARG;
  if ((outputs & (VGF_FIELD_CENTERED | VGF_FIELD_GRADIENT_KERNEL)) && !(outputs & VGF_OUT_E))
    return VGF_ERR_INVALID_ARG;
  if ((outputs & VGF_FIELD_CENTERED) && (outputs & VGF_FIELD_GRADIENT_KERNEL)) return VGF_ERR_INVALID_ARG;
  if ((outputs & VGF_FIELD_GRADIENT_KERNEL) && method != VGF_METHOD_VGF) return VGF_ERR_INVALID_ARG;
  for (int a = 0; a < dim; ++a) {
    if (!(h[a] > 0.0) || !std::isfinite(h[a])) return VGF_ERR_INVALID_ARG;
    if (n[a] <= 0) return VGF_ERR_INVALID_ARG;
  }
  const bool wide = dim == 2 && !(outputs & VGF_LAYOUT_AXIS0);
  for (int a = 0; a < dim; ++a)
    if (!size_supported(n[a], wide)) return VGF_ERR_UNSUPPORTED_SIZE;

  double diam2 = 0.0, upper = INFINITY;
  for (int a = 0; a < dim; ++a) {
    const double ext = (double)(n[a] - 1) * h[a];
    diam2 += ext * ext;
    upper = std::min(upper, 4.0 * (double)n[a] * h[a] - ext);
  }
  const double diam = std::sqrt(diam2);
  double Lp = 0.0;
  if (method == VGF_METHOD_VGF) {
    if (std::isnan(L)) return VGF_ERR_L_WINDOW;
    Lp = (L > 0.0) ? L : 1.1 * diam;
    if (!(Lp > diam) || !(Lp < upper) || !std::isfinite(Lp)) return VGF_ERR_L_WINDOW;
  }

  vgf_plan p = new (std::nothrow) vgf_plan_s();
  if (!p) return VGF_ERR_OUT_OF_MEMORY;
  p->dim = dim;
  for (int a = 0; a < dim; ++a) {
    p->n[a] = n[a];
    p->h[a] = h[a];
    p->P[a] = 2 * n[a];
  }
  p->H = n[dim - 1] + 1;
  {
    const int64_t align = prec == VGF_F32 ? 16 : 8;  // complex values per 128 bytes
    p->Hs = (p->H + align - 1) / align * align;
  }
  p->method = method;
  p->prec = prec;
  p->L = Lp;
  p->outputs = outputs;
  p->nf_max = ((outputs & VGF_OUT_PHI) ? 1 : 0) + ((outputs & VGF_OUT_E) ? dim : 0);
  p->fd = (outputs & VGF_FIELD_CENTERED) != 0;
  p->gradk = (outputs & VGF_FIELD_GRADIENT_KERNEL) != 0;
  p->stream_min = stream_min_env();
  p->tile_y = tile_y_env();
  // the multiply pass runs along the contiguous axis unless asked otherwise
  p->contig = !(outputs & VGF_LAYOUT_AXIS0);

  const size_t rb = prec == VGF_F32 ? 4 : 8, cb = 2 * rb;
  const int64_t N0 = n[0], N1 = n[1], H = p->Hs;
  int64_t oct = 1, vol = 1;
  for (int a = 0; a < dim; ++a) {
    oct *= (n[a] + 1);
    vol *= n[a];
  }
  // Y holds the axis-0 outputs (phi's spectrum, and E_0's when E is
  // requested); Z the axis-1 outputs (phi, E_1, E_0). The adjoint reuses
  // the same regions in the mirrored order.
  // (A finite-difference field needs phi's spectrum only, and phi itself in
  // a real array when the caller does not ask for it.)
  // With gradient kernels every field is its own spectrum after axis 0.
  const bool fourier_E = (outputs & VGF_OUT_E) && !p->fd;
  size_t ny = fourier_E ? 2 : 1, nz = fourier_E ? 3 : 1;
  if (p->gradk) ny = nz = (size_t)(1 + dim);
  size_t x1 = 0, x2 = 0, y = 0, z = 0;
  if (p->contig) {
    // half spectrum along axis 0: [N0 + 1][N1]([N2]), no padding needed
    const int64_t H0 = N0 + 1;
    if (dim == 3) {
      x1 = (size_t)(H0 * N1 * n[2]);
      x2 = (size_t)(H0 * p->P[1] * n[2]);
      y = ny * x2;
      z = nz * x1;
    } else {
      x1 = (size_t)(H0 * N1);
      y = ny * x1;
    }
  } else if (dim == 3) {
    x1 = (size_t)(N0 * N1 * H);
    x2 = (size_t)(N0 * p->P[1] * H);
    y = ny * x2;
    z = nz * x1;
  } else {
    x1 = (size_t)(N0 * H);
    y = ny * x1;
  }
  auto align = [](size_t v) { return (v + 255) & ~(size_t)255; };
  p->off_x1 = 0;
  p->off_x2 = align(x1 * cb);
  p->off_y = p->off_x2 + align(x2 * cb);
  p->off_z = p->off_y + align(y * cb);
  p->off_phi = p->off_z + align(z * cb);
  const size_t ws_bytes = p->off_phi + (p->fd ? align((size_t)vol * rb) : 0);
  p->ws_bytes = ws_bytes;
  size_t tw_bytes = 0;
  for (int a = 0; a < dim; ++a) tw_bytes += (size_t)2 * p->P[a] * cb;
  p->bytes = ws_bytes + tw_bytes + (size_t)oct * (rb + 8) + (size_t)vol * 8;
  if (p->gradk) p->bytes += (size_t)dim * ((size_t)oct * (rb + 8) + (size_t)vol * 8);
  if (p->bytes > max_workspace_env()) {
    release(p);
    return VGF_ERR_OUT_OF_MEMORY;
  }

  hipError_t err = hipSuccess;
  vgf_status st = VGF_OK;
  do {
    if ((err = hipMalloc(&p->ws, ws_bytes)) != hipSuccess) break;
    if ((err = hipMalloc(&p->spec, (size_t)oct * rb)) != hipSuccess) break;
    if ((err = hipMalloc((void**)&p->spec64, (size_t)oct * 8)) != hipSuccess) break;
    if ((err = hipMalloc((void**)&p->w64, (size_t)vol * 8)) != hipSuccess) break;
    if (p->gradk) {
      if ((err = hipMalloc((void**)&p->wgrad64, (size_t)dim * vol * 8)) != hipSuccess) break;
      if ((err = hipMalloc((void**)&p->specg64, (size_t)dim * oct * 8)) != hipSuccess) break;
      if ((err = hipMalloc(&p->specg, (size_t)dim * oct * rb)) != hipSuccess) break;
    }
    for (int a = 0; a < dim && err == hipSuccess; ++a) {
      err = hipMalloc(&p->tw[a], (size_t)2 * p->P[a] * cb);
      if (err != hipSuccess) break;
      if (prec == VGF_F32) {
        std::vector<float2> t;
        if (!make_stage_twiddles<float>((int)p->P[a], t)) err = hipErrorInvalidValue;
        else err = hipMemcpy(p->tw[a], t.data(), t.size() * sizeof(t[0]), hipMemcpyHostToDevice);
      } else {
        std::vector<double2> t;
        if (!make_stage_twiddles<double>((int)p->P[a], t)) err = hipErrorInvalidValue;
        else err = hipMemcpy(p->tw[a], t.data(), t.size() * sizeof(t[0]), hipMemcpyHostToDevice);
      }
    }
  } while (false);
  if (err != hipSuccess) {
    st = err == hipErrorOutOfMemory ? VGF_ERR_OUT_OF_MEMORY : VGF_ERR_HIP;
    release(p);
    (void)hipGetLastError();
    return st;
  }
  st = precompute(p, stream);
  if (st != VGF_OK) {
    release(p);
    (void)hipGetLastError();
    return st;
  }
  {
    // set-up of vgf_solve_noalloc on this device: its scratch address is
    // looked up here, outside any solve (a failure is reported by that call)
    void* scratch_dev = nullptr;
    if (scratch_address(&scratch_dev) != hipSuccess) (void)hipGetLastError();
  }
  *out = p;
  return VGF_OK;
}

vgf_status vgf_solve(vgf_plan p, const void* rho, void* phi, void* E, hipStream_t stream) {
  vgf_status st = check_solve_args(p, rho, phi, E);
  if (st != VGF_OK) return st;
  if (p->prec == VGF_F32)
    return solve_t<float>(p, (const float*)rho, (float*)phi, (float*)E, stream, (char*)p->ws);
  return solve_t<double>(p, (const double*)rho, (double*)phi, (double*)E, stream, (char*)p->ws);
}

vgf_status vgf_solve_noalloc(vgf_plan p, const void* rho, void* phi, void* E, hipStream_t stream) {
  vgf_status st = check_solve_args(p, rho, phi, E);
  if (st != VGF_OK) return st;
  if (p->ws_bytes > kScratchBytes) return VGF_ERR_SCRATCH_LIMIT;
  void* ws = nullptr;
  hipError_t e = scratch_address(&ws);
  if (e != hipSuccess) return hip_status(p, e);
  if (p->prec == VGF_F32)
    return solve_t<float>(p, (const float*)rho, (float*)phi, (float*)E, stream, (char*)ws);
  return solve_t<double>(p, (const double*)rho, (double*)phi, (double*)E, stream, (char*)ws);
}

vgf_status vgf_solve_adjoint(vgf_plan p, const void* g_phi, const void* g_E, void* g_rho,
                             hipStream_t stream) {
  if (!p || !g_rho || (!g_phi && !g_E)) return VGF_ERR_INVALID_ARG;
  if (g_phi && !(p->outputs & VGF_OUT_PHI)) return VGF_ERR_NOT_REQUESTED;
  if (g_E && !(p->outputs & VGF_OUT_E)) return VGF_ERR_NOT_REQUESTED;
  if (p->fd && g_E) {
    // E = -D phi, so the field's cotangent reaches phi as -D^T g_E
    void* tmp = (char*)p->ws + p->off_phi;
    hipError_t e = p->prec == VGF_F32
                       ? vgf::launch_fd_adjoint<float>((const float*)g_phi, (const float*)g_E, (float*)tmp,
                                                       fd_geom(p), stream)
                       : vgf::launch_fd_adjoint<double>((const double*)g_phi, (const double*)g_E,
                                                        (double*)tmp, fd_geom(p), stream);
    if (e != hipSuccess) return hip_status(p, e);
    g_phi = tmp;
    g_E = nullptr;
  }
  if (p->prec == VGF_F32)
    return adjoint_t<float>(p, (const float*)g_phi, (const float*)g_E, (float*)g_rho, stream);
  return adjoint_t<double>(p, (const double*)g_phi, (const double*)g_E, (double*)g_rho, stream);
}

vgf_status vgf_solve_batched(const vgf_plan* plans, int count, const void* const* rho,
                             void* const* phi, void* const* E, hipStream_t stream) {
  if (count < 0 || (count > 0 && (!plans || !rho))) return VGF_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i) {
    vgf_status st = check_solve_args(plans[i], rho[i], phi ? phi[i] : nullptr, E ? E[i] : nullptr);
    if (st != VGF_OK) return st;
  }
  for (int i = 0; i < count; ++i) {
    vgf_status st = vgf_solve(plans[i], rho[i], phi ? phi[i] : nullptr, E ? E[i] : nullptr, stream);
    if (st != VGF_OK) return st;
  }
  return VGF_OK;
}

vgf_status vgf_plan_autotune(vgf_plan p, const void* rho, void* phi, void* E, int reps, hipStream_t stream) {
  vgf_status st = check_solve_args(p, rho, phi, E);
  if (st != VGF_OK) return st;
  if (reps <= 0) return VGF_ERR_INVALID_ARG;
  if (p->fd && E) {  // the tuned passes compute phi; the field is a separate kernel
    if (!phi) phi = (char*)p->ws + p->off_phi;
    E = nullptr;
  }
  auto run = [&](const int* sched, hipEvent_t* ev, int* tg) -> vgf_status {
    if (p->prec == VGF_F32) {
      Entries<float> en;
      en.ws = (char*)p->ws;
      en.rho = (const float*)rho;
      en.phi = (float*)phi;
      en.E = (float*)E;
      en.want_phi = phi != nullptr;
      en.want_E = E != nullptr;
      return enqueue_solve<float>(p, en, stream, false, sched, ev, tg);
    }
    Entries<double> en;
    en.ws = (char*)p->ws;
    en.rho = (const double*)rho;
    en.phi = (double*)phi;
    en.E = (double*)E;
    en.want_phi = phi != nullptr;
    en.want_E = E != nullptr;
    return enqueue_solve<double>(p, en, stream, false, sched, ev, tg);
  };
  hipError_t herr = hipSuccess;
  st = tune_cached(p, phi != nullptr, E != nullptr, 1, reps, stream, run, p->schedule, &herr);
  if (herr != hipSuccess) p->last_err = herr;
  return st;
}

vgf_status vgf_plan_get_schedule(vgf_plan p, int* schedule) {
  if (!p || !schedule) return VGF_ERR_INVALID_ARG;
  for (int k = 0; k < kPasses; ++k) schedule[k] = p->schedule[k];
  return VGF_OK;
}

vgf_status vgf_plan_set_schedule(vgf_plan p, const int* schedule) {
  if (!p || !schedule) return VGF_ERR_INVALID_ARG;
  for (int k = 0; k < kPasses; ++k) {
    if (schedule[k] < 0 || schedule[k] >= kScheduleValues) return VGF_ERR_INVALID_ARG;
    if (schedule[k] != 0 && !pass_tunable(p, k)) return VGF_ERR_INVALID_ARG;
  }
  for (int k = 0; k < kPasses; ++k) p->schedule[k] = schedule[k];
  return VGF_OK;
}

vgf_status vgf_plan_get_L(vgf_plan p, double* L) {
  if (!p || !L) return VGF_ERR_INVALID_ARG;
  *L = p->L;
  return VGF_OK;
}

vgf_status vgf_plan_workspace_bytes(vgf_plan p, size_t* bytes) {
  if (!p || !bytes) return VGF_ERR_INVALID_ARG;
  *bytes = p->bytes;
  return VGF_OK;
}

vgf_status vgf_plan_get_kernel(vgf_plan p, double* host_out) {
  if (!p || !host_out) return VGF_ERR_INVALID_ARG;
  const size_t cnt = (size_t)prod(p->n, p->dim);
  return hip_status(p, hipMemcpy(host_out, p->w64, cnt * sizeof(double), hipMemcpyDeviceToHost));
}

vgf_status vgf_plan_get_spectrum(vgf_plan p, double* host_out) {
  if (!p || !host_out) return VGF_ERR_INVALID_ARG;
  size_t cnt = 1;
  for (int a = 0; a < p->dim; ++a) cnt *= (size_t)(p->n[a] + 1);
  return hip_status(p, hipMemcpy(host_out, p->spec64, cnt * sizeof(double), hipMemcpyDeviceToHost));
}

vgf_status vgf_plan_get_gradient_kernel(vgf_plan p, int axis, double* host_out) {
  if (!p || !host_out || axis < 0 || axis >= p->dim) return VGF_ERR_INVALID_ARG;
  if (!p->gradk) return VGF_ERR_NOT_REQUESTED;
  const size_t cnt = (size_t)prod(p->n, p->dim);
  return hip_status(p, hipMemcpy(host_out, p->wgrad64 + axis * cnt, cnt * sizeof(double),
                                 hipMemcpyDeviceToHost));
}

vgf_status vgf_plan_get_gradient_spectrum(vgf_plan p, int axis, double* host_out) {
  if (!p || !host_out || axis < 0 || axis >= p->dim) return VGF_ERR_INVALID_ARG;
  if (!p->gradk) return VGF_ERR_NOT_REQUESTED;
  size_t cnt = 1;
  for (int a = 0; a < p->dim; ++a) cnt *= (size_t)(p->n[a] + 1);
  return hip_status(p, hipMemcpy(host_out, p->specg64 + axis * cnt, cnt * sizeof(double),
                                 hipMemcpyDeviceToHost));
}

vgf_status vgf_plan_profile_begin(vgf_plan p, int max_solves) {
  if (!p || max_solves <= 0 || p->profiling) return VGF_ERR_INVALID_ARG;
  p->prof_events.assign((size_t)max_solves * kMaxMarks, nullptr);
  p->prof_tags.assign((size_t)max_solves * kMaxMarks, -1);
  for (size_t i = 0; i < p->prof_events.size(); ++i) {
    hipError_t e = hipEventCreate(&p->prof_events[i]);
    if (e != hipSuccess) {
      for (size_t k = 0; k < i; ++k) (void)hipEventDestroy(p->prof_events[k]);
      p->prof_events.clear();
      return hip_status(p, e);
    }
  }
  p->prof_cap = max_solves;
  p->prof_used = 0;
  p->prof_nlaunch = 0;
  p->profiling = true;
  return VGF_OK;
}

vgf_status vgf_plan_profile_end(vgf_plan p, double* launch_ms, int* launch_pass, int* nlaunch, int* nsolves) {
  if (!p || !launch_ms || !launch_pass || !nlaunch || !nsolves || !p->profiling) return VGF_ERR_INVALID_ARG;
  hipError_t err = hipSuccess;
  const int nl = p->prof_nlaunch;
  for (int k = 0; k < kMaxLaunches; ++k) {
    launch_ms[k] = 0.0;
    launch_pass[k] = -1;
  }
  for (int sIdx = 0; sIdx < p->prof_used && err == hipSuccess; ++sIdx) {
    hipEvent_t* ev = &p->prof_events[(size_t)sIdx * kMaxMarks];
    err = hipEventSynchronize(ev[nl]);
    for (int k = 0; k < nl && err == hipSuccess; ++k) {
      float ms = 0.f;
      err = hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
      launch_ms[k] += ms;
    }
  }
  if (err == hipSuccess && p->prof_used > 0)
    for (int k = 0; k < nl; ++k) {
      launch_ms[k] /= p->prof_used;
      launch_pass[k] = p->prof_tags[k];
    }
  *nlaunch = nl;
  *nsolves = p->prof_used;
  for (hipEvent_t ev : p->prof_events) (void)hipEventDestroy(ev);
  p->prof_events.clear();
  p->prof_tags.clear();
  p->profiling = false;
  p->prof_cap = p->prof_used = 0;
  return hip_status(p, err);
}

int vgf_plan_hip_error(vgf_plan p) { return p ? (int)p->last_err : (int)hipErrorInvalidValue; }

void vgf_plan_destroy(vgf_plan p) { release(p); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches: many right-hand sides, possibly of different plans (uneven grid
// sizes). Entries that share a plan form a group, and each pass of a group
// runs as one launch over all of its entries (workspaces one entry apart,
// per-entry rho / phi / E base pointers in device tables). Groups are
// independent, so with VGF_BATCH_GRAPH they are captured as parallel
// branches of one hipGraph, which every later solve replays; the tables are
// refreshed on the solve stream before the replay whenever the caller's
// pointers change.
// ---------------------------------------------------------------------------
struct vgf_batch_s {
  struct Group {
    vgf_plan plan = nullptr;
    std::vector<int> idx;        // entry indices, in order
    void* ws = nullptr;          // idx.size() x plan->ws_bytes
    void** tab = nullptr;        // device [3][count]: rho, phi, E
    hipStream_t st = nullptr;    // capture branch
    hipEvent_t done = nullptr;
    int schedule[5] = {0, 0, 0, 0, 0};  // tile variants of the group's launches
  };
  int count = 0;
  unsigned flags = 0;
  std::vector<Group> groups;
  std::vector<void*> cur;        // pointers in the tables, group order [3][count]
  bool tab_valid = false;
  hipStream_t cs = nullptr;      // capture origin
  hipEvent_t fork = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_outputs = -1;        // outputs of the captured graph
  size_t bytes = 0;
  hipError_t last_err = hipSuccess;
};

namespace {

vgf_status batch_hip(vgf_batch b, hipError_t e) {
  if (e == hipSuccess) return VGF_OK;
  b->last_err = e;
  return VGF_ERR_HIP;
}

void batch_drop_graph(vgf_batch b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_outputs = -1;
}

void batch_release(vgf_batch b) {
  if (!b) return;
  batch_drop_graph(b);
  for (auto& g : b->groups) {
    if (g.ws) (void)hipFree(g.ws);
    if (g.tab) (void)hipFree(g.tab);
    if (g.st) (void)hipStreamDestroy(g.st);
    if (g.done) (void)hipEventDestroy(g.done);
  }
  if (b->cs) (void)hipStreamDestroy(b->cs);
  if (b->fork) (void)hipEventDestroy(b->fork);
  delete b;
}

// the passes of one group, all entries per launch
template <typename T>
vgf_status batch_group_enqueue(const vgf_batch_s::Group& g, bool want_phi, bool want_E, hipStream_t s,
                               const int* sched = nullptr, hipEvent_t* marks = nullptr, int* tags = nullptr) {
  const vgf_plan p = g.plan;
  const int c = (int)g.idx.size();
  Entries<T> en;
  en.count = c;
  en.ws = (char*)g.ws;
  en.es = (int64_t)(p->ws_bytes / sizeof(cplx<T>));
  en.rho_tab = (const T* const*)g.tab;
  en.phi_tab = want_phi ? (T* const*)(g.tab + c) : nullptr;
  en.E_tab = want_E ? (T* const*)(g.tab + 2 * c) : nullptr;
  en.want_phi = want_phi;
  en.want_E = want_E;
  if (!(p->fd && want_E)) return enqueue_solve<T>(p, en, s, false, sched ? sched : g.schedule, marks, tags);
  // finite-difference field: phi of every entry (the tables hold the
  // workspace arrays when phi is not wanted), then E = -D phi over all entries
  en.phi_tab = (T* const*)(g.tab + c);
  en.want_phi = true;
  en.E_tab = nullptr;
  en.want_E = false;
  vgf_status st = enqueue_solve<T>(p, en, s, false, sched ? sched : g.schedule, marks, tags);
  if (st != VGF_OK) return st;
  return hip_status(p, vgf::launch_fd_field_entries<T>((const T* const*)(g.tab + c), (T* const*)(g.tab + 2 * c),
                                                       c, fd_geom(p), s));
}

// Adjoint of every entry of a default-layout group with Fourier fields in
// one launch per pass (tables: [g_rho | g_phi | g_E]).
template <typename T>
vgf_status batch_group_adjoint(const vgf_batch_s::Group& g, bool has_phi, bool has_E, hipStream_t s) {
  const vgf_plan p = g.plan;
  const int c = (int)g.idx.size();
  AdjEntries<T> en;
  en.count = c;
  en.ws = (char*)g.ws;
  en.es = (int64_t)(p->ws_bytes / sizeof(cplx<T>));
  en.g_rho_tab = (T* const*)g.tab;
  en.g_phi_tab = has_phi ? (const T* const*)(g.tab + c) : nullptr;
  en.g_E_tab = has_E ? (const T* const*)(g.tab + 2 * c) : nullptr;
  en.has_phi = has_phi;
  en.has_E = has_E;
  return adjoint_c_entries<T>(p, en, g.schedule, s);
}

vgf_status batch_enqueue_groups(vgf_batch b, bool want_phi, bool want_E, bool branches, hipStream_t s) {
  for (auto& g : b->groups) {
    hipStream_t gs = branches ? g.st : s;
    if (branches) {
      hipError_t e = hipStreamWaitEvent(gs, b->fork, 0);
      if (e != hipSuccess) return batch_hip(b, e);
    }
    vgf_status st = g.plan->prec == VGF_F32 ? batch_group_enqueue<float>(g, want_phi, want_E, gs)
                                            : batch_group_enqueue<double>(g, want_phi, want_E, gs);
    if (st != VGF_OK) {
      if (st == VGF_ERR_HIP) b->last_err = g.plan->last_err;
      return st;
    }
    if (branches) {
      hipError_t e = hipEventRecord(g.done, gs);
      if (e == hipSuccess) e = hipStreamWaitEvent(b->cs, g.done, 0);
      if (e != hipSuccess) return batch_hip(b, e);
    }
  }
  return VGF_OK;
}

vgf_status batch_capture(vgf_batch b, bool want_phi, bool want_E) {
  batch_drop_graph(b);
  hipError_t e = hipStreamBeginCapture(b->cs, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) return batch_hip(b, e);
  vgf_status st = VGF_OK;
  // several groups run as parallel branches (fork / join events); a single
  // group is captured as one chain of launches, without event nodes
  const bool branches = b->groups.size() > 1;
  if (branches) {
    e = hipEventRecord(b->fork, b->cs);
    if (e != hipSuccess) st = batch_hip(b, e);
  }
  if (st == VGF_OK) st = batch_enqueue_groups(b, want_phi, want_E, branches, b->cs);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(b->cs, &graph);  // always ends the capture
  if (st == VGF_OK && e != hipSuccess) st = batch_hip(b, e);
  if (st != VGF_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    return st;
  }
  b->graph = graph;
  e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    batch_drop_graph(b);
    return batch_hip(b, e);
  }
  b->graph_outputs = (want_phi ? 1 : 0) | (want_E ? 2 : 0);
  return VGF_OK;
}

vgf_status batch_write_tables(vgf_batch b, const std::vector<void*>& ptrs, hipStream_t stream);

// Validates one call's pointers and refreshes the device pointer tables on
// `stream` when they differ from the last ones written.
vgf_status batch_set_tables(vgf_batch b, const void* const* rho, void* const* phi, void* const* E,
                            hipStream_t stream) {
  if (!b || !rho || (!phi && !E)) return VGF_ERR_INVALID_ARG;
  const bool want_phi = phi != nullptr, want_E = E != nullptr;
  const int n = b->count;
  std::vector<void*> ptrs((size_t)3 * n, nullptr);
  size_t k = 0;
  for (auto& g : b->groups) {
    const size_t c = g.idx.size();
    for (size_t j = 0; j < c; ++j) {
      const int i = g.idx[j];
      vgf_status st = check_solve_args(g.plan, rho[i], want_phi ? phi[i] : nullptr, want_E ? E[i] : nullptr);
      if (st != VGF_OK) return st;
      if (want_phi != (phi && phi[i]) || want_E != (E && E[i])) return VGF_ERR_INVALID_ARG;
      ptrs[k + j] = const_cast<void*>(rho[i]);
      // a finite-difference group always has a phi per entry: the field is
      // taken from it (the entry's workspace array when phi is not wanted)
      ptrs[k + c + j] = want_phi ? phi[i]
                        : g.plan->fd ? (char*)g.ws + j * g.plan->ws_bytes + g.plan->off_phi
                                     : nullptr;
      ptrs[k + 2 * c + j] = want_E ? E[i] : nullptr;
    }
    k += 3 * c;
  }
  return batch_write_tables(b, ptrs, stream);
}

// Writes the per-group pointer tables ([3][count] per group, group order)
// on `stream` unless they already hold `ptrs`.
vgf_status batch_write_tables(vgf_batch b, const std::vector<void*>& ptrs, hipStream_t stream) {
  if (b->tab_valid && ptrs == b->cur) return VGF_OK;
  size_t k = 0;
  for (auto& g : b->groups) {
    const size_t c3 = 3 * g.idx.size();
    for (size_t o = 0; o < c3; o += vgf::PtrChunk::kMax) {
      vgf::PtrChunk ch{};
      ch.n = (int)std::min<size_t>(vgf::PtrChunk::kMax, c3 - o);
      for (int j = 0; j < ch.n; ++j) ch.p[j] = ptrs[k + o + j];
      hipError_t e = vgf::launch_set_pointers(g.tab + o, ch, stream);
      if (e != hipSuccess) {
        b->tab_valid = false;
        return batch_hip(b, e);
      }
    }
    k += c3;
  }
  b->cur = ptrs;
  b->tab_valid = true;
  return VGF_OK;
}

}  // namespace

extern "C" {

vgf_status vgf_batch_create(vgf_batch* out, const vgf_plan* plans, int count, unsigned flags) {
  if (!out) return VGF_ERR_INVALID_ARG;
  *out = nullptr;
  if (count <= 0 || !plans || (flags & ~(unsigned)VGF_BATCH_GRAPH)) return VGF_ERR_INVALID_ARG;
  for (int i = 0; i < count; ++i)
    if (!plans[i]) return VGF_ERR_INVALID_ARG;
  vgf_batch b = new (std::nothrow) vgf_batch_s();
  if (!b) return VGF_ERR_OUT_OF_MEMORY;
  b->count = count;
  b->flags = flags;
  // group by plan, first appearance order; a group's strided launches cover
  // (n0 + 1) x entries batches, at most 65535
  for (int i = 0; i < count; ++i) {
    const vgf_plan p = plans[i];
    const int cap = (int)std::max<int64_t>(1, 65535 / (p->n[0] + 1));
    vgf_batch_s::Group* hit = nullptr;
    for (auto& g : b->groups)
      if (g.plan == p && (int)g.idx.size() < cap) hit = &g;
    if (!hit) {
      b->groups.emplace_back();
      hit = &b->groups.back();
      hit->plan = p;
      for (int k = 0; k < kPasses; ++k) hit->schedule[k] = p->schedule[k];
    }
    hit->idx.push_back(i);
  }
  hipError_t e = hipSuccess;
  for (auto& g : b->groups) {
    const size_t c = g.idx.size();
    const size_t wsb = c * g.plan->ws_bytes;
    if (b->bytes + wsb > max_workspace_env()) {
      batch_release(b);
      return VGF_ERR_OUT_OF_MEMORY;
    }
    b->bytes += wsb + 3 * c * sizeof(void*);
    if ((e = hipMalloc(&g.ws, wsb)) != hipSuccess) break;
    if ((e = hipMalloc((void**)&g.tab, 3 * c * sizeof(void*))) != hipSuccess) break;
    if ((e = hipStreamCreateWithFlags(&g.st, hipStreamNonBlocking)) != hipSuccess) break;
    if ((e = hipEventCreateWithFlags(&g.done, hipEventDisableTiming)) != hipSuccess) break;
  }
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  if (e != hipSuccess) {
    batch_release(b);
    (void)hipGetLastError();
    return e == hipErrorOutOfMemory ? VGF_ERR_OUT_OF_MEMORY : VGF_ERR_HIP;
  }
  *out = b;
  return VGF_OK;
}

vgf_status vgf_batch_solve(vgf_batch b, const void* const* rho, void* const* phi, void* const* E,
                           hipStream_t stream) {
  vgf_status st = batch_set_tables(b, rho, phi, E, stream);
  if (st != VGF_OK) return st;
  const bool want_phi = phi != nullptr, want_E = E != nullptr;
  if (!(b->flags & VGF_BATCH_GRAPH)) return batch_enqueue_groups(b, want_phi, want_E, false, stream);
  const int outs = (want_phi ? 1 : 0) | (want_E ? 2 : 0);
  if (!b->exec || b->graph_outputs != outs) {
    st = batch_capture(b, want_phi, want_E);
    if (st != VGF_OK) return st;
  }
  return batch_hip(b, hipGraphLaunch(b->exec, stream));
}

vgf_status vgf_batch_adjoint(vgf_batch b, const void* const* g_phi, const void* const* g_E, void* const* g_rho,
                             hipStream_t stream) {
  if (!b || !g_rho || (!g_phi && !g_E)) return VGF_ERR_INVALID_ARG;
  // validate every entry before anything is enqueued
  for (auto& g : b->groups)
    for (int i : g.idx) {
      if (!g_rho[i] || (g_phi && !g_phi[i]) || (g_E && !g_E[i])) return VGF_ERR_INVALID_ARG;
      if (g_phi && !(g.plan->outputs & VGF_OUT_PHI)) return VGF_ERR_NOT_REQUESTED;
      if (g_E && !(g.plan->outputs & VGF_OUT_E)) return VGF_ERR_NOT_REQUESTED;
    }
  std::vector<void*> ptrs((size_t)3 * b->count, nullptr);
  size_t k = 0;
  for (auto& g : b->groups) {
    const size_t c = g.idx.size();
    for (size_t j = 0; j < c; ++j) {
      const int i = g.idx[j];
      ptrs[k + j] = g_rho[i];
      ptrs[k + c + j] = g_phi ? const_cast<void*>(g_phi[i]) : nullptr;
      ptrs[k + 2 * c + j] = g_E ? const_cast<void*>(g_E[i]) : nullptr;
    }
    k += 3 * c;
  }
  vgf_status st = batch_write_tables(b, ptrs, stream);
  if (st != VGF_OK) return st;
  for (auto& g : b->groups) {
    const vgf_plan p = g.plan;
    if (p->contig && !p->fd && !p->gradk) {
      st = p->prec == VGF_F32 ? batch_group_adjoint<float>(g, g_phi != nullptr, g_E != nullptr, stream)
                              : batch_group_adjoint<double>(g, g_phi != nullptr, g_E != nullptr, stream);
      if (st == VGF_ERR_HIP) b->last_err = p->last_err;
      if (st != VGF_OK) return st;
      continue;
    }
    // other plans: one adjoint per entry on the plan's own workspace
    for (int i : g.idx) {
      st = vgf_solve_adjoint(p, g_phi ? g_phi[i] : nullptr, g_E ? g_E[i] : nullptr, g_rho[i], stream);
      if (st == VGF_ERR_HIP) b->last_err = p->last_err;
      if (st != VGF_OK) return st;
    }
  }
  return VGF_OK;
}

vgf_status vgf_batch_autotune(vgf_batch b, const void* const* rho, void* const* phi, void* const* E,
                              int reps, hipStream_t stream) {
  if (!b || reps <= 0) return VGF_ERR_INVALID_ARG;
  vgf_status st = batch_set_tables(b, rho, phi, E, stream);
  if (st != VGF_OK) return st;
  for (auto& g : b->groups) {
    const int count = (int)g.idx.size();
    // a finite-difference group tunes the passes of phi (the field is a
    // separate kernel; the tables hold a phi for every entry)
    const bool want_phi = phi != nullptr || g.plan->fd, want_E = E != nullptr && !g.plan->fd;
    auto run = [&](const int* sched, hipEvent_t* ev, int* tg) -> vgf_status {
      vgf_status r = g.plan->prec == VGF_F32
                         ? batch_group_enqueue<float>(g, want_phi, want_E, stream, sched, ev, tg)
                         : batch_group_enqueue<double>(g, want_phi, want_E, stream, sched, ev, tg);
      if (r == VGF_ERR_HIP) b->last_err = g.plan->last_err;
      return r;
    };
    hipError_t herr = hipSuccess;
    st = tune_cached(g.plan, want_phi, want_E, count, reps, stream, run, g.schedule, &herr);
    if (st != VGF_OK) {
      if (herr != hipSuccess) b->last_err = herr;
      return st;
    }
  }
  batch_drop_graph(b);  // the next solve captures the tuned launches
  return VGF_OK;
}

vgf_status vgf_batch_get_schedule(vgf_batch b, int group, int* schedule) {
  if (!b || !schedule || group < 0 || group >= (int)b->groups.size()) return VGF_ERR_INVALID_ARG;
  for (int k = 0; k < kPasses; ++k) schedule[k] = b->groups[(size_t)group].schedule[k];
  return VGF_OK;
}

vgf_status vgf_batch_workspace_bytes(vgf_batch b, size_t* bytes) {
  if (!b || !bytes) return VGF_ERR_INVALID_ARG;
  *bytes = b->bytes;
  return VGF_OK;
}

int vgf_batch_groups(vgf_batch b) { return b ? (int)b->groups.size() : 0; }

int vgf_batch_hip_error(vgf_batch b) { return b ? (int)b->last_err : (int)hipErrorInvalidValue; }

void vgf_batch_destroy(vgf_batch b) { batch_release(b); }

}  // extern "C"
