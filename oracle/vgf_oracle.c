/*
 * vgf_oracle.c -- plain, slow, FP64 CPU oracle for the free-space Poisson
 * solvers compared in Zou, Kim & Cerfon, "FFT-based free space Poisson
 * solvers: why Vico-Greengard-Ferrando should replace Hockney-Eastwood"
 * (arXiv:2103.08531).
 *
 * THIS FILE IS TEST INFRASTRUCTURE. Only the test suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it. It shares no code, table
 * or helper with the GPU library, and the GPU library never calls it.
 *
 * Everything is double precision, written as the plain definitions:
 *   - the windowed-kernel spectrum in closed form (Eqs. 7-8, Sec. II);
 *   - the VGF "numerical Green's function": the inverse DFT of that spectrum
 *     on the 4N-oversampled grid, restricted to offsets |n_a| <= N_a-1
 *     (Sec. II, last paragraph), evaluated as explicit cosine sums;
 *   - the Hockney-Eastwood kernel h^d G(|n h|) with the origin regularised
 *     (Eq. 3 and the text after it, Sec. I);
 *   - the potential as the direct discrete convolution of that kernel with
 *     rho (the trapezoidal discretisation of Eq. 2 / Eq. 6);
 *   - the field E = -grad phi by Fourier differentiation on the 2N solve grid
 *     (Sec. III.A), written without an FFT as the periodic spectral
 *     differentiation stencil (Trefethen, Spectral Methods in MATLAB, ch. 3);
 *   - an independent naive mixed-radix (2,3) FFT used for the 2N and the 4N
 *     ("in principle", Sec. II) paths, so that direct sums, the 2N path and
 *     the 4N path check each other;
 *   - the adjoint operators, by direct transposed sums;
 *   - the closed-form Gaussian potentials used in Sec. III (Eqs. 10-11,
 *     14-15), and a 1-D integral for the anisotropic Gaussian.
 *
 * Arrays are C-contiguous, last axis fastest. dim is 2 or 3. For dim == 2
 * only n[0], n[1] (and h[0], h[1]) are read.
 *
 *   - the Hockney-Eastwood variants of the comparison figures (Sec. III.A):
 *     "nearby value" (G at half a spacing) and "cell average" (the integral
 *     of G over the origin cell, by pyramids and Gauss-Legendre), and the
 *     second-order finite-difference field and its transpose.
 *
 * Parity unpinned: the Hockney-Eastwood origin constant G0 (1/(4 pi) in 3D,
 * 1/(2 pi) in 2D) is a reading of the paper's "G(0)=1" and its figure legend;
 * nothing outside the paper fixes it. Likewise the "nearby value" distance
 * (half the smallest spacing) is a reading of a figure legend.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define ORC_PI 3.14159265358979323846264338327950288
#define ORC_PI_L 3.14159265358979323846264338327950288L
#define ORC_EULER_GAMMA 0.57721566490153286060651209008240243

/* ------------------------------------------------------------------------ */
/* small helpers                                                             */
/* ------------------------------------------------------------------------ */

static int64_t prod(int dim, const int64_t* n) {
  int64_t p = 1;
  for (int a = 0; a < dim; ++a) p *= n[a];
  return p;
}

/* linear index -> multi-index for a C-contiguous array of shape n[0..dim) */
static void unravel(int dim, const int64_t* n, int64_t lin, int64_t* idx) {
  for (int a = dim - 1; a >= 0; --a) {
    idx[a] = lin % n[a];
    lin /= n[a];
  }
}

static int64_t ravel(int dim, const int64_t* n, const int64_t* idx) {
  int64_t lin = 0;
  for (int a = 0; a < dim; ++a) lin = lin * n[a] + idx[a];
  return lin;
}

/* Neumaier compensated summation */
typedef struct { double s, c; } ksum;
static inline void kadd(ksum* k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x))
    k->c += (k->s - t) + x;
  else
    k->c += (x - t) + k->s;
  k->s = t;
}
static inline double kval(const ksum* k) { return k->s + k->c; }

/* cos and sin of 2*pi*t/n with t reduced modulo n, evaluated in long double
 * and rounded once, so every table entry is (close to) correctly rounded. */
static void cis_frac(int64_t t, int64_t n, double* c, double* s) {
  t %= n;
  if (t < 0) t += n;
  long double ang = 2.0L * ORC_PI_L * (long double)t / (long double)n;
  *c = (double)cosl(ang);
  *s = (double)sinl(ang);
}

/* ------------------------------------------------------------------------ */
/* Windowed Green's function spectrum, Eqs. (7) and (8) (Sec. II)            */
/* ------------------------------------------------------------------------ */

/* F{G^L}(k) for the kernel G truncated at radius L.
 * 3D: 2 (sin(L k / 2) / k)^2, limit L^2/2 at k = 0.
 * 2D: (1 - J0(L k)) / k^2 - L ln(L) J1(L k) / k, limit L^2/4 - L^2 ln(L)/2. */
double orc_ghat(int dim, double L, double k) {
  if (dim == 3) {
    if (k == 0.0) return 0.5 * L * L;
    double s = sin(0.5 * L * k) / k;
    return 2.0 * s * s;
  }
  if (k == 0.0) return 0.25 * L * L - 0.5 * L * L * log(L);
  double x = L * k;
  return (1.0 - j0(x)) / (k * k) - L * log(L) * j1(x) / k;
}

/* Admissible window for L. The lower bound is the largest source-target
 * distance in the box (the paper's L > sqrt(d) for the unit box, Sec. II).
 * The upper bound keeps the period-(4 N_a h_a) images of the truncated kernel
 * away from the box, which is why the oversampled grid is 4N (Sec. II). */
void orc_window(int dim, const int64_t* n, const double* h, double* Lmin,
                double* Lmax) {
  double d2 = 0.0, up = INFINITY;
  for (int a = 0; a < dim; ++a) {
    double ext = (double)(n[a] - 1) * h[a];
    d2 += ext * ext;
    double u = 4.0 * (double)n[a] * h[a] - ext;
    if (u < up) up = u;
  }
  *Lmin = sqrt(d2);
  *Lmax = up;
}

/* ------------------------------------------------------------------------ */
/* Kernels on the solve grid                                                 */
/* ------------------------------------------------------------------------ */

/* VGF restricted kernel (Sec. II, last paragraph): the inverse DFT of
 * F{G^L}(k_m) over the (4N)^d grid, k_{m,a} = 2 pi m_a / (4 N_a h_a),
 * m_a in [-2N_a, 2N_a), kept at offsets n_a in [0, N_a) (it is even in each
 * axis, so this octant holds all of |n_a| <= N_a - 1):
 *
 *   w[n] = prod_a (4 N_a)^{-1} * sum_m F{G^L}(|k_m|) prod_a cos(2 pi m_a n_a / (4 N_a)).
 *
 * The spectrum is even in every m_a, so the sum over m_a in [-2N_a, 2N_a) is
 * f(0) + 2 sum_{m=1}^{2N-1} f(m) + f(2N) cos(pi n) (the -2N term appears once).
 * The d-fold sum factorises over axes in the cosine weights and is taken one
 * axis at a time, with compensated sums. w carries the h^d quadrature weight
 * implicitly. Output shape n[0..dim). */
static int vgf_kernel_impl(int dim, const int64_t* n, const double* h, double L, int odd_axis,
                           double* w);

int orc_vgf_kernel(int dim, const int64_t* n, const double* h, double L,
                   double* w) {
  return vgf_kernel_impl(dim, n, h, L, -1, w);
}

/* Gradient kernel of the field reading that transforms -i k_a times the
 * windowed spectrum instead of differentiating the potential on the 2N grid
 * (the alternative reading of "multiplying by the wavevector", Sec. III.A):
 *   w_a[n] = (prod_b 4N_b)^{-1} sum_m (-i k_{m,a}) Ghat(|k_m|) e^{i k_m . x_n},
 * restricted to n in [0, N)^d. The sum is real: pairing m_a with -m_a gives
 * 2 k_{m,a} sin(2 pi m_a n_a / 4N_a) along axis a (the m_a = 0 and -2N_a
 * terms vanish), the cosine weights of orc_vgf_kernel along the others.
 * w_a is odd in n_a and even in the other offsets; E_a = w_a * rho. */
int orc_vgf_grad_kernel(int dim, const int64_t* n, const double* h, double L, int axis,
                        double* w) {
  if (axis < 0 || axis >= dim) return -1;
  return vgf_kernel_impl(dim, n, h, L, axis, w);
}

static int vgf_kernel_impl(int dim, const int64_t* n, const double* h, double L, int odd_axis,
                           double* w) {
  if (dim != 2 && dim != 3) return -1;
  int64_t ms[3], cur[3];
  for (int a = 0; a < dim; ++a) ms[a] = 2 * n[a] + 1;
  int64_t total = prod(dim, ms);
  double* buf = (double*)malloc(sizeof(double) * (size_t)total);
  if (!buf) return -2;

  /* spectrum samples on the non-negative octant m in [0, 2N]^d */
#pragma omp parallel for schedule(static)
  for (int64_t lin = 0; lin < total; ++lin) {
    int64_t m[3];
    unravel(dim, ms, lin, m);
    double k2 = 0.0;
    for (int a = 0; a < dim; ++a) {
      double ka = 2.0 * ORC_PI * (double)m[a] / (4.0 * (double)n[a] * h[a]);
      k2 += ka * ka;
    }
    buf[lin] = orc_ghat(dim, L, sqrt(k2));
  }

  /* one axis at a time: m_a in [0, 2N_a] -> n_a in [0, N_a) */
  for (int a = 0; a < dim; ++a) cur[a] = ms[a];
  for (int a = 0; a < dim; ++a) {
    int64_t N = n[a], M = 4 * n[a];
    int64_t outer = 1, inner = 1;
    for (int b = 0; b < a; ++b) outer *= cur[b];
    for (int b = a + 1; b < dim; ++b) inner *= cur[b];
    int64_t in_len = cur[a];
    double* cosm = (double*)malloc(sizeof(double) * (size_t)(in_len * N));
    double* out = (double*)malloc(sizeof(double) * (size_t)(outer * N * inner));
    if (!cosm || !out) {
      free(cosm);
      free(out);
      free(buf);
      return -2;
    }
    for (int64_t m = 0; m < in_len; ++m)
      for (int64_t j = 0; j < N; ++j) {
        double c, s;
        cis_frac(m * j, M, &c, &s);
        if (a == odd_axis) {
          const double km = 2.0 * ORC_PI * (double)m / ((double)M * h[a]);
          cosm[m * N + j] = (m == 0 || m == 2 * N) ? 0.0 : 2.0 * km * s / (double)M;
        } else {
          double wgt = (m == 0 || m == 2 * N) ? 1.0 : 2.0;
          cosm[m * N + j] = wgt * c / (double)M;
        }
      }
    /* every output is one compensated sum over m in increasing order; the
     * loops run m outside i only so that rows are read contiguously */
#pragma omp parallel
    {
      ksum* acc = (ksum*)malloc(sizeof(ksum) * (size_t)inner);
#pragma omp for collapse(2) schedule(static)
      for (int64_t o = 0; o < outer; ++o)
        for (int64_t j = 0; j < N; ++j) {
          for (int64_t i = 0; i < inner; ++i) acc[i].s = acc[i].c = 0.0;
          for (int64_t m = 0; m < in_len; ++m) {
            const double cm = cosm[m * N + j];
            const double* row = buf + (o * in_len + m) * inner;
            for (int64_t i = 0; i < inner; ++i) kadd(&acc[i], cm * row[i]);
          }
          for (int64_t i = 0; i < inner; ++i) out[(o * N + j) * inner + i] = kval(&acc[i]);
        }
      free(acc);
    }
    free(cosm);
    free(buf);
    buf = out;
    cur[a] = N;
  }
  memcpy(w, buf, sizeof(double) * (size_t)prod(dim, n));
  free(buf);
  return 0;
}

/* Hockney-Eastwood kernel (Eq. 3): w[n] = (prod_a h_a) G(|n o h|) with
 * G = 1/(4 pi r) in 3D and -ln(r)/(2 pi) in 2D (Eq. 2). At the origin the
 * singular factor (1/r, resp. -ln r) is replaced by 1, i.e.
 * G0 = 1/(4 pi) in 3D and 1/(2 pi) in 2D (Sec. I, "G(0)=1", and the figure
 * legend of Sec. III.A). Parity unpinned beyond this convention.
 * Octant n_a in [0, N_a). */
/* Gauss-Legendre nodes and weights on [0, 1] (m points): Newton iteration
 * on P_m from the Chebyshev guesses, the three-term recurrence for P_m. */
static void gauss_legendre01(int m, double* x, double* wt) {
  for (int i = 0; i < m; ++i) {
    double z = cos(ORC_PI * (i + 0.75) / (m + 0.5)), dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= m; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = m * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= m; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = m * (z * p1 - p0) / (z * z - 1.0);
    }
    x[i] = 0.5 * (1.0 - z);
    wt[i] = 1.0 / ((1.0 - z * z) * dp * dp);  /* 2/((1-z^2)P'^2), halved for [0,1] */
  }
}

/* Integral of G over the cell prod_a [-h_a/2, h_a/2] around the origin,
 * by symmetry 2^d times the integral over the corner box [0, h_a/2]. The
 * corner box is split into d pyramids with apex at the origin, one per far
 * face; on the pyramid over the face x_a = c_a the points are t * (face
 * point), t in [0, 1]. The t-integral is done in closed form, leaving a
 * smooth integral over the face, done with tensor Gauss-Legendre:
 *   3D, G = 1/(4 pi r): int_0^1 t^2 c_a /(t R) dt = c_a / (2 R);
 *   2D, G = -ln(r)/(2 pi): int_0^1 t c_a (-ln t - ln R) dt = c_a (1/4 - ln(R)/2);
 * R = |face point|. */
double orc_cell_average_integral(int dim, const double* h) {
  enum { M = 48 };
  double x[M], wt[M];
  gauss_legendre01(M, x, wt);
  double c[3];
  for (int a = 0; a < dim; ++a) c[a] = 0.5 * h[a];
  double total = 0.0;
  if (dim == 3) {
    for (int a = 0; a < 3; ++a) {
      const double ca = c[a], cb = c[(a + 1) % 3], cc = c[(a + 2) % 3];
      double acc = 0.0;
      for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) {
          const double y = cb * x[i], z = cc * x[j];
          acc += wt[i] * wt[j] * ca / (2.0 * sqrt(ca * ca + y * y + z * z));
        }
      total += acc * cb * cc;
    }
    return 8.0 * total / (4.0 * ORC_PI);
  }
  for (int a = 0; a < 2; ++a) {
    const double ca = c[a], cb = c[1 - a];
    double acc = 0.0;
    for (int i = 0; i < M; ++i) {
      const double y = cb * x[i];
      acc += wt[i] * ca * (0.25 - 0.5 * log(sqrt(ca * ca + y * y)));
    }
    total += acc * cb;
  }
  return 4.0 * total / (2.0 * ORC_PI);
}

/* Origin weight w[0] of the Hockney-Eastwood kernel (Sec. I and the legends
 * of Sec. III.A):
 *   mode 0: the singular factor (1/r, -ln r) replaced by 1: vol * G0 with
 *           G0 = 1/(4 pi) in 3D, 1/(2 pi) in 2D;
 *   mode 1: "nearby value": vol * G(r0), r0 = half the smallest spacing;
 *   mode 2: "cell average": the integral of G over the cell around the
 *           origin (vol times the average of G over it). */
double orc_he_origin(int dim, const double* h, int mode) {
  double vol = 1.0, hmin = h[0];
  for (int a = 0; a < dim; ++a) {
    vol *= h[a];
    if (h[a] < hmin) hmin = h[a];
  }
  if (mode == 1) {
    const double r0 = 0.5 * hmin;
    return vol * (dim == 3 ? 1.0 / (4.0 * ORC_PI * r0) : -log(r0) / (2.0 * ORC_PI));
  }
  if (mode == 2) return orc_cell_average_integral(dim, h);
  return vol * ((dim == 3) ? 1.0 / (4.0 * ORC_PI) : 1.0 / (2.0 * ORC_PI));
}

int orc_he_kernel_mode(int dim, const int64_t* n, const double* h, int mode, double* w);

int orc_he_kernel(int dim, const int64_t* n, const double* h, double* w) {
  return orc_he_kernel_mode(dim, n, h, 0, w);
}

int orc_he_kernel_mode(int dim, const int64_t* n, const double* h, int mode, double* w) {
  if (dim != 2 && dim != 3) return -1;
  if (mode < 0 || mode > 2) return -1;
  double vol = 1.0;
  for (int a = 0; a < dim; ++a) vol *= h[a];
  int64_t total = prod(dim, n);
  for (int64_t lin = 0; lin < total; ++lin) {
    int64_t idx[3];
    unravel(dim, n, lin, idx);
    double r2 = 0.0;
    for (int a = 0; a < dim; ++a) {
      double x = (double)idx[a] * h[a];
      r2 += x * x;
    }
    if (lin == 0) {
      w[0] = orc_he_origin(dim, h, mode);
      continue;
    }
    const double g = (dim == 3) ? 1.0 / (4.0 * ORC_PI * sqrt(r2)) : -log(sqrt(r2)) / (2.0 * ORC_PI);
    w[lin] = vol * g;
  }
  return 0;
}

/* Finite-difference field E = -D phi (Sec. III.A, the "Finite Diff" curves):
 * along each axis a second-order centred difference (phi[i+1] - phi[i-1]) /
 * (2 h_a) at interior points and the second-order one-sided differences
 * (-3 phi[0] + 4 phi[1] - phi[2]) / (2 h_a) and
 * (3 phi[N-1] - 4 phi[N-2] + phi[N-3]) / (2 h_a) on the two end planes.
 * Needs N_a >= 3. E is planar [dim][n]. */
static double fd_coef(int64_t N, int64_t i, int64_t j) {
  /* D[i][j] * 2h */
  if (i == 0) return j == 0 ? -3.0 : (j == 1 ? 4.0 : (j == 2 ? -1.0 : 0.0));
  if (i == N - 1) return j == N - 1 ? 3.0 : (j == N - 2 ? -4.0 : (j == N - 3 ? 1.0 : 0.0));
  return j == i + 1 ? 1.0 : (j == i - 1 ? -1.0 : 0.0);
}

int orc_fd_field(int dim, const int64_t* n, const double* h, const double* phi, double* E) {
  if (dim != 2 && dim != 3) return -1;
  for (int a = 0; a < dim; ++a)
    if (n[a] < 3) return -1;
  const int64_t total = prod(dim, n);
  for (int a = 0; a < dim; ++a) {
    int64_t stride = 1;
    for (int b = a + 1; b < dim; ++b) stride *= n[b];
    for (int64_t lin = 0; lin < total; ++lin) {
      int64_t idx[3];
      unravel(dim, n, lin, idx);
      const int64_t i = idx[a], N = n[a];
      double acc = 0.0;
      for (int64_t j = 0; j < N; ++j) {
        const double c = fd_coef(N, i, j);
        if (c != 0.0) acc += c * phi[lin + (j - i) * stride];
      }
      E[a * total + lin] = -acc / (2.0 * h[a]);
    }
  }
  return 0;
}

/* Transpose: gphi = -sum_a D_a^T gE[a], by scattering each row's
 * coefficients (no use of the stencil's structure). */
int orc_fd_field_T(int dim, const int64_t* n, const double* h, const double* gE, double* gphi) {
  if (dim != 2 && dim != 3) return -1;
  for (int a = 0; a < dim; ++a)
    if (n[a] < 3) return -1;
  const int64_t total = prod(dim, n);
  memset(gphi, 0, sizeof(double) * (size_t)total);
  for (int a = 0; a < dim; ++a) {
    int64_t stride = 1;
    for (int b = a + 1; b < dim; ++b) stride *= n[b];
    for (int64_t lin = 0; lin < total; ++lin) {
      int64_t idx[3];
      unravel(dim, n, lin, idx);
      const int64_t i = idx[a], N = n[a];
      for (int64_t j = 0; j < N; ++j) {
        const double c = fd_coef(N, i, j);
        if (c != 0.0) gphi[lin + (j - i) * stride] -= c * gE[a * total + lin] / (2.0 * h[a]);
      }
    }
  }
  return 0;
}

/* 2N-periodic embedding of an even octant kernel: shape P_a = 2 N_a,
 * W[p] = w[|s|] with s_a the signed offset (p_a or p_a - P_a) when every
 * |s_a| <= N_a - 1, and W = 0 wherever some |s_a| = N_a (that offset is
 * never used by outputs in [0, N); fixing it to zero fixes the spectrum). */
void orc_periodic_kernel(int dim, const int64_t* n, const double* w_oct,
                         double* W) {
  int64_t P[3];
  for (int a = 0; a < dim; ++a) P[a] = 2 * n[a];
  int64_t total = prod(dim, P);
  for (int64_t lin = 0; lin < total; ++lin) {
    int64_t p[3], q[3];
    unravel(dim, P, lin, p);
    int zero = 0;
    for (int a = 0; a < dim; ++a) {
      if (p[a] == n[a]) zero = 1;
      q[a] = (p[a] < n[a]) ? p[a] : P[a] - p[a];
    }
    W[lin] = zero ? 0.0 : w_oct[ravel(dim, n, q)];
  }
}

/* Field kernel v_a = -D_a W on the 2N-periodic grid, where D_a is the
 * periodic spectral differentiation matrix along axis a (period P = 2N,
 * spacing h): (D u)[p] = sum_q d[p - q] u[q], d[0] = 0,
 * d[j] = (pi / (P h)) (-1)^j cot(pi j / P). This is Fourier differentiation
 * (multiplication by i k before the inverse transform, Sec. III.A) with the
 * Nyquist wavenumber's factor set to zero, written without an FFT. */
void orc_field_kernel(int dim, const int64_t* n, const double* h,
                      const double* W, int axis, double* v) {
  int64_t P[3];
  for (int a = 0; a < dim; ++a) P[a] = 2 * n[a];
  int64_t Pa = P[axis];
  double* d = (double*)malloc(sizeof(double) * (size_t)Pa);
  d[0] = 0.0;
  for (int64_t j = 1; j < Pa; ++j) {
    long double ang = ORC_PI_L * (long double)j / (long double)Pa;
    double cot = (double)(cosl(ang) / sinl(ang));
    double sgn = (j % 2 == 0) ? 1.0 : -1.0;
    d[j] = (ORC_PI / ((double)Pa * h[axis])) * sgn * cot;
  }
  int64_t total = prod(dim, P);
#pragma omp parallel for schedule(static)
  for (int64_t lin = 0; lin < total; ++lin) {
    int64_t p[3], q[3];
    unravel(dim, P, lin, p);
    for (int a = 0; a < dim; ++a) q[a] = p[a];
    ksum acc = {0.0, 0.0};
    for (int64_t t = 0; t < Pa; ++t) {
      q[axis] = t;
      int64_t j = ((p[axis] - t) % Pa + Pa) % Pa;
      kadd(&acc, d[j] * W[ravel(dim, P, q)]);
    }
    v[lin] = -kval(&acc);
  }
  free(d);
}

/* ------------------------------------------------------------------------ */
/* Direct discrete convolutions (the definitions the FFT paths must match)   */
/* ------------------------------------------------------------------------ */

/* phi_i = sum_{j in [0,N)^d} w[|i - j|] rho_j, w an even octant kernel. */
void orc_conv_direct(int dim, const int64_t* n, const double* w_oct,
                     const double* rho, double* phi) {
  int64_t total = prod(dim, n);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t li = 0; li < total; ++li) {
    int64_t i[3], j[3], q[3];
    unravel(dim, n, li, i);
    ksum acc = {0.0, 0.0};
    for (int64_t lj = 0; lj < total; ++lj) {
      unravel(dim, n, lj, j);
      for (int a = 0; a < dim; ++a) q[a] = i[a] >= j[a] ? i[a] - j[a] : j[a] - i[a];
      kadd(&acc, w_oct[ravel(dim, n, q)] * rho[lj]);
    }
    phi[li] = kval(&acc);
  }
}

/* out_i = sum_{j in [0,N)^d} V[(i - j) mod P] x_j, V a full 2N-periodic
 * kernel (shape 2 n). */
/* 2N-periodic embedding of a kernel odd in axis `axis` and even in the
 * others: W[p] = sign * w[|s|] with sign = -1 when s_axis < 0, and 0
 * wherever some |s_a| = N_a. */
void orc_periodic_kernel_odd(int dim, const int64_t* n, const double* w_oct, int axis,
                             double* W) {
  int64_t P[3];
  for (int a = 0; a < dim; ++a) P[a] = 2 * n[a];
  int64_t total = prod(dim, P);
  for (int64_t lin = 0; lin < total; ++lin) {
    int64_t p[3], q[3];
    unravel(dim, P, lin, p);
    int zero = 0;
    double sign = 1.0;
    for (int a = 0; a < dim; ++a) {
      if (p[a] == n[a]) zero = 1;
      q[a] = (p[a] < n[a]) ? p[a] : P[a] - p[a];
      if (a == axis && p[a] > n[a]) sign = -1.0;
    }
    W[lin] = zero ? 0.0 : sign * w_oct[ravel(dim, n, q)];
  }
}

void orc_conv_periodic(int dim, const int64_t* n, const double* V,
                       const double* x, double* out) {
  int64_t P[3];
  for (int a = 0; a < dim; ++a) P[a] = 2 * n[a];
  int64_t total = prod(dim, n);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t li = 0; li < total; ++li) {
    int64_t i[3], j[3], q[3];
    unravel(dim, n, li, i);
    ksum acc = {0.0, 0.0};
    for (int64_t lj = 0; lj < total; ++lj) {
      unravel(dim, n, lj, j);
      for (int a = 0; a < dim; ++a) q[a] = ((i[a] - j[a]) % P[a] + P[a]) % P[a];
      kadd(&acc, V[ravel(dim, P, q)] * x[lj]);
    }
    out[li] = kval(&acc);
  }
}

/* Transpose of the previous operator: out_j = sum_i V[(i - j) mod P] g_i. */
void orc_conv_periodic_T(int dim, const int64_t* n, const double* V,
                         const double* g, double* out) {
  int64_t P[3];
  for (int a = 0; a < dim; ++a) P[a] = 2 * n[a];
  int64_t total = prod(dim, n);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t lj = 0; lj < total; ++lj) {
    int64_t i[3], j[3], q[3];
    unravel(dim, n, lj, j);
    ksum acc = {0.0, 0.0};
    for (int64_t li = 0; li < total; ++li) {
      unravel(dim, n, li, i);
      for (int a = 0; a < dim; ++a) q[a] = ((i[a] - j[a]) % P[a] + P[a]) % P[a];
      kadd(&acc, V[ravel(dim, P, q)] * g[li]);
    }
    out[lj] = kval(&acc);
  }
}

/* One output point of the direct potential, for sampled checks on grids too
 * large for the full O(N^{2d}) sum. */
double orc_conv_direct_point(int dim, const int64_t* n, const double* w_oct,
                             const double* rho, const int64_t* i) {
  int64_t total = prod(dim, n);
  ksum acc = {0.0, 0.0};
  for (int64_t lj = 0; lj < total; ++lj) {
    int64_t j[3], q[3];
    unravel(dim, n, lj, j);
    for (int a = 0; a < dim; ++a) q[a] = i[a] >= j[a] ? i[a] - j[a] : j[a] - i[a];
    kadd(&acc, w_oct[ravel(dim, n, q)] * rho[lj]);
  }
  return kval(&acc);
}

/* ------------------------------------------------------------------------ */
/* Naive FFT (recursive decimation in time, radices 2 and 3, direct DFT for  */
/* any other factor). Unnormalised: y[k] = sum_j x[j] exp(sign 2 pi i jk/n).*/
/* ------------------------------------------------------------------------ */

/* Twiddle table of a top-level length n0: tab[t] = exp(sign 2 pi i t / n0),
 * t in [0, n0), each entry from cis_frac (long double, rounded once). A
 * sub-transform of length n = n0 / stride_t reads tab[(t mod n) * tstep]. */
static cplx* make_table(int64_t n0, int sign) {
  cplx* tab = (cplx*)malloc(sizeof(cplx) * (size_t)n0);
  for (int64_t t = 0; t < n0; ++t) {
    double c, s;
    cis_frac(t, n0, &c, &s);
    tab[t] = c + sign * s * I;
  }
  return tab;
}

static void fft_rec(int64_t n, const cplx* x, int64_t stride, cplx* y, const cplx* tab,
                    int64_t tstep) {
  if (n == 1) {
    y[0] = x[0];
    return;
  }
  int64_t r = (n % 2 == 0) ? 2 : ((n % 3 == 0) ? 3 : n);
  int64_t m = n / r;
  if (r == n) { /* direct DFT */
    for (int64_t k = 0; k < n; ++k) {
      cplx acc = 0.0;
      for (int64_t j = 0; j < n; ++j) acc += x[j * stride] * tab[((j * k) % n) * tstep];
      y[k] = acc;
    }
    return;
  }
  for (int64_t s = 0; s < r; ++s)
    fft_rec(m, x + s * stride, stride * r, y + s * m, tab, tstep * r);
  cplx t[3];
  for (int64_t k = 0; k < m; ++k) {
    for (int64_t s = 0; s < r; ++s) t[s] = y[s * m + k] * tab[((s * k) % n) * tstep];
    for (int64_t q = 0; q < r; ++q) {
      cplx acc = 0.0;
      for (int64_t s = 0; s < r; ++s) acc += t[s] * tab[((s * q * m) % n) * tstep];
      y[q * m + k] = acc;
    }
  }
}

/* In-place 1-D transform of length n (buffer passed as interleaved re,im). */
void orc_fft1d(int64_t n, double* xy, int sign) {
  cplx* x = (cplx*)xy;
  cplx* y = (cplx*)malloc(sizeof(cplx) * (size_t)n);
  cplx* tab = make_table(n, sign);
  fft_rec(n, x, 1, y, tab, 1);
  memcpy(x, y, sizeof(cplx) * (size_t)n);
  free(y);
  free(tab);
}

/* Textbook O(n^2) DFT, the brute-force check of orc_fft1d. */
void orc_dft1d(int64_t n, double* xy, int sign) {
  cplx* x = (cplx*)xy;
  cplx* y = (cplx*)malloc(sizeof(cplx) * (size_t)n);
  for (int64_t k = 0; k < n; ++k) {
    cplx acc = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      double c, s;
      cis_frac(j * k, n, &c, &s);
      acc += x[j] * (c + sign * s * I);
    }
    y[k] = acc;
  }
  memcpy(x, y, sizeof(cplx) * (size_t)n);
  free(y);
}

/* Unnormalised d-dimensional transform, one axis after the other. */
static void fftnd(int dim, const int64_t* shape, cplx* x, int sign) {
  for (int a = 0; a < dim; ++a) {
    int64_t len = shape[a], inner = 1, outer = 1;
    for (int b = a + 1; b < dim; ++b) inner *= shape[b];
    for (int b = 0; b < a; ++b) outer *= shape[b];
    cplx* tab = make_table(len, sign);
#pragma omp parallel
    {
      cplx* line = (cplx*)malloc(sizeof(cplx) * (size_t)len);
      cplx* res = (cplx*)malloc(sizeof(cplx) * (size_t)len);
#pragma omp for collapse(2) schedule(static)
      for (int64_t o = 0; o < outer; ++o)
        for (int64_t i = 0; i < inner; ++i) {
          cplx* base = x + o * len * inner + i;
          for (int64_t j = 0; j < len; ++j) line[j] = base[j * inner];
          fft_rec(len, line, 1, res, tab, 1);
          for (int64_t j = 0; j < len; ++j) base[j * inner] = res[j];
        }
      free(line);
      free(res);
    }
    free(tab);
  }
}

void orc_fftnd(int dim, const int64_t* shape, double* xy, int sign) {
  fftnd(dim, shape, (cplx*)xy, sign);
}

/* zero-pad a real [0,N)^d array into a complex array of shape `big` */
static cplx* pad_complex(int dim, const int64_t* n, const int64_t* big,
                         const double* x) {
  int64_t tb = prod(dim, big), tn = prod(dim, n);
  cplx* X = (cplx*)calloc((size_t)tb, sizeof(cplx));
  for (int64_t lin = 0; lin < tn; ++lin) {
    int64_t idx[3];
    unravel(dim, n, lin, idx);
    X[ravel(dim, big, idx)] = x[lin];
  }
  return X;
}

/* real part of the [0,N)^d corner of a complex array of shape `big`, scaled */
static void restrict_real(int dim, const int64_t* n, const int64_t* big,
                          const cplx* X, double scale, double* out) {
  int64_t tn = prod(dim, n);
  for (int64_t lin = 0; lin < tn; ++lin) {
    int64_t idx[3];
    unravel(dim, n, lin, idx);
    out[lin] = creal(X[ravel(dim, big, idx)]) * scale;
  }
}

/* signed frequency of index p on a length-P grid, with the Nyquist index
 * P/2 mapped to 0 when zero_nyquist is set (used for differentiation). */
static double signed_freq(int64_t p, int64_t P, int zero_nyquist) {
  if (2 * p == P) return zero_nyquist ? 0.0 : -(double)p;
  return (2 * p < P) ? (double)p : (double)(p - P);
}

/* Spectrum of the 2N-periodic kernel, What = DFT_{2N}(W), returned on the
 * octant kappa in [0, N]^d (real part), plus the largest |imag| seen. */
int orc_kernel_spectrum(int dim, const int64_t* n, const double* w_oct,
                        double* what_oct, double* max_imag) {
  int64_t P[3], H[3];
  for (int a = 0; a < dim; ++a) {
    P[a] = 2 * n[a];
    H[a] = n[a] + 1;
  }
  int64_t tp = prod(dim, P);
  double* W = (double*)malloc(sizeof(double) * (size_t)tp);
  cplx* X = (cplx*)malloc(sizeof(cplx) * (size_t)tp);
  orc_periodic_kernel(dim, n, w_oct, W);
  for (int64_t i = 0; i < tp; ++i) X[i] = W[i];
  fftnd(dim, P, X, -1);
  double mi = 0.0;
  for (int64_t i = 0; i < tp; ++i)
    if (fabs(cimag(X[i])) > mi) mi = fabs(cimag(X[i]));
  int64_t th = prod(dim, H);
  for (int64_t lin = 0; lin < th; ++lin) {
    int64_t idx[3];
    unravel(dim, H, lin, idx);
    what_oct[lin] = creal(X[ravel(dim, P, idx)]);
  }
  if (max_imag) *max_imag = mi;
  free(W);
  free(X);
  return 0;
}

/* 2N path: phi = restrict IDFT_{2N}( DFT_{2N}(W) . DFT_{2N}(pad rho) ) and
 * E_a = restrict IDFT_{2N}( -i k_a DFT_{2N}(W) . DFT_{2N}(pad rho) ), with
 * k_a = 2 pi s_a / (2 N_a h_a), s_a the signed frequency and k_a := 0 at the
 * Nyquist index. phi and/or E (planar [dim][n...]) may be NULL. */
int orc_solve_fft2n(int dim, const int64_t* n, const double* h,
                    const double* w_oct, const double* rho, double* phi,
                    double* E) {
  int64_t P[3];
  for (int a = 0; a < dim; ++a) P[a] = 2 * n[a];
  int64_t tp = prod(dim, P), tn = prod(dim, n);
  double* W = (double*)malloc(sizeof(double) * (size_t)tp);
  cplx* What = (cplx*)malloc(sizeof(cplx) * (size_t)tp);
  cplx* F = (cplx*)malloc(sizeof(cplx) * (size_t)tp);
  if (!W || !What || !F) return -2;
  orc_periodic_kernel(dim, n, w_oct, W);
  for (int64_t i = 0; i < tp; ++i) What[i] = W[i];
  fftnd(dim, P, What, -1);
  cplx* R = pad_complex(dim, n, P, rho);
  fftnd(dim, P, R, -1);
  double scale = 1.0 / (double)tp;
  if (phi) {
    for (int64_t i = 0; i < tp; ++i) F[i] = What[i] * R[i];
    fftnd(dim, P, F, +1);
    restrict_real(dim, n, P, F, scale, phi);
  }
  if (E) {
    for (int a = 0; a < dim; ++a) {
      for (int64_t lin = 0; lin < tp; ++lin) {
        int64_t p[3];
        unravel(dim, P, lin, p);
        double ka = 2.0 * ORC_PI * signed_freq(p[a], P[a], 1) / ((double)P[a] * h[a]);
        F[lin] = (-I * ka) * What[lin] * R[lin];
      }
      fftnd(dim, P, F, +1);
      restrict_real(dim, n, P, F, scale, E + (int64_t)a * tn);
    }
  }
  free(W);
  free(What);
  free(F);
  free(R);
  return 0;
}

/* out = restriction to [0, N) of the 2N-periodic convolution of V (full
 * 2N-periodic real kernel) with rho zero-padded to 2N, through the naive
 * FFT: pad, DFT, multiply by DFT(V), inverse DFT, restrict. */
int orc_conv_fft2n(int dim, const int64_t* n, const double* V, const double* rho, double* out) {
  int64_t P[3] = {1, 1, 1};
  for (int a = 0; a < dim; ++a) P[a] = 2 * n[a];
  const int64_t tp = prod(dim, P);
  cplx* R = pad_complex(dim, n, P, rho);
  cplx* K = (cplx*)malloc(sizeof(cplx) * (size_t)tp);
  if (!R || !K) {
    free(R);
    free(K);
    return -2;
  }
  for (int64_t i = 0; i < tp; ++i) K[i] = V[i];
  fftnd(dim, P, R, -1);
  fftnd(dim, P, K, -1);
  for (int64_t i = 0; i < tp; ++i) R[i] *= K[i];
  fftnd(dim, P, R, +1);
  restrict_real(dim, n, P, R, 1.0 / (double)tp, out);
  free(R);
  free(K);
  return 0;
}

/* The "in principle" 4N path for the gradient-kernel field: pad rho to 4N,
 * multiply its DFT by -i k_a Ghat(|k|) (k_m from the signed index m), invert,
 * restrict to [0, N) and keep the real part. */
int orc_solve_fft4n_grad(int dim, const int64_t* n, const double* h, double L, int axis,
                         const double* rho, double* Ea) {
  int64_t M[3];
  for (int a = 0; a < dim; ++a) M[a] = 4 * n[a];
  int64_t tm = prod(dim, M);
  cplx* R = pad_complex(dim, n, M, rho);
  if (!R) return -2;
  fftnd(dim, M, R, -1);
#pragma omp parallel for schedule(static)
  for (int64_t lin = 0; lin < tm; ++lin) {
    int64_t m[3];
    unravel(dim, M, lin, m);
    double k2 = 0.0, kax = 0.0;
    for (int a = 0; a < dim; ++a) {
      double ka = 2.0 * ORC_PI * signed_freq(m[a], M[a], 0) / ((double)M[a] * h[a]);
      k2 += ka * ka;
      if (a == axis) kax = ka;
    }
    R[lin] *= -I * kax * orc_ghat(dim, L, sqrt(k2));
  }
  fftnd(dim, M, R, +1);
  restrict_real(dim, n, M, R, 1.0 / (double)tm, Ea);
  free(R);
  return 0;
}

/* 4N path for the VGF potential ("in principle" computation of Sec. II):
 * pad rho to (4N)^d, multiply its DFT by F{G^L}(k_m), k_{m,a} = 2 pi s_a /
 * (4 N_a h_a) with s_a in [-2N_a, 2N_a), inverse DFT, restrict to [0,N)^d. */
int orc_solve_fft4n(int dim, const int64_t* n, const double* h, double L,
                    const double* rho, double* phi) {
  int64_t M[3];
  for (int a = 0; a < dim; ++a) M[a] = 4 * n[a];
  int64_t tm = prod(dim, M);
  cplx* R = pad_complex(dim, n, M, rho);
  if (!R) return -2;
  fftnd(dim, M, R, -1);
#pragma omp parallel for schedule(static)
  for (int64_t lin = 0; lin < tm; ++lin) {
    int64_t m[3];
    unravel(dim, M, lin, m);
    double k2 = 0.0;
    for (int a = 0; a < dim; ++a) {
      double ka = 2.0 * ORC_PI * signed_freq(m[a], M[a], 0) / ((double)M[a] * h[a]);
      k2 += ka * ka;
    }
    R[lin] *= orc_ghat(dim, L, sqrt(k2));
  }
  fftnd(dim, M, R, +1);
  restrict_real(dim, n, M, R, 1.0 / (double)tm, phi);
  free(R);
  return 0;
}

/* Adjoint by the FFT route, without using any symmetry of the kernels:
 * g_rho = K^T g_phi + sum_a K_a^T g_E[a], where K (resp. K_a) is the 2N path
 * operator for phi (resp. E_a); in Fourier space the transpose multiplies by
 * the complex conjugate of the forward multiplier. g_phi or g_E may be NULL. */
int orc_adjoint_fft2n(int dim, const int64_t* n, const double* h,
                      const double* w_oct, const double* g_phi,
                      const double* g_E, double* g_rho) {
  int64_t P[3];
  for (int a = 0; a < dim; ++a) P[a] = 2 * n[a];
  int64_t tp = prod(dim, P), tn = prod(dim, n);
  double* W = (double*)malloc(sizeof(double) * (size_t)tp);
  cplx* What = (cplx*)malloc(sizeof(cplx) * (size_t)tp);
  cplx* acc = (cplx*)calloc((size_t)tp, sizeof(cplx));
  orc_periodic_kernel(dim, n, w_oct, W);
  for (int64_t i = 0; i < tp; ++i) What[i] = W[i];
  fftnd(dim, P, What, -1);
  if (g_phi) {
    cplx* G = pad_complex(dim, n, P, g_phi);
    fftnd(dim, P, G, -1);
    for (int64_t i = 0; i < tp; ++i) acc[i] += conj(What[i]) * G[i];
    free(G);
  }
  if (g_E) {
    for (int a = 0; a < dim; ++a) {
      cplx* G = pad_complex(dim, n, P, g_E + (int64_t)a * tn);
      fftnd(dim, P, G, -1);
      for (int64_t lin = 0; lin < tp; ++lin) {
        int64_t p[3];
        unravel(dim, P, lin, p);
        double ka = 2.0 * ORC_PI * signed_freq(p[a], P[a], 1) / ((double)P[a] * h[a]);
        acc[lin] += conj((-I * ka) * What[lin]) * G[lin];
      }
      free(G);
    }
  }
  fftnd(dim, P, acc, +1);
  restrict_real(dim, n, P, acc, 1.0 / (double)tp, g_rho);
  free(W);
  free(What);
  free(acc);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Closed-form Gaussian potentials (Sec. III) and special functions          */
/* ------------------------------------------------------------------------ */

/* Ein(u) = sum_{k>=1} (-1)^{k+1} u^k / (k k!) = E1(u) + gamma + ln u.
 * Power series for u <= 2; for larger u, E1 from its continued fraction
 * (Abramowitz & Stegun 5.1.22, in the even-contracted form
 * E1(u) = e^{-u} / (u + 1 - 1^2/(u + 3 - 2^2/(u + 5 - ...)))), evaluated
 * with the modified Lentz method. */
double orc_expint_e1(double u);

double orc_ein(double u) {
  if (u <= 2.0) {
    double term = u, sum = 0.0;
    for (int k = 1; k < 200; ++k) {
      double t = term / (double)k;
      sum += (k % 2 == 1) ? t : -t;
      term *= u / (double)(k + 1);
      if (fabs(t) < 1e-18 * fabs(sum)) break;
    }
    return sum;
  }
  return orc_expint_e1(u) + ORC_EULER_GAMMA + log(u);
}

double orc_expint_e1(double u) {
  if (u <= 1.0) return orc_ein(u) - ORC_EULER_GAMMA - log(u);
  const double tiny = 1e-300;
  double f = u + 1.0, C = f, D = 0.0;
  for (int i = 1; i < 1000; ++i) {
    double a = -(double)i * (double)i, b = u + 2.0 * i + 1.0;
    D = b + a * D;
    if (fabs(D) < tiny) D = tiny;
    C = b + a / C;
    if (fabs(C) < tiny) C = tiny;
    D = 1.0 / D;
    double delta = C * D;
    f *= delta;
    if (fabs(delta - 1.0) < 1e-17) break;
  }
  return exp(-u) / f;
}

/* 3D unit Gaussian of width sigma centred at c (Eq. 14): potential Eq. (15)
 * phi = erf(r / (sqrt2 sigma)) / (4 pi r), phi(0) = 1 / ((2 pi)^{3/2} sigma);
 * field E = Q(s) / (4 pi r^2) * (x - c) / r with Q(s) = erf(s) - (2/sqrt pi)
 * s e^{-s^2} the charge inside radius r, s = r / (sqrt2 sigma); Q by its
 * series (4/sqrt pi) sum_k (-1)^k s^{2k+3} / (k! (2k+3)) for s < 0.5. */
void orc_gauss3d_point(double sigma, const double* c, const double* x,
                       double* phi, double* E) {
  double d[3], r2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    d[a] = x[a] - c[a];
    r2 += d[a] * d[a];
  }
  double r = sqrt(r2), s = r / (sqrt(2.0) * sigma);
  if (phi) {
    if (r == 0.0)
      *phi = 1.0 / (pow(2.0 * ORC_PI, 1.5) * sigma);
    else
      *phi = erf(s) / (4.0 * ORC_PI * r);
  }
  if (E) {
    if (r == 0.0) {
      E[0] = E[1] = E[2] = 0.0;
      return;
    }
    double Q;
    if (s < 0.5) {
      double sum = 0.0, pw = s * s * s, fact = 1.0;
      for (int k = 0; k < 40; ++k) {
        if (k > 0) fact *= (double)k;
        double t = pw / (fact * (2.0 * k + 3.0));
        sum += (k % 2 == 0) ? t : -t;
        pw *= s * s;
      }
      Q = 4.0 / sqrt(ORC_PI) * sum;
    } else {
      Q = erf(s) - 2.0 / sqrt(ORC_PI) * s * exp(-s * s);
    }
    double Er = Q / (4.0 * ORC_PI * r2);
    for (int a = 0; a < 3; ++a) E[a] = Er * d[a] / r;
  }
}

/* 2D unit Gaussian of width sigma centred at c (Eq. 10). Potential Eq. (11)
 * read with the exponential integral E1 (the formula as printed uses "Ei";
 * only E1 gives a function that solves the problem):
 *   phi = -(E1(u) + ln r^2) / (4 pi), u = r^2 / (2 sigma^2),
 * evaluated as (gamma - ln(2 sigma^2) - Ein(u)) / (4 pi), which is finite at
 * r = 0. Field E = (1 - e^{-u}) / (2 pi r^2) (x - c). */
void orc_gauss2d_point(double sigma, const double* c, const double* x,
                       double* phi, double* E) {
  double d0 = x[0] - c[0], d1 = x[1] - c[1];
  double r2 = d0 * d0 + d1 * d1, u = r2 / (2.0 * sigma * sigma);
  if (phi)
    *phi = (ORC_EULER_GAMMA - log(2.0 * sigma * sigma) - orc_ein(u)) / (4.0 * ORC_PI);
  if (E) {
    if (r2 == 0.0) {
      E[0] = E[1] = 0.0;
      return;
    }
    double f = -expm1(-u) / (2.0 * ORC_PI * r2);
    E[0] = f * d0;
    E[1] = f * d1;
  }
}

/* 3D anisotropic unit Gaussian with widths sig[3] centred at c. From
 * 1/r = (2/sqrt pi) int_0^inf exp(-r^2 t^2) dt, the potential is
 *   phi = (2 pi^{3/2})^{-1} int_0^inf prod_a (1 + 2 sig_a^2 t^2)^{-1/2}
 *         exp(-sum_a d_a^2 t^2 / (1 + 2 sig_a^2 t^2)) dt,   d = x - c,
 * and E_a carries the extra factor 2 d_a t^2 / (1 + 2 sig_a^2 t^2).
 * The integral is taken with the exp-sinh substitution t = exp(pi/2 sinh s)
 * and the trapezoidal rule in s (double-exponential quadrature). */
void orc_gauss3d_aniso_point(const double* sig, const double* c,
                             const double* x, double step, double* phi,
                             double* E) {
  double d[3];
  for (int a = 0; a < 3; ++a) d[a] = x[a] - c[a];
  ksum sp = {0, 0}, se[3] = {{0, 0}, {0, 0}, {0, 0}};
  const double smax = 4.75;
  int64_t K = (int64_t)ceil(smax / step);
  for (int64_t q = -K; q <= K; ++q) {
    double s = (double)q * step;
    double t = exp(0.5 * ORC_PI * sinh(s));
    double dt = t * 0.5 * ORC_PI * cosh(s);
    if (!(t > 0.0) || !isfinite(t) || !isfinite(dt)) continue;
    double t2 = t * t, pref = 1.0, ex = 0.0, fac[3];
    for (int a = 0; a < 3; ++a) {
      double den = 1.0 + 2.0 * sig[a] * sig[a] * t2;
      pref /= sqrt(den);
      ex += d[a] * d[a] * t2 / den;
      fac[a] = 2.0 * d[a] * t2 / den;
    }
    double f = pref * exp(-ex) * dt;
    kadd(&sp, f);
    for (int a = 0; a < 3; ++a) kadd(&se[a], f * fac[a]);
  }
  double norm = step / (2.0 * pow(ORC_PI, 1.5));
  if (phi) *phi = kval(&sp) * norm;
  if (E)
    for (int a = 0; a < 3; ++a) E[a] = kval(&se[a]) * norm;
}

/* Analytic phi and E of a mixture of Gaussians on the grid
 * x_{a,j} = x0_a + j h_a. sig holds dim widths per Gaussian; iso != 0 uses
 * the closed forms (requires equal widths), otherwise (3D only) the
 * integral. phi (shape n) and E (planar [dim][n...]) may be NULL. */
int orc_gauss_mixture_grid(int dim, const int64_t* n, const double* x0,
                           const double* h, int count, const double* centers,
                           const double* sig, const double* weights, int iso,
                           double* phi, double* E) {
  int64_t tn = prod(dim, n);
  if (!iso && dim != 3) return -1;
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t lin = 0; lin < tn; ++lin) {
    int64_t idx[3];
    double x[3], p = 0.0, e[3] = {0, 0, 0};
    unravel(dim, n, lin, idx);
    for (int a = 0; a < dim; ++a) x[a] = x0[a] + (double)idx[a] * h[a];
    for (int g = 0; g < count; ++g) {
      double pg, eg[3];
      const double* c = centers + g * dim;
      const double* sg = sig + g * dim;
      if (dim == 3 && iso)
        orc_gauss3d_point(sg[0], c, x, &pg, eg);
      else if (dim == 3)
        orc_gauss3d_aniso_point(sg, c, x, 1.0 / 64.0, &pg, eg);
      else
        orc_gauss2d_point(sg[0], c, x, &pg, eg);
      p += weights[g] * pg;
      for (int a = 0; a < dim; ++a) e[a] += weights[g] * eg[a];
    }
    if (phi) phi[lin] = p;
    if (E)
      for (int a = 0; a < dim; ++a) E[(int64_t)a * tn + lin] = e[a];
  }
  return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_num_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}
