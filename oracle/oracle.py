"""ctypes front end of the FP64 CPU oracle (test infrastructure only).

Each function marshals numpy float64 arrays to the C definitions in
vgf_oracle.c and returns numpy arrays. Shapes follow the solve grid: `n` is
the tuple of points per axis (last axis fastest), `h` the spacings.
"""
import ctypes as C
import math
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        d, i64p, dp = C.c_double, C.POINTER(C.c_int64), C.POINTER(C.c_double)
        L.orc_ghat.restype = d
        L.orc_ghat.argtypes = [C.c_int, d, d]
        L.orc_window.argtypes = [C.c_int, i64p, dp, dp, dp]
        L.orc_vgf_kernel.argtypes = [C.c_int, i64p, dp, d, dp]
        L.orc_he_kernel.argtypes = [C.c_int, i64p, dp, dp]
        L.orc_he_kernel_mode.argtypes = [C.c_int, i64p, dp, C.c_int, dp]
        L.orc_he_origin.restype = d
        L.orc_he_origin.argtypes = [C.c_int, dp, C.c_int]
        L.orc_cell_average_integral.restype = d
        L.orc_cell_average_integral.argtypes = [C.c_int, dp]
        L.orc_fd_field.argtypes = [C.c_int, i64p, dp, dp, dp]
        L.orc_vgf_grad_kernel.argtypes = [C.c_int, i64p, dp, d, C.c_int, dp]
        L.orc_periodic_kernel_odd.argtypes = [C.c_int, i64p, dp, C.c_int, dp]
        L.orc_conv_fft2n.argtypes = [C.c_int, i64p, dp, dp, dp]
        L.orc_solve_fft4n_grad.argtypes = [C.c_int, i64p, dp, d, C.c_int, dp, dp]
        L.orc_fd_field_T.argtypes = [C.c_int, i64p, dp, dp, dp]
        L.orc_periodic_kernel.argtypes = [C.c_int, i64p, dp, dp]
        L.orc_field_kernel.argtypes = [C.c_int, i64p, dp, dp, C.c_int, dp]
        L.orc_conv_direct.argtypes = [C.c_int, i64p, dp, dp, dp]
        L.orc_conv_periodic.argtypes = [C.c_int, i64p, dp, dp, dp]
        L.orc_conv_periodic_T.argtypes = [C.c_int, i64p, dp, dp, dp]
        L.orc_conv_direct_point.restype = d
        L.orc_conv_direct_point.argtypes = [C.c_int, i64p, dp, dp, i64p]
        L.orc_fft1d.argtypes = [C.c_int64, dp, C.c_int]
        L.orc_dft1d.argtypes = [C.c_int64, dp, C.c_int]
        L.orc_fftnd.argtypes = [C.c_int, i64p, dp, C.c_int]
        L.orc_kernel_spectrum.argtypes = [C.c_int, i64p, dp, dp, dp]
        L.orc_solve_fft2n.argtypes = [C.c_int, i64p, dp, dp, dp, dp, dp]
        L.orc_solve_fft4n.argtypes = [C.c_int, i64p, dp, d, dp, dp]
        L.orc_adjoint_fft2n.argtypes = [C.c_int, i64p, dp, dp, dp, dp, dp]
        L.orc_ein.restype = d
        L.orc_ein.argtypes = [d]
        L.orc_expint_e1.restype = d
        L.orc_expint_e1.argtypes = [d]
        L.orc_gauss3d_point.argtypes = [d, dp, dp, dp, dp]
        L.orc_gauss2d_point.argtypes = [d, dp, dp, dp, dp]
        L.orc_gauss3d_aniso_point.argtypes = [dp, dp, dp, d, dp, dp]
        L.orc_gauss_mixture_grid.argtypes = [C.c_int, i64p, dp, dp, C.c_int, dp, dp, dp,
                                             C.c_int, dp, dp]
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        _lib = L
    return _lib


def _i64(seq):
    a = np.ascontiguousarray(np.asarray(seq, dtype=np.int64))
    return a, a.ctypes.data_as(C.POINTER(C.c_int64))


def _f64(arr):
    a = np.ascontiguousarray(np.asarray(arr, dtype=np.float64))
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _out(shape):
    a = np.zeros(shape, dtype=np.float64)
    return a, a.ctypes.data_as(C.POINTER(C.c_double))


def _np(x):
    return None if x is None else x


NULL = C.POINTER(C.c_double)()


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(t):
    lib().orc_set_num_threads(int(t))


def ghat(dim, L, k):
    """F{G^L}(|k|), Eqs. (7)-(8)."""
    return lib().orc_ghat(int(dim), float(L), float(k))


def window(n, h):
    """(Lmin, Lmax): admissible open interval for the truncation radius L."""
    dim = len(n)
    n_, pn = _i64(n)
    h_, ph = _f64(h)
    lo, hi = C.c_double(), C.c_double()
    lib().orc_window(dim, pn, ph, C.byref(lo), C.byref(hi))
    return lo.value, hi.value


def default_L(n, h):
    """1.1 times the box diameter (inside the window for every grid used here)."""
    lo, hi = window(n, h)
    L = 1.1 * lo
    assert lo < L < hi, (lo, L, hi)
    return L


def vgf_kernel(n, h, L):
    """Restricted VGF kernel w on offsets [0, N_a) (even octant)."""
    dim = len(n)
    n_, pn = _i64(n)
    h_, ph = _f64(h)
    w, pw = _out(tuple(n))
    rc = lib().orc_vgf_kernel(dim, pn, ph, float(L), pw)
    assert rc == 0
    return w


HE_MODES = {"he": 0, "he_nearby": 1, "he_cellavg": 2}


def he_kernel(n, h, mode=0):
    """Hockney-Eastwood kernel; mode 0 (G0 convention), 1 (nearby value),
    2 (cell average) for the origin weight."""
    dim = len(n)
    n_, pn = _i64(n)
    h_, ph = _f64(h)
    w, pw = _out(tuple(n))
    assert lib().orc_he_kernel_mode(dim, pn, ph, int(mode), pw) == 0
    return w


def he_origin(h, mode):
    h_, ph = _f64(h)
    return lib().orc_he_origin(len(h), ph, int(mode))


def cell_average_integral(h):
    """Integral of G over the cell prod_a [-h_a/2, h_a/2]."""
    h_, ph = _f64(h)
    return lib().orc_cell_average_integral(len(h), ph)


def vgf_grad_kernel(n, h, L, axis):
    """Restricted inverse 4N DFT of -i k_axis Ghat: octant [0, N)^d, odd in axis."""
    dim = len(n)
    n_, pn = _i64(n)
    h_, ph = _f64(h)
    w, pw = _out(tuple(n))
    assert lib().orc_vgf_grad_kernel(dim, pn, ph, float(L), int(axis), pw) == 0
    return w


def periodic_kernel_odd(n, w_oct, axis):
    dim = len(n)
    n_, pn = _i64(n)
    w_, pw = _f64(w_oct)
    W, pW = _out(tuple(2 * x for x in n))
    lib().orc_periodic_kernel_odd(dim, pn, pw, int(axis), pW)
    return W


def conv_fft2n(n, V, rho):
    """Restriction of the 2N-periodic convolution of V with zero-padded rho (FFT route)."""
    dim = len(n)
    n_, pn = _i64(n)
    v_, pv = _f64(V)
    r_, pr = _f64(rho)
    out, po = _out(tuple(n))
    assert lib().orc_conv_fft2n(dim, pn, pv, pr, po) == 0
    return out


def solve_fft4n_grad(n, h, L, axis, rho):
    dim = len(n)
    n_, pn = _i64(n)
    h_, ph = _f64(h)
    r_, pr = _f64(rho)
    out, po = _out(tuple(n))
    assert lib().orc_solve_fft4n_grad(dim, pn, ph, float(L), int(axis), pr, po) == 0
    return out


def solve_grad_kernel(n, h, L, rho, w=None, want_phi=True):
    """phi (2N path, kernel w) and E_a = w_a * rho with the gradient kernels."""
    dim = len(n)
    if w is None and want_phi:
        w = vgf_kernel(n, h, L)
    phi = conv_fft2n(n, periodic_kernel(n, w), rho) if want_phi else None
    E = np.stack([conv_fft2n(n, periodic_kernel_odd(n, vgf_grad_kernel(n, h, L, a), a), rho)
                  for a in range(dim)])
    return phi, E


def fd_field(n, h, phi):
    """E = -D phi, second-order differences (centred inside, one-sided ends)."""
    dim = len(n)
    n_, pn = _i64(n)
    h_, ph = _f64(h)
    p_, pp = _f64(phi)
    E, pE = _out((dim,) + tuple(n))
    assert lib().orc_fd_field(dim, pn, ph, pp, pE) == 0
    return E


def fd_field_T(n, h, gE):
    """-sum_a D_a^T gE[a]: the transpose of fd_field."""
    dim = len(n)
    n_, pn = _i64(n)
    h_, ph = _f64(h)
    g_, pg = _f64(gE)
    out, po = _out(tuple(n))
    assert lib().orc_fd_field_T(dim, pn, ph, pg, po) == 0
    return out


def periodic_kernel(n, w_oct):
    dim = len(n)
    n_, pn = _i64(n)
    w_, pw = _f64(w_oct)
    W, pW = _out(tuple(2 * x for x in n))
    lib().orc_periodic_kernel(dim, pn, pw, pW)
    return W


def field_kernel(n, h, W, axis):
    dim = len(n)
    n_, pn = _i64(n)
    h_, ph = _f64(h)
    W_, pW = _f64(W)
    v, pv = _out(W_.shape)
    lib().orc_field_kernel(dim, pn, ph, pW, int(axis), pv)
    return v


def conv_direct(n, w_oct, rho):
    dim = len(n)
    n_, pn = _i64(n)
    w_, pw = _f64(w_oct)
    r_, pr = _f64(rho)
    phi, pp = _out(tuple(n))
    lib().orc_conv_direct(dim, pn, pw, pr, pp)
    return phi


def conv_periodic(n, V, x):
    dim = len(n)
    n_, pn = _i64(n)
    V_, pV = _f64(V)
    x_, px = _f64(x)
    out, po = _out(tuple(n))
    lib().orc_conv_periodic(dim, pn, pV, px, po)
    return out


def conv_periodic_T(n, V, g):
    dim = len(n)
    n_, pn = _i64(n)
    V_, pV = _f64(V)
    g_, pg = _f64(g)
    out, po = _out(tuple(n))
    lib().orc_conv_periodic_T(dim, pn, pV, pg, po)
    return out


def conv_direct_point(n, w_oct, rho, idx):
    dim = len(n)
    n_, pn = _i64(n)
    w_, pw = _f64(w_oct)
    r_, pr = _f64(rho)
    i_, pi = _i64(idx)
    return lib().orc_conv_direct_point(dim, pn, pw, pr, pi)


def _complex_call(fn, x, *args):
    a = np.ascontiguousarray(np.asarray(x, dtype=np.complex128)).copy()
    fn(*args[:-1], a.ctypes.data_as(C.POINTER(C.c_double)), args[-1])
    return a


def fft1d(x, sign=-1):
    x = np.asarray(x, dtype=np.complex128)
    return _complex_call(lib().orc_fft1d, x, C.c_int64(x.size), int(sign))


def dft1d(x, sign=-1):
    x = np.asarray(x, dtype=np.complex128)
    return _complex_call(lib().orc_dft1d, x, C.c_int64(x.size), int(sign))


def fftnd(x, sign=-1):
    x = np.ascontiguousarray(np.asarray(x, dtype=np.complex128)).copy()
    s_, ps = _i64(x.shape)
    lib().orc_fftnd(x.ndim, ps, x.ctypes.data_as(C.POINTER(C.c_double)), int(sign))
    return x


def kernel_spectrum(n, w_oct):
    """Octant [0, N_a] of DFT_{2N}(W) (real part) and the largest |imag part|."""
    dim = len(n)
    n_, pn = _i64(n)
    w_, pw = _f64(w_oct)
    s, ps = _out(tuple(x + 1 for x in n))
    mi = C.c_double()
    lib().orc_kernel_spectrum(dim, pn, pw, ps, C.byref(mi))
    return s, mi.value


def solve_fft2n(n, h, w_oct, rho, want_phi=True, want_E=True):
    dim = len(n)
    n_, pn = _i64(n)
    h_, ph = _f64(h)
    w_, pw = _f64(w_oct)
    r_, pr = _f64(rho)
    phi, pp = _out(tuple(n)) if want_phi else (None, NULL)
    E, pE = _out((dim,) + tuple(n)) if want_E else (None, NULL)
    assert lib().orc_solve_fft2n(dim, pn, ph, pw, pr, pp, pE) == 0
    return phi, E


def solve_fft4n(n, h, L, rho):
    dim = len(n)
    n_, pn = _i64(n)
    h_, ph = _f64(h)
    r_, pr = _f64(rho)
    phi, pp = _out(tuple(n))
    assert lib().orc_solve_fft4n(dim, pn, ph, float(L), pr, pp) == 0
    return phi


def adjoint_fft2n(n, h, w_oct, g_phi=None, g_E=None):
    dim = len(n)
    n_, pn = _i64(n)
    h_, ph = _f64(h)
    w_, pw = _f64(w_oct)
    if g_phi is not None:
        gp_, pgp = _f64(g_phi)
    else:
        pgp = NULL
    if g_E is not None:
        ge_, pge = _f64(g_E)
    else:
        pge = NULL
    out, po = _out(tuple(n))
    assert lib().orc_adjoint_fft2n(dim, pn, ph, pw, pgp, pge, po) == 0
    return out


def ein(u):
    return lib().orc_ein(float(u))


def expint_e1(u):
    return lib().orc_expint_e1(float(u))


def gauss3d_point(sigma, c, x):
    c_, pc = _f64(c)
    x_, px = _f64(x)
    p = C.c_double()
    E, pE = _out((3,))
    lib().orc_gauss3d_point(float(sigma), pc, px, C.byref(p), pE)
    return p.value, E


def gauss2d_point(sigma, c, x):
    c_, pc = _f64(c)
    x_, px = _f64(x)
    p = C.c_double()
    E, pE = _out((2,))
    lib().orc_gauss2d_point(float(sigma), pc, px, C.byref(p), pE)
    return p.value, E


def gauss3d_aniso_point(sig, c, x, step=1.0 / 64.0):
    s_, ps = _f64(sig)
    c_, pc = _f64(c)
    x_, px = _f64(x)
    p = C.c_double()
    E, pE = _out((3,))
    lib().orc_gauss3d_aniso_point(ps, pc, px, float(step), C.byref(p), pE)
    return p.value, E


def gauss_mixture_grid(n, x0, h, centers, sigmas, weights, iso=True,
                       want_phi=True, want_E=True):
    """Analytic phi / E of a Gaussian mixture sampled at x0 + j h.

    centers: (count, dim); sigmas: (count, dim) widths; weights: (count,).
    """
    dim = len(n)
    n_, pn = _i64(n)
    x0_, px0 = _f64(x0)
    h_, ph = _f64(h)
    c_, pc = _f64(np.asarray(centers, dtype=np.float64).reshape(-1, dim))
    s_, ps = _f64(np.asarray(sigmas, dtype=np.float64).reshape(-1, dim))
    w_, pw = _f64(np.asarray(weights, dtype=np.float64).reshape(-1))
    phi, pp = _out(tuple(n)) if want_phi else (None, NULL)
    E, pE = _out((dim,) + tuple(n)) if want_E else (None, NULL)
    rc = lib().orc_gauss_mixture_grid(dim, pn, px0, ph, int(w_.size), pc, ps, pw,
                                      1 if iso else 0, pp, pE)
    assert rc == 0
    return phi, E


def kernel(method, n, h, L=None):
    """Octant kernel for 'vgf' or 'he'."""
    if method == "vgf":
        return vgf_kernel(n, h, default_L(n, h) if L is None else L)
    if method in HE_MODES:
        return he_kernel(n, h, HE_MODES[method])
    raise ValueError(method)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = math.sqrt(float(np.sum(b * b)))
    return math.sqrt(float(np.sum((a - b) ** 2))) / den if den > 0 else math.sqrt(float(np.sum(a * a)))
