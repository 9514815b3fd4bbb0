"""Pins of the oracle's kernel spectrum (Eqs. 7-8) and restricted kernels.

The closed forms are checked against the Fourier transform of the truncated
Green's function taken by numerical quadrature from its definition (Eqs. 2
and 4), against their Taylor expansions at k = 0, and the restricted kernel
against an inverse FFT of the same samples on the full 4N grid."""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as ss


def ft_truncated_green(dim, L, k):
    """Radial Fourier transform of G * 1(r <= L) by quadrature (definition)."""
    if dim == 3:
        G = lambda r: 1.0 / (4 * math.pi * r)
        f = lambda r: 4 * math.pi * r * r * G(r) * (np.sinc(k * r / math.pi))
    else:
        G = lambda r: -math.log(r) / (2 * math.pi) if r > 0 else 0.0
        f = lambda r: 2 * math.pi * r * G(r) * ss.j0(k * r)
    val, err = si.quad(f, 0.0, L, limit=400, epsabs=1e-14, epsrel=1e-13)
    return val


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("L", [0.7, 1.0, 1.9, 3.81])
@pytest.mark.parametrize("k", [0.0, 0.3, 1.7, 6.0, 23.0])
def test_ghat_matches_quadrature_of_definition(orc, dim, L, k):
    a = orc.ghat(dim, L, k)
    b = ft_truncated_green(dim, L, k)
    assert abs(a - b) <= 1e-10 * max(1.0, abs(b)), (a, b)


def test_ghat_small_k_taylor(orc):
    for L in (0.9, 2.0, 3.81):
        k = 1e-3
        # 3D: (1 - cos(Lk)) / k^2
        t3 = L**2 / 2 - L**4 * k**2 / 24 + L**6 * k**4 / 720
        assert abs(orc.ghat(3, L, k) - t3) < 1e-13 * t3
        assert orc.ghat(3, L, 0.0) == pytest.approx(L * L / 2, rel=1e-15)
        # 2D: series of (1 - J0(x))/k^2 - L ln L J1(x)/k, x = L k
        x = L * k
        one_m_j0 = x**2 / 4 - x**4 / 64 + x**6 / 2304
        j1 = x / 2 - x**3 / 16 + x**5 / 384
        t2 = one_m_j0 / k**2 - L * math.log(L) * j1 / k
        assert abs(orc.ghat(2, L, k) - t2) < 1e-9 * abs(t2)
        assert orc.ghat(2, L, 0.0) == pytest.approx(L * L / 4 - L * L * math.log(L) / 2, rel=1e-14)


@pytest.mark.parametrize("x", [0.1, 1.0, 5.0, 37.5, 410.0, 3500.0])
def test_libm_bessel_vs_integral_representation(orc, x):
    # Bessel's integral J_n(x) = (1/pi) int_0^pi cos(n t - x sin t) dt; the
    # trapezoidal rule on this periodic integrand converges exponentially.
    m = int(2 * x) + 200
    t = np.linspace(0.0, math.pi, m + 1)
    wts = np.full(m + 1, math.pi / m)
    wts[0] = wts[-1] = 0.5 * math.pi / m
    j0i = float(np.sum(wts * np.cos(x * np.sin(t)))) / math.pi
    j1i = float(np.sum(wts * np.cos(t - x * np.sin(t)))) / math.pi
    # the oracle's 2D spectrum evaluated against these values
    L = 1.0
    k = x / L
    g = orc.ghat(2, L, k)  # ln(1) = 0, so only (1 - J0)/k^2 survives
    assert abs(g - (1.0 - j0i) / k**2) < 1e-13 * max(1.0, 1.0 / k**2)
    assert abs(ss.j0(x) - j0i) < 1e-13 and abs(ss.j1(x) - j1i) < 1e-13
    L = 2.0
    k = x / L
    g = orc.ghat(2, L, k)
    ref = (1.0 - j0i) / k**2 - L * math.log(L) * j1i / k
    assert abs(g - ref) < 2e-13 * max(1.0, L * L)


def test_window_bounds(orc):
    N = 32
    h = 2.0 / (N - 1)
    lo, hi = orc.window((N, N, N), (h, h, h))
    assert lo == pytest.approx(2.0 * math.sqrt(3.0), rel=1e-15)
    assert hi == pytest.approx(4 * N * h - 2.0, rel=1e-15)
    lo, hi = orc.window((N, N), (h, h))
    assert lo == pytest.approx(2.0 * math.sqrt(2.0), rel=1e-15)


@pytest.mark.parametrize("n,h", [((6, 8, 9), (0.31, 0.27, 0.22)), ((10, 12), (0.11, 0.09)),
                                 ((8, 8, 8), (0.25, 0.25, 0.25))])
def test_vgf_kernel_equals_4n_inverse_fft(orc, n, h):
    """Cosine sums (the restricted kernel) == inverse FFT of the same samples
    on the full (4N)^d grid, restricted to offsets [0, N)."""
    dim = len(n)
    L = orc.default_L(n, h)
    w = orc.vgf_kernel(n, h, L)
    M = [4 * x for x in n]
    k2 = np.zeros(M)
    for a in range(dim):
        s = np.arange(M[a])
        s = np.where(s < 2 * n[a], s, s - M[a]).astype(np.float64)
        ka = 2 * math.pi * s / (M[a] * h[a])
        shp = [1] * dim
        shp[a] = M[a]
        k2 = k2 + (ka ** 2).reshape(shp)
    G = np.vectorize(lambda kk: orc.ghat(dim, L, kk))(np.sqrt(k2))
    full = orc.fftnd(G.astype(np.complex128), +1) / np.prod(M)
    sl = tuple(slice(0, x) for x in n)
    ref = full[sl]
    assert np.max(np.abs(ref.imag)) < 1e-15 * np.max(np.abs(w)) * 100
    assert np.max(np.abs(w - ref.real)) < 1e-14 * np.max(np.abs(w))
    # P3: sum over the whole 4N grid of the inverse transform is the k=0 value
    assert abs(full.sum().real - orc.ghat(dim, L, 0.0)) < 1e-13 * orc.ghat(dim, L, 0.0)


def test_vgf_kernel_symmetry_and_real_spectrum(orc):
    n = (8, 8, 8)
    h = (2 / 7,) * 3
    w = orc.vgf_kernel(n, h, orc.default_L(n, h))
    for perm in [(1, 0, 2), (0, 2, 1), (2, 1, 0)]:
        assert np.max(np.abs(w - w.transpose(perm))) < 1e-15 * np.max(np.abs(w)) * 10
    s, mi = orc.kernel_spectrum(n, w)
    assert mi < 1e-15 * np.max(np.abs(s)) * 100
    # the spectrum of the even periodic kernel equals the cosine transform
    W = orc.periodic_kernel(n, w)
    ref = np.fft.fftn(W).real[:9, :9, :9]
    assert np.max(np.abs(s - ref)) < 1e-13 * np.max(np.abs(ref))


def test_he_kernel_values(orc):
    n = (5, 6, 7)
    h = (0.1, 0.2, 0.3)
    w = orc.he_kernel(n, h)
    vol = 0.1 * 0.2 * 0.3
    assert w[0, 0, 0] == pytest.approx(vol / (4 * math.pi), rel=1e-15)
    r = math.sqrt((2 * 0.1) ** 2 + (3 * 0.2) ** 2 + (4 * 0.3) ** 2)
    assert w[2, 3, 4] == pytest.approx(vol / (4 * math.pi * r), rel=1e-15)
    w2 = orc.he_kernel((4, 4), (0.5, 0.25))
    assert w2[0, 0] == pytest.approx(0.125 / (2 * math.pi), rel=1e-15)
    r = math.hypot(3 * 0.5, 2 * 0.25)
    assert w2[3, 2] == pytest.approx(-0.125 * math.log(r) / (2 * math.pi), rel=1e-14)


def test_field_kernel_is_spectral_derivative(orc):
    """P8: the cot stencil equals multiplication by i k with the Nyquist
    factor zeroed, applied with numpy's FFT to the periodic kernel."""
    n = (6, 8, 5)
    h = (0.3, 0.2, 0.25)
    w = orc.vgf_kernel(n, h, orc.default_L(n, h))
    W = orc.periodic_kernel(n, w)
    F = np.fft.fftn(W)
    for a in range(3):
        v = orc.field_kernel(n, h, W, a)
        P = 2 * n[a]
        s = np.fft.fftfreq(P, d=1.0 / P)
        s[P // 2] = 0.0
        k = 2 * math.pi * s / (P * h[a])
        shp = [1, 1, 1]
        shp[a] = P
        ref = np.fft.ifftn(-1j * k.reshape(shp) * F)
        assert np.max(np.abs(ref.imag)) < 1e-13 * np.max(np.abs(v))
        assert np.max(np.abs(v - ref.real)) < 1e-13 * np.max(np.abs(v))
        # odd in its own axis
        idx = [slice(None)] * 3
        rev = np.roll(np.flip(v, axis=a), 1, axis=a)
        assert np.max(np.abs(v + rev)) < 1e-13 * np.max(np.abs(v))
