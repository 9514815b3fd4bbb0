"""Pins of the oracle's Hockney-Eastwood variants and finite-difference field
(the comparison curves of Sec. III.A: "nearby value", "cell average",
"Finite Diff").

* The cell-average origin weight (integral of G over the origin cell,
  computed by pyramids and Gauss-Legendre) against closed forms for the
  cube and square (3 ln(2 + sqrt 3) - pi/2 for the unit cube; ln 2 - 3 + pi/2
  for the unit square's integral of ln(x^2 + y^2) over [0, 1]^2) and against
  scipy's adaptive quadrature on rectangular cells.
* Every HE variant differs from the others at the origin only, and every one
  converges like h^2 to the closed-form Gaussian potential, while VGF beats
  them all once N >= 24.
* The finite-difference field is exact on quadratics (second-order stencils,
  one-sided ends included), converges like h^2 on a smooth field, and its
  transpose satisfies <D x, y> = <x, D^T y>.
"""
import math

import numpy as np
import pytest

from paper_2103_08531_amd import workloads as W


def test_cell_average_cube_and_square(orc):
    c3 = 3.0 * math.log(2.0 + math.sqrt(3.0)) - math.pi / 2.0  # int over unit cube of 1/r
    for h in (1.0, 0.1, 2.0 / 255):
        v = orc.cell_average_integral((h, h, h))
        assert abs(v - h * h * c3 / (4 * math.pi)) <= 1e-14 * abs(v)
    # int over [-1/2,1/2]^2 of ln r = (ln 2 - 3 + pi/2) / 2 + ln(1/2) / 2 ... by scaling
    i_unit = 0.5 * (math.log(2.0) - 3.0 + math.pi / 2.0)  # int over [0,1]^2 of ln r
    # [-h/2, h/2]^2 = 4 copies of [0, h/2]^2; int_[0,a]^2 ln r = a^2 (i_unit + ln a)
    for h in (1.0, 0.1, 2.0 / 511):
        a = 0.5 * h
        ref = -4.0 * a * a * (i_unit + math.log(a)) / (2.0 * math.pi)
        v = orc.cell_average_integral((h, h))
        assert abs(v - ref) <= 1e-13 * abs(ref), (h, v, ref)


def test_cell_average_rectangular_vs_scipy(orc):
    integrate = pytest.importorskip("scipy.integrate")
    a, b, c = 0.03, 0.05, 0.07
    ref, _ = integrate.tplquad(lambda z, y, x: 1.0 / math.sqrt(x * x + y * y + z * z),
                               0, a, 0, b, 0, c, epsabs=1e-13, epsrel=1e-12)
    v = orc.cell_average_integral((2 * a, 2 * b, 2 * c))
    assert abs(v - 8 * ref / (4 * math.pi)) <= 1e-9 * abs(v)
    ref2, _ = integrate.dblquad(lambda y, x: -0.5 * math.log(x * x + y * y) / (2 * math.pi),
                                0, a, 0, c, epsabs=1e-14, epsrel=1e-12)
    v2 = orc.cell_average_integral((2 * a, 2 * c))
    assert abs(v2 - 4 * ref2) <= 1e-9 * abs(v2)


@pytest.mark.parametrize("dim", [2, 3])
def test_he_variants_differ_only_at_origin(orc, dim):
    n = (8, 12, 10)[:dim]
    h = (0.1, 0.08, 0.12)[:dim]
    ws = [orc.he_kernel(n, h, m) for m in (0, 1, 2)]
    for m in (1, 2):
        d = ws[m] - ws[0]
        d.flat[0] = 0.0
        assert np.all(d == 0.0)
    origins = [w.flat[0] for w in ws]
    assert len(set(origins)) == 3
    vol = float(np.prod(h))
    r0 = 0.5 * min(h)
    g = (lambda r: 1 / (4 * math.pi * r)) if dim == 3 else (lambda r: -math.log(r) / (2 * math.pi))
    assert abs(origins[1] - vol * g(r0)) <= 1e-15 * abs(origins[1])


def _slope(Ns, errs):
    return -np.polyfit(np.log(Ns), np.log(errs), 1)[0]


@pytest.mark.parametrize("method", ["he", "he_nearby", "he_cellavg"])
def test_he_variants_converge_second_order_3d(orc, method):
    Ns, errs, vgf = (16, 24, 32, 48), [], []
    for N in Ns:
        n, h, x0 = W.cube_grid(3, N, -1.0, 1.0)
        c, s = np.zeros((1, 3)), np.full((1, 3), 0.1)
        rho = W.gaussian_density(n, x0, h, c, s, np.ones(1))
        pa, _ = orc.gauss_mixture_grid(n, x0, h, c, s, np.ones(1), want_E=False)
        phi, _ = orc.solve_fft2n(n, h, orc.kernel(method, n, h), rho, want_E=False)
        errs.append(orc.rel_l2(phi, pa))
        if N >= 24:
            pv, _ = orc.solve_fft2n(n, h, orc.kernel("vgf", n, h), rho, want_E=False)
            vgf.append(orc.rel_l2(pv, pa))
    p = _slope(Ns, errs)
    assert 1.7 < p < 2.5, (method, errs, p)
    assert all(v < e for v, e in zip(vgf, errs[1:])), (vgf, errs)


@pytest.mark.parametrize("method", ["he", "he_nearby", "he_cellavg"])
def test_he_variants_converge_second_order_2d(orc, method):
    """The paper's 2D setup: sigma = 0.05 on [-1/2, 1/2]^2."""
    Ns, errs = (24, 32, 48, 64), []
    for N in Ns:
        n, h, x0 = W.cube_grid(2, N, -0.5, 0.5)
        c, s = np.zeros((1, 2)), np.full((1, 2), 0.05)
        rho = W.gaussian_density(n, x0, h, c, s, np.ones(1))
        pa, _ = orc.gauss_mixture_grid(n, x0, h, c, s, np.ones(1), want_E=False)
        phi, _ = orc.solve_fft2n(n, h, orc.kernel(method, n, h), rho, want_E=False)
        errs.append(orc.rel_l2(phi, pa))
    p = _slope(Ns, errs)
    assert 1.6 < p < 2.6, (method, errs, p)


@pytest.mark.parametrize("dim", [2, 3])
def test_fd_field_exact_on_quadratics(orc, dim):
    n = (9, 12, 10)[:dim]
    h = (0.11, 0.07, 0.13)[:dim]
    x = np.meshgrid(*[np.arange(m) * hh - 0.4 for m, hh in zip(n, h)], indexing="ij")
    rng = np.random.default_rng(1)
    A = rng.normal(size=(dim, dim))
    A = A + A.T
    b = rng.normal(size=dim)
    phi = sum(b[a] * x[a] for a in range(dim)) + 0.5 * sum(A[a, c] * x[a] * x[c]
                                                         for a in range(dim) for c in range(dim))
    grad = [b[a] + sum(A[a, c] * x[c] for c in range(dim)) for a in range(dim)]
    E = orc.fd_field(n, h, phi)
    for a in range(dim):
        assert np.max(np.abs(E[a] + grad[a])) < 1e-12 * (1 + np.max(np.abs(grad[a])))


def test_fd_field_second_order_and_transpose(orc):
    errs = []
    for N in (16, 32, 64):
        n = (N, N)
        h = (1.0 / (N - 1), 1.0 / (N - 1))
        x = np.meshgrid(*[np.arange(N) * h[0] for _ in range(2)], indexing="ij")
        phi = np.sin(2.0 * x[0]) * np.cos(1.5 * x[1])
        ex = -2.0 * np.cos(2.0 * x[0]) * np.cos(1.5 * x[1])
        E = orc.fd_field(n, h, phi)
        errs.append(np.max(np.abs(E[0] - ex)))
    p = _slope((16, 32, 64), errs)
    assert 1.8 < p < 2.3, (errs, p)
    n, h = (8, 11, 9), (0.1, 0.2, 0.15)
    rng = np.random.default_rng(2)
    xv = rng.normal(size=n)
    yv = rng.normal(size=(3,) + n)
    lhs = float(np.vdot(orc.fd_field(n, h, xv), yv))
    rhs = float(np.vdot(xv, orc.fd_field_T(n, h, yv)))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


# ---------------------------------------------------------------------------
# Gradient-kernel field (the alternative reading of "multiplying by the
# wavevector": transform -i k_a Ghat on the 4N grid and restrict, Sec. II /
# Sec. III.A).
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_grad_kernel_4n_path_equals_restricted_kernel(orc, dim):
    """The restricted odd kernel convolved on the 2N grid equals the 4N
    "in principle" computation with -i k_a Ghat (both from the oracle, by
    different routes: cosine/sine sums + FFT convolution vs. a 4N FFT)."""
    n = (12, 16, 8)[:dim]
    h = (0.1, 0.09, 0.12)[:dim]
    L = orc.default_L(n, h)
    rho = W.random_field(3, n)
    _, E = orc.solve_grad_kernel(n, h, L, rho, want_phi=False)
    for a in range(dim):
        e4 = orc.solve_fft4n_grad(n, h, L, a, rho)
        assert orc.rel_l2(E[a], e4) < 1e-13, a


def test_grad_kernel_symmetry_and_direct_sum(orc):
    n, h = (8, 10, 12), (0.11, 0.1, 0.09)
    L = orc.default_L(n, h)
    rho = W.random_field(4, n)
    for a in range(3):
        w = orc.vgf_grad_kernel(n, h, L, a)
        idx = [slice(None)] * 3
        idx[a] = 0
        assert np.all(w[tuple(idx)] == 0.0)  # odd in n_a
        V = orc.periodic_kernel_odd(n, w, a)
        direct = orc.conv_periodic(n, V, rho)
        assert orc.rel_l2(orc.conv_fft2n(n, V, rho), direct) < 1e-13


def test_grad_kernel_converges_to_analytic_field(orc):
    errs, errs_ik = [], []
    for N in (16, 24, 32, 48):
        n, h, x0 = W.cube_grid(3, N, -1.0, 1.0)
        c, s = np.zeros((1, 3)), np.full((1, 3), 0.1)
        rho = W.gaussian_density(n, x0, h, c, s, np.ones(1))
        _, Ea = orc.gauss_mixture_grid(n, x0, h, c, s, np.ones(1))
        L = orc.default_L(n, h)
        _, E = orc.solve_grad_kernel(n, h, L, rho, want_phi=False)
        _, E2 = orc.solve_fft2n(n, h, orc.vgf_kernel(n, h, L), rho, want_phi=False)
        errs.append(orc.rel_l2(E, Ea))
        errs_ik.append(orc.rel_l2(E2, Ea))
    assert errs[0] / errs[1] > 30 and errs[1] / errs[2] > 100, errs  # spectral
    assert errs[3] < 1e-11, errs
    # the two readings differ at moderate N (both are converged at N = 48)
    assert abs(errs[2] - errs_ik[2]) > 1e-7, (errs, errs_ik)
