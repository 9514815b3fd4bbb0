"""Pins of the oracle's closed-form Gaussian potentials (Sec. III, Eqs. 10-11,
14-15) and of its special functions. Each analytic solution is checked to
solve the problem itself: -Laplace(phi) = rho and E = -grad(phi) by finite
differences, the far field tends to the free-space Green's function, and the
special functions agree with scipy's independent implementations."""
import math

import numpy as np
import pytest
import scipy.integrate as si
import scipy.special as ss

EULER = 0.5772156649015329


@pytest.mark.parametrize("u", list(np.logspace(-4, 2.6, 37)))
def test_e1_and_ein_match_scipy(orc, u):
    assert orc.expint_e1(u) == pytest.approx(ss.exp1(u), rel=2e-14, abs=1e-300)
    assert orc.ein(u) == pytest.approx(ss.exp1(u) + EULER + math.log(u), rel=2e-14)


def _laplacian_fd(f, x, d):
    """Fourth-order central differences."""
    x = np.asarray(x, dtype=np.float64)
    tot = 0.0
    for a in range(x.size):
        e = np.zeros_like(x)
        e[a] = d
        tot += (-f(x + 2 * e) + 16 * f(x + e) - 30 * f(x) + 16 * f(x - e) - f(x - 2 * e)) / (12 * d * d)
    return tot


def _grad_fd(f, x, d):
    x = np.asarray(x, dtype=np.float64)
    g = np.zeros_like(x)
    for a in range(x.size):
        e = np.zeros_like(x)
        e[a] = d
        g[a] = (-f(x + 2 * e) + 8 * f(x + e) - 8 * f(x - e) + f(x - 2 * e)) / (12 * d)
    return g


PTS3 = [(0.05, -0.02, 0.03), (0.11, 0.07, -0.09), (0.3, -0.2, 0.25), (0.0, 0.0, 0.21)]
PTS2 = [(0.05, -0.02), (0.11, 0.07), (0.3, -0.2), (0.0, 0.21)]


@pytest.mark.parametrize("x", PTS3)
def test_gauss3d_solves_poisson(orc, x):
    sig, c = 0.1, np.array([0.01, -0.02, 0.005])
    rho = lambda p: math.exp(-np.sum((p - c) ** 2) / (2 * sig * sig)) / ((2 * math.pi) ** 1.5 * sig**3)
    phi = lambda p: orc.gauss3d_point(sig, c, p)[0]
    lap = _laplacian_fd(phi, x, 1e-3)
    assert abs(-lap - rho(np.array(x))) < 2e-5 * max(1.0, rho(np.array(x)))
    g = _grad_fd(phi, x, 1e-4)
    E = orc.gauss3d_point(sig, c, x)[1]
    assert np.max(np.abs(E + g)) < 1e-8 * max(1.0, np.max(np.abs(E)))
    # closed form against scipy's erf
    r = np.linalg.norm(np.array(x) - c)
    assert phi(np.array(x)) == pytest.approx(ss.erf(r / (math.sqrt(2) * sig)) / (4 * math.pi * r), rel=1e-15)


@pytest.mark.parametrize("x", PTS2)
def test_gauss2d_solves_poisson(orc, x):
    """Also pins the reading E1 (not Ei) of the printed 2D potential."""
    sig, c = 0.05, np.array([0.01, -0.02])
    rho = lambda p: math.exp(-np.sum((p - c) ** 2) / (2 * sig * sig)) / (2 * math.pi * sig * sig)
    phi = lambda p: orc.gauss2d_point(sig, c, p)[0]
    lap = _laplacian_fd(phi, x, 5e-4)
    assert abs(-lap - rho(np.array(x))) < 1e-4 * max(1.0, rho(np.array(x)))
    g = _grad_fd(phi, x, 1e-4)
    E = orc.gauss2d_point(sig, c, x)[1]
    assert np.max(np.abs(E + g)) < 1e-8 * max(1.0, np.max(np.abs(E)))
    r2 = float(np.sum((np.array(x) - c) ** 2))
    ref = -(ss.exp1(r2 / (2 * sig * sig)) + math.log(r2)) / (4 * math.pi)
    assert phi(np.array(x)) == pytest.approx(ref, rel=1e-13)


def test_far_field_is_green_function(orc):
    for r in (3.0, 10.0):
        p3, _ = orc.gauss3d_point(0.05, np.zeros(3), np.array([r, 0, 0]))
        assert p3 == pytest.approx(1 / (4 * math.pi * r), rel=1e-15)
        p2, _ = orc.gauss2d_point(0.05, np.zeros(2), np.array([0, r]))
        assert p2 == pytest.approx(-math.log(r) / (2 * math.pi), rel=1e-14)


def test_centre_values_closed_form(orc):
    """P12: phi*(0) = 1/((2 pi)^{3/2} sigma) in 3D, (gamma - ln 2 sigma^2)/(4 pi) in 2D."""
    for s in (0.05, 0.1, 0.3):
        p3, E3 = orc.gauss3d_point(s, np.zeros(3), np.zeros(3))
        assert p3 == pytest.approx(1 / ((2 * math.pi) ** 1.5 * s), rel=1e-15)
        assert np.all(E3 == 0.0)
        p2, E2 = orc.gauss2d_point(s, np.zeros(2), np.zeros(2))
        assert p2 == pytest.approx((EULER - math.log(2 * s * s)) / (4 * math.pi), rel=1e-15)
        # continuity at the origin
        p3b, _ = orc.gauss3d_point(s, np.zeros(3), np.array([1e-7, 0, 0]))
        assert p3b == pytest.approx(p3, rel=1e-12)


@pytest.mark.parametrize("x", PTS3 + [(0.0, 0.0, 0.0), (0.9, -0.9, 0.95)])
def test_aniso_integral_reduces_to_erf(orc, x):
    """P9: the 1-D integral with equal widths equals the erf closed form."""
    c = np.array([0.02, 0.0, -0.01])
    for s in (0.05, 0.1):
        pa, Ea = orc.gauss3d_aniso_point([s, s, s], c, x)
        pi, Ei = orc.gauss3d_point(s, c, np.array(x))
        assert pa == pytest.approx(pi, rel=1e-14)
        assert np.max(np.abs(Ea - Ei)) < 1e-13 * max(1.0, np.max(np.abs(Ei)))


@pytest.mark.parametrize("x", [(0.02, 0.01, 0.2), (0.3, -0.1, 0.6), (-0.7, 0.5, -0.9)])
def test_aniso_integral_vs_quad_and_poisson(orc, x):
    sig = np.array([0.05, 0.05, 0.3])
    c = np.array([0.01, -0.02, 0.03])
    d = np.array(x) - c

    def integrand(t):
        den = 1 + 2 * sig**2 * t * t
        return np.prod(den**-0.5) * math.exp(-np.sum(d * d * t * t / den))

    ref, _ = si.quad(integrand, 0, np.inf, limit=500, epsabs=0, epsrel=1e-13)
    ref /= 2 * math.pi**1.5
    p, E = orc.gauss3d_aniso_point(sig, c, x)
    assert p == pytest.approx(ref, rel=1e-11)
    # step halving leaves the value unchanged (quadrature converged)
    p2, E2 = orc.gauss3d_aniso_point(sig, c, x, step=1.0 / 128.0)
    assert p2 == pytest.approx(p, rel=1e-15)
    assert np.max(np.abs(E2 - E)) < 1e-14 * np.max(np.abs(E))
    phi = lambda q: orc.gauss3d_aniso_point(sig, c, q)[0]
    rho = lambda q: math.exp(-np.sum((q - c) ** 2 / (2 * sig**2))) / ((2 * math.pi) ** 1.5 * np.prod(sig))
    lap = _laplacian_fd(phi, x, 1e-3)
    assert abs(-lap - rho(np.array(x))) < 1e-4 * max(1.0, rho(np.array(x)))
    g = _grad_fd(phi, x, 1e-4)
    assert np.max(np.abs(E + g)) < 1e-8 * max(1.0, np.max(np.abs(E)))


def test_mixture_grid_is_superposition(orc):
    n, x0, h = (5, 6, 4), (-1.0, -1.0, -1.0), (0.5, 0.4, 0.6)
    cen = np.array([[0.1, 0.2, -0.1], [-0.3, 0.0, 0.2]])
    sig = np.array([[0.1] * 3, [0.2] * 3])
    w = np.array([1.0, -1.0])
    phi, E = orc.gauss_mixture_grid(n, x0, h, cen, sig, w)
    x = np.array([x0[0] + 3 * h[0], x0[1] + 2 * h[1], x0[2] + 1 * h[2]])
    p0, E0 = orc.gauss3d_point(0.1, cen[0], x)
    p1, E1 = orc.gauss3d_point(0.2, cen[1], x)
    assert phi[3, 2, 1] == pytest.approx(p0 - p1, rel=1e-15)
    assert np.allclose(E[:, 3, 2, 1], E0 - E1, rtol=1e-15, atol=0)
