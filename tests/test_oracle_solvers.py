"""Pins of the oracle's solvers.

P1  VGF converges spectrally to the closed-form Gaussian potential/field
    (Sec. III), on cubic and on rectangular grids.
P2  Hockney-Eastwood converges like h^2 (Sec. I, Sec. III).
P5  direct discrete convolution == 2N FFT path == 4N FFT path (Sec. II).
P6  the VGF result does not depend on L inside the admissible window.
P7  linearity and integer-shift equivariance.
P8  Fourier-differentiated field == direct cot-stencil convolution.
P10 adjoint identities <K x, y> = <x, K^T y>, K^T = K, K_a^T = -K_a.
P4  symmetry of phi and antisymmetry of E for a centred Gaussian.
"""
import math

import numpy as np
import pytest

from paper_2103_08531_amd import workloads as W


def _gauss_case(orc, dim, N, sigma, lo=-1.0, hi=1.0, center=None):
    n, h, x0 = W.cube_grid(dim, N, lo, hi)
    c = np.zeros((1, dim)) if center is None else np.asarray(center).reshape(1, dim)
    s = np.full((1, dim), sigma)
    rho = W.gaussian_density(n, x0, h, c, s, np.ones(1))
    phi_a, E_a = orc.gauss_mixture_grid(n, x0, h, c, s, np.ones(1))
    return n, h, x0, rho, phi_a, E_a


def test_p1_vgf_spectral_convergence_3d(orc):
    errs, errE = [], []
    for N in (16, 24, 32):
        n, h, x0, rho, pa, Ea = _gauss_case(orc, 3, N, 0.1)
        w = orc.vgf_kernel(n, h, orc.default_L(n, h))
        phi, E = orc.solve_fft2n(n, h, w, rho)
        errs.append(orc.rel_l2(phi, pa))
        errE.append(orc.rel_l2(E, Ea))
    assert errs[0] < 1e-3 and errs[1] < 1e-5 and errs[2] < 1e-8, errs
    assert errs[0] / errs[1] > 50 and errs[1] / errs[2] > 300, errs  # faster than any power
    assert errE[2] < 1e-5 and errE[0] > errE[1] > errE[2], errE


def test_p1_vgf_converges_to_rounding_3d(orc):
    n, h, x0, rho, pa, Ea = _gauss_case(orc, 3, 48, 0.1)
    w = orc.vgf_kernel(n, h, orc.default_L(n, h))
    phi, E = orc.solve_fft2n(n, h, w, rho)
    assert orc.rel_l2(phi, pa) < 1e-14
    assert orc.rel_l2(E, Ea) < 1e-9


def test_p1_vgf_paper_2d_setup(orc):
    """The 2D test of Sec. III.A: sigma = 0.05 on [-0.5, 0.5]^2."""
    errs = []
    for N in (17, 33, 49):
        n, h, x0, rho, pa, Ea = _gauss_case(orc, 2, N, 0.05, -0.5, 0.5)
        w = orc.vgf_kernel(n, h, orc.default_L(n, h))
        phi, E = orc.solve_fft2n(n, h, w, rho)
        errs.append(orc.rel_l2(phi, pa))
        if N == 49:
            assert orc.rel_l2(E, Ea) < 1e-10
            # the paper's metric, Eq. (12): max pointwise relative error
            assert np.max(np.abs((phi - pa) / pa)) < 1e-13
    assert errs[1] < 1e-7 and errs[2] < 1e-14, errs


def test_p1_vgf_rectangular_grid(orc):
    """Different N_a and h_a per axis: an axis mix-up anywhere breaks this."""
    n = (28, 32, 36)
    lo = (-0.9, -1.0, -1.1)
    h = tuple(-2 * l / (m - 1) for l, m in zip(lo, n))
    c = np.array([[0.03, -0.02, 0.05]])
    s = np.full((1, 3), 0.1)
    rho = W.gaussian_density(n, lo, h, c, s, np.ones(1))
    pa, Ea = orc.gauss_mixture_grid(n, lo, h, c, s, np.ones(1))
    w = orc.vgf_kernel(n, h, orc.default_L(n, h))
    phi, E = orc.solve_fft2n(n, h, w, rho)
    assert orc.rel_l2(phi, pa) < 1e-8
    for a in range(3):
        assert orc.rel_l2(E[a], Ea[a]) < 1e-5


def test_p2_he_second_order(orc):
    Ns = (16, 24, 32, 48, 64)
    hs, errs = [], []
    for N in Ns:
        n, h, x0, rho, pa, Ea = _gauss_case(orc, 3, N, 0.1)
        phi, _ = orc.solve_fft2n(n, h, orc.he_kernel(n, h), rho, want_E=False)
        hs.append(h[0])
        errs.append(orc.rel_l2(phi, pa))
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert 1.8 < slope < 2.2, (slope, errs)


def test_p2_he_second_order_2d(orc):
    Ns = (17, 25, 33, 49, 65)
    hs, errs = [], []
    for N in Ns:
        n, h, x0, rho, pa, Ea = _gauss_case(orc, 2, N, 0.05, -0.5, 0.5)
        phi, _ = orc.solve_fft2n(n, h, orc.he_kernel(n, h), rho, want_E=False)
        hs.append(h[0])
        errs.append(orc.rel_l2(phi, pa))
    slope = np.polyfit(np.log(hs), np.log(errs), 1)[0]
    assert 1.7 < slope < 2.3, (slope, errs)


CASES = [((6, 8, 9), (0.31, 0.27, 0.22)), ((8, 8, 8), (2 / 7,) * 3), ((12, 16), (0.11, 0.09)),
         ((9, 6), (0.2, 0.3))]


@pytest.mark.parametrize("n,h", CASES)
@pytest.mark.parametrize("method", ["vgf", "he"])
def test_p5_direct_equals_2n_equals_4n(orc, n, h, method):
    rho = W.random_field(11, n)
    L = orc.default_L(n, h)
    w = orc.kernel(method, n, h, L)
    direct = orc.conv_direct(n, w, rho)
    phi2, E2 = orc.solve_fft2n(n, h, w, rho)
    scale = np.max(np.abs(direct))
    assert np.max(np.abs(phi2 - direct)) < 1e-14 * scale * 10
    if method == "vgf":
        phi4 = orc.solve_fft4n(n, h, L, rho)
        assert np.max(np.abs(phi4 - direct)) < 1e-14 * scale * 10
    # P8: the field from i k on the 2N grid equals the direct cot-stencil sums
    Wp = orc.periodic_kernel(n, w)
    for a in range(len(n)):
        v = orc.field_kernel(n, h, Wp, a)
        Ed = orc.conv_periodic(n, v, rho)
        assert np.max(np.abs(E2[a] - Ed)) < 1e-13 * np.max(np.abs(Ed))
    # the periodic embedding reproduces the even-kernel sums
    assert np.max(np.abs(orc.conv_periodic(n, Wp, rho) - direct)) < 1e-14 * scale * 10
    # sampled single points
    for idx in [(0,) * len(n), tuple(x - 1 for x in n), tuple(x // 2 for x in n)]:
        assert orc.conv_direct_point(n, w, rho, idx) == pytest.approx(direct[idx], rel=1e-14, abs=1e-14 * scale)


def test_p6_L_independence(orc):
    n, h, x0, rho, pa, Ea = _gauss_case(orc, 3, 40, 0.1, center=[0.02, -0.01, 0.03])
    lo, hi = orc.window(n, h)
    assert 1.4 * lo < hi
    p1, E1 = orc.solve_fft2n(n, h, orc.vgf_kernel(n, h, 1.1 * lo), rho)
    p2, E2 = orc.solve_fft2n(n, h, orc.vgf_kernel(n, h, 1.4 * lo), rho)
    assert orc.rel_l2(p1, p2) < 1e-11
    assert orc.rel_l2(E1, E2) < 1e-8


def test_p7_linearity_and_shift(orc):
    n, h = (10, 12, 8), (0.2, 0.15, 0.25)
    w = orc.vgf_kernel(n, h, orc.default_L(n, h))
    a, b = W.random_field(1, n), W.random_field(2, n)
    pa, Ea = orc.solve_fft2n(n, h, w, a)
    pb, Eb = orc.solve_fft2n(n, h, w, b)
    pc, Ec = orc.solve_fft2n(n, h, w, 2.5 * a - 0.75 * b)
    assert np.max(np.abs(pc - (2.5 * pa - 0.75 * pb))) < 1e-13 * np.max(np.abs(pc))
    assert np.max(np.abs(Ec - (2.5 * Ea - 0.75 * Eb))) < 1e-13 * np.max(np.abs(Ec))
    # integer shift: rho supported away from the last plane, shifted by one
    r = W.random_field(3, n)
    r[-1, :, :] = 0.0
    s = np.zeros_like(r)
    s[1:, :, :] = r[:-1, :, :]
    pr, _ = orc.solve_fft2n(n, h, w, r, want_E=False)
    ps, _ = orc.solve_fft2n(n, h, w, s, want_E=False)
    assert np.max(np.abs(ps[1:] - pr[:-1])) < 1e-13 * np.max(np.abs(pr))


@pytest.mark.parametrize("n,h", [((6, 8, 5), (0.3, 0.2, 0.25)), ((10, 7), (0.2, 0.3))])
def test_p10_adjoint_identities(orc, n, h):
    dim = len(n)
    w = orc.vgf_kernel(n, h, orc.default_L(n, h))
    Wp = orc.periodic_kernel(n, w)
    x, y = W.random_field(5, n), W.random_field(6, n)
    gE = W.random_field(7, (dim,) + n)
    Kx = orc.conv_periodic(n, Wp, x)
    KTy = orc.conv_periodic_T(n, Wp, y)
    assert abs(np.vdot(Kx, y) - np.vdot(x, KTy)) < 1e-13 * abs(np.vdot(Kx, y)) + 1e-14
    assert np.max(np.abs(KTy - orc.conv_periodic(n, Wp, y))) < 1e-13 * np.max(np.abs(KTy))
    total = KTy.copy()
    for a in range(dim):
        v = orc.field_kernel(n, h, Wp, a)
        KaT = orc.conv_periodic_T(n, v, gE[a])
        Ka = orc.conv_periodic(n, v, gE[a])
        assert np.max(np.abs(KaT + Ka)) < 1e-12 * np.max(np.abs(Ka))
        Kax = orc.conv_periodic(n, v, x)
        assert abs(np.vdot(Kax, gE[a]) - np.vdot(x, KaT)) < 1e-12 * np.max(np.abs(Kax)) * x.size
        total += KaT
    # the FFT-route adjoint equals the direct transposed sums
    g_rho = orc.adjoint_fft2n(n, h, w, y, gE)
    assert np.max(np.abs(g_rho - total)) < 1e-13 * np.max(np.abs(total))


def test_p4_symmetry_centred_gaussian(orc):
    n, h, x0, rho, pa, Ea = _gauss_case(orc, 3, 24, 0.1)
    w = orc.vgf_kernel(n, h, orc.default_L(n, h))
    phi, E = orc.solve_fft2n(n, h, w, rho)
    for a in range(3):
        assert np.max(np.abs(phi - np.flip(phi, axis=a))) < 1e-13 * np.max(np.abs(phi))
        assert np.max(np.abs(E[a] + np.flip(E[a], axis=a))) < 1e-12 * np.max(np.abs(E[a]))
    assert np.max(np.abs(phi - phi.transpose(1, 0, 2))) < 1e-13 * np.max(np.abs(phi))
