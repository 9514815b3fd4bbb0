"""Behavioural pins of the admissible window of the truncation radius L
(Sec. II): the oracle's window (Lmin, Lmax) is checked by what happens to the
discrete VGF solution at L just inside and just outside each end, not by
restating its formula.

Lmin: below the largest source-target distance the truncated kernel drops
source-target pairs, so the solution changes. Lmax: above it the images of
the truncated kernel that the 4N-periodic inverse DFT creates reach the box,
so the solution changes. Strictly inside, the solution for a charge that is
smooth and contained in the box does not depend on L (to rounding), because
the grid-band-limited kernel and the band-limited charge only see the kernel
inside radius L.

A wrong bound fails one of these: a bound too loose by more than the margin
lets a departing L in (the "agree" check at 0.98 Lmax or 1.02 Lmin fails);
a bound too strict by more than the margin makes the "depart" check at
1.05 Lmax or 0.9 Lmin land inside the true window, where nothing departs.
The charges are placed so that the relevant source-target pairs carry mass:
near a face for the images, in a corner for the longest distances.
"""
import numpy as np
import pytest

from paper_2103_08531_amd import workloads as W


def _charge(dim, N, center, sigma):
    n, h, x0 = W.cube_grid(dim, N)
    c = np.asarray(center, dtype=np.float64).reshape(1, dim)
    rho = W.gaussian_density(n, x0, h, c, np.full((1, dim), sigma), np.ones(1))
    return n, h, rho


def _solve(orc, n, h, rho, L):
    return orc.solve_fft2n(n, h, orc.vgf_kernel(n, h, L), rho)


def _maxrel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _departures(orc, n, h, rho, Ls):
    lo, _ = orc.window(n, h)
    p0, E0 = _solve(orc, n, h, rho, 1.1 * lo)
    out = []
    for L in Ls:
        p, E = _solve(orc, n, h, rho, L)
        out.append((_maxrel(p, p0), _maxrel(E, E0)))
    return out


def test_window_2d_both_ends(orc):
    """2D, 256^2 on [-1,1]^2, sigma = 0.025 at (-0.8, -0.8): 8 sigma from the
    two near faces (contained), and half its mass farther than 0.9 D from
    the far corner; its images at 1.05 Lmax land on the far faces."""
    n, h, rho = _charge(2, 256, [-0.8, -0.8], 0.025)
    lo, hi = orc.window(n, h)
    assert 1.3 * lo < 0.98 * hi
    (a_lo, a_hi, a_mid, d_lo, d_hi) = _departures(orc, n, h, rho,
                                                  [1.02 * lo, 0.98 * hi, 1.3 * lo, 0.9 * lo, 1.05 * hi])
    for p, E in (a_lo, a_hi, a_mid):
        assert p < 1e-13 and E < 1e-12, (a_lo, a_hi, a_mid)
    for p, E in (d_lo, d_hi):
        assert p > 1e-2 and E > 1e-2, (d_lo, d_hi)


def test_window_3d_upper_end(orc):
    """3D, 64^3, sigma = 0.065 at (-0.5, 0.05, 0): contained (7.7 sigma from
    the nearest face); sources below x0 = -0.69 reach the targets near
    x0 = 1 through the images once L passes 1.05 Lmax."""
    n, h, rho = _charge(3, 64, [-0.5, 0.05, 0.0], 0.065)
    lo, hi = orc.window(n, h)
    (a_lo, a_hi, d_hi) = _departures(orc, n, h, rho, [1.02 * lo, 0.98 * hi, 1.05 * hi])
    for p, E in (a_lo, a_hi):
        assert p < 1e-11 and E < 1e-10, (a_lo, a_hi)
    assert d_hi[0] > 1e-6 and d_hi[1] > 1e-5, d_hi


def test_window_3d_lower_end(orc):
    """3D, 32^3, sigma = 0.1 at (-0.8, -0.8, -0.8): a contained charge cannot
    reach 0.9 D from a corner target on a grid this size, so this one sits
    in the corner and is cut by the faces. Its solution then varies with L
    inside the window at the 1e-6 level (the cut makes it less than
    band-limited), far below what dropping source-target pairs does."""
    n, h, rho = _charge(3, 32, [-0.8, -0.8, -0.8], 0.1)
    lo, _ = orc.window(n, h)
    (a_lo, d_lo) = _departures(orc, n, h, rho, [1.02 * lo, 0.9 * lo])
    assert a_lo[0] < 1e-5 and a_lo[1] < 1e-4, a_lo
    assert d_lo[0] > 1e-3 and d_lo[1] > 1e-3, d_lo
    assert d_lo[0] > 1e3 * a_lo[0] and d_lo[1] > 1e3 * a_lo[1]


def test_window_rectangular_grid(orc):
    """The upper end is set by the axis with the smallest 4 N_a h_a - extent_a:
    on a 2D grid with unequal N and h, a charge near the low face of that
    axis departs at 1.05 Lmax and agrees at 0.98 Lmax."""
    n, h = (96, 128), (2.0 / 95, 2.6 / 127)
    x0 = (-1.0, -1.3)
    lims = [4 * n[a] * h[a] - (n[a] - 1) * h[a] for a in range(2)]
    a = int(np.argmin(lims))
    c = np.zeros((1, 2))
    c[0, a] = x0[a] + 0.2 * (n[a] - 1) * h[a]  # 8 sigma from the face
    rho = W.gaussian_density(n, x0, h, c, np.full((1, 2), 0.05), np.ones(1))
    lo, hi = orc.window(n, h)
    p0, E0 = _solve(orc, n, h, rho, 1.1 * lo)
    pa, Ea = _solve(orc, n, h, rho, 0.98 * hi)
    pd, Ed = _solve(orc, n, h, rho, 1.05 * hi)
    assert _maxrel(pa, p0) < 1e-12 and _maxrel(Ea, E0) < 1e-11
    assert _maxrel(pd, p0) > 1e-6 and _maxrel(Ed, E0) > 1e-5
