"""Seeded synthetic charge densities (inputs only; no solver arithmetic).

Both the GPU path and the CPU oracle are fed from here, so this module holds
nothing but the random draws and the evaluation of Gaussian charge densities
on the grid x_{a,j} = x0_a + j h_a. The Gaussians are unit-mass and
normalised as in the paper's test sources (Sec. III, Eqs. 10 and 14); the
anisotropic one generalises Eq. (14) to per-axis widths.

Workloads (draws in the order listed, numpy.random.default_rng(seed)):
  gaussian_3d_32      3D, N=32 on [-1,1]^3, one Gaussian sigma=0.1 at 0.
  mixture_2d_512      2D, N=512 on [-1,1]^2, 8 Gaussians:
                      centres U[-.5,.5]^2 (8x2), sigma U[.05,.15] (8),
                      weights Rademacher (8).
  beam_3d_256         3D, N=256 on [-1,1]^3, anisotropic unit Gaussian
                      sigma=(0.05,0.05,0.3), centroid uniform in the ball of
                      radius 0.05 (rejection from the cube [-1,1]^3, scaled).
  batch_3d_mixed      64 right-hand sides, N_b from {32,48,64,96,128}, then
                      per rhs: K_b in {1..4}, centres U[-.5,.5]^3 (K_b x 3),
                      sigma U[.05,.2] (K_b), weights Rademacher (K_b).
  diff_3d_128         8 right-hand sides at N=128 drawn as in batch_3d_mixed
                      (without the N draw); the target field comes from a
                      3-Gaussian mixture drawn the same way from seed+1000.
"""
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np


@dataclass
class Charge:
    """A Gaussian mixture on a uniform grid."""
    n: Tuple[int, ...]
    h: Tuple[float, ...]
    x0: Tuple[float, ...]
    centers: np.ndarray          # (count, dim)
    sigmas: np.ndarray           # (count, dim) per-axis widths
    weights: np.ndarray          # (count,)
    isotropic: bool = True
    meta: dict = field(default_factory=dict)

    @property
    def dim(self):
        return len(self.n)

    def rho(self, dtype=np.float64) -> np.ndarray:
        return gaussian_density(self.n, self.x0, self.h, self.centers, self.sigmas,
                                self.weights).astype(dtype)


def cube_grid(dim: int, N: int, lo: float = -1.0, hi: float = 1.0):
    """N points per axis including both ends of [lo, hi]."""
    h = (hi - lo) / (N - 1)
    return (N,) * dim, (h,) * dim, (lo,) * dim


def gaussian_density(n, x0, h, centers, sigmas, weights) -> np.ndarray:
    """sum_g w_g prod_a (2 pi s_{g,a}^2)^{-1/2} exp(-(x_a - c_{g,a})^2 / (2 s_{g,a}^2))."""
    dim = len(n)
    centers = np.asarray(centers, dtype=np.float64).reshape(-1, dim)
    sigmas = np.asarray(sigmas, dtype=np.float64).reshape(-1, dim)
    weights = np.asarray(weights, dtype=np.float64).reshape(-1)
    out = np.zeros(tuple(n), dtype=np.float64)
    axes = [x0[a] + np.arange(n[a], dtype=np.float64) * h[a] for a in range(dim)]
    for g in range(weights.size):
        fac = []
        for a in range(dim):
            s = sigmas[g, a]
            d = axes[a] - centers[g, a]
            fac.append(np.exp(-d * d / (2.0 * s * s)) / np.sqrt(2.0 * np.pi * s * s))
        if dim == 2:
            out += weights[g] * np.multiply.outer(fac[0], fac[1])
        else:
            out += weights[g] * np.multiply.outer(np.multiply.outer(fac[0], fac[1]), fac[2])
    return out


def gaussian_3d_32(seed: int = 0, N: int = 32, sigma: float = 0.1) -> Charge:
    n, h, x0 = cube_grid(3, N)
    return Charge(n, h, x0, np.zeros((1, 3)), np.full((1, 3), sigma), np.ones(1),
                  meta={"workload": f"gaussian_3d_{N}", "seed": seed})


def mixture_2d_512(seed: int = 0, N: int = 512) -> Charge:
    rng = np.random.default_rng(seed)
    c = rng.uniform(-0.5, 0.5, (8, 2))
    s = rng.uniform(0.05, 0.15, 8)
    w = rng.choice([-1.0, 1.0], 8)
    n, h, x0 = cube_grid(2, N)
    return Charge(n, h, x0, c, np.repeat(s[:, None], 2, axis=1), w,
                  meta={"workload": f"mixture_2d_{N}", "seed": seed})


def beam_3d_256(seed: int = 0, N: int = 256) -> Charge:
    rng = np.random.default_rng(seed)
    while True:
        u = rng.uniform(-1.0, 1.0, 3)
        if float(np.dot(u, u)) <= 1.0:
            break
    c = 0.05 * u
    n, h, x0 = cube_grid(3, N)
    return Charge(n, h, x0, c[None, :], np.array([[0.05, 0.05, 0.3]]), np.ones(1),
                  isotropic=False, meta={"workload": f"beam_3d_{N}", "seed": seed})


def _random_mixture(rng, N: int, kmax: int = 4) -> Charge:
    K = int(rng.integers(1, kmax + 1))
    c = rng.uniform(-0.5, 0.5, (K, 3))
    s = rng.uniform(0.05, 0.2, K)
    w = rng.choice([-1.0, 1.0], K)
    n, h, x0 = cube_grid(3, N)
    return Charge(n, h, x0, c, np.repeat(s[:, None], 3, axis=1), w)


BATCH_SIZES = (32, 48, 64, 96, 128)


def batch_3d_mixed(seed: int = 0, count: int = 64, sizes=BATCH_SIZES) -> List[Charge]:
    rng = np.random.default_rng(seed)
    Ns = rng.choice(np.asarray(sizes), count)
    out = []
    for b in range(count):
        ch = _random_mixture(rng, int(Ns[b]))
        ch.meta = {"workload": "batch_3d_mixed", "seed": seed, "index": b}
        out.append(ch)
    return out


def diff_3d_128(seed: int = 0, batch: int = 8, N: int = 128):
    """Returns (list of rhs Charges, target Charge of 3 Gaussians)."""
    rng = np.random.default_rng(seed)
    rhs = [_random_mixture(rng, N) for _ in range(batch)]
    trng = np.random.default_rng(seed + 1000)
    c = trng.uniform(-0.5, 0.5, (3, 3))
    s = trng.uniform(0.05, 0.2, 3)
    w = trng.choice([-1.0, 1.0], 3)
    n, h, x0 = cube_grid(3, N)
    target = Charge(n, h, x0, c, np.repeat(s[:, None], 3, axis=1), w,
                    meta={"workload": "diff_3d_target", "seed": seed + 1000})
    return rhs, target


def fd_directions(seed: int, shape, count: int, like: np.ndarray) -> np.ndarray:
    """count directions u ~ N(0, I), each rescaled to the 2-norm of `like`."""
    rng = np.random.default_rng(seed + 2000)
    u = rng.standard_normal((count,) + tuple(shape))
    nrm = np.sqrt(np.sum(u.reshape(count, -1) ** 2, axis=1))
    return u * (np.linalg.norm(like.ravel()) / nrm).reshape((count,) + (1,) * len(shape))


def random_field(seed: int, shape) -> np.ndarray:
    """Generic seeded N(0,1) array (used for linearity / adjoint checks)."""
    return np.random.default_rng(seed).standard_normal(tuple(shape))
