"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and the FP64 oracle on the same seeded input."""
import math
import sys

import numpy as np
import pytest

import oracle as orc
from paper_2103_08531_amd import workloads as W

FP64_TOL = 1e-12
FP32_TOL = 1e-5


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2103_08531_amd import vgf
    vgf.lib()
    return torch, vgf


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return math.sqrt(float(np.sum((a - b) ** 2)) / float(np.sum(b * b)))


def gpu_solve(plan, rho_np, want_phi=True, want_E=True):
    torch, vgf = need_gpu()
    rho = torch.from_numpy(np.ascontiguousarray(rho_np)).to(device="cuda", dtype=plan.dtype)
    phi, E = plan.solve(rho, want_phi=want_phi, want_E=want_E)
    torch.cuda.synchronize()
    return (None if phi is None else phi.double().cpu().numpy(),
            None if E is None else E.double().cpu().numpy())


def oracle_kernel(method, n, h, L):
    return orc.kernel(method, n, h, L)


def oracle_solve(method, n, h, L, rho_np, want_E=True):
    w = oracle_kernel(method, n, h, L)
    return orc.solve_fft2n(n, h, w, np.asarray(rho_np, dtype=np.float64), want_E=want_E)


def rounded_input(rho_np, precision):
    """The exact values the GPU receives, widened back to FP64 for the oracle."""
    return rho_np.astype(np.float32).astype(np.float64) if precision == "f32" else rho_np


def check_fields(phi_g, E_g, phi_o, E_o, tol, label):
    out = {}
    if phi_o is not None:
        e = rel_l2(phi_g, phi_o)
        out["phi"] = e
        say("%s phi rel-L2 %.3e" % (label, e))
        assert e <= tol, (label, "phi", e)
    if E_o is not None:
        for a in range(E_o.shape[0]):
            e = rel_l2(E_g[a], E_o[a])
            out["E%d" % a] = e
            say("%s E%d rel-L2 %.3e" % (label, a, e))
            assert e <= tol, (label, "E%d" % a, e)
    return out
