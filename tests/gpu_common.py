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


def gpu_plan(vgf, n, h, method="vgf", **kw):
    """A plan whose truncation radius is the oracle's default L, passed
    explicitly (VGF) and read back: both sides then solve with the same L by
    construction, never with whatever the library would choose."""
    L = kw.pop("L", None)
    if method == "vgf" and L is None:
        L = orc.default_L(n, h)
    plan = vgf.Plan(n, h, method=method, L=L, **kw)
    if method == "vgf":
        assert plan.L == L, (plan.L, L)
    return plan


def max_rel(a, b):
    """max |a - b| over max |b|: element-wise, so one wrong plane or row of a
    large grid cannot hide in a norm over all points."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b))) / float(np.max(np.abs(b)))


def err(a, b):
    """The larger of rel-L2 and the element-wise max_rel of a against b."""
    return max(rel_l2(a, b), max_rel(a, b))


def check_fields(phi_g, E_g, phi_o, E_o, tol, label, elem_tol=None):
    """Per field: rel-L2 <= tol and max |gpu - ref| <= elem_tol * max |ref|
    (elem_tol defaults to tol)."""
    elem_tol = tol if elem_tol is None else elem_tol
    out = {}
    pairs = []
    if phi_o is not None:
        pairs.append(("phi", phi_g, phi_o))
    if E_o is not None:
        pairs += [("E%d" % a, E_g[a], E_o[a]) for a in range(E_o.shape[0])]
    for name, g, o in pairs:
        e = rel_l2(g, o)
        m = max_rel(g, o)
        out[name] = e
        out[name + "_max"] = m
        say("%s %s rel-L2 %.3e max %.3e" % (label, name, e, m))
        assert e <= tol, (label, name, e)
        assert m <= elem_tol, (label, name, "max", m)
    return out
