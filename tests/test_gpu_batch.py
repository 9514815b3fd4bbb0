"""Batched solves (vgf_batch_*): entries of several plans, one launch per pass
and per plan, optionally replayed as one captured hipGraph. Every entry must
equal vgf_solve on the same plan bit for bit (the same kernels in the same
arithmetic order), across graph replays with eager work between them, new
pointers and new output sets; and a mixed batch must match the FP64 oracle."""
import ctypes as C

import numpy as np
import pytest

import oracle as orc
from gpu_common import FP32_TOL, FP64_TOL, check_fields, need_gpu, rounded_input, gpu_plan, say
from paper_2103_08531_amd import workloads as W

pytestmark = pytest.mark.gpu


def _plans(vgf, specs):
    plans = {}
    for n, prec, method in specs:
        key = (n, prec, method)
        if key not in plans:
            h = tuple(2.0 / (x - 1) for x in n)
            plans[key] = gpu_plan(vgf, n, h, method=method, precision=prec)
    return plans


def _entries(torch, plans, keys, seed):
    rhos = []
    for i, k in enumerate(keys):
        p = plans[k]
        rhos.append(torch.from_numpy(W.random_field(seed + i, p.n)).to("cuda", p.dtype))
    return rhos


def _outputs(torch, plans, keys):
    phis = [torch.full(plans[k].n, float("nan"), dtype=plans[k].dtype, device="cuda") for k in keys]
    Es = [torch.full((plans[k].dim,) + plans[k].n, float("nan"), dtype=plans[k].dtype, device="cuda")
          for k in keys]
    return phis, Es


# 3D and 2D, both precisions, VGF and HE, repeated plans (groups of 1..3)
KEYS = [((32, 32, 32), "f32", "vgf"), ((48, 48, 48), "f32", "vgf"), ((32, 32, 32), "f32", "vgf"),
        ((16, 24, 32), "f64", "vgf"), ((32, 32, 32), "f32", "vgf"), ((64, 48), "f64", "he"),
        ((96, 96, 96), "f32", "vgf"), ((64, 48), "f64", "he"), ((24, 24, 24), "f64", "vgf")]


@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_single_solves(graph):
    torch, vgf = need_gpu()
    plans = _plans(vgf, KEYS)
    batch = vgf.Batch([plans[k] for k in KEYS], graph=graph)
    assert batch.groups == len(set(KEYS))
    say("batch of %d entries, %d groups, graph=%s, %.1f MB" % (len(KEYS), batch.groups, graph,
                                                                batch.workspace_bytes / 1e6))
    for rep in range(3):
        rhos = _entries(torch, plans, KEYS, seed=100 * rep)
        phis, Es = _outputs(torch, plans, KEYS)
        batch.solve(rhos, phis, Es)
        # eager work between replays on the same stream
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for i, k in enumerate(KEYS):
            p1, E1 = plans[k].solve(rhos[i])
            torch.cuda.synchronize()
            assert torch.equal(phis[i], p1), (rep, i, k)
            assert torch.equal(Es[i], E1), (rep, i, k)
        say("  replay %d: all %d entries bit-identical to vgf_solve" % (rep, len(KEYS)))
    # a different output set re-captures; E only, then phi only
    rhos = _entries(torch, plans, KEYS, seed=7)
    phis, Es = _outputs(torch, plans, KEYS)
    batch.solve(rhos, None, Es)
    torch.cuda.synchronize()
    for i, k in enumerate(KEYS):
        _, E1 = plans[k].solve(rhos[i], want_phi=False)
        torch.cuda.synchronize()
        assert torch.equal(Es[i], E1), ("E only", i)
        assert torch.isnan(phis[i]).all()
    batch.solve(rhos, phis, None)
    torch.cuda.synchronize()
    for i, k in enumerate(KEYS):
        p1, _ = plans[k].solve(rhos[i], want_E=False)
        torch.cuda.synchronize()
        assert torch.equal(phis[i], p1), ("phi only", i)
    batch.close()
    for p in plans.values():
        p.close()


# plans of every field mode and layout in one batch: centred differences,
# gradient kernels (both layouts), the axis-0 layout with Fourier fields, and
# the default; 3D and 2D, both precisions, groups of 1 and 2 entries
MODE_SPECS = [((24, 32, 16), "f64", "centered", "contiguous"), ((48, 64), "f32", "centered", "contiguous"),
              ((32, 32, 32), "f32", "gradient_kernel", "axis0"), ((64, 48), "f64", "gradient_kernel", "axis0"),
              ((24, 24, 24), "f64", "fourier", "axis0"), ((32, 32, 32), "f32", "fourier", "contiguous"),
              ((24, 32, 16), "f32", "gradient_kernel", "contiguous"), ((48, 64), "f64", "gradient_kernel", "contiguous")]
MODE_ENTRIES = [0, 1, 2, 3, 4, 5, 2, 0, 3, 6, 7, 6]


@pytest.mark.parametrize("graph", [False, True])
def test_batch_field_modes_equal_single_solves(graph):
    """Batches of finite-difference and gradient-kernel plans (mixed with
    the other layouts) give every entry exactly what vgf_solve gives, for
    phi + E, E only and phi only, across new pointers and after autotuning."""
    torch, vgf = need_gpu()
    plans = []
    for n, prec, field, layout in MODE_SPECS:
        h = tuple(2.0 / (x - 1) for x in n)
        plans.append(gpu_plan(vgf, n, h, precision=prec, field=field, layout=layout))
    ents = [plans[i] for i in MODE_ENTRIES]
    batch = vgf.Batch(ents, graph=graph)
    assert batch.groups == len(MODE_SPECS)

    def run(seed, want_phi, want_E, tune=False):
        rhos = [torch.from_numpy(W.random_field(seed + i, p.n)).to("cuda", p.dtype) for i, p in enumerate(ents)]
        phis = [torch.full(p.n, float("nan"), dtype=p.dtype, device="cuda") for p in ents]
        Es = [torch.full((p.dim,) + p.n, float("nan"), dtype=p.dtype, device="cuda") for p in ents]
        args = (rhos, phis if want_phi else None, Es if want_E else None)
        if tune:
            say("  schedules after autotune: %s" % (batch.autotune(*args, reps=2),))
        batch.solve(*args)
        junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between solves
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for i, p in enumerate(ents):
            p1, E1 = p.solve(rhos[i], want_phi=want_phi, want_E=want_E)
            torch.cuda.synchronize()
            tag = (seed, want_phi, want_E, i, p.n, p.field, p.layout)
            if want_phi:
                assert torch.equal(phis[i], p1), tag
            else:
                assert torch.isnan(phis[i]).all(), tag
            if want_E:
                assert torch.equal(Es[i], E1), tag
            else:
                assert torch.isnan(Es[i]).all(), tag
        say("  seed %d phi=%s E=%s: all %d entries bit-identical to vgf_solve" % (seed, want_phi, want_E, len(ents)))

    say("field-mode batch: %d entries, %d groups, graph=%s" % (len(ents), batch.groups, graph))
    run(0, True, True)
    run(10, True, True)
    run(20, False, True)
    run(30, True, False)
    run(40, True, True, tune=True)
    batch.close()
    for p in plans:
        p.close()


@pytest.mark.parametrize("graph", [False, True])
def test_batch_adjoint_equals_single_adjoints(graph):
    """vgf_batch_adjoint gives every entry exactly what vgf_solve_adjoint
    gives (batched groups and per-entry groups alike), for both cotangents
    and each alone; a solve of the same batch afterwards (its graph replayed
    with the solve's pointers restored) still equals vgf_solve."""
    torch, vgf = need_gpu()
    plans = []
    for n, prec, field, layout in MODE_SPECS:
        h = tuple(2.0 / (x - 1) for x in n)
        plans.append(gpu_plan(vgf, n, h, precision=prec, field=field, layout=layout))
    ents = [plans[i] for i in MODE_ENTRIES] + [plans[5], plans[5]]  # a group of three
    batch = vgf.Batch(ents, graph=graph)
    rhos = [torch.from_numpy(W.random_field(60 + i, p.n)).to("cuda", p.dtype) for i, p in enumerate(ents)]
    phis = [torch.empty(p.n, dtype=p.dtype, device="cuda") for p in ents]
    Es = [torch.empty((p.dim,) + p.n, dtype=p.dtype, device="cuda") for p in ents]
    batch.solve(rhos, phis, Es)  # captures the graph with the solve's pointers
    for seed, wp, wE in ((70, True, True), (80, False, True), (90, True, False)):
        gps = [torch.from_numpy(W.random_field(seed + i, p.n)).to("cuda", p.dtype) for i, p in enumerate(ents)]
        gEs = [torch.from_numpy(W.random_field(seed + 50 + i, (p.dim,) + p.n)).to("cuda", p.dtype)
               for i, p in enumerate(ents)]
        grs = [torch.full(p.n, float("nan"), dtype=p.dtype, device="cuda") for p in ents]
        batch.adjoint(gps if wp else None, gEs if wE else None, grs)
        torch.cuda.synchronize()
        for i, p in enumerate(ents):
            ref = p.adjoint(gps[i] if wp else None, gEs[i] if wE else None)
            torch.cuda.synchronize()
            assert torch.equal(grs[i], ref), (seed, wp, wE, i, p.n, p.field, p.layout)
        say("  adjoint g_phi=%s g_E=%s: all %d entries bit-identical to vgf_solve_adjoint"
            % (wp, wE, len(ents)))
    rhos = [torch.from_numpy(W.random_field(95 + i, p.n)).to("cuda", p.dtype) for i, p in enumerate(ents)]
    batch.solve(rhos, phis, Es)
    torch.cuda.synchronize()
    for i, p in enumerate(ents):
        p1, E1 = p.solve(rhos[i])
        torch.cuda.synchronize()
        assert torch.equal(phis[i], p1) and torch.equal(Es[i], E1), ("solve after adjoint", i)
    say("  solve after the adjoint: bit-identical (graph=%s)" % graph)
    batch.close()
    for p in plans:
        p.close()


def test_batch_autograd_equals_per_entry_autograd():
    """Gradients through vgf.solve_batch (batched solve and adjoint) equal
    those through vgf.solve per entry, bit for bit, for phi + E plans of
    several kinds and for an E-only group (the differentiable workload's
    shape), including entries whose phi does not enter the loss."""
    torch, vgf = need_gpu()
    specs = [((32, 32, 32), "f32", "fourier", ("phi", "E")), ((64, 48), "f64", "fourier", ("phi", "E")),
             ((24, 32, 16), "f64", "centered", ("phi", "E")), ((32, 32, 32), "f32", "fourier", ("E",))]
    plans = []
    for n, prec, field, outs in specs:
        h = tuple(2.0 / (x - 1) for x in n)
        plans.append(gpu_plan(vgf, n, h, precision=prec, field=field, outputs=outs))
    for ents in ([plans[0], plans[1], plans[0], plans[2]], [plans[3]] * 3):
        batch = vgf.Batch(ents, graph=True)
        rhos = [torch.from_numpy(W.random_field(200 + i, p.n)).to("cuda", p.dtype) for i, p in enumerate(ents)]
        tE = [torch.from_numpy(W.random_field(300 + i, (p.dim,) + p.n)).to("cuda", p.dtype) for i, p in enumerate(ents)]

        def loss_of(phis, Es):
            total = 0.0
            for i in range(len(ents)):
                total = total + ((Es[i] - tE[i]) ** 2).sum().double()
                if phis is not None and i % 2 == 0:  # phi of the odd entries stays out of the loss
                    total = total + (phis[i] ** 2).sum().double()
            return total

        xs = [r.clone().requires_grad_(True) for r in rhos]
        phis, Es = vgf.solve_batch(batch, xs)
        loss_of(phis, Es).backward()
        ys = [r.clone().requires_grad_(True) for r in rhos]
        outs = [vgf.solve(y, p) for y, p in zip(ys, ents)]
        has_phi = all("phi" in p.outputs for p in ents)
        loss_of([o[0] for o in outs] if has_phi else None, [o[1] for o in outs]).backward()
        torch.cuda.synchronize()
        for i in range(len(ents)):
            assert torch.equal(xs[i].grad, ys[i].grad), (i, ents[i].n, ents[i].field, ents[i].outputs)
        say("  batched autograd over %d entries: gradients bit-identical to per-entry autograd" % len(ents))
        batch.close()
    for p in plans:
        p.close()


def test_batch_adjoint_rejects_bad_arguments():
    """Partial cotangent lists, a missing g_rho and cotangents of outputs a
    plan was not created for are refused before anything is enqueued."""
    torch, vgf = need_gpu()
    n = (32, 32, 32)
    h = tuple(2.0 / (x - 1) for x in n)
    full = gpu_plan(vgf, n, h, precision="f32")
    e_only = gpu_plan(vgf, n, h, precision="f32", outputs=("E",))
    VP = C.c_void_p
    for plans, expect_phi in (([full, full], 0), ([full, e_only], -6)):
        batch = vgf.Batch(plans, graph=False)
        gp = [torch.randn(n, device="cuda") for _ in plans]
        gE = [torch.randn((3,) + n, device="cuda") for _ in plans]
        gr = [torch.full(n, float("nan"), device="cuda") for _ in plans]
        arr = lambda xs: (VP * len(xs))(*[x.data_ptr() if x is not None else None for x in xs])
        L = vgf.lib()
        assert L.vgf_batch_adjoint(batch.handle, None, None, arr(gr), None) == -1
        assert L.vgf_batch_adjoint(batch.handle, arr([gp[0], None]), None, arr(gr), None) == -1
        assert L.vgf_batch_adjoint(batch.handle, None, arr(gE), arr([gr[0], None]), None) == -1
        assert L.vgf_batch_adjoint(batch.handle, None, arr(gE), None, None) == -1
        st = L.vgf_batch_adjoint(batch.handle, arr(gp), None, arr(gr), None)
        assert st == expect_phi
        torch.cuda.synchronize()
        if st != 0:
            for x in gr:
                assert torch.isnan(x).all()  # nothing was enqueued
        batch.close()
    full.close()
    e_only.close()


def test_batch_rejects_partial_outputs():
    torch, vgf = need_gpu()
    keys = KEYS[:3]
    plans = _plans(vgf, keys)
    batch = vgf.Batch([plans[k] for k in keys], graph=True)
    rhos = _entries(torch, plans, keys, seed=1)
    phis, Es = _outputs(torch, plans, keys)
    VP = C.c_void_p
    rh = (VP * 3)(*[r.data_ptr() for r in rhos])
    ph = (VP * 3)(phis[0].data_ptr(), None, phis[2].data_ptr())
    assert vgf.lib().vgf_batch_solve(batch.handle, rh, ph, None, None) == -1
    rh_bad = (VP * 3)(rhos[0].data_ptr(), None, rhos[2].data_ptr())
    ph = (VP * 3)(*[x.data_ptr() for x in phis])
    assert vgf.lib().vgf_batch_solve(batch.handle, rh_bad, ph, None, None) == -1
    torch.cuda.synchronize()
    for x in phis:
        assert torch.isnan(x).all()  # nothing was enqueued
    batch.close()
    for p in plans.values():
        p.close()


def test_batch_3d_mixed_graph_vs_oracle():
    """The 64-entry mixed-size FP32 workload through one graph launch."""
    torch, vgf = need_gpu()
    charges = W.batch_3d_mixed(seed=0, count=64)
    plans = {}
    kernels = {}
    for ch in charges:
        if ch.n not in plans:
            plans[ch.n] = gpu_plan(vgf, ch.n, ch.h, method="vgf", precision="f32")
            kernels[ch.n] = orc.vgf_kernel(ch.n, ch.h, plans[ch.n].L)
    pl = [plans[ch.n] for ch in charges]
    batch = vgf.Batch(pl, graph=True)
    assert batch.groups == len(plans)
    rhos = [torch.from_numpy(ch.rho()).to("cuda", torch.float32) for ch in charges]
    phis = [torch.empty(ch.n, dtype=torch.float32, device="cuda") for ch in charges]
    Es = [torch.empty((3,) + ch.n, dtype=torch.float32, device="cuda") for ch in charges]
    batch.solve(rhos, phis, Es)
    torch.cuda.synchronize()
    worst = 0.0
    for b, ch in enumerate(charges):
        rho = rounded_input(ch.rho(), "f32")
        phi_o, E_o = orc.solve_fft2n(ch.n, ch.h, kernels[ch.n], rho)
        errs = check_fields(phis[b].double().cpu().numpy(), Es[b].double().cpu().numpy(), phi_o, E_o,
                            FP32_TOL, "graph batch[%d] N=%d" % (b, ch.n[0]))
        worst = max(worst, max(errs.values()))
    say("graph batch worst rel-L2 %.3e" % worst)
    batch.close()
    for p in plans.values():
        p.close()


def test_batch_fp64_vs_oracle():
    torch, vgf = need_gpu()
    keys = [((24, 24, 24), "f64", "vgf"), ((32, 32, 32), "f64", "he"), ((24, 24, 24), "f64", "vgf"),
            ((48, 32), "f64", "vgf")]
    plans = _plans(vgf, keys)
    batch = vgf.Batch([plans[k] for k in keys], graph=True)
    rho_np = [W.random_field(50 + i, plans[k].n) for i, k in enumerate(keys)]
    rhos = [torch.from_numpy(r).to("cuda", torch.float64) for r in rho_np]
    phis, Es = _outputs(torch, plans, keys)
    batch.solve(rhos, phis, Es)
    torch.cuda.synchronize()
    for i, k in enumerate(keys):
        n, _, method = k
        h = plans[k].h
        w = orc.vgf_kernel(n, h, plans[k].L) if method == "vgf" else orc.he_kernel(n, h)
        phi_o, E_o = orc.solve_fft2n(n, h, w, rho_np[i])
        check_fields(phis[i].cpu().numpy(), Es[i].cpu().numpy(), phi_o, E_o, FP64_TOL,
                     "f64 batch[%d] %s %s" % (i, n, method))
    batch.close()
    for p in plans.values():
        p.close()


def test_batch_splits_groups_beyond_launch_limit():
    """A plan whose strided launches would exceed 65535 batches is split into
    several groups; every entry still equals vgf_solve (2D, n0 = 512: at most
    127 entries per group)."""
    torch, vgf = need_gpu()
    n = (512, 8)
    plan = gpu_plan(vgf, n, (2.0 / 511, 2.0 / 7), precision="f32")
    count = 130
    batch = vgf.Batch([plan] * count, graph=True)
    assert batch.groups == 2
    rhos = [torch.from_numpy(W.random_field(300 + i, n)).to("cuda", torch.float32) for i in range(count)]
    phis = [torch.empty(n, dtype=torch.float32, device="cuda") for _ in range(count)]
    Es = [torch.empty((2,) + n, dtype=torch.float32, device="cuda") for _ in range(count)]
    batch.solve(rhos, phis, Es)
    torch.cuda.synchronize()
    for i in (0, 1, 126, 127, 128, 129):
        p1, E1 = plan.solve(rhos[i])
        torch.cuda.synchronize()
        assert torch.equal(phis[i], p1) and torch.equal(Es[i], E1), i
    batch.close()
    plan.close()
