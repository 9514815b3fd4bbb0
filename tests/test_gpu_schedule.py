"""Tile schedules and the autotuner: every schedule must give results
bit-identical to the default one (a schedule only changes how many columns a
workgroup transforms, never the arithmetic of a line), for the solve and its
adjoint; the tuner must return a valid schedule, cache it, and leave the
results unchanged, for plans and for batches."""
import numpy as np
import pytest

from gpu_common import need_gpu, gpu_plan, say
from paper_2103_08531_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = [((32, 32, 32), "f32", "contiguous"), ((48, 48, 48), "f32", "contiguous"),
         ((24, 16, 32), "f64", "contiguous"), ((64, 48), "f64", "contiguous"),
         ((128, 128), "f32", "contiguous"), ((64, 64, 64), "f64", "contiguous"),
         ((32, 32, 32), "f32", "axis0"), ((24, 16, 32), "f64", "axis0"), ((64, 48), "f64", "axis0"),
         ((36, 18, 54), "f64", "contiguous"), ((72, 144), "f32", "contiguous"), ((36, 18, 54), "f32", "axis0")]


def _tunable(dim, layout):
    """Passes with schedules: the strided ones of each layout (the axis-0
    transforms of the default layout, the axis-0 multiply pass of the axis-0
    layout), in 3D the axis-1 transforms, and the contiguous multiply pass of
    the default layout (lanes per line, walk length)."""
    own = [2] if layout == "axis0" else [0, 2, 4]
    return own + ([1, 3] if dim == 3 else [])


def _schedules(dim, layout):
    """Every value (two bits: first launch, later launches) of one tunable
    pass at a time, all-half-width, and a seeded sample of combinations."""
    tun = _tunable(dim, layout)
    out = {(0,) * 5}
    for k in tun:
        for v in (1, 2, 3):
            out.add(tuple(v if i == k else 0 for i in range(5)))
    out.add(tuple(3 if i in tun else 0 for i in range(5)))
    rng = np.random.default_rng(17)
    for _ in range(12):
        out.add(tuple(int(rng.integers(0, 4)) if i in tun else 0 for i in range(5)))
    return sorted(out)


@pytest.mark.parametrize("n,prec,layout", CASES)
def test_every_schedule_is_bit_identical(n, prec, layout):
    torch, vgf = need_gpu()
    h = tuple(2.0 / (x - 1) for x in n)
    plan = gpu_plan(vgf, n, h, precision=prec, layout=layout)
    assert plan.schedule == (0, 0, 0, 0, 0)
    rho = torch.from_numpy(W.random_field(3, n)).to("cuda", plan.dtype)
    g_phi = torch.from_numpy(W.random_field(4, n)).to("cuda", plan.dtype)
    g_E = torch.from_numpy(W.random_field(5, (len(n),) + n)).to("cuda", plan.dtype)
    phi0, E0 = plan.solve(rho)
    adj0 = plan.adjoint(g_phi, g_E)
    torch.cuda.synchronize()
    for sched in _schedules(len(n), layout):
        plan.schedule = sched
        assert plan.schedule == sched
        phi, E = plan.solve(rho)
        adj = plan.adjoint(g_phi, g_E)
        torch.cuda.synchronize()
        assert torch.equal(phi, phi0) and torch.equal(E, E0), sched
        assert torch.equal(adj, adj0), sched
    say("%s %s %s: %d schedules bit-identical" % (n, prec, layout, len(_schedules(len(n), layout))))
    for k in range(5):
        if k not in _tunable(len(n), layout):
            with pytest.raises(vgf.VGFError):
                plan.schedule = tuple(1 if i == k else 0 for i in range(5))  # one schedule only
    with pytest.raises(vgf.VGFError):
        plan.schedule = tuple(4 if i == _tunable(len(n), layout)[0] else 0 for i in range(5))
    plan.close()


def _plan_env(vgf, n, prec, stream_min):
    """A plan created with VGF_STREAM_MIN_BYTES = stream_min (read at creation)."""
    import os
    old = os.environ.get("VGF_STREAM_MIN_BYTES")
    os.environ["VGF_STREAM_MIN_BYTES"] = str(stream_min)
    try:
        return gpu_plan(vgf, n, tuple(2.0 / (x - 1) for x in n), precision=prec)
    finally:
        if old is None:
            del os.environ["VGF_STREAM_MIN_BYTES"]
        else:
            os.environ["VGF_STREAM_MIN_BYTES"] = old


STREAM_CASES = [((32, 32, 32), "f32"), ((24, 16, 32), "f64"), ((64, 48), "f64"), ((128, 128), "f32"),
                ((48, 64, 24), "f32")]


@pytest.mark.parametrize("n,prec", STREAM_CASES)
def test_streaming_accesses_are_bit_identical(n, prec):
    """Non-temporal loads and stores (forced on for a small grid) change no
    bit of any output, with either tile schedule and every output set, for
    single solves and for a batch of the plan."""
    torch, vgf = need_gpu()
    on = _plan_env(vgf, n, prec, 0)
    off = _plan_env(vgf, n, prec, 1 << 62)
    rho = torch.from_numpy(W.random_field(8, n)).to("cuda", on.dtype)
    half = tuple(3 if i in _tunable(len(n), "contiguous") else 0 for i in range(5))
    for sched in ((0,) * 5, half):
        on.schedule = sched
        off.schedule = sched
        for wp, wE in ((True, True), (False, True), (True, False)):
            a = on.solve(rho, want_phi=wp, want_E=wE)
            b = off.solve(rho, want_phi=wp, want_E=wE)
            torch.cuda.synchronize()
            for x, y in zip(a, b):
                assert (x is None) == (y is None)
                if x is not None:
                    assert torch.equal(x, y), (n, prec, sched, wp, wE)
    rhos = [torch.from_numpy(W.random_field(20 + i, n)).to("cuda", on.dtype) for i in range(3)]
    outs = {}
    for name, plan in (("on", on), ("off", off)):
        batch = vgf.Batch([plan] * 3, graph=False)
        phis = [torch.empty(n, dtype=plan.dtype, device="cuda") for _ in range(3)]
        Es = [torch.empty((len(n),) + n, dtype=plan.dtype, device="cuda") for _ in range(3)]
        batch.solve(rhos, phis, Es)
        torch.cuda.synchronize()
        outs[name] = (phis, Es)
        batch.close()
    for i in range(3):
        assert torch.equal(outs["on"][0][i], outs["off"][0][i]) and torch.equal(outs["on"][1][i], outs["off"][1][i])
    say("%s %s: streaming and plain accesses bit-identical (solve, 2 schedules, 3 output sets, batch)" % (n, prec))
    on.close()
    off.close()


def test_plan_autotune_is_cached_and_exact():
    torch, vgf = need_gpu()
    n = (128, 128, 128)
    h = tuple(2.0 / (x - 1) for x in n)
    plan = gpu_plan(vgf, n, h, precision="f32")
    rho = torch.from_numpy(W.random_field(9, n)).to("cuda", torch.float32)
    phi0, E0 = plan.solve(rho)
    phi = torch.empty_like(phi0)
    E = torch.empty_like(E0)
    sched = plan.autotune(rho, phi, E, reps=3)
    say("autotuned 128^3 f32 schedule %s" % (sched,))
    assert len(sched) == 5 and all(0 <= v <= 3 for v in sched)
    torch.cuda.synchronize()
    assert torch.equal(phi, phi0) and torch.equal(E, E0)  # the tuning solves' results
    phi, E = plan.solve(rho)
    torch.cuda.synchronize()
    assert torch.equal(phi, phi0) and torch.equal(E, E0)
    # an identical plan takes the cached choice without enqueueing anything:
    # the output buffers, which every tuning solve writes, keep their marker
    plan2 = gpu_plan(vgf, n, h, precision="f32")
    phi_m = torch.full_like(phi0, float("nan"))
    E_m = torch.full_like(E0, float("nan"))
    assert plan2.autotune(rho, phi_m, E_m, reps=3) == sched
    torch.cuda.synchronize()
    assert bool(torch.isnan(phi_m).all()) and bool(torch.isnan(E_m).all())
    assert plan2.schedule == sched
    plan.close()
    plan2.close()


def test_batch_autotune_keeps_results():
    torch, vgf = need_gpu()
    keys = [(32, 32, 32), (64, 64, 64), (32, 32, 32), (96, 96, 96), (64, 64, 64)]
    plans = {}
    for n in keys:
        if n not in plans:
            plans[n] = gpu_plan(vgf, n, tuple(2.0 / (x - 1) for x in n), precision="f32")
    pl = [plans[n] for n in keys]
    rhos = [torch.from_numpy(W.random_field(20 + i, n)).to("cuda", torch.float32) for i, n in enumerate(keys)]
    phis = [torch.empty(n, dtype=torch.float32, device="cuda") for n in keys]
    Es = [torch.empty((3,) + n, dtype=torch.float32, device="cuda") for n in keys]
    batch = vgf.Batch(pl, graph=True)
    batch.solve(rhos, phis, Es)  # captured with the default schedules
    torch.cuda.synchronize()
    ref = [(p.clone(), E.clone()) for p, E in zip(phis, Es)]
    scheds = batch.autotune(rhos, phis, Es, reps=2)
    say("batch schedules per group: %s" % scheds)
    assert len(scheds) == batch.groups == 3
    for rep in range(2):
        for x in phis + Es:
            x.fill_(float("nan"))
        batch.solve(rhos, phis, Es)  # recaptured with the tuned schedules
        torch.cuda.synchronize()
        for i in range(len(keys)):
            assert torch.equal(phis[i], ref[i][0]) and torch.equal(Es[i], ref[i][1]), (rep, i)
    batch.close()
    for p in plans.values():
        p.close()


# tiled: (16, 24, 128), (48, 64, 96), (64, 32, 256), and (8, 512, 64) with
# half-width blocks (P1 = 1024); plain rows kept: (24, 16, 32) (8 butterflies
# in the last inverse stage), (36, 18, 54) (54 not a multiple of 8)
@pytest.mark.parametrize("n,prec", [((16, 24, 128), "f32"), ((48, 64, 96), "f64"), ((64, 32, 256), "f32"),
                                    ((8, 512, 64), "f32"), ((24, 16, 32), "f32"), ((36, 18, 54), "f64")])
def test_tiled_handoff_is_bit_identical(n, prec, monkeypatch):
    """The multiply pass (forward and adjoint) writes the axis-1 inverse's
    tile order unless VGF_TILED_Y=0 (read at plan creation); only addresses
    differ, so the fields and the adjoint match plain rows bit for bit, under
    several schedules of the two passes and in a batch."""
    torch, vgf = need_gpu()
    h = tuple(2.0 / (x - 1) for x in n)
    plans = {}
    for v in ("0", "1"):
        monkeypatch.setenv("VGF_TILED_Y", v)
        plans[v] = gpu_plan(vgf, n, h, precision=prec)
    rho = torch.from_numpy(W.random_field(8, n)).to("cuda", plans["0"].dtype)
    g_phi = torch.from_numpy(W.random_field(10, n)).to("cuda", rho.dtype)
    g_E = torch.from_numpy(W.random_field(11, (3,) + n)).to("cuda", rho.dtype)
    phi0, E0 = plans["0"].solve(rho)
    adj0 = plans["0"].adjoint(g_phi, g_E)
    for sched in [(0, 0, 0, 0, 0), (0, 0, 1, 0, 0), (0, 0, 2, 1, 0), (0, 0, 3, 3, 0), (0, 1, 0, 2, 0)]:
        plans["1"].schedule = sched
        phi1, E1 = plans["1"].solve(rho)
        adj1 = plans["1"].adjoint(g_phi, g_E)
        torch.cuda.synchronize()
        assert torch.equal(phi0, phi1) and torch.equal(E0, E1), sched
        assert torch.equal(adj0, adj1), sched
    plans["1"].schedule = (0, 0, 0, 0, 0)
    rhos = [rho, torch.from_numpy(W.random_field(9, n)).to("cuda", rho.dtype)]
    outs = vgf.Batch([plans["1"], plans["1"]], graph=False)
    phis = [torch.empty_like(r) for r in rhos]
    Es = [torch.empty((3,) + n, dtype=rho.dtype, device="cuda") for _ in rhos]
    outs.solve(rhos, phis, Es)
    torch.cuda.synchronize()
    for r, p, E in zip(rhos, phis, Es):
        pr, Er = plans["0"].solve(r)
        torch.cuda.synchronize()
        assert torch.equal(p, pr) and torch.equal(E, Er)
    outs.close()
    for p in plans.values():
        p.close()


@pytest.mark.parametrize("n,prec", [((48, 64, 96), "f64"), ((64, 32, 256), "f32")])
def test_tiled_handoff_gradient_kernel_is_bit_identical(n, prec, monkeypatch):
    """The gradient-kernel multiply pass writes every field in the axis-1
    inverse's tile order unless VGF_TILED_Y=0: fields bit-identical, in a
    batch too."""
    torch, vgf = need_gpu()
    h = tuple(2.0 / (x - 1) for x in n)
    plans = {}
    for v in ("0", "1"):
        monkeypatch.setenv("VGF_TILED_Y", v)
        plans[v] = gpu_plan(vgf, n, h, precision=prec, field="gradient_kernel")
    rhos = [torch.from_numpy(W.random_field(s, n)).to("cuda", plans["0"].dtype) for s in (12, 13)]
    ref = [plans["0"].solve(r) for r in rhos]
    for sched in [(0, 0, 0, 0, 0), (0, 0, 0, 3, 0)]:
        plans["1"].schedule = sched
        phi1, E1 = plans["1"].solve(rhos[0])
        torch.cuda.synchronize()
        assert torch.equal(ref[0][0], phi1) and torch.equal(ref[0][1], E1), sched
    plans["1"].schedule = (0, 0, 0, 0, 0)
    b = vgf.Batch([plans["1"], plans["1"]], graph=False)
    phis = [torch.empty_like(r) for r in rhos]
    Es = [torch.empty((3,) + n, dtype=rhos[0].dtype, device="cuda") for _ in rhos]
    b.solve(rhos, phis, Es)
    torch.cuda.synchronize()
    for (pr, Er), p, E in zip(ref, phis, Es):
        assert torch.equal(p, pr) and torch.equal(E, Er)
    b.close()
    for p in plans.values():
        p.close()
