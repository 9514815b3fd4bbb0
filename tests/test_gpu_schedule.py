"""Tile schedules and the autotuner: every schedule must give results
bit-identical to the default one (a schedule only changes how many columns a
workgroup transforms, never the arithmetic of a line), for the solve and its
adjoint; the tuner must return a valid schedule, cache it, and leave the
results unchanged, for plans and for batches."""
import itertools
import time

import pytest

from gpu_common import need_gpu, say
from paper_2103_08531_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = [((32, 32, 32), "f32"), ((48, 48, 48), "f32"), ((24, 16, 32), "f64"), ((64, 48), "f64"),
         ((128, 128), "f32"), ((64, 64, 64), "f64")]


def _schedules(dim):
    if dim == 2:
        return [(0, 0, v, 0, 0) for v in (0, 1)]
    return [(0, a, b, c, 0) for a, b, c in itertools.product((0, 1), repeat=3)]


@pytest.mark.parametrize("n,prec", CASES)
def test_every_schedule_is_bit_identical(n, prec):
    torch, vgf = need_gpu()
    h = tuple(2.0 / (x - 1) for x in n)
    plan = vgf.Plan(n, h, precision=prec)
    assert plan.schedule == (0, 0, 0, 0, 0)
    rho = torch.from_numpy(W.random_field(3, n)).to("cuda", plan.dtype)
    g_phi = torch.from_numpy(W.random_field(4, n)).to("cuda", plan.dtype)
    g_E = torch.from_numpy(W.random_field(5, (len(n),) + n)).to("cuda", plan.dtype)
    phi0, E0 = plan.solve(rho)
    adj0 = plan.adjoint(g_phi, g_E)
    torch.cuda.synchronize()
    for sched in _schedules(len(n)):
        plan.schedule = sched
        assert plan.schedule == sched
        phi, E = plan.solve(rho)
        adj = plan.adjoint(g_phi, g_E)
        torch.cuda.synchronize()
        assert torch.equal(phi, phi0) and torch.equal(E, E0), sched
        assert torch.equal(adj, adj0), sched
    say("%s %s: %d schedules bit-identical" % (n, prec, len(_schedules(len(n)))))
    with pytest.raises(vgf.VGFError):
        plan.schedule = (1, 0, 0, 0, 0)  # r2c has one schedule only
    with pytest.raises(vgf.VGFError):
        plan.schedule = (0, 0, 2, 0, 0)
    if len(n) == 2:
        with pytest.raises(vgf.VGFError):
            plan.schedule = (0, 1, 0, 0, 0)  # no middle pass in 2D
    plan.close()


def test_plan_autotune_is_cached_and_exact():
    torch, vgf = need_gpu()
    n = (128, 128, 128)
    h = tuple(2.0 / (x - 1) for x in n)
    plan = vgf.Plan(n, h, precision="f32")
    rho = torch.from_numpy(W.random_field(9, n)).to("cuda", torch.float32)
    phi0, E0 = plan.solve(rho)
    t0 = time.perf_counter()
    sched = plan.autotune(rho, reps=3)
    t_tune = time.perf_counter() - t0
    say("autotuned 128^3 f32 schedule %s in %.1f ms" % (sched, 1e3 * t_tune))
    assert len(sched) == 5 and sched[0] == 0 and sched[4] == 0 and all(v in (0, 1) for v in sched)
    phi, E = plan.solve(rho)
    torch.cuda.synchronize()
    assert torch.equal(phi, phi0) and torch.equal(E, E0)
    # an identical plan takes the cached choice without timing anything
    plan2 = vgf.Plan(n, h, precision="f32")
    t0 = time.perf_counter()
    assert plan2.autotune(rho, reps=3) == sched
    t_cached = time.perf_counter() - t0
    say("cached: %.3f ms" % (1e3 * t_cached))
    assert t_cached < 0.5 * t_tune
    plan.close()
    plan2.close()


def test_batch_autotune_keeps_results():
    torch, vgf = need_gpu()
    keys = [(32, 32, 32), (64, 64, 64), (32, 32, 32), (96, 96, 96), (64, 64, 64)]
    plans = {}
    for n in keys:
        if n not in plans:
            plans[n] = vgf.Plan(n, tuple(2.0 / (x - 1) for x in n), precision="f32")
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
