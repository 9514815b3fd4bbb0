"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs. FP64 must agree to rel-L2 <= 1e-12 per field, FP32 to
<= 1e-5 (the FP32 run gets the FP32-rounded rho, and the oracle the same
values widened to FP64)."""
import numpy as np
import pytest

import oracle as orc
from gpu_common import (FP32_TOL, FP64_TOL, check_fields, err, gpu_plan, gpu_solve, need_gpu, oracle_kernel,
                        oracle_solve, rel_l2, rounded_input, say)
from paper_2103_08531_amd import workloads as W

pytestmark = pytest.mark.gpu


def make_plan(n, h, method="vgf", precision="f64", outputs=("phi", "E"), L=None):
    torch, vgf = need_gpu()
    return gpu_plan(vgf, n, h, method=method, precision=precision, outputs=outputs, L=L)


KERNEL_CASES = [((8, 8, 8), "vgf"), ((12, 12, 12), "he"), ((32, 32, 32), "vgf"), ((32, 32, 32), "he"),
                ((16, 24, 32), "vgf"), ((16, 16), "vgf"), ((64, 48), "he"), ((512, 512), "vgf"),
                ((1024, 1024), "vgf")]


@pytest.mark.parametrize("n,method", KERNEL_CASES)
def test_precompute_kernel_and_spectrum(n, method):
    h = tuple(2.0 / (x - 1) for x in n)
    say("precompute", n, method)
    plan = make_plan(n, h, method)
    L = plan.L
    w_o = oracle_kernel(method, n, h, L)
    w_g = plan.kernel()
    err = np.max(np.abs(w_g - w_o)) / np.max(np.abs(w_o))
    say("  kernel max rel %.3e" % err)
    assert err <= FP64_TOL
    s_o, _ = orc.kernel_spectrum(n, w_o)
    s_g = plan.spectrum()
    err = np.max(np.abs(s_g - s_o)) / np.max(np.abs(s_o))
    say("  spectrum max rel %.3e" % err)
    assert err <= FP64_TOL
    plan.close()


DIRECT_CASES = [((8, 8, 8), "vgf"), ((12, 12, 12), "he"), ((8, 12, 16), "vgf"), ((16, 16), "vgf"),
                ((24, 16), "he"), ((48, 32), "vgf")]


@pytest.mark.parametrize("n,method", DIRECT_CASES)
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_small_grids_against_direct_sums(n, method, precision):
    """Random rho (no structure to hide behind) against the plain convolution
    sums and the cot-stencil field, computed without any FFT."""
    h = tuple((2.0 + 0.2 * a) / (x - 1) for a, x in enumerate(n))
    say("direct", n, method, precision)
    plan = make_plan(n, h, method, precision)
    rho = rounded_input(W.random_field(42, n), precision)
    phi_g, E_g = gpu_solve(plan, rho)
    w = oracle_kernel(method, n, h, plan.L)
    phi_o = orc.conv_direct(n, w, rho)
    Wp = orc.periodic_kernel(n, w)
    E_o = np.stack([orc.conv_periodic(n, orc.field_kernel(n, h, Wp, a), rho) for a in range(len(n))])
    tol = FP64_TOL if precision == "f64" else FP32_TOL
    check_fields(phi_g, E_g, phi_o, E_o, tol, "direct %s %s %s" % (n, method, precision))
    plan.close()


@pytest.mark.parametrize("method", ["vgf", "he"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_gaussian_3d_32(method, precision):
    """3D N=32 on [-1,1]^3, unit Gaussian sigma=0.1 at the origin."""
    ch = W.gaussian_3d_32()
    say("gaussian_3d_32", method, precision)
    plan = make_plan(ch.n, ch.h, method, precision)
    rho = rounded_input(ch.rho(), precision)
    phi_g, E_g = gpu_solve(plan, rho)
    phi_o, E_o = oracle_solve(method, ch.n, ch.h, plan.L, rho)
    tol = FP64_TOL if precision == "f64" else FP32_TOL
    check_fields(phi_g, E_g, phi_o, E_o, tol, "cfg1 %s %s" % (method, precision))
    pa, Ea = orc.gauss_mixture_grid(ch.n, ch.x0, ch.h, ch.centers, ch.sigmas, ch.weights)
    ea = rel_l2(phi_g, pa)
    say("  vs analytic phi %.3e E %.3e" % (ea, rel_l2(E_g, Ea)))
    if method == "vgf":
        # discretisation error 3e-9; FP32 rounding (~1e-7) dominates in FP32
        assert ea < (1e-8 if precision == "f64" else 1e-6)
    else:
        assert 5e-3 < ea < 5e-2
    plan.close()


@pytest.mark.parametrize("method", ["vgf", "he"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_mixture_2d_512(method, precision):
    """2D N=512 on [-1,1]^2, 8 seeded Gaussians, phi and E."""
    ch = W.mixture_2d_512(seed=0)
    say("mixture_2d_512", method, precision)
    plan = make_plan(ch.n, ch.h, method, precision)
    rho = rounded_input(ch.rho(), precision)
    phi_g, E_g = gpu_solve(plan, rho)
    phi_o, E_o = oracle_solve(method, ch.n, ch.h, plan.L, rho)
    tol = FP64_TOL if precision == "f64" else FP32_TOL
    check_fields(phi_g, E_g, phi_o, E_o, tol, "cfg2 %s %s" % (method, precision))
    plan.close()


SIZE_CASES = [(2, 96), (2, 192), (2, 384), (3, 24), (3, 48), (3, 64),
              # lengths 2N with two or more factors 3 (radix plans 4-3-3, 8-3-3, 2-3-3-3, ...)
              (2, 18), (2, 36), (2, 54), (2, 72), (2, 108), (2, 144), (2, 162), (2, 216), (2, 288),
              (2, 324), (2, 432), (2, 486), (3, 18), (3, 36), (3, 54), (3, 72)]


@pytest.mark.parametrize("dim,N", SIZE_CASES)
def test_fft_lengths(dim, N):
    """Every radix mix (8/6/4/2/3) of the supported lengths, ragged column tiles."""
    n = (N,) * dim
    h = (2.0 / (N - 1),) * dim
    rng = np.random.default_rng(N)
    c = rng.uniform(-0.4, 0.4, (3, dim))
    s = np.repeat(rng.uniform(0.08, 0.2, 3)[:, None], dim, axis=1)
    rho = W.gaussian_density(n, (-1.0,) * dim, h, c, s, np.array([1.0, -0.5, 0.7]))
    say("lengths", dim, N)
    for precision, tol in (("f64", FP64_TOL), ("f32", FP32_TOL)):
        plan = make_plan(n, h, "vgf", precision)
        r = rounded_input(rho, precision)
        phi_g, E_g = gpu_solve(plan, r)
        phi_o, E_o = oracle_solve("vgf", n, h, plan.L, r)
        check_fields(phi_g, E_g, phi_o, E_o, tol, "len %dD %d %s" % (dim, N, precision))
        plan.close()


LONG_AXIS_CASES = [(384, 8, 12), (8, 384, 8), (8, 12, 384), (512, 8, 8), (8, 512, 12), (12, 8, 512),
                   (288, 8, 12), (8, 288, 8), (8, 12, 288), (486, 8, 8), (8, 432, 12), (12, 8, 324),
                   # lengths 384 and 432 (radix plans 8-8-6 and 8-6-3-3) on each axis
                   (192, 8, 12), (8, 192, 8), (12, 8, 192), (216, 8, 8), (8, 216, 12), (8, 12, 216)]


@pytest.mark.parametrize("n", LONG_AXIS_CASES)
def test_fft_lengths_3d_long_axes(n):
    """Transform lengths 384 to 1024 on each 3D axis (the axis-1 passes meet
    them only in 3D), thin grids so the oracle stays fast."""
    h = tuple(2.0 / (x - 1) for x in n)
    rho = W.random_field(sum(n), n)
    say("long axis", n)
    for precision, tol in (("f64", FP64_TOL), ("f32", FP32_TOL)):
        plan = make_plan(n, h, "vgf", precision)
        r = rounded_input(rho, precision)
        phi_g, E_g = gpu_solve(plan, r)
        phi_o, E_o = oracle_solve("vgf", n, h, plan.L, r)
        check_fields(phi_g, E_g, phi_o, E_o, tol, "long %s %s" % (n, precision))
        plan.close()


# 2D grids of 576 .. 1024 points per axis: FFT lengths 1152 .. 2048, which the
# library builds for the 2D default layout only
WIDE_2D_CASES = [((1024, 1024), "f64"), ((1024, 1024), "f32"), ((576, 648), "f64"), ((768, 972), "f32"),
                 ((864, 96), "f64"), ((96, 1024), "f32")]


def _mixture(n, h, seed):
    """Eight Gaussians of the 2D example's recipe (centres in [-0.5, 0.5]^2,
    sigma in [0.05, 0.15], weights +-1) on the grid starting at -1."""
    rng = np.random.default_rng(seed)
    c = rng.uniform(-0.5, 0.5, (8, 2))
    s = rng.uniform(0.05, 0.15, 8)
    q = rng.choice([-1.0, 1.0], 8)
    return W.gaussian_density(n, (-1.0, -1.0), h, c, np.repeat(s[:, None], 2, axis=1), q)


@pytest.mark.parametrize("n,precision", WIDE_2D_CASES)
def test_wide_2d_grids(n, precision):
    """phi + E against the oracle, and at 1024^2 FP64 the adjoint too. FP64
    takes the 2D example's Gaussian mixture: with white noise the fields are
    dominated by the highest frequencies, where the kernel spectrum is
    smallest, so the rounding of the two precomputes (GEMMs here, direct sums
    in the oracle; the kernels agree to 1e-14 relative) reaches ~2e-12 in E
    at 1024^2. FP32 takes white noise (its own rounding dominates)."""
    torch, vgf = need_gpu()
    h = (2.0 / (n[0] - 1), 2.2 / (n[1] - 1))
    tol = FP64_TOL if precision == "f64" else FP32_TOL
    src = _mixture(n, h, sum(n)) if precision == "f64" else W.random_field(sum(n) + 1, n)
    rho = rounded_input(src, precision)
    say("wide 2D", n, precision)
    plan = make_plan(n, h, "vgf", precision)
    phi_g, E_g = gpu_solve(plan, rho)
    w = orc.vgf_kernel(n, h, plan.L)
    phi_o, E_o = orc.solve_fft2n(n, h, w, rho)
    check_fields(phi_g, E_g, phi_o, E_o, tol, "wide %s %s" % (n, precision))
    if n == (1024, 1024) and precision == "f64":
        y = _mixture(n, h, 5)
        z = np.stack([_mixture(n, h, 6), _mixture(n, h, 7)])
        dt = plan.dtype
        g = plan.adjoint(torch.from_numpy(y).to("cuda", dt), torch.from_numpy(z).to("cuda", dt))
        e = err(g.double().cpu().numpy(), orc.adjoint_fft2n(n, h, w, y, z))
        say("  adjoint vs oracle %.3e" % e)
        assert e <= tol
    plan.close()


def test_rectangular_grid():
    n = (16, 24, 32)
    lo = (-0.9, -1.0, -1.1)
    h = tuple(-2 * l / (m - 1) for l, m in zip(lo, n))
    c = np.array([[0.03, -0.02, 0.05]])
    s = np.full((1, 3), 0.12)
    rho = W.gaussian_density(n, lo, h, c, s, np.ones(1))
    for precision, tol in (("f64", FP64_TOL), ("f32", FP32_TOL)):
        plan = make_plan(n, h, "vgf", precision)
        r = rounded_input(rho, precision)
        phi_g, E_g = gpu_solve(plan, r)
        phi_o, E_o = oracle_solve("vgf", n, h, plan.L, r)
        check_fields(phi_g, E_g, phi_o, E_o, tol, "rect %s" % precision)
        plan.close()


@pytest.mark.parametrize("outputs", [("phi",), ("E",)])
def test_output_subsets(outputs):
    torch, vgf = need_gpu()
    ch = W.gaussian_3d_32()
    plan = make_plan(ch.n, ch.h, "vgf", "f64", outputs=outputs)
    rho = ch.rho()
    phi_g, E_g = gpu_solve(plan, rho)
    phi_o, E_o = oracle_solve("vgf", ch.n, ch.h, plan.L, rho)
    if outputs == ("phi",):
        assert E_g is None
        check_fields(phi_g, None, phi_o, None, FP64_TOL, "phi-only")
        with pytest.raises(vgf.VGFError) as ei:
            r = torch.from_numpy(rho).cuda()
            E = torch.empty((3,) + ch.n, dtype=torch.float64, device="cuda")
            vgf.lib()  # the C call itself must refuse the E output
            import ctypes as C
            st = vgf.lib().vgf_solve(plan.handle, C.c_void_p(r.data_ptr()), None,
                                     C.c_void_p(E.data_ptr()), None)
            vgf._check(st, "vgf_solve")
        assert ei.value.status == -6
    else:
        assert phi_g is None
        check_fields(None, E_g, None, E_o, FP64_TOL, "E-only")
    plan.close()


def test_repeat_solves_are_bitwise_identical():
    torch, vgf = need_gpu()
    ch = W.mixture_2d_512(seed=1)
    plan = make_plan(ch.n, ch.h, "vgf", "f32")
    a = gpu_solve(plan, ch.rho())
    b = gpu_solve(plan, ch.rho())
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    plan.close()


@pytest.mark.parametrize("n", [(16, 16, 16), (8, 12, 16), (32, 24)])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_adjoint(n, precision):
    """<K x, y> + sum_a <K_a x, z_a> = <x, K^T y + sum_a K_a^T z_a>, and the
    GPU adjoint against the oracle's adjoint."""
    torch, vgf = need_gpu()
    dim = len(n)
    h = tuple((2.0 + 0.15 * a) / (x - 1) for a, x in enumerate(n))
    plan = make_plan(n, h, "vgf", precision)
    x = rounded_input(W.random_field(1, n), precision)
    y = rounded_input(W.random_field(2, n), precision)
    z = rounded_input(W.random_field(3, (dim,) + n), precision)
    phi_g, E_g = gpu_solve(plan, x)
    dt = plan.dtype
    g = plan.adjoint(torch.from_numpy(y).to("cuda", dt), torch.from_numpy(z).to("cuda", dt))
    torch.cuda.synchronize()
    g = g.double().cpu().numpy()
    lhs = np.vdot(phi_g, y) + np.vdot(E_g, z)
    rhs = np.vdot(x, g)
    tol = FP64_TOL if precision == "f64" else FP32_TOL
    say("adjoint %s %s dot lhs %.16e rhs %.16e" % (n, precision, lhs, rhs))
    assert abs(lhs - rhs) <= tol * (np.linalg.norm(phi_g) * np.linalg.norm(y) + np.linalg.norm(E_g) * np.linalg.norm(z))
    w = orc.vgf_kernel(n, h, plan.L)
    g_o = orc.adjoint_fft2n(n, h, w, y, z)
    e = err(g, g_o)
    say("  vs oracle adjoint %.3e" % e)
    assert e <= tol
    # phi-only and E-only adjoints
    g1 = plan.adjoint(torch.from_numpy(y).to("cuda", dt), None).double().cpu().numpy()
    assert err(g1, orc.adjoint_fft2n(n, h, w, y, None)) <= tol
    g2 = plan.adjoint(None, torch.from_numpy(z).to("cuda", dt)).double().cpu().numpy()
    assert err(g2, orc.adjoint_fft2n(n, h, w, None, z)) <= tol
    plan.close()


def test_batched_matches_single():
    torch, vgf = need_gpu()
    charges = W.batch_3d_mixed(seed=0, count=6, sizes=(32, 48, 64))
    plans = {}
    for ch in charges:
        if ch.n not in plans:
            plans[ch.n] = make_plan(ch.n, ch.h, "vgf", "f32")
    rhos = [torch.from_numpy(ch.rho()).to("cuda", torch.float32) for ch in charges]
    pl = [plans[ch.n] for ch in charges]
    phis = [torch.empty(ch.n, dtype=torch.float32, device="cuda") for ch in charges]
    Es = [torch.empty((3,) + ch.n, dtype=torch.float32, device="cuda") for ch in charges]
    vgf.solve_batched(pl, rhos, phis, Es)
    torch.cuda.synchronize()
    for ch, r, p, E, plan in zip(charges, rhos, phis, Es, pl):
        p1, E1 = plan.solve(r)
        torch.cuda.synchronize()
        assert torch.equal(p, p1) and torch.equal(E, E1)
        phi_o, E_o = oracle_solve("vgf", ch.n, ch.h, plan.L, rounded_input(ch.rho(), "f32"))
        check_fields(p.double().cpu().numpy(), E.double().cpu().numpy(), phi_o, E_o, FP32_TOL,
                     "batched %s" % (ch.n,))
    for p in plans.values():
        p.close()


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_degenerate_inputs(precision):
    """rho = 0 gives exactly zero fields; a unit charge at the origin corner
    gives phi = the kernel itself (phi[i] = w[i]) and E = the field kernel,
    against the oracle's kernel and its cot-stencil field kernel."""
    torch, vgf = need_gpu()
    n = (12, 16, 8)
    h = (0.15, 0.12, 0.2)
    plan = make_plan(n, h, "vgf", precision)
    phi, E = gpu_solve(plan, np.zeros(n))
    assert np.all(phi == 0.0) and np.all(E == 0.0)
    delta = np.zeros(n)
    delta[0, 0, 0] = 1.0
    phi, E = gpu_solve(plan, delta)
    w = orc.vgf_kernel(n, h, plan.L)
    tol = FP64_TOL if precision == "f64" else FP32_TOL
    assert err(phi, w) <= tol
    Wp = orc.periodic_kernel(n, w)
    for a in range(3):
        V = orc.field_kernel(n, h, Wp, a)
        Ea = V[:n[0], :n[1], :n[2]]  # E_a[i] = V_a[i - 0]
        assert err(E[a], Ea) <= tol, a
    plan.close()


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_largest_grid_512(precision):
    """The largest supported grid, 512^3: a contained Gaussian (sigma = 0.1)
    against its closed-form potential and field on a stride-16 subsample.
    VGF is converged far below FP32 rounding here, so the bound is the
    arithmetic's."""
    torch, vgf = need_gpu()
    ch = W.gaussian_3d_32(N=512)
    say("512^3", precision, "plan ...")
    plan = make_plan(ch.n, ch.h, "vgf", precision)
    rho = ch.rho()
    phi_g, E_g = gpu_solve(plan, rounded_input(rho, precision))
    plan.close()
    sub = tuple(slice(0, 512, 16) for _ in range(3))
    n_s = (32, 32, 32)
    h_s = tuple(16 * x for x in ch.h)
    pa, Ea = orc.gauss_mixture_grid(n_s, ch.x0, h_s, ch.centers, ch.sigmas, ch.weights)
    ep = rel_l2(phi_g[sub], pa)
    eE = rel_l2(E_g[(slice(None),) + sub], Ea)
    say("  512^3 %s vs analytic: phi %.3e E %.3e" % (precision, ep, eE))
    bound = 1e-12 if precision == "f64" else 1e-5
    assert ep <= bound and eE <= bound


LAYOUT_CASES = [((16, 24, 32), "vgf"), ((24, 12, 48), "he"), ((64, 48), "vgf"), ((96, 64), "he_cellavg")]


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("n,method", LAYOUT_CASES)
def test_axis0_layout_matches_oracle(n, method, precision):
    """The axis-0 layout (multiply inside the strided axis-0 pass), solve and
    adjoint, against the oracle, next to the default layout."""
    h = tuple((2.0 + 0.1 * a) / (x - 1) for a, x in enumerate(n))
    torch, vgf = need_gpu()
    tol = FP64_TOL if precision == "f64" else FP32_TOL
    rho = rounded_input(W.random_field(61, n), precision)
    g_phi = rounded_input(W.random_field(62, n), precision)
    g_E = rounded_input(W.random_field(63, (len(n),) + n), precision)
    res = {}
    for layout in ("axis0", "contiguous"):
        plan = gpu_plan(vgf, n, h, method=method, precision=precision, layout=layout)
        w = oracle_kernel(method, n, h, plan.L)
        phi_g, E_g = gpu_solve(plan, rho)
        phi_o, E_o = orc.solve_fft2n(n, h, w, rho)
        check_fields(phi_g, E_g, phi_o, E_o, tol, "%s %s %s %s" % (layout, n, method, precision))
        gp = torch.from_numpy(g_phi).to("cuda", plan.dtype)
        ge = torch.from_numpy(g_E).to("cuda", plan.dtype)
        g_rho = plan.adjoint(gp, ge).double().cpu().numpy()
        ref = orc.adjoint_fft2n(n, h, w, g_phi, g_E)
        assert err(g_rho, ref) <= tol, (layout, err(g_rho, ref))
        res[layout] = phi_g
        plan.close()
    assert rel_l2(res["axis0"], res["contiguous"]) <= 2 * tol


def test_solve_follows_the_current_stream():
    """With no stream argument the binding enqueues on torch's current stream:
    inside a side-stream context the solve runs there, with the same result."""
    torch, vgf = need_gpu()
    n = (32, 24, 16)
    h = tuple(2.0 / (x - 1) for x in n)
    plan = make_plan(n, h)
    rho = torch.from_numpy(W.random_field(31, n)).to("cuda", torch.float64)
    phi0, E0 = plan.solve(rho)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    # c_void_p(0).value is None: the default stream's handle is 0
    assert (vgf._stream().value or 0) == torch.cuda.current_stream().cuda_stream
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        assert (vgf._stream().value or 0) == side.cuda_stream != 0
        phi1, E1 = plan.solve(rho)
    side.synchronize()
    assert torch.equal(phi0, phi1) and torch.equal(E0, E1)
    plan.close()
