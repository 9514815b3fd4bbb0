"""C-ABI checks that need no GPU: the library loads, exports every function
include/vgf.h declares, and rejects bad arguments with status codes before
touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def V():
    from paper_2103_08531_amd import vgf
    if not os.path.exists(vgf.LIB_PATH):
        from paper_2103_08531_amd import build
        build.build()
    return vgf


def declared_functions():
    text = open(os.path.join(ROOT, "include", "vgf.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vgf_[A-Za-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(V):
    names = declared_functions()
    assert len(names) >= 11
    lib = V.lib()
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(V.EXPORTS) == names


def test_status_strings(V):
    for st in V.STATUS:
        s = V.lib().vgf_status_string(st)
        assert isinstance(s, bytes) and len(s) > 0
    assert V.lib().vgf_status_string(12345) == b"unknown status"


def _create(V, dim=3, n=(32, 32, 32), h=None, method=0, prec=0, L=0.0, outputs=3, null_out=False):
    h = h or tuple(2.0 / (x - 1) for x in n)
    handle = C.c_void_p(12345)
    n_arr = (C.c_int64 * len(n))(*n)
    h_arr = (C.c_double * len(h))(*h)
    st = V.lib().vgf_plan_create(None if null_out else C.byref(handle), dim, n_arr, h_arr,
                                 method, prec, L, outputs, None)
    return st, handle


def test_plan_create_rejects_bad_arguments(V):
    assert _create(V, null_out=True)[0] == -1
    assert _create(V, dim=4, n=(32,) * 4)[0] == -1
    assert _create(V, dim=1, n=(32,))[0] == -1
    assert _create(V, method=7)[0] == -1
    assert _create(V, prec=3)[0] == -1
    assert _create(V, outputs=0)[0] == -1
    assert _create(V, outputs=8)[0] == -1
    assert _create(V, h=(0.1, -0.1, 0.1))[0] == -1
    assert _create(V, h=(0.1, float("nan"), 0.1))[0] == -1
    st, handle = _create(V, n=(33, 32, 32))
    assert st == -2 and handle.value is None  # *out is cleared on error
    assert _create(V, n=(7, 8, 8))[0] == -2
    assert _create(V, n=(1024, 32, 32))[0] == -2
    assert _create(V, dim=2, n=(640, 64))[0] == -2
    # odd sizes and factors other than 2 and 3 are outside the rule
    for bad in ((9, 16, 16), (27, 16, 16), (16, 20, 16), (16, 16, 1024), (40, 16, 16), (16, 16, 243)):
        assert _create(V, n=bad)[0] == -2, bad
    # 576 .. 1024 points only for 2D plans in the default layout
    for bad in ((576, 32, 32), (32, 648, 32)):
        assert _create(V, n=bad)[0] == -2, bad
    for bad in ((2048, 64), (64, 1152), (1000, 64), (1536, 64)):
        assert _create(V, dim=2, n=bad)[0] == -2, bad
    assert _create(V, dim=2, n=(1024, 64), outputs=3 | 64)[0] == -2
    for good in ((1024, 1024), (576, 648), (768, 864), (972, 64)):
        st, handle = _create(V, dim=2, n=good)
        assert st != -2, good
        if st == 0:
            V.lib().vgf_plan_destroy(handle)


def test_plan_create_rejects_L_outside_window(V, orc):
    """The library rejects L just outside the oracle's window, whose ends are
    pinned by behaviour (tests/test_oracle_window.py), on cubic, 2D and
    rectangular grids; NaN and infinite L are rejected too (HE ignores L)."""
    cases = [(3, (32, 32, 32), (2.0 / 31,) * 3), (2, (64, 64), (2 / 63, 2 / 63)),
             (3, (16, 48, 24), (0.13, 0.05, 0.09)), (2, (96, 128), (2.0 / 95, 2.6 / 127))]
    for dim, n, h in cases:
        lo, hi = orc.window(n, h)
        for L in (0.99 * lo, lo, hi, 1.01 * hi, float("nan"), float("inf"), 1e300):
            assert _create(V, dim=dim, n=n, h=h, L=L)[0] == -3, (n, h, L, lo, hi)
        _not_window_error(V, _create(V, dim=dim, n=n, h=h, L=float("nan"), method=1))
    # L <= 0 selects the default, inside the window
    _not_window_error(V, _create(V, n=(32, 32, 32), h=(2.0 / 31,) * 3, L=-1.0))


def _not_window_error(V, created):
    """No L_WINDOW status; without a device the call fails later (HIP error),
    with one it succeeds and the plan is released here."""
    st, handle = created
    assert st != -3
    if st == 0:
        V.lib().vgf_plan_destroy(handle)


def test_null_plan_calls_fail_cleanly(V):
    L = V.lib()
    assert L.vgf_solve(None, None, None, None, None) == -1
    assert L.vgf_solve_noalloc(None, None, None, None, None) == -1
    assert L.vgf_solve_adjoint(None, None, None, None, None) == -1
    assert L.vgf_solve_batched(None, -1, None, None, None, None) == -1
    assert L.vgf_solve_batched(None, 0, None, None, None, None) == 0
    v = C.c_double()
    assert L.vgf_plan_get_L(None, C.byref(v)) == -1
    s = C.c_size_t()
    assert L.vgf_plan_workspace_bytes(None, C.byref(s)) == -1
    assert L.vgf_plan_get_kernel(None, None) == -1
    assert L.vgf_plan_get_spectrum(None, None) == -1
    L.vgf_plan_destroy(None)


def test_workspace_cap_is_enforced(V, monkeypatch):
    """VGF_MAX_WORKSPACE forces VGF_ERR_OUT_OF_MEMORY before any allocation."""
    monkeypatch.setenv("VGF_MAX_WORKSPACE", "1024")
    st, handle = _create(V)
    assert st == -4 and handle.value is None


def test_null_batch_calls_fail_cleanly(V):
    L = V.lib()
    VP = C.c_void_p
    handle = VP(12345)
    assert L.vgf_batch_create(None, None, 1, 0) == -1
    assert L.vgf_batch_create(C.byref(handle), None, 1, 0) == -1
    assert handle.value is None  # *out is cleared on error
    plans = (VP * 2)(None, None)
    assert L.vgf_batch_create(C.byref(handle), plans, 2, 0) == -1  # NULL plan entries
    assert L.vgf_batch_create(C.byref(handle), plans, 0, 0) == -1
    assert L.vgf_batch_create(C.byref(handle), plans, -3, 0) == -1
    assert L.vgf_batch_create(C.byref(handle), plans, 2, 4) == -1  # unknown flag
    ptrs = (VP * 1)(None)
    assert L.vgf_batch_solve(None, ptrs, ptrs, None, None) == -1
    assert L.vgf_batch_adjoint(None, ptrs, None, ptrs, None) == -1
    s = C.c_size_t()
    assert L.vgf_batch_workspace_bytes(None, C.byref(s)) == -1
    assert L.vgf_batch_groups(None) == 0
    L.vgf_batch_destroy(None)


def test_null_schedule_calls_fail_cleanly(V):
    L = V.lib()
    sched = (C.c_int * 5)()
    assert L.vgf_plan_get_schedule(None, sched) == -1
    assert L.vgf_plan_set_schedule(None, sched) == -1
    assert L.vgf_plan_autotune(None, None, None, None, 3, None) == -1
    assert L.vgf_batch_autotune(None, None, None, None, 3, None) == -1
    assert L.vgf_batch_get_schedule(None, 0, sched) == -1


def test_field_mode_flags_are_checked(V):
    # centred and gradient-kernel fields need E; they exclude each other; the
    # gradient kernel needs the VGF method
    assert _create(V, outputs=1 | 16)[0] == -1
    assert _create(V, outputs=1 | 32)[0] == -1
    assert _create(V, outputs=3 | 16 | 32)[0] == -1
    assert _create(V, method=1, outputs=3 | 32)[0] == -1
    assert _create(V, outputs=3 | 128)[0] == -1
    L = V.lib()
    out = (C.c_double * 8)()
    assert L.vgf_plan_get_gradient_kernel(None, 0, out) == -1
    assert L.vgf_plan_get_gradient_spectrum(None, 0, out) == -1
