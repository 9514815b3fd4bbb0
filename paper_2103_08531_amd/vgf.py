"""Thin ctypes binding of libvgf.so (include/vgf.h).

Only argument marshalling lives here: every step of the solve runs in the HIP
kernels of libvgf.so. torch provides device memory (tensors are passed by
data_ptr) and the current HIP stream. There is no CPU fallback: if the
library is missing or no GPU is present, the calls raise.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# VGF_LIB selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("VGF_LIB") or os.path.join(HERE, "libvgf.so")

OK = 0
STATUS = {0: "VGF_OK", -1: "VGF_ERR_INVALID_ARG", -2: "VGF_ERR_UNSUPPORTED_SIZE",
          -3: "VGF_ERR_L_WINDOW", -4: "VGF_ERR_OUT_OF_MEMORY", -5: "VGF_ERR_HIP",
          -6: "VGF_ERR_NOT_REQUESTED", -7: "VGF_ERR_SCRATCH_LIMIT"}
NOALLOC_SCRATCH_BYTES = 64 << 20
METHODS = {"vgf": 0, "he": 1, "he_nearby": 2, "he_cellavg": 3}
PRECISIONS = {"f64": 0, "f32": 1}
OUT_PHI, OUT_E, FIELD_CENTERED, FIELD_GRADIENT_KERNEL, LAYOUT_AXIS0 = 1, 2, 16, 32, 64
EXPORTS = ["vgf_plan_create", "vgf_solve", "vgf_solve_adjoint", "vgf_solve_batched",
           "vgf_plan_get_L", "vgf_plan_workspace_bytes", "vgf_plan_get_kernel",
           "vgf_plan_get_spectrum", "vgf_plan_hip_error", "vgf_plan_destroy",
           "vgf_status_string", "vgf_plan_profile_begin", "vgf_plan_profile_end",
           "vgf_batch_create", "vgf_batch_solve", "vgf_batch_workspace_bytes", "vgf_batch_groups",
           "vgf_batch_hip_error", "vgf_batch_destroy", "vgf_plan_autotune", "vgf_plan_get_schedule",
           "vgf_plan_set_schedule", "vgf_batch_autotune", "vgf_batch_get_schedule",
           "vgf_plan_get_gradient_kernel", "vgf_plan_get_gradient_spectrum", "vgf_batch_adjoint",
           "vgf_solve_noalloc"]
BATCH_GRAPH = 1
PASS_NAMES = {3: ["r2c", "c2c_fwd", "fused", "c2c_inv", "c2r"],
              2: ["r2c", "fused", "c2r"]}
PASS_IDS = ["r2c", "c2c_fwd", "fused", "c2c_inv", "c2r"]  # VGF_PASS_* order
MAX_LAUNCHES = 16


class VGFError(RuntimeError):
    def __init__(self, status, what=""):
        self.status = status
        super().__init__("%s: %s (%s)" % (what, STATUS.get(status, status),
                                          lib().vgf_status_string(status).decode()))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libvgf.so not built (run paper_2103_08531_amd/build.py): %s" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        vp, i64p, dp = C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)
        L.vgf_plan_create.restype = C.c_int
        L.vgf_plan_create.argtypes = [C.POINTER(vp), C.c_int, i64p, dp, C.c_int, C.c_int,
                                      C.c_double, C.c_uint, vp]
        L.vgf_solve.restype = C.c_int
        L.vgf_solve.argtypes = [vp, vp, vp, vp, vp]
        L.vgf_solve_noalloc.restype = C.c_int
        L.vgf_solve_noalloc.argtypes = [vp, vp, vp, vp, vp]
        L.vgf_solve_adjoint.restype = C.c_int
        L.vgf_solve_adjoint.argtypes = [vp, vp, vp, vp, vp]
        L.vgf_solve_batched.restype = C.c_int
        L.vgf_solve_batched.argtypes = [C.POINTER(vp), C.c_int, C.POINTER(vp), C.POINTER(vp),
                                        C.POINTER(vp), vp]
        L.vgf_plan_get_L.restype = C.c_int
        L.vgf_plan_get_L.argtypes = [vp, dp]
        L.vgf_plan_workspace_bytes.restype = C.c_int
        L.vgf_plan_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.vgf_plan_get_kernel.restype = C.c_int
        L.vgf_plan_get_kernel.argtypes = [vp, dp]
        L.vgf_plan_get_spectrum.restype = C.c_int
        L.vgf_plan_get_spectrum.argtypes = [vp, dp]
        L.vgf_plan_hip_error.restype = C.c_int
        L.vgf_plan_hip_error.argtypes = [vp]
        L.vgf_plan_destroy.restype = None
        L.vgf_plan_destroy.argtypes = [vp]
        L.vgf_plan_profile_begin.restype = C.c_int
        L.vgf_plan_profile_begin.argtypes = [vp, C.c_int]
        L.vgf_plan_profile_end.restype = C.c_int
        L.vgf_plan_profile_end.argtypes = [vp, dp, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                           C.POINTER(C.c_int)]
        L.vgf_status_string.restype = C.c_char_p
        L.vgf_status_string.argtypes = [C.c_int]
        L.vgf_batch_create.restype = C.c_int
        L.vgf_batch_create.argtypes = [C.POINTER(vp), C.POINTER(vp), C.c_int, C.c_uint]
        L.vgf_batch_solve.restype = C.c_int
        L.vgf_batch_solve.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), vp]
        L.vgf_batch_adjoint.restype = C.c_int
        L.vgf_batch_adjoint.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), vp]
        L.vgf_batch_workspace_bytes.restype = C.c_int
        L.vgf_batch_workspace_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
        L.vgf_batch_groups.restype = C.c_int
        L.vgf_batch_groups.argtypes = [vp]
        L.vgf_batch_hip_error.restype = C.c_int
        L.vgf_batch_hip_error.argtypes = [vp]
        L.vgf_batch_destroy.restype = None
        L.vgf_batch_destroy.argtypes = [vp]
        ip = C.POINTER(C.c_int)
        L.vgf_plan_autotune.restype = C.c_int
        L.vgf_plan_autotune.argtypes = [vp, vp, vp, vp, C.c_int, vp]
        L.vgf_plan_get_schedule.restype = C.c_int
        L.vgf_plan_get_schedule.argtypes = [vp, ip]
        L.vgf_plan_set_schedule.restype = C.c_int
        L.vgf_plan_set_schedule.argtypes = [vp, ip]
        L.vgf_batch_autotune.restype = C.c_int
        L.vgf_batch_autotune.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.c_int, vp]
        L.vgf_batch_get_schedule.restype = C.c_int
        L.vgf_batch_get_schedule.argtypes = [vp, C.c_int, ip]
        L.vgf_plan_get_gradient_kernel.restype = C.c_int
        L.vgf_plan_get_gradient_kernel.argtypes = [vp, C.c_int, dp]
        L.vgf_plan_get_gradient_spectrum.restype = C.c_int
        L.vgf_plan_get_gradient_spectrum.argtypes = [vp, C.c_int, dp]
        _lib = L
    return _lib


def _check(st, what):
    if st != OK:
        raise VGFError(st, what)


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    if stream is not None:
        return C.c_void_p(stream.cuda_stream)
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:
        # the current stream's handle without building a Stream object (a few
        # microseconds per call, which small solves notice)
        return C.c_void_p(raw(torch.cuda.current_device()))
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


class Plan:
    """A solver plan for one grid (Sec. II: precompute once, then solve per rho).

    n: points per axis (2 or 3 values); h: spacings; method 'vgf', 'he', 'he_nearby' or
    'he_cellavg';
    precision 'f64' or 'f32'; L: VGF truncation radius (None: 1.1 x diameter);
    outputs: subset of {'phi', 'E'}; field: 'fourier' (default), 'centered'
    (E by second-order finite differences of phi) or 'gradient_kernel' (E_a =
    w_a * rho with the restricted 4N transform of -i k_a Ghat; VGF only);
    layout: 'contiguous' (default: the spectral multiply runs along the
    contiguous last axis) or 'axis0' (inside the strided axis-0 pass).
    """

    def __init__(self, n, h, method="vgf", precision="f64", L=None, outputs=("phi", "E"),
                 stream=None, field="fourier", layout="contiguous"):
        torch = _torch()
        self.n = tuple(int(x) for x in n)
        self.h = tuple(float(x) for x in h)
        self.dim = len(self.n)
        self.method = method
        self.precision = precision
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.outputs = tuple(outputs)
        if field not in ("fourier", "centered", "gradient_kernel"):
            raise ValueError("field must be 'fourier', 'centered' or 'gradient_kernel'")
        self.field = field
        flags = (OUT_PHI if "phi" in outputs else 0) | (OUT_E if "E" in outputs else 0)
        if field == "centered":
            flags |= FIELD_CENTERED
        elif field == "gradient_kernel":
            flags |= FIELD_GRADIENT_KERNEL
        if layout not in ("contiguous", "axis0"):
            raise ValueError("layout must be 'contiguous' or 'axis0'")
        self.layout = layout
        if layout == "axis0":
            flags |= LAYOUT_AXIS0
        n_arr = (C.c_int64 * self.dim)(*self.n)
        h_arr = (C.c_double * self.dim)(*self.h)
        handle = C.c_void_p()
        self._h = None
        st = lib().vgf_plan_create(C.byref(handle), self.dim, n_arr, h_arr,
                                   METHODS[method], PRECISIONS[precision],
                                   0.0 if L is None else float(L), flags, _stream(stream))
        _check(st, "vgf_plan_create")
        self._h = handle

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("plan destroyed")
        return self._h

    @property
    def L(self):
        v = C.c_double()
        _check(lib().vgf_plan_get_L(self.handle, C.byref(v)), "vgf_plan_get_L")
        return v.value

    @property
    def workspace_bytes(self):
        v = C.c_size_t()
        _check(lib().vgf_plan_workspace_bytes(self.handle, C.byref(v)), "vgf_plan_workspace_bytes")
        return v.value

    def kernel(self):
        out = np.zeros(self.n, dtype=np.float64)
        _check(lib().vgf_plan_get_kernel(self.handle, out.ctypes.data_as(C.POINTER(C.c_double))),
               "vgf_plan_get_kernel")
        return out

    def spectrum(self):
        out = np.zeros(tuple(x + 1 for x in self.n), dtype=np.float64)
        _check(lib().vgf_plan_get_spectrum(self.handle, out.ctypes.data_as(C.POINTER(C.c_double))),
               "vgf_plan_get_spectrum")
        return out

    def gradient_kernel(self, axis):
        out = np.zeros(self.n, dtype=np.float64)
        _check(lib().vgf_plan_get_gradient_kernel(self.handle, int(axis),
                                                  out.ctypes.data_as(C.POINTER(C.c_double))),
               "vgf_plan_get_gradient_kernel")
        return out

    def gradient_spectrum(self, axis):
        out = np.zeros(tuple(x + 1 for x in self.n), dtype=np.float64)
        _check(lib().vgf_plan_get_gradient_spectrum(self.handle, int(axis),
                                                    out.ctypes.data_as(C.POINTER(C.c_double))),
               "vgf_plan_get_gradient_spectrum")
        return out

    def _check_tensor(self, t, shape, name):
        if t.dtype != self.dtype or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shape:
            raise ValueError("%s must be a contiguous %s CUDA tensor of shape %s (got %s %s %s)"
                             % (name, self.dtype, shape, t.dtype, tuple(t.shape), t.device))

    def solve(self, rho, phi=None, E=None, want_phi=True, want_E=True, stream=None):
        """Returns (phi, E); fields not wanted come back as None."""
        torch = _torch()
        self._check_tensor(rho, self.n, "rho")
        want_phi = want_phi and "phi" in self.outputs
        want_E = want_E and "E" in self.outputs
        if want_phi and phi is None:
            phi = torch.empty(self.n, dtype=self.dtype, device=rho.device)
        if want_E and E is None:
            E = torch.empty((self.dim,) + self.n, dtype=self.dtype, device=rho.device)
        if not want_phi:
            phi = None
        if not want_E:
            E = None
        if phi is not None:
            self._check_tensor(phi, self.n, "phi")
        if E is not None:
            self._check_tensor(E, (self.dim,) + self.n, "E")
        st = lib().vgf_solve(self.handle, _ptr(rho), _ptr(phi), _ptr(E), _stream(stream))
        _check(st, "vgf_solve")
        return phi, E

    def solve_noalloc(self, rho, phi=None, E=None, stream=None):
        """vgf_solve_noalloc: the solve on the library's static scratch; the
        caller passes every output it wants (this call allocates nothing)."""
        self._check_tensor(rho, self.n, "rho")
        if phi is not None:
            self._check_tensor(phi, self.n, "phi")
        if E is not None:
            self._check_tensor(E, (self.dim,) + self.n, "E")
        st = lib().vgf_solve_noalloc(self.handle, _ptr(rho), _ptr(phi), _ptr(E), _stream(stream))
        _check(st, "vgf_solve_noalloc")
        return phi, E

    def adjoint(self, g_phi=None, g_E=None, g_rho=None, stream=None):
        torch = _torch()
        ref = g_phi if g_phi is not None else g_E
        if ref is None:
            raise ValueError("adjoint needs g_phi or g_E")
        if g_phi is not None:
            self._check_tensor(g_phi, self.n, "g_phi")
        if g_E is not None:
            self._check_tensor(g_E, (self.dim,) + self.n, "g_E")
        if g_rho is None:
            g_rho = torch.empty(self.n, dtype=self.dtype, device=ref.device)
        self._check_tensor(g_rho, self.n, "g_rho")
        st = lib().vgf_solve_adjoint(self.handle, _ptr(g_phi), _ptr(g_E), _ptr(g_rho),
                                     _stream(stream))
        _check(st, "vgf_solve_adjoint")
        return g_rho

    @property
    def schedule(self):
        """Tile variant per pass (r2c, c2c fwd, fused axis 0, c2c inv, c2r)."""
        v = (C.c_int * 5)()
        _check(lib().vgf_plan_get_schedule(self.handle, v), "vgf_plan_get_schedule")
        return tuple(v)

    @schedule.setter
    def schedule(self, sched):
        v = (C.c_int * 5)(*[int(x) for x in sched])
        _check(lib().vgf_plan_set_schedule(self.handle, v), "vgf_plan_set_schedule")

    def autotune(self, rho, phi=None, E=None, reps=3, stream=None):
        """Measure every tile schedule on this call's buffers and keep the fastest per pass."""
        torch = _torch()
        self._check_tensor(rho, self.n, "rho")
        if phi is None and "phi" in self.outputs:
            phi = torch.empty(self.n, dtype=self.dtype, device=rho.device)
        if E is None and "E" in self.outputs:
            E = torch.empty((self.dim,) + self.n, dtype=self.dtype, device=rho.device)
        _check(lib().vgf_plan_autotune(self.handle, _ptr(rho), _ptr(phi), _ptr(E), int(reps), _stream(stream)),
               "vgf_plan_autotune")
        return self.schedule

    def profile_begin(self, max_solves):
        _check(lib().vgf_plan_profile_begin(self.handle, int(max_solves)), "vgf_plan_profile_begin")

    def profile_end(self):
        """({pass name: mean ms}, [(pass name, mean ms) per launch], solves recorded)
        over the solves recorded since profile_begin."""
        ms = (C.c_double * MAX_LAUNCHES)()
        tags = (C.c_int * MAX_LAUNCHES)()
        nl, nsol = C.c_int(), C.c_int()
        _check(lib().vgf_plan_profile_end(self.handle, ms, tags, C.byref(nl), C.byref(nsol)),
               "vgf_plan_profile_end")
        launches = [(PASS_IDS[tags[k]], ms[k]) for k in range(nl.value)]
        passes = {}
        for name, t in launches:
            passes[name] = passes.get(name, 0.0) + t
        return passes, launches, nsol.value

    def close(self):
        if self._h is not None:
            lib().vgf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def solve_batched(plans, rhos, phis=None, Es=None, stream=None):
    """One vgf_solve_batched call over parallel lists (phis / Es entries may be None)."""
    count = len(plans)
    VP = C.c_void_p
    pl = (VP * count)(*[p.handle.value for p in plans])
    rh = (VP * count)(*[r.data_ptr() for r in rhos])
    ph = (VP * count)(*[(x.data_ptr() if x is not None else None) for x in phis]) if phis is not None else None
    ee = (VP * count)(*[(x.data_ptr() if x is not None else None) for x in Es]) if Es is not None else None
    st = lib().vgf_solve_batched(pl, count, rh, ph, ee, _stream(stream))
    _check(st, "vgf_solve_batched")


class Batch:
    """Many right-hand sides over fixed plans (vgf_batch_*): entries sharing a
    plan run as one launch per pass; with graph=True the whole batch is
    captured once and replayed as one hipGraph per solve."""

    def __init__(self, plans, graph=True):
        self.plans = list(plans)  # keeps the plans alive
        count = len(self.plans)
        VP = C.c_void_p
        pl = (VP * count)(*[p.handle.value for p in self.plans])
        handle = C.c_void_p()
        self._h = None
        _check(lib().vgf_batch_create(C.byref(handle), pl, count, BATCH_GRAPH if graph else 0),
               "vgf_batch_create")
        self._h = handle

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("batch destroyed")
        return self._h

    @property
    def groups(self):
        return lib().vgf_batch_groups(self.handle)

    @property
    def workspace_bytes(self):
        v = C.c_size_t()
        _check(lib().vgf_batch_workspace_bytes(self.handle, C.byref(v)), "vgf_batch_workspace_bytes")
        return v.value

    def solve(self, rhos, phis=None, Es=None, stream=None):
        """rhos, phis, Es: lists of tensors shaped for each entry's plan
        (phis / Es None: that output is skipped for every entry)."""
        rh, ph, ee = self._arrays(rhos, phis, Es)
        _check(lib().vgf_batch_solve(self.handle, rh, ph, ee, _stream(stream)), "vgf_batch_solve")

    def _arrays(self, rhos, phis, Es):
        # a replay loop passes the same tensors every time: reuse the pointer
        # arrays of the last call when every tensor and its storage are the same
        key = tuple((id(x), x.data_ptr()) for lst in (rhos, phis, Es) if lst is not None for x in lst) + (
            phis is None, Es is None)
        last = getattr(self, "_last_arrays", None)
        if last is not None and last[0] == key:
            return last[2]
        count = len(self.plans)
        if len(rhos) != count or (phis is not None and len(phis) != count) or (
                Es is not None and len(Es) != count):
            raise ValueError("one rho (and phi / E) per entry")
        for i, p in enumerate(self.plans):
            p._check_tensor(rhos[i], p.n, "rho[%d]" % i)
            if phis is not None:
                p._check_tensor(phis[i], p.n, "phi[%d]" % i)
            if Es is not None:
                p._check_tensor(Es[i], (p.dim,) + p.n, "E[%d]" % i)
        VP = C.c_void_p
        rh = (VP * count)(*[r.data_ptr() for r in rhos])
        ph = (VP * count)(*[x.data_ptr() for x in phis]) if phis is not None else None
        ee = (VP * count)(*[x.data_ptr() for x in Es]) if Es is not None else None
        # the tensors are kept with the key, so their ids cannot be reused
        self._last_arrays = (key, (list(rhos), phis and list(phis), Es and list(Es)), (rh, ph, ee))
        return rh, ph, ee

    def adjoint(self, g_phis=None, g_Es=None, g_rhos=None, stream=None):
        """Adjoint of every entry (vgf_batch_adjoint): g_phis / g_Es are lists
        of cotangents (None: zero for every entry); returns g_rhos (allocated
        when not given)."""
        torch = _torch()
        count = len(self.plans)
        if g_phis is None and g_Es is None:
            raise ValueError("adjoint needs g_phis or g_Es")
        if g_rhos is None:
            ref = g_phis if g_phis is not None else g_Es
            g_rhos = [torch.empty(p.n, dtype=p.dtype, device=ref[i].device) for i, p in enumerate(self.plans)]
        if len(g_rhos) != count or (g_phis is not None and len(g_phis) != count) or (
                g_Es is not None and len(g_Es) != count):
            raise ValueError("one g_rho (and g_phi / g_E) per entry")
        for i, p in enumerate(self.plans):
            p._check_tensor(g_rhos[i], p.n, "g_rho[%d]" % i)
            if g_phis is not None:
                p._check_tensor(g_phis[i], p.n, "g_phi[%d]" % i)
            if g_Es is not None:
                p._check_tensor(g_Es[i], (p.dim,) + p.n, "g_E[%d]" % i)
        VP = C.c_void_p
        gr = (VP * count)(*[x.data_ptr() for x in g_rhos])
        gp = (VP * count)(*[x.data_ptr() for x in g_phis]) if g_phis is not None else None
        ge = (VP * count)(*[x.data_ptr() for x in g_Es]) if g_Es is not None else None
        _check(lib().vgf_batch_adjoint(self.handle, gp, ge, gr, _stream(stream)), "vgf_batch_adjoint")
        return g_rhos

    def autotune(self, rhos, phis=None, Es=None, reps=3, stream=None):
        """Tune every group's tile schedule on these buffers; returns the schedules."""
        rh, ph, ee = self._arrays(rhos, phis, Es)
        _check(lib().vgf_batch_autotune(self.handle, rh, ph, ee, int(reps), _stream(stream)),
               "vgf_batch_autotune")
        return self.schedules()

    def schedules(self):
        out = []
        for g in range(self.groups):
            v = (C.c_int * 5)()
            _check(lib().vgf_batch_get_schedule(self.handle, g, v), "vgf_batch_get_schedule")
            out.append(tuple(v))
        return out

    def close(self):
        self._last_arrays = None
        if self._h is not None:
            lib().vgf_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def _autograd_function():
    torch = _torch()

    class VGFSolve(torch.autograd.Function):
        """(phi, E) = solve(rho); backward applies the hand-written adjoint."""

        @staticmethod
        def forward(ctx, rho, plan):
            ctx.plan = plan
            phi, E = plan.solve(rho.contiguous())
            return phi, E

        @staticmethod
        def backward(ctx, g_phi, g_E):
            plan = ctx.plan
            gp = g_phi.contiguous() if (g_phi is not None and "phi" in plan.outputs) else None
            ge = g_E.contiguous() if (g_E is not None and "E" in plan.outputs) else None
            if gp is None and ge is None:
                return None, None
            return plan.adjoint(gp, ge), None

    return VGFSolve


_VGFSolve = None


def VGFSolve():
    global _VGFSolve
    if _VGFSolve is None:
        _VGFSolve = _autograd_function()
    return _VGFSolve


def solve(rho, plan):
    """Differentiable solve: returns (phi, E) with autograd through the adjoint."""
    return VGFSolve().apply(rho, plan)


def _batch_autograd_function():
    torch = _torch()

    class VGFBatchSolve(torch.autograd.Function):
        """The solves of every entry of a Batch; backward applies the batched
        hand-written adjoint (vgf_batch_adjoint)."""

        @staticmethod
        def forward(ctx, batch, want_phi, want_E, *rhos):
            ctx.batch = batch
            ctx.want = (want_phi, want_E)
            plans = batch.plans
            phis = [torch.empty(p.n, dtype=p.dtype, device=rhos[i].device)
                    for i, p in enumerate(plans)] if want_phi else None
            Es = [torch.empty((p.dim,) + p.n, dtype=p.dtype, device=rhos[i].device)
                  for i, p in enumerate(plans)] if want_E else None
            batch.solve([r.contiguous() for r in rhos], phis, Es)
            return tuple((phis or []) + (Es or []))

        @staticmethod
        def backward(ctx, *grads):
            batch = ctx.batch
            want_phi, want_E = ctx.want
            plans = batch.plans
            count = len(plans)

            def cotangents(gs, shape_of):
                if all(g is None for g in gs):
                    return None
                return [g.contiguous() if g is not None else
                        torch.zeros(shape_of(p), dtype=p.dtype, device=next(x for x in gs if x is not None).device)
                        for g, p in zip(gs, plans)]

            gp = cotangents(grads[:count], lambda p: p.n) if want_phi else None
            ge = cotangents(grads[count if want_phi else 0:], lambda p: (p.dim,) + p.n) if want_E else None
            if gp is None and ge is None:
                return (None, None, None) + (None,) * count
            return (None, None, None) + tuple(batch.adjoint(gp, ge))

    return VGFBatchSolve


_VGFBatchSolve = None


def solve_batch(batch, rhos, want_phi=True, want_E=True):
    """Differentiable solves of a Batch's entries: returns (phis, Es), lists
    (None for an output not wanted), with autograd through the batched
    adjoint."""
    global _VGFBatchSolve
    if _VGFBatchSolve is None:
        _VGFBatchSolve = _batch_autograd_function()
    want_phi = want_phi and all("phi" in p.outputs for p in batch.plans)
    want_E = want_E and all("E" in p.outputs for p in batch.plans)
    if not (want_phi or want_E):
        raise ValueError("no output wanted")
    outs = _VGFBatchSolve.apply(batch, want_phi, want_E, *rhos)
    count = len(batch.plans)
    phis = list(outs[:count]) if want_phi else None
    Es = list(outs[count if want_phi else 0:]) if want_E else None
    return phis, Es
