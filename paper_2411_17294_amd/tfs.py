"""Python binding of libtfs.so: argument marshalling only.

Every step of the update runs in the library's HIP kernels; this module only
passes device pointers, sizes and the stream.  PyTorch supplies device memory
and streams.  Importing it without the built library raises immediately: there
is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtfs.so")

TFS_OK, TFS_EINVAL, TFS_ENOMEM, TFS_EHIP, TFS_ENUMERIC, TFS_EUNSUPPORTED = range(6)
TFS_FP64, TFS_FP32_MODES = 0, 1
TFS_SCHEME_BDF2, TFS_SCHEME_EXP = 0, 1
TFS_KAPPA_FP64, TFS_KAPPA_FP32 = 0, 1
TFS_MODE_FORM_AUTO, TFS_MODE_FORM_Y, TFS_MODE_FORM_Z = 0, 1, 2
TFS_FLAG_CHECK_SYNC = 1

EXPORTS = ("tfs_plan_create", "tfs_plan_destroy", "tfs_plan_set_stream", "tfs_plan_set_spatial", "tfs_step",
           "tfs_step_noalloc", "tfs_step_levels", "tfs_step_adjoint", "tfs_plan_set_field", "tfs_field_eval", "tfs_run_fused", "tfs_pbar_size", "tfs_pbar_to_params", "tfs_pbar_rate_gradient",
           "tfs_modes_to_plain", "tfs_plan_x_levels",
           "tfs_plan_tables", "tfs_plan_stride", "tfs_plan_tile", "tfs_plan_tune", "tfs_soe_fit", "tfs_soe_gl_log",
           "tfs_status_string", "tfs_last_error",
           "tfs_ns_create", "tfs_ns_destroy", "tfs_ns_spectral_size", "tfs_ns_batched", "tfs_ns_set_batched", "tfs_ns_set_transport", "tfs_ns_init",
           "tfs_ns_step", "tfs_transport_create", "tfs_transport_destroy", "tfs_transport_step",
           "tfs_transport_batched", "tfs_transport_set_batched", "tfs_transport_set_method",
           "tfs_transport_set_tolerance", "tfs_transport_last_iterations",
           "tfs_spectral_create", "tfs_spectral_destroy", "tfs_spectral_npoints", "tfs_spectral_rate",
           "tfs_spectral_to_points", "tfs_spectral_to_grid")


# Mode-ring tile (points) used when the caller does not choose one: 32 KB mode planes
# (4096 FP64 or 8192 FP32 points), measured best on MI355X in 2-D and 3-D for both precisions.
def default_tile(dim, precision):
    return 8192 if precision == TFS_FP32_MODES else 4096


class TfsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(msg)
        self.status = status


class PlanDesc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nmodes", C.c_int32), ("npoints", C.c_int64), ("stride", C.c_int64),
                ("tile", C.c_int64),
                ("alpha", C.c_double), ("De", C.c_double), ("eta_p", C.c_double), ("dt", C.c_double),
                ("max_steps", C.c_int64), ("w", C.POINTER(C.c_double)), ("lam", C.POINTER(C.c_double)),
                ("precision", C.c_int32), ("flags", C.c_uint32), ("stream", C.c_void_p),
                ("scheme", C.c_int32), ("kappa_precision", C.c_int32), ("mode_form", C.c_int32)]


class FieldDesc(C.Structure):
    _fields_ = [("nterms", C.c_int32), ("grid", C.c_int64), ("point0", C.c_int64), ("k", C.POINTER(C.c_double)),
                ("phase", C.POINTER(C.c_double)), ("omega", C.POINTER(C.c_double)),
                ("coef", C.POINTER(C.c_double))]


_lib = None


def lib():
    """Load libtfs.so (built in-tree by paper_2411_17294_amd.build); raise if absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2411_17294_amd.build` "
                          "(there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, dp, i64, i32 = C.c_void_p, C.POINTER(C.c_double), C.c_int64, C.c_int32
    L.tfs_plan_create.argtypes = [C.POINTER(PlanDesc), C.POINTER(C.c_void_p)]
    L.tfs_plan_destroy.argtypes = [vp]
    L.tfs_plan_set_stream.argtypes = [vp, vp]
    L.tfs_plan_set_spatial.argtypes = [vp, vp, i64]
    L.tfs_plan_set_field.argtypes = [vp, C.POINTER(FieldDesc)]
    L.tfs_run_fused.argtypes = [vp, i64, i64, vp, vp, vp]
    L.tfs_field_eval.argtypes = [vp, C.c_double, vp, vp]
    L.tfs_step.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
    L.tfs_step_noalloc.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp]
    L.tfs_step_levels.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.tfs_step_adjoint.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.tfs_pbar_size.argtypes = [vp]
    L.tfs_pbar_size.restype = i64
    L.tfs_pbar_to_params.argtypes = [vp, dp, dp, dp, dp, dp, dp, dp, dp]
    L.tfs_pbar_rate_gradient.argtypes = [vp, dp, dp]
    L.tfs_modes_to_plain.argtypes = [vp, i64, vp, vp, vp]
    L.tfs_plan_x_levels.argtypes = [vp]
    L.tfs_plan_x_levels.restype = i32
    L.tfs_plan_tables.argtypes = [vp, dp, dp, dp]
    L.tfs_plan_stride.argtypes = [vp]
    L.tfs_plan_stride.restype = i64
    L.tfs_plan_tile.argtypes = [vp]
    L.tfs_plan_tile.restype = i64
    L.tfs_plan_tune.argtypes = [vp, C.c_char_p, i64]
    L.tfs_soe_fit.argtypes = [C.c_double, i32, C.c_double, C.c_double, dp, dp, dp, dp, dp]
    L.tfs_soe_gl_log.argtypes = [C.c_double, i32, C.c_double, C.c_double, dp, dp, dp, dp]
    L.tfs_status_string.argtypes = [C.c_int]
    L.tfs_status_string.restype = C.c_char_p
    L.tfs_last_error.restype = C.c_char_p
    L.tfs_ns_create.argtypes = [C.c_int, C.POINTER(i64), dp, C.c_double, C.c_double, i64, C.POINTER(C.c_void_p)]
    L.tfs_ns_destroy.argtypes = [vp]
    L.tfs_ns_spectral_size.argtypes = [vp]
    L.tfs_ns_spectral_size.restype = i64
    L.tfs_ns_batched.argtypes = [vp]
    L.tfs_ns_batched.restype = C.c_int
    L.tfs_ns_set_batched.argtypes = [vp, C.c_int]
    L.tfs_ns_set_transport.argtypes = [vp, vp]
    L.tfs_transport_create.argtypes = [C.c_int, C.POINTER(i64), dp, C.c_double, i64, C.c_int, C.POINTER(C.c_void_p)]
    L.tfs_transport_destroy.argtypes = [vp]
    L.tfs_transport_step.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp]
    L.tfs_transport_batched.argtypes = [vp]
    L.tfs_transport_batched.restype = C.c_int
    L.tfs_transport_set_batched.argtypes = [vp, C.c_int]
    L.tfs_transport_set_method.argtypes = [vp, C.c_int]
    L.tfs_transport_set_tolerance.argtypes = [vp, C.c_double, C.c_int]
    L.tfs_transport_last_iterations.argtypes = [vp]
    L.tfs_transport_last_iterations.restype = C.c_int
    L.tfs_ns_init.argtypes = [vp, vp, vp, vp, vp]
    L.tfs_ns_step.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp]
    L.tfs_spectral_create.argtypes = [C.c_int, C.POINTER(i64), dp, C.POINTER(C.c_void_p)]
    L.tfs_spectral_destroy.argtypes = [vp]
    L.tfs_spectral_npoints.argtypes = [vp]
    L.tfs_spectral_npoints.restype = i64
    L.tfs_spectral_rate.argtypes = [vp, C.c_double, vp, i64, vp]
    L.tfs_spectral_to_points.argtypes = [vp, vp, i64, i64, vp, i64, vp]
    L.tfs_spectral_to_grid.argtypes = [vp, vp, i64, i64, vp, i64, vp]
    for name in ("tfs_plan_create", "tfs_plan_destroy", "tfs_plan_set_stream", "tfs_plan_set_spatial", "tfs_step",
                 "tfs_step_levels", "tfs_plan_set_field", "tfs_field_eval", "tfs_run_fused",
                 "tfs_step_adjoint", "tfs_pbar_to_params", "tfs_pbar_rate_gradient", "tfs_modes_to_plain",
                 "tfs_plan_tables", "tfs_plan_tune", "tfs_soe_fit", "tfs_soe_gl_log",
                 "tfs_ns_create", "tfs_ns_destroy", "tfs_ns_set_batched", "tfs_ns_set_transport", "tfs_ns_init", "tfs_ns_step",
                 "tfs_transport_create", "tfs_transport_destroy", "tfs_transport_step",
           "tfs_transport_batched", "tfs_transport_set_batched", "tfs_transport_set_method",
           "tfs_transport_set_tolerance", "tfs_transport_last_iterations",
                 "tfs_spectral_create", "tfs_spectral_destroy", "tfs_spectral_rate", "tfs_spectral_to_points",
                 "tfs_spectral_to_grid"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(status: int):
    if status != TFS_OK:
        L = lib()
        raise TfsError(status, f"{L.tfs_status_string(status).decode()}: {L.tfs_last_error().decode()}")


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _tptr(t) -> Optional[int]:
    """Device address of a torch tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor required")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor required")
    return t.data_ptr()


def soe_fit(alpha: float, m: int, dt: float, T: float):
    """Product SOE fit (GL-log, Laplace-symbol window); returns (w, lam, dw, dlam, info)."""
    w, lam, dw, dl, info = np.zeros(m), np.zeros(m), np.zeros(m), np.zeros(m), np.zeros(4)
    check(lib().tfs_soe_fit(float(alpha), int(m), float(dt), float(T), _dptr(w), _dptr(lam), _dptr(dw),
                            _dptr(dl), _dptr(info)))
    return w, lam, dw, dl, {"y_lo": info[0], "y_hi": info[1], "symbol_relerr": info[2], "kernel_relerr": info[3]}


def soe_gl_log(alpha: float, m: int, y_lo: float, y_hi: float):
    w, lam, dw, dl = np.zeros(m), np.zeros(m), np.zeros(m), np.zeros(m)
    check(lib().tfs_soe_gl_log(float(alpha), int(m), float(y_lo), float(y_hi), _dptr(w), _dptr(lam), _dptr(dw),
                               _dptr(dl)))
    return w, lam, dw, dl


class Plan:
    """One tfs_plan: dim, m, npoints, parameters and the (w, lambda) table."""

    def __init__(self, dim, npoints, w, lam, alpha, De, eta_p, dt, max_steps, precision="fp64",
                 stride=0, tile=None, flags=0, stream=None, scheme="bdf2", kappa="fp64", mode_form="auto"):
        import torch
        self.dim = int(dim)
        self.c = self.dim * (self.dim + 1) // 2
        self.w = np.ascontiguousarray(w, dtype=np.float64)
        self.lam = np.ascontiguousarray(lam, dtype=np.float64)
        self.m = int(self.w.size)
        self.npoints = int(npoints)
        self.alpha, self.De, self.eta_p, self.dt = float(alpha), float(De), float(eta_p), float(dt)
        self.max_steps = int(max_steps)
        self.precision = {"fp64": TFS_FP64, "fp32_modes": TFS_FP32_MODES}[precision] \
            if isinstance(precision, str) else int(precision)
        self.mode_dtype = torch.float64 if self.precision == TFS_FP64 else torch.float32
        # storage precision of the velocity gradients the steps read (kappabar stays FP64)
        self.kappa_precision = {"fp64": TFS_KAPPA_FP64, "fp32": TFS_KAPPA_FP32}[kappa] \
            if isinstance(kappa, str) else int(kappa)
        self.kappa_dtype = torch.float32 if self.kappa_precision == TFS_KAPPA_FP32 else torch.float64
        self.scheme = {"bdf2": TFS_SCHEME_BDF2, "exp": TFS_SCHEME_EXP}[scheme] \
            if isinstance(scheme, str) else int(scheme)
        # mode levels the caller keeps: a two-slot ring (BDF2) or one level updated in place
        self.mode_levels = 1 if self.scheme == TFS_SCHEME_EXP else 2
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        if tile is None:
            tile = default_tile(self.dim, self.precision)
        d = PlanDesc(self.dim, self.m, self.npoints, int(stride), int(tile), self.alpha, self.De, self.eta_p, self.dt,
                     self.max_steps, _dptr(self.w), _dptr(self.lam), self.precision, int(flags),
                     C.c_void_p(stream), self.scheme, self.kappa_precision,
                     {"auto": TFS_MODE_FORM_AUTO, "y": TFS_MODE_FORM_Y, "z": TFS_MODE_FORM_Z}[mode_form]
                     if isinstance(mode_form, str) else int(mode_form))
        h = C.c_void_p()
        check(lib().tfs_plan_create(C.byref(d), C.byref(h)))
        self._h = h
        self.stride = int(lib().tfs_plan_stride(h))
        self.tile = int(lib().tfs_plan_tile(h))
        # slots of the X ring and of the adjoint's Xbar ring (3 for the shifted mode form)
        self.x_levels = int(lib().tfs_plan_x_levels(h))

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            check(lib().tfs_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        check(lib().tfs_plan_set_stream(self._h, C.c_void_p(stream)))

    def set_spatial(self, rate=None, source_point=-1):
        """Spatial form (tfs_plan_set_spatial): rate is a device FP64 tensor of at least
        stride elements (eps |xi|^2 per point) or None; source_point is the point holding
        the constant function's coefficient, or -1.  The plan keeps a reference to rate."""
        import torch
        self._need(rate, "rate", self.stride, torch.float64)
        check(lib().tfs_plan_set_spatial(self._h, _tptr(rate), int(source_point)))
        self._sp_rate = rate

    def set_field(self, k, phase, omega, coef, grid, point0=0):
        """Analytic velocity gradient of the fused launches (tfs_plan_set_field): host arrays
        k [NF][d], phase [NF], omega [NF], coef [NF][d][d] (kappa_ij = sum_n coef_nij
        sin(k_n . x + phase_n + omega_n t) on the grid of `grid` points per axis)."""
        d = self.dim
        k = np.ascontiguousarray(k, dtype=np.float64).reshape(-1, d)
        nf = k.shape[0]
        ph = np.ascontiguousarray(phase, dtype=np.float64).reshape(nf)
        om = np.ascontiguousarray(omega, dtype=np.float64).reshape(nf)
        cf = np.ascontiguousarray(coef, dtype=np.float64).reshape(nf, d * d)
        desc = FieldDesc(nf, int(grid), int(point0), _dptr(k), _dptr(ph), _dptr(om), _dptr(cf))
        check(lib().tfs_plan_set_field(self._h, C.byref(desc)))

    def field_eval(self, t, out, add=None):
        """out [d*d][stride] (kappa_dtype) = the plan's field at time t (+ add, FP64) (tfs_field_eval)."""
        import torch
        n = self.dim * self.dim * self.stride
        self._need(out, "kappa_out", n, self.kappa_dtype)
        self._need(add, "add", n, torch.float64)
        check(lib().tfs_field_eval(self._h, float(t), _tptr(add), _tptr(out)))
        return out

    def run_fused(self, n0, nsteps, X, Y, tau=None):
        """Levels n0 -> n0 + nsteps in one launch, kappa from the plan's field (tfs_run_fused)."""
        import torch
        if self.npoints > 0:
            st, c = self.stride, self.c
            self._need(X, "X", self.x_levels * c * st, torch.float64)
            self._need(Y, "Y", self.mode_levels * self.m * c * st, self.mode_dtype)
            self._need(tau, "tau", c * st, torch.float64)
        check(lib().tfs_run_fused(self._h, int(n0), int(nsteps), _tptr(X), _tptr(Y), _tptr(tau)))

    def tune(self, key: str, value: int):
        check(lib().tfs_plan_tune(self._h, key.encode(), int(value)))

    # -- buffers -------------------------------------------------------------------------
    def alloc(self, device="cuda"):
        """Zeroed X ring ([x_levels][c][stride]), Y ring (flat, in the plan's tiled layout), tau and
        diag tensors."""
        import torch
        st = self.stride
        X = torch.zeros((self.x_levels, self.c, st), dtype=torch.float64, device=device)
        Y = torch.zeros((self.mode_levels * self.m * self.c * st,), dtype=self.mode_dtype, device=device)
        tau = torch.zeros((self.c, st), dtype=torch.float64, device=device)
        diag = torch.zeros(6, dtype=torch.float64, device=device)
        return X, Y, tau, diag

    # -- entry points --------------------------------------------------------------------
    def _need(self, t, name, numel, dtype):
        """The C ABI takes raw pointers; refuse tensors smaller than the plan's layout."""
        if t is None:
            return
        if t.dtype != dtype:
            raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
        if t.numel() < numel:
            raise ValueError(f"{name}: {t.numel()} elements, the plan's layout needs {numel}")

    def step(self, n, kappa_a, kappa_b, X, Y, tau=None, diag=None):
        self._step(lib().tfs_step, n, kappa_a, kappa_b, X, Y, tau, diag)

    def step_noalloc(self, n, kappa_a, kappa_b, X, Y, tau=None, diag=None):
        """tfs_step_noalloc: tfs_step with the diagnostics partials in the library's static
        device scratch (no device allocation by the call)."""
        self._step(lib().tfs_step_noalloc, n, kappa_a, kappa_b, X, Y, tau, diag)

    def _step(self, fn, n, kappa_a, kappa_b, X, Y, tau, diag):
        import torch
        if self.npoints > 0:
            st, c, d = self.stride, self.c, self.dim
            self._need(kappa_a, "kappa_a", d * d * st, self.kappa_dtype)
            self._need(kappa_b, "kappa_b", d * d * st, self.kappa_dtype)
            self._need(X, "X", self.x_levels * c * st, torch.float64)
            self._need(Y, "Y", self.mode_levels * self.m * c * st, self.mode_dtype)
            self._need(tau, "tau", c * st, torch.float64)
        self._need(diag, "diag", 6, torch.float64)
        check(fn(self._h, int(n), _tptr(kappa_a), _tptr(kappa_b), _tptr(X), _tptr(Y), _tptr(tau), _tptr(diag)))

    def step_levels(self, n, kappa_a, kappa_b, X_n, X_nm1, X_out, Y_n, Y_nm1, Y_out, tau=None, diag=None,
                    X_nm2=None):
        """tfs_step_levels; X_nm2 (level n-2) is read by shifted-mode-form plans at n >= 2."""
        import torch
        if self.npoints > 0:
            st, c, d = self.stride, self.c, self.dim
            for t, nm in ((kappa_a, "kappa_a"), (kappa_b, "kappa_b")):
                self._need(t, nm, d * d * st, self.kappa_dtype)
            for t, nm in ((X_n, "X_n"), (X_nm1, "X_nm1"), (X_nm2, "X_nm2"), (X_out, "X_out"), (tau, "tau")):
                self._need(t, nm, c * st, torch.float64)
            for t, nm in ((Y_n, "Y_n"), (Y_nm1, "Y_nm1"), (Y_out, "Y_out")):
                self._need(t, nm, self.m * c * st, self.mode_dtype)
        self._need(diag, "diag", 6, torch.float64)
        check(lib().tfs_step_levels(self._h, int(n), _tptr(kappa_a), _tptr(kappa_b), _tptr(X_n), _tptr(X_nm1),
                                    _tptr(X_nm2), _tptr(X_out), _tptr(Y_n), _tptr(Y_nm1), _tptr(Y_out), _tptr(tau),
                                    _tptr(diag)))

    @property
    def pbar_size(self):
        return int(lib().tfs_pbar_size(self._h))

    def step_adjoint(self, n, kappa_a, kappa_b, X_n, X_nm1, X_np1, Y_n, Y_nm1, Xbar, Hbar, pbar,
                     taubar=None, kappabar_a=None, kappabar_b=None, X_nm2=None):
        """tfs_step_adjoint; X_nm2 (forward level n-2) is read by shifted-mode-form plans at n >= 2,
        whose Xbar ring has x_levels = 3 slots."""
        import torch
        if self.npoints > 0:
            st, c, d = self.stride, self.c, self.dim
            for t, nm in ((kappa_a, "kappa_a"), (kappa_b, "kappa_b")):
                self._need(t, nm, d * d * st, self.kappa_dtype)
            for t, nm in ((kappabar_a, "kappabar_a"), (kappabar_b, "kappabar_b")):
                self._need(t, nm, d * d * st, torch.float64)
            for t, nm in ((X_n, "X_n"), (X_nm1, "X_nm1"), (X_nm2, "X_nm2"), (X_np1, "X_np1"), (taubar, "taubar")):
                self._need(t, nm, c * st, torch.float64)
            for t, nm in ((Y_n, "Y_n"), (Y_nm1, "Y_nm1")):
                self._need(t, nm, self.m * c * st, self.mode_dtype)
            self._need(Xbar, "Xbar", self.x_levels * c * st, torch.float64)
            self._need(Hbar, "Hbar", self.mode_levels * self.m * c * st, self.mode_dtype)
        self._need(pbar, "pbar", self.pbar_size, torch.float64)
        check(lib().tfs_step_adjoint(self._h, int(n), _tptr(kappa_a), _tptr(kappa_b), _tptr(X_n), _tptr(X_nm1),
                                     _tptr(X_nm2), _tptr(X_np1), _tptr(Y_n), _tptr(Y_nm1), _tptr(Xbar), _tptr(Hbar),
                                     _tptr(taubar), _tptr(kappabar_a), _tptr(kappabar_b), _tptr(pbar)))

    def pbar_to_params(self, pbar_host, dw_dalpha=None, dlambda_dalpha=None):
        """(dL/dw [m], dL/dlambda [m], dL/dDe, dL/deta_p, dL/dalpha) from a host copy of pbar;
        dL/dalpha (chained in the library) is None unless the rule's derivatives are given."""
        pb = np.ascontiguousarray(pbar_host, dtype=np.float64)
        if pb.size < self.pbar_size:
            raise ValueError("pbar too short")
        dw, dl = np.zeros(self.m), np.zeros(self.m)
        dDe, dep, da = C.c_double(0.0), C.c_double(0.0), C.c_double(0.0)
        want_a = dw_dalpha is not None and dlambda_dalpha is not None
        dwa = np.ascontiguousarray(dw_dalpha, dtype=np.float64) if want_a else None
        dla = np.ascontiguousarray(dlambda_dalpha, dtype=np.float64) if want_a else None
        if want_a and (dwa.size != self.m or dla.size != self.m):
            raise ValueError("dw/dalpha and dlambda/dalpha need m entries")
        check(lib().tfs_pbar_to_params(self._h, _dptr(pb), _dptr(dwa) if want_a else None,
                                       _dptr(dla) if want_a else None, _dptr(dw), _dptr(dl), C.pointer(dDe),
                                       C.pointer(dep), C.pointer(da) if want_a else None))
        return dw, dl, dDe.value, dep.value, (da.value if want_a else None)

    def pbar_rate_gradient(self, pbar_host):
        """sum_p rate_p dL/drate_p of the spatial form (eps dL/deps for rate = eps |xi|^2)."""
        pb = np.ascontiguousarray(pbar_host, dtype=np.float64)
        if pb.size < self.pbar_size:
            raise ValueError("pbar too short")
        out = C.c_double(0.0)
        check(lib().tfs_pbar_rate_gradient(self._h, _dptr(pb), C.pointer(out)))
        return out.value

    def modes_to_plain(self, level, X, Y, out):
        """Plain modes of time level `level` from the X and mode rings (tfs_modes_to_plain)."""
        import torch
        st, c = self.stride, self.c
        self._need(X, "X", self.x_levels * c * st, torch.float64)
        self._need(Y, "Y", self.mode_levels * self.m * c * st, self.mode_dtype)
        self._need(out, "out", self.m * c * st, torch.float64)
        check(lib().tfs_modes_to_plain(self._h, int(level), _tptr(X), _tptr(Y), _tptr(out)))

    def kappa_tensor(self, kappa=None, device="cuda"):
        """[d*d][stride] device tensor in the plan's kappa precision, optionally filled from a
        host [d*d][npoints] array (rounded to that precision)."""
        import torch
        t = torch.zeros((self.dim * self.dim, self.stride), dtype=self.kappa_dtype, device=device)
        if kappa is not None:
            t[:, :self.npoints] = torch.as_tensor(np.ascontiguousarray(kappa)).to(device).to(self.kappa_dtype)
        return t

    def tables(self):
        t = np.zeros((5, self.m))
        s = np.zeros(8)
        z = np.zeros(self.max_steps + 1)
        check(lib().tfs_plan_tables(self._h, _dptr(t), _dptr(s), _dptr(z)))
        return {"d": t[0], "c": t[1], "eta_k": t[2], "u": t[3], "v": t[4], "eta": s[0], "s_ec": s[1],
                "a_diag": s[2], "tau_scale": s[3], "theta": s[4], "rho": s[5], "sigma1": s[6], "sigma2": s[7],
                "zeta": z}
