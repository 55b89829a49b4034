"""Binding of the stress update with the MFP equation's transport terms
(include/tfs_transport.h): advection by a velocity field and centre-of-mass diffusion inside
the implicit operator, on a periodic grid.  Argument marshalling only: every transform and
kernel runs in libtfs.so."""
from __future__ import annotations

import ctypes as C

from . import tfs


class Transport:
    """One tfs_transport object for the grid fields of `plan` (a BDF2 tfs.Plan with one point
    per grid point, C order): box `shape` / `extent`, diffusion `eps`, `iters` splitting
    iterations per implicit solve."""

    def __init__(self, plan: tfs.Plan, shape, extent, eps, iters=30):
        self.plan = plan
        self.dim = len(shape)
        if len(extent) != self.dim:
            raise ValueError("shape and extent differ in length")
        sh = (C.c_int64 * self.dim)(*[int(n) for n in shape])
        ex = (C.c_double * self.dim)(*[float(L) for L in extent])
        h = C.c_void_p()
        tfs.check(tfs.lib().tfs_transport_create(self.dim, sh, ex, float(eps), int(plan.stride), int(iters),
                                                 C.byref(h)))
        self._h = h

    @property
    def batched(self):
        return bool(tfs.lib().tfs_transport_batched(self._h))

    def set_batched(self, on: bool):
        """Transform whole fields in batched plans (True) or one plane at a time (False)."""
        tfs.check(tfs.lib().tfs_transport_set_batched(self._h, int(bool(on))))

    def set_method(self, method: str):
        """"splitting" (the default) or "gmres" for the implicit solve."""
        tfs.check(tfs.lib().tfs_transport_set_method(self._h, {"splitting": 0, "gmres": 1}[method]))

    def set_tolerance(self, tol: float, every: int = 5):
        """Early exit of the solves at relative tolerance tol (0: fixed iteration counts)."""
        tfs.check(tfs.lib().tfs_transport_set_tolerance(self._h, float(tol), int(every)))

    @property
    def last_iterations(self) -> int:
        return int(tfs.lib().tfs_transport_last_iterations(self._h))

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            tfs.check(tfs.lib().tfs_transport_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n, kappa_a, kappa_b, u_a, u_b, X, Y, tau, diag=None):
        """Step n -> n+1 (tfs_transport_step); kappa_b / u_b None for given levels; diag an
        optional device [6] FP64 tensor for the diagnostics of level n+1."""
        import torch
        p, st = self.plan, self.plan.stride
        for t, nm, k in ((kappa_a, "kappa_a", p.dim * p.dim), (kappa_b, "kappa_b", p.dim * p.dim),
                         (u_a, "u_a", p.dim), (u_b, "u_b", p.dim), (tau, "tau", p.c)):
            p._need(t, nm, k * st, torch.float64)
        p._need(X, "X", 2 * p.c * st, torch.float64)
        p._need(Y, "Y", p.mode_levels * p.m * p.c * st, p.mode_dtype)
        p._need(diag, "diag", 6, torch.float64)
        ptr = lambda t: None if t is None else t.data_ptr()
        tfs.check(tfs.lib().tfs_transport_step(self._h, p.handle, int(n), ptr(kappa_a), ptr(kappa_b), ptr(u_a),
                                               ptr(u_b), X.data_ptr(), Y.data_ptr(), tau.data_ptr(), ptr(diag)))
