"""Binding of the coupled step (include/tfs_ns.h): the pseudo-spectral projection method for
the Navier-Stokes equations on a periodic box, coupled to the stress update of a tfs.Plan.
Argument marshalling only: every transform and kernel runs in libtfs.so."""
from __future__ import annotations

import ctypes as C

from . import tfs


class Solver:
    """One tfs_ns object: a periodic box of `shape` points and `extent` lengths, viscosity
    nu = beta/Re and step dt, for grid fields of the plane stride of `plan` (a tfs.Plan with
    one point per grid point, C order)."""

    def __init__(self, plan: tfs.Plan, shape, extent, nu, dt):
        self.plan = plan
        self.dim = len(shape)
        if len(extent) != self.dim:
            raise ValueError("shape and extent differ in length")
        self.shape = tuple(int(n) for n in shape)
        sh = (C.c_int64 * self.dim)(*self.shape)
        ex = (C.c_double * self.dim)(*[float(L) for L in extent])
        h = C.c_void_p()
        tfs.check(tfs.lib().tfs_ns_create(self.dim, sh, ex, float(nu), float(dt), int(plan.stride), C.byref(h)))
        self._h = h
        self.nc = int(tfs.lib().tfs_ns_spectral_size(h))
        self.batched = bool(tfs.lib().tfs_ns_batched(h))

    def set_batched(self, on: bool):
        """Transform whole fields in batched plans (True) or one plane at a time (False)."""
        tfs.check(tfs.lib().tfs_ns_set_batched(self._h, int(bool(on))))
        self.batched = bool(tfs.lib().tfs_ns_batched(self._h))

    def set_transport(self, tr):
        """Stress update with the MFP transport terms (a transport.Transport), or None for the
        pointwise update."""
        self._transport = tr                     # kept alive while the solver uses it
        tfs.check(tfs.lib().tfs_ns_set_transport(self._h, None if tr is None else tr.handle))

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            tfs.check(tfs.lib().tfs_ns_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def alloc(self, device="cuda"):
        """(u [d][stride], kappa [d*d][stride], uh ring, fh ring) device buffers, zeroed; the
        rings are [2][d][nc] complex128."""
        import torch
        d, st = self.dim, self.plan.stride
        u = torch.zeros((d, st), dtype=torch.float64, device=device)
        kappa = torch.zeros((d * d, st), dtype=torch.float64, device=device)
        uh = torch.zeros((2, d, self.nc), dtype=torch.complex128, device=device)
        fh = torch.zeros((2, d, self.nc), dtype=torch.complex128, device=device)
        return u, kappa, uh, fh

    def _check(self, t, name, numel, dtype):
        if t is None or not t.is_cuda or not t.is_contiguous() or t.dtype != dtype or t.numel() < numel:
            raise ValueError(f"{name}: need a contiguous CUDA {dtype} tensor of >= {numel} elements")

    def init(self, u, uh, kappa):
        """Level 0 from the grid velocity in u (overwritten with its solenoidal in-band part)."""
        import torch
        d, st = self.dim, self.plan.stride
        self._check(u, "u", d * st, torch.float64)
        self._check(kappa, "kappa", d * d * st, torch.float64)
        self._check(uh, "uh", 2 * d * self.nc, torch.complex128)
        tfs.check(tfs.lib().tfs_ns_init(self._h, self.plan.handle, u.data_ptr(), uh.data_ptr(), kappa.data_ptr()))

    def step(self, n, u, uh, fh, kappa, X, Y, tau, diag=None):
        """Coupled step n -> n+1 (tfs_ns_step)."""
        import torch
        d, st, p = self.dim, self.plan.stride, self.plan
        self._check(u, "u", d * st, torch.float64)
        self._check(kappa, "kappa", d * d * st, torch.float64)
        self._check(uh, "uh", 2 * d * self.nc, torch.complex128)
        self._check(fh, "fh", 2 * d * self.nc, torch.complex128)
        self._check(X, "X", 2 * p.c * st, torch.float64)
        self._check(Y, "Y", p.mode_levels * p.m * p.c * st, p.mode_dtype)
        self._check(tau, "tau", p.c * st, torch.float64)
        if diag is not None:
            self._check(diag, "diag", 6, torch.float64)
        tfs.check(tfs.lib().tfs_ns_step(self._h, p.handle, int(n), u.data_ptr(), uh.data_ptr(), fh.data_ptr(),
                                        kappa.data_ptr(), X.data_ptr(), Y.data_ptr(), tau.data_ptr(),
                                        None if diag is None else diag.data_ptr()))
