"""Binding of the spectral layout of the spatial form on a periodic grid (include/tfs.h,
tfs_spectral_*): input and output preparation for tfs_plan_set_spatial.

With u = 0 and a velocity gradient that is the same at every grid point, the operator of
eq. FP_discrete, L = -eps Laplace - A(kappa), acts on each Fourier mode of the fields
separately, and on a mode of wave vector xi the diffusion is the number eps |xi|^2.  The
plan then advances Fourier coefficients instead of grid values, one real number per
point.  The layout is the half spectrum of a real-to-complex transform normalised so that
the constant function's coefficient is the field's mean, each complex coefficient taking
two consecutive points (real part, then imaginary part).  The library writes the rate
field eps |xi|^2 and converts fields between the grid and the layout (hipFFT plans of its
own); this module only marshals arguments.
"""
from __future__ import annotations

import ctypes as C
import math

from . import tfs


class PeriodicGrid:
    """A periodic box of `shape` grid points and `extent` length per axis (C order).  The
    library object behind it is made on first use, on the current device."""

    def __init__(self, shape, extent):
        if len(shape) != len(extent) or len(shape) not in (2, 3):
            raise ValueError("shape and extent must both have 2 or 3 entries")
        self.shape = tuple(int(n) for n in shape)
        self.extent = tuple(float(L) for L in extent)
        self.dim = len(shape)
        self.half = self.shape[:-1] + (self.shape[-1] // 2 + 1,)
        self.npoints = 2 * math.prod(self.half)
        self.ngrid = math.prod(self.shape)
        self.source_point = 0          # real part of the zero wave vector
        self._h = None

    def _handle(self):
        if self._h is None:
            sh = (C.c_int64 * self.dim)(*self.shape)
            ex = (C.c_double * self.dim)(*self.extent)
            h = C.c_void_p()
            tfs.check(tfs.lib().tfs_spectral_create(self.dim, sh, ex, C.byref(h)))
            self._h = h
            if tfs.lib().tfs_spectral_npoints(h) != self.npoints:
                raise RuntimeError("the library's layout size differs from the binding's")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            tfs.check(tfs.lib().tfs_spectral_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _stream():
        import torch
        return torch.cuda.current_stream().cuda_stream

    def rate(self, eps, stride=None, device="cuda"):
        """The plan's rate field eps |xi|^2 per point of the layout, zero on the padding up
        to `stride` points ([stride] FP64 on the device)."""
        import torch
        st = int(stride or self.npoints)
        out = torch.empty(st, dtype=torch.float64, device=device)
        tfs.check(tfs.lib().tfs_spectral_rate(self._handle(), float(eps), tfs._tptr(out), st, self._stream()))
        return out

    def to_points(self, fields):
        """[..., *shape] real grid fields (device) -> [..., npoints] coefficients in the layout."""
        import torch
        lead = fields.shape[:fields.dim() - self.dim]
        if tuple(fields.shape[fields.dim() - self.dim:]) != self.shape:
            raise ValueError(f"fields must end in the grid shape {self.shape}")
        g = fields.to(torch.float64).contiguous().reshape(-1, self.ngrid)
        out = torch.empty((g.shape[0], self.npoints), dtype=torch.float64, device=g.device)
        tfs.check(tfs.lib().tfs_spectral_to_points(self._handle(), tfs._tptr(g), g.shape[0], self.ngrid,
                                                   tfs._tptr(out), self.npoints, self._stream()))
        return out.reshape(*lead, self.npoints)

    def to_grid(self, points):
        """[..., >= npoints] coefficients in the layout (device) -> [..., *shape] grid fields."""
        import torch
        lead = points.shape[:-1]
        if points.shape[-1] < self.npoints:
            raise ValueError(f"need at least {self.npoints} points per field")
        z = points[..., :self.npoints].to(torch.float64).reshape(-1, self.npoints)
        if z.stride(-1) != 1 or (z.shape[0] > 1 and z.stride(0) < self.npoints):
            z = z.contiguous()
        if not z.is_cuda:
            raise ValueError("device tensor required")
        out = torch.empty((z.shape[0], self.ngrid), dtype=torch.float64, device=z.device)
        ps = z.stride(0) if z.shape[0] > 1 else self.npoints
        tfs.check(tfs.lib().tfs_spectral_to_grid(self._handle(), z.data_ptr(), z.shape[0], ps,
                                                 tfs._tptr(out), self.ngrid, self._stream()))
        return out.reshape(*lead, *self.shape)
