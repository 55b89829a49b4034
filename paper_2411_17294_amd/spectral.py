"""Spectral layout of the spatial form on a periodic grid (input and output preparation).

With u = 0 and a velocity gradient that is the same at every grid point, the operator of
eq. FP_discrete, L = -eps Laplace - A(kappa), acts on each Fourier mode of the fields
separately, and on a mode of wave vector xi the diffusion is the number eps |xi|^2.  The
plan then advances Fourier coefficients instead of grid values, one real number per
point (tfs_plan_set_spatial).

This module fixes that layout: the half spectrum of torch.fft.rfftn with norm="forward"
(so the constant function's coefficient is the field's mean), each complex coefficient
taking two consecutive points (real part, then imaginary part).  It builds the rate field
eps |xi|^2 and converts fields between the grid and the layout.  The conversions are a
change of basis before and after a run (torch.fft, i.e. rocFFT), not part of a step.
"""
from __future__ import annotations

import math


class PeriodicGrid:
    """A periodic box of `shape` grid points and `extent` length per axis (C order)."""

    def __init__(self, shape, extent):
        if len(shape) != len(extent) or len(shape) not in (2, 3):
            raise ValueError("shape and extent must both have 2 or 3 entries")
        self.shape = tuple(int(n) for n in shape)
        self.extent = tuple(float(L) for L in extent)
        self.dim = len(shape)
        self.half = self.shape[:-1] + (self.shape[-1] // 2 + 1,)
        self.npoints = 2 * math.prod(self.half)
        self.source_point = 0          # real part of the zero wave vector

    def _axes(self):
        return tuple(range(-self.dim, 0))

    def wavenumber_squared(self, device="cpu"):
        """|xi|^2 per point of the layout, [npoints] FP64."""
        import torch
        ks = []
        for j, (n, L) in enumerate(zip(self.shape, self.extent)):
            f = torch.fft.rfftfreq(n, d=L / n, dtype=torch.float64) if j == self.dim - 1 else \
                torch.fft.fftfreq(n, d=L / n, dtype=torch.float64)
            ks.append(2.0 * math.pi * f)
        grids = torch.meshgrid(*ks, indexing="ij")
        k2 = sum(g * g for g in grids).reshape(-1)
        return k2.repeat_interleave(2).to(device)

    def rate(self, eps, stride=None, device="cuda"):
        """The plan's rate field eps |xi|^2, padded with zeros to `stride` points."""
        import torch
        r = eps * self.wavenumber_squared(device)
        st = stride or self.npoints
        out = torch.zeros(st, dtype=torch.float64, device=device)
        out[:self.npoints] = r
        return out

    def to_points(self, fields):
        """[..., *shape] real grid fields -> [..., npoints] coefficients in the layout."""
        import torch
        F = torch.fft.rfftn(fields.to(torch.float64), dim=self._axes(), norm="forward")
        lead = fields.shape[:-self.dim]
        return torch.view_as_real(F).reshape(*lead, self.npoints)

    def to_grid(self, points):
        """[..., >= npoints] coefficients in the layout -> [..., *shape] grid fields."""
        import torch
        lead = points.shape[:-1]
        z = points[..., :self.npoints].contiguous().reshape(*lead, *self.half, 2)
        return torch.fft.irfftn(torch.view_as_complex(z), s=self.shape, dim=self._axes(), norm="forward")
