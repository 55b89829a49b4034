"""Device-side synthesis of the seeded inputs (plumbing, not the method).

Evaluates the same divergence-free Fourier velocity-gradient field as
``inputs.FourierField.kappa_at`` on the whole grid with the library's field kernel
(tfs_field_eval), and lays out X0 in the X ring.  No part of the update runs here.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import inputs as I
from . import tfs


class DeviceKappa:
    """kappa(x, t) of a FourierField on a periodic grid (or a slab of consecutive grid points
    from flat index `offset`), written into [d*d][stride] device tensors by the library's field
    evaluation (tfs_field_eval: every term's phase and sine and the sums in FP64, rounded once
    to the tensor's precision, FP64 or FP32).  The evaluation runs through a one-mode plan per
    (stride, precision) that serves only this purpose."""

    def __init__(self, ff: I.FourierField, grid: int, npoints: int, device="cuda", offset=0):
        self.ff = ff
        self.grid = grid
        self.dim = ff.dim
        self.npoints = npoints
        self.offset = int(offset)   # first flat grid index (a slab of the grid)
        self.device = device
        self._plans = {}

    def _plan(self, stride, dtype):
        key = (stride, dtype)
        if key not in self._plans:
            f32 = dtype == torch.float32
            p = tfs.Plan(self.dim, self.npoints, [1.0], [0.0], 1.0, 1.0, 0.0, 1.0, 1,
                         precision="fp32_modes" if f32 else "fp64", stride=stride, tile=0,
                         kappa="fp32" if f32 else "fp64")
            p.set_field(*self.ff.table(self.grid, self.offset))
            self._plans[key] = p
        return self._plans[key]

    def fill(self, out: torch.Tensor, t: float):
        """out: [d*d][stride] FP64 or FP32; column j gets grid point offset + j, j < npoints."""
        if out.dim() != 2 or out.shape[0] != self.dim * self.dim or out.shape[1] < self.npoints:
            raise ValueError("out must be [d*d][stride >= npoints]")
        self._plan(int(out.shape[1]), out.dtype).field_eval(t, out)
        return out


def x0_ring(wl: I.Workload, stride: int, device="cuda", points=None, levels=2):
    """X ring [levels][c][stride] with X0 of workload wl in slot 0 (all points, or the given
    subset); levels is the plan's x_levels."""
    X0 = I.initial_state(wl, points)
    P = X0.shape[1]
    X = torch.zeros((levels, wl.c, stride), dtype=torch.float64, device=device)
    X[0, :, :P] = torch.from_numpy(X0).to(device)
    return X


def synthetic_velocity(d, n, seed, k0=4.0):
    """A seeded random grid velocity on [0, 2 pi)^d with the isotropic spectrum shape
    E(k) ~ k^4 exp(-2 (k/k0)^2) of synthetic decaying-turbulence initial data, rms 1 per
    component ([d][n^d], C order; the solver keeps its solenoidal part)."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    f = torch.randn((d,) + (n,) * d, dtype=torch.float64, device="cuda", generator=g)
    F = torch.fft.rfftn(f, dim=tuple(range(1, d + 1)))
    ks = [torch.fft.fftfreq(n, 1.0 / n, dtype=torch.float64, device="cuda")] * (d - 1) + \
        [torch.fft.rfftfreq(n, 1.0 / n, dtype=torch.float64, device="cuda")]
    K2 = sum(k * k for k in torch.meshgrid(*ks, indexing="ij"))
    F = F * (K2 * torch.exp(-K2 / (k0 * k0)))
    u = torch.fft.irfftn(F, s=(n,) * d, dim=tuple(range(1, d + 1)))
    u = u / u.pow(2).mean(dim=tuple(range(1, d + 1)), keepdim=True).sqrt()
    return u.reshape(d, n ** d)
