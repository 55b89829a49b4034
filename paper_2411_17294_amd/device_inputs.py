"""Device-side synthesis of the seeded inputs (plumbing, not the method).

Evaluates the same divergence-free Fourier velocity-gradient field as
``inputs.FourierField.kappa_at`` on the whole grid with torch FP64 operations,
chunked over points, and lays out X0 in the X ring.  No part of the update runs
here.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import inputs as I


class DeviceKappa:
    """kappa(x, t) of a FourierField on a full periodic grid, written into [d*d][stride] tensors."""

    def __init__(self, ff: I.FourierField, grid: int, npoints: int, device="cuda", chunk=1 << 22, offset=0):
        self.ff = ff
        self.grid = grid
        self.dim = ff.dim
        self.npoints = npoints
        self.offset = int(offset)   # first flat grid index (a slab of the grid)
        self.device = device
        self.chunk = chunk
        self.k = torch.tensor(ff.k.T.astype(np.float64), device=device)                    # [d, NF]
        self.B = torch.tensor(ff.coef().reshape(len(ff.amp), ff.dim * ff.dim), device=device)  # [NF, d*d]
        self.phase = torch.tensor(ff.phase, device=device)
        self.omega = torch.tensor(ff.omega, device=device)
        # k . x + phase of every point, kept when it fits one chunk (slabs evaluated at many t)
        self.theta0 = self._theta0(0, npoints) if npoints <= chunk else None

    def _theta0(self, p0, p1):
        d, g = self.dim, self.grid
        flat = torch.arange(self.offset + p0, self.offset + p1, device=self.device, dtype=torch.int64)
        idx = torch.empty((p1 - p0, d), device=self.device, dtype=torch.float64)
        r = flat.clone()
        for a in range(d):
            idx[:, a] = (r % g).to(torch.float64)
            r = r // g
        return (idx * (2.0 * math.pi / g)) @ self.k + self.phase[None, :]

    def fill(self, out: torch.Tensor, t: float):
        """out: [d*d][stride] FP64; column j gets grid point offset + j, j < npoints."""
        if self.theta0 is not None:
            out[:, :self.npoints] = (torch.sin(self.theta0 + self.omega[None, :] * t) @ self.B).T
            return out
        for p0 in range(0, self.npoints, self.chunk):
            p1 = min(self.npoints, p0 + self.chunk)
            theta = self._theta0(p0, p1) + self.omega[None, :] * t
            out[:, p0:p1] = (torch.sin(theta) @ self.B).T
        return out


def x0_ring(wl: I.Workload, stride: int, device="cuda", points=None):
    """X ring [2][c][stride] with X0 of workload wl in slot 0 (all points, or the given subset)."""
    X0 = I.initial_state(wl, points)
    P = X0.shape[1]
    X = torch.zeros((2, wl.c, stride), dtype=torch.float64, device=device)
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
