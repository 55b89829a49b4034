"""Seeded synthetic inputs for the time-fractional extra-stress update.

This module holds no arithmetic of the method itself.  It only describes the
five workloads and draws their inputs:

* the prescribed velocity gradient kappa = grad u of a divergence-free,
  periodic Fourier velocity field (a kinematic-simulation sum), and
* the initial conformation deviation X0 = C0 - I (identity conformation plus
  small seeded symmetric noise).

The paper measures on finite-element meshes that are not available here; these
synthetic periodic fields stand in for the velocity gradients its coupled
Navier--Stokes solve would hand to the Fokker--Planck update (Sec. 4.1: the MFP
step only consumes grad u at the new level).  Both the device path and the CPU
oracle receive exactly these arrays.

Layouts (structure of arrays, point index fastest):
  kappa  [d*d][N]  row-major ij, kappa_ij = d u_i / d x_j
  X      [c][N]    packed symmetric: 2-D (xx, yy, xy); 3-D (xx, yy, zz, xy, xz, yz)
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

# packed symmetric component order, shared by every producer and consumer
PACK2 = ((0, 0), (1, 1), (0, 1))
PACK3 = ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))


def packed_pairs(dim: int):
    return PACK2 if dim == 2 else PACK3


def ncomp(dim: int) -> int:
    return dim * (dim + 1) // 2


@dataclasses.dataclass(frozen=True)
class Workload:
    """One parameter set of the five benchmark workloads."""
    cid: int
    name: str
    dim: int
    grid: int                 # points per axis
    alphas: tuple             # fractional orders run by this workload
    nmodes: int               # exponential modes m
    nsteps: int
    dt: float
    precision: str            # "fp64" or "fp32_modes"
    kmin: float
    kmax: float
    spectrum: Optional[float]  # E(k) ~ k^-p exponent; None = C1 literal amplitudes
    nfourier: int
    time_varying: bool
    De: float = 1.0            # Weissenberg number 1 -> relaxation time 1
    eta_p: float = 0.1         # polymer viscosity ratio (1-beta)/Re with Re = 1
    adjoint: bool = False
    ckpt_every: int = 0
    target_alpha: Optional[float] = None
    target_De_factor: float = 1.0

    @property
    def c(self) -> int:
        return ncomp(self.dim)

    @property
    def npoints(self) -> int:
        return self.grid ** self.dim


WORKLOADS = {
    1: Workload(1, "fp64_2d_64sq_m20", 2, 64, (0.5,), 20, 200, 1e-3, "fp64",
                1.0, 4.0, None, 8, False),
    2: Workload(2, "fp64_2d_1024sq_m32", 2, 1024, (0.3, 0.7), 32, 1000, 5e-4, "fp64",
                4.0, 256.0, 3.0, 64, True),
    3: Workload(3, "fp32modes_3d_256cube_m40", 3, 256, (0.4,), 40, 500, 2e-4, "fp32_modes",
                2.0, 128.0, 5.0 / 3.0, 64, False),
    4: Workload(4, "adjoint_3d_128cube_m32", 3, 128, (0.6,), 32, 400, 2.5e-4, "fp32_modes",
                2.0, 64.0, 5.0 / 3.0, 64, False, adjoint=True, ckpt_every=50,
                target_alpha=0.55, target_De_factor=1.05),
    5: Workload(5, "fp32modes_adjoint_3d_384cube_m48", 3, 384, (0.2,), 48, 2000, 1e-4, "fp32_modes",
                2.0, 192.0, 5.0 / 3.0, 64, True, adjoint=True, ckpt_every=100),
}


@dataclasses.dataclass
class FourierField:
    """u(x,t) = sum_n A_n e_n cos(k_n . x + phi_n + omega_n t) on [0, 2 pi)^d."""
    dim: int
    k: np.ndarray       # [NF, d] integer wavevectors
    e: np.ndarray       # [NF, d] unit vectors, e_n . k_n = 0
    amp: np.ndarray     # [NF]
    phase: np.ndarray   # [NF]
    omega: np.ndarray   # [NF]

    def coef(self) -> np.ndarray:
        """[NF, d, d] coefficient B_n,ij = -A_n e_n,i k_n,j of sin(theta_n) in kappa_ij."""
        return -(self.amp[:, None, None] * self.e[:, :, None] * self.k[:, None, :])

    def table(self, grid: int, point0: int = 0) -> tuple:
        """(k, phase, omega, coef, grid, point0): the field as tfs_plan_set_field takes it,
        on the grid of `grid` points per axis with the plan's point 0 at flat index point0."""
        return (self.k.astype(np.float64), self.phase, self.omega, self.coef(), int(grid), int(point0))

    def kappa_at(self, idx: np.ndarray, grid: int, t: float) -> np.ndarray:
        """kappa at the grid points with multi-indices idx [P, d] and time t -> [d*d, P] fp64."""
        d = self.dim
        x = (2.0 * math.pi / grid) * np.asarray(idx, dtype=np.float64)      # [P, d]
        theta = x @ self.k.T.astype(np.float64) + self.phase[None, :] + self.omega[None, :] * t  # [P, NF]
        s = np.sin(theta)
        B = self.coef().reshape(len(self.amp), d * d)                        # [NF, d*d]
        return np.ascontiguousarray((s @ B).T)                               # [d*d, P]

    def kappa_levels(self, idx: np.ndarray, grid: int, times) -> np.ndarray:
        """kappa at many times -> [T, d*d, P]; sin(a + w t) by angle addition (one sin/cos
        table per point and mode), so it is faster than kappa_at per level but not bitwise
        equal to it."""
        d = self.dim
        x = (2.0 * math.pi / grid) * np.asarray(idx, dtype=np.float64)
        theta = x @ self.k.T.astype(np.float64) + self.phase[None, :]
        st, ct = np.sin(theta), np.cos(theta)
        B = self.coef().reshape(len(self.amp), d * d)
        out = np.empty((len(times), d * d, idx.shape[0]))
        for i, t in enumerate(times):
            s = st * np.cos(self.omega * t)[None, :] + ct * np.sin(self.omega * t)[None, :]
            out[i] = (s @ B).T
        return out


def _draw_wavevectors(rng, dim, kmin, kmax, nf, grid, log_uniform):
    ks = []
    seen = set()
    tries = 0
    while len(ks) < nf:
        tries += 1
        if tries > 200000:
            raise RuntimeError("could not draw distinct wavevectors")
        if log_uniform:
            mag = math.exp(rng.uniform(math.log(kmin), math.log(kmax)))
            v = rng.standard_normal(dim)
            v = v / np.linalg.norm(v) * mag
            kv = np.rint(v).astype(np.int64)
        else:
            kv = rng.integers(-int(kmax), int(kmax) + 1, size=dim)
        kn = float(np.linalg.norm(kv))
        if kn < kmin - 1e-12 or kn > kmax + 1e-12 or kn == 0.0:
            continue
        if np.any(np.abs(kv) >= grid // 2):          # stay strictly below Nyquist
            continue
        key = tuple(int(a) for a in kv)
        neg = tuple(-a for a in key)
        if key in seen or neg in seen:               # distinct up to sign
            continue
        seen.add(key)
        ks.append(kv)
    return np.array(ks, dtype=np.int64)


def _perp_unit(rng, k):
    d = len(k)
    kf = k.astype(np.float64)
    if d == 2:
        e = np.array([-kf[1], kf[0]]) / np.linalg.norm(kf)
        return e if rng.uniform() < 0.5 else -e
    while True:
        v = rng.standard_normal(d)
        v = v - (v @ kf) / (kf @ kf) * kf
        nv = np.linalg.norm(v)
        if nv > 1e-6:
            return v / nv


def fourier_field(wl: Workload, seed: Optional[int] = None) -> FourierField:
    """Seeded divergence-free periodic velocity field for workload wl."""
    rng = np.random.Generator(np.random.PCG64(1000 + wl.cid if seed is None else seed))
    d = wl.dim
    log_uniform = wl.spectrum is not None
    k = _draw_wavevectors(rng, d, wl.kmin, wl.kmax, wl.nfourier, wl.grid, log_uniform)
    e = np.stack([_perp_unit(rng, kv) for kv in k])
    kn = np.linalg.norm(k.astype(np.float64), axis=1)
    if wl.spectrum is None:
        amp = rng.standard_normal(len(k)) * kn ** -2.0
    else:
        dk = kn * math.log(wl.kmax / wl.kmin) / len(k)
        amp = np.sqrt(2.0 * kn ** (-wl.spectrum) * dk)
        # distinct, sub-Nyquist wavevectors: grid mean of sin^2 is 1/2, cross terms vanish
        rms = math.sqrt(0.5 * float(np.sum(amp ** 2 * kn ** 2)))
        amp = amp / rms
    phase = rng.uniform(0.0, 2.0 * math.pi, size=len(k))
    omega = rng.uniform(0.5, 2.0, size=len(k)) if wl.time_varying else np.zeros(len(k))
    return FourierField(d, k, e, amp, phase, omega)


def grid_multi_index(grid: int, dim: int, flat: np.ndarray) -> np.ndarray:
    """Flat point index (x fastest) -> multi-index [P, d]."""
    flat = np.asarray(flat, dtype=np.int64)
    out = np.empty((flat.size, dim), dtype=np.int64)
    r = flat.copy()
    for a in range(dim):
        out[:, a] = r % grid
        r //= grid
    return out


def initial_state(wl: Workload, points: Optional[np.ndarray] = None, seed: Optional[int] = None) -> np.ndarray:
    """X0 = 1e-3 * packed N(0,1) noise [c][P] (identity conformation plus noise)."""
    rng = np.random.Generator(np.random.PCG64(2000 + wl.cid if seed is None else seed))
    full = rng.standard_normal((wl.c, wl.npoints)) * 1e-3
    if points is None:
        return full
    return np.ascontiguousarray(full[:, points])


def subdomain_points(wl: Workload) -> np.ndarray:
    """Flat indices of the strided parity subdomain of each workload."""
    g, d = wl.grid, wl.dim
    step = {1: 1, 2: 32, 3: 8, 4: 8, 5: 12}[wl.cid]
    ax = np.arange(0, g, step, dtype=np.int64)
    if d == 2:
        jj, ii = np.meshgrid(ax, ax, indexing="ij")
        return (jj * g + ii).ravel()
    kk, jj, ii = np.meshgrid(ax, ax, ax, indexing="ij")
    return ((kk * g + jj) * g + ii).ravel()


def random_symmetric_case(dim: int, npts: int, seed: int, kscale: float = 1.0, xscale: float = 1e-3):
    """Small unstructured case for tests: random kappa [d*d][P] and X0 [c][P]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kappa = rng.standard_normal((dim * dim, npts)) * kscale
    X0 = rng.standard_normal((ncomp(dim), npts)) * xscale
    return np.ascontiguousarray(kappa), np.ascontiguousarray(X0)
