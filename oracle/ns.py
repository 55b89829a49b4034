"""Oracle of the coupled step (test infrastructure only: tests, the smoke check and the
benchmark's CPU-baseline leg may use it; the product path never does).

What it computes: the incompressible Navier-Stokes equations of Sec. 2 (eq. Navier_Stokes)
on a periodic box,

    d/dt u + (u . grad) u + grad p - nu Laplace u = div tau,   div u = 0,   nu = beta / Re,

advanced by the projection method of Sec. 4.1 and coupled to the stress update of the same
section: once the velocity of level n+1 is known, the pointwise scheme (the pinned
pointwise oracle) advances the stress with kappa^{n+1} = grad u^{n+1}, kappa_ij = d u_i / d x_j.
One step n -> n+1 of the velocity, in the paper's order and notation
(eqs. BDF_and_extrapolation, velocity_correction, time_discretization_NS, NS_Poisson,
NS_Helmholtz), with g = 1 at the first step (no level -1) and g = 2 after:

    Xi^{n+1}  = sum_{j=1..g} (b_j/dt) u^{n+1-j} + E^{n+1}( nu curl curl u + (u.grad)u - div tau )
    Laplace p^{n+1} = -(b_0/dt) div u^{n+1} - div Xi^{n+1},   div u^{n+1} = 0,  mean(p) = 0
    (b_0/dt) u^{n+1} - nu Laplace u^{n+1}
              = -grad p^{n+1} - sum_{j=1..g} (b_j/dt) u^{n+1-j} + E^{n+1}( -(u.grad)u + div tau )

with E^{n+1} f = sum_{j=1..g} a_j f^{n+1-j}: (b_0, b_1) = (1, -1), a_1 = 1 for g = 1;
(b_0, b_1, b_2) = (3/2, -2, 1/2), (a_1, a_2) = (2, -1) for g = 2.

Space (the paper uses finite elements; on a periodic box the operators are Fourier
multipliers): the full complex DFT of numpy.fft.fftn with coefficients normalised by the
number of points, derivatives as multiplication by i xi, products on the grid.  The
explicit term -(u.grad)u + div tau and the initial velocity are restricted to the 2/3 band
(|k_j| < n_j / 3 on every axis, k_j the integer wave number), which keeps every level of
the velocity free of aliasing in the quadratic term and of the Nyquist modes.  The initial
velocity is also made divergence-free (its gradient part removed).  tau^0 = 0, the
pointwise scheme's stress at level 0.

The stress update is either the pointwise scheme without transport terms (the pinned
pointwise oracle) or, with eps given, the MFP equation of eq. FP_discrete in full, advection
by u and centre-of-mass diffusion eps Laplace included (the pinned spatial oracle,
oracle/mfp.py; with startup="exp" both run the exponential-mode scheme).  Either runs with
the velocity levels and their gradients as given levels
(no extrapolation: step n -> n+1 uses u^{n+1} and kappa^{n+1}), re-run from level 0 at every
step so that each of its steps sees exactly the levels the coupled scheme has produced by
then.  Its cost is quadratic in the number of steps: small cases only.
"""
from __future__ import annotations

import math

import numpy as np

from . import mfp as _spatial
from . import oracle as _pointwise

# packed symmetric components, the order of the pointwise path: (xx, yy, xy) and
# (xx, yy, zz, xy, xz, yz)
PAIRS = {2: ((0, 0), (1, 1), (0, 1)), 3: ((0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2))}

# (b_0 .. b_g), (a_1 .. a_g) of eq. BDF_and_extrapolation
BDF = {1: ((1.0, -1.0), (1.0,)), 2: ((1.5, -2.0, 0.5), (2.0, -1.0))}


class Box:
    """A periodic box of `shape` points and `extent` length per axis (C order)."""

    def __init__(self, shape, extent):
        self.shape = tuple(int(n) for n in shape)
        self.extent = tuple(float(L) for L in extent)
        self.d = len(self.shape)
        self.P = int(np.prod(self.shape))
        ks = [np.fft.fftfreq(n, 1.0 / n) for n in self.shape]          # integer wave numbers
        K = np.meshgrid(*ks, indexing="ij")
        self.xi = [2.0 * math.pi / L * k for k, L in zip(K, self.extent)]
        self.xi2 = sum(x * x for x in self.xi)
        self.band = np.ones(self.shape, dtype=bool)
        for k, n in zip(K, self.shape):
            self.band &= 3.0 * np.abs(k) < n
        self.axes = tuple(range(-self.d, 0))

    def fft(self, f):
        """Grid fields [..., *shape] -> coefficients normalised by the number of points."""
        return np.fft.fftn(f, axes=self.axes) / self.P

    def ifft(self, fh):
        return np.real(np.fft.ifftn(fh, axes=self.axes) * self.P)

    def grid(self, flat):
        return np.asarray(flat).reshape(flat.shape[:-1] + self.shape)

    def flat(self, g):
        return np.asarray(g).reshape(g.shape[:-self.d] + (self.P,))

    def gradient(self, uh):
        """kappa_ij = d u_i / d x_j on the grid, [d*d][*shape] with index i*d + j."""
        d = self.d
        return np.stack([self.ifft(1j * self.xi[j] * uh[i]) for i in range(d) for j in range(d)])

    def div_tensor(self, tauh_packed):
        """(div tau)_i = sum_j d tau_ij / d x_j, from packed symmetric coefficients."""
        d = self.d
        full = [[None] * d for _ in range(d)]
        for s, (i, j) in enumerate(PAIRS[d]):
            full[i][j] = full[j][i] = tauh_packed[s]
        return np.stack([sum(1j * self.xi[j] * full[i][j] for j in range(d)) for i in range(d)])

    def curl_curl(self, uh):
        """curl curl u = grad(div u) - Laplace u."""
        div = sum(1j * self.xi[j] * uh[j] for j in range(self.d))
        return np.stack([1j * self.xi[i] * div + self.xi2 * uh[i] for i in range(self.d)])

    def project(self, uh):
        """Remove the gradient part: u - xi (xi . u) / |xi|^2 (the mean kept)."""
        dot = sum(self.xi[j] * uh[j] for j in range(self.d))
        safe = np.where(self.xi2 > 0, self.xi2, 1.0)
        return np.stack([uh[i] - np.where(self.xi2 > 0, self.xi[i] * dot / safe, 0.0) for i in range(self.d)])


def explicit_term(box, uh, tau_grid):
    """F = -(u.grad)u + div tau of one level, in the 2/3 band: coefficients [d][*shape]."""
    d = box.d
    u = np.stack([box.ifft(uh[i]) for i in range(d)])
    kap = box.gradient(uh)
    adv = np.stack([sum(u[j] * kap[i * d + j] for j in range(d)) for i in range(d)])
    F = -box.fft(adv) + box.div_tensor(box.fft(tau_grid))
    return F * box.band


def velocity_step(box, nu, dt, uh_levels, F_levels, C_levels):
    """u^{n+1} from the levels u^{n+1-j}, F^{n+1-j} and C^{n+1-j} = nu curl curl u^{n+1-j}
    (newest first; their count g is the order used).  Returns (u^{n+1}, p^{n+1}) coefficients."""
    g = len(F_levels)
    b, a = BDF[g]
    hist = sum(b[j] / dt * uh_levels[j - 1] for j in range(1, g + 1))
    Xi = hist + sum(a[j - 1] * (C_levels[j - 1] - F_levels[j - 1]) for j in range(1, g + 1))
    # Laplace p = -(b0/dt) div u^{n+1} - div Xi with div u^{n+1} = 0: -|xi|^2 p = -i xi . Xi
    divXi = sum(1j * box.xi[j] * Xi[j] for j in range(box.d))
    safe = np.where(box.xi2 > 0, box.xi2, 1.0)
    ph = np.where(box.xi2 > 0, divXi / safe, 0.0)
    rhs = np.stack([-1j * box.xi[i] * ph for i in range(box.d)]) - hist + sum(
        a[j - 1] * F_levels[j - 1] for j in range(1, g + 1))
    return rhs / (b[0] / dt + nu * box.xi2), ph


def initial_velocity(box, u0_grid):
    """Divergence-free, 2/3-band part of a grid velocity [d][*shape] (coefficients)."""
    return box.project(box.fft(u0_grid)) * box.band


def run(d, shape, extent, nu, w, lam, De, eta_p, dt, nsteps, u0, X0, startup="sdirk2", want_levels=False,
        eps=None):
    """Coupled run.  u0: [d][P] grid velocity (C-order points), X0: [c][P]; eps: None for
    the pointwise stress update, else the MFP equation with advection and diffusion eps.
    Returns dict: u [d][P] and kappa [d*d][P] of level N, uh (coefficients [d][*shape]),
    p (pressure coefficients of the last step, None if N = 0), tau [c][P], X [2][c][P]
    (levels N, N-1 of the pointwise scheme), modes [2][m][c][P], div (max |div u^N|), and
    with want_levels the velocity coefficients of every level."""
    box = Box(shape, extent)
    assert box.d == d
    uh = initial_velocity(box, box.grid(np.asarray(u0, dtype=np.float64)))
    kappas = [box.flat(box.gradient(uh))]
    vels = [np.stack([box.flat(box.ifft(uh[i])) for i in range(d)])]
    tau = np.zeros((d * (d + 1) // 2, box.P))
    uh_hist, F_hist, C_hist = [uh], [], []
    levels = [uh] if want_levels else None
    res = None
    ph = None
    for n in range(nsteps):
        F_hist.insert(0, explicit_term(box, uh_hist[0], box.grid(tau)))
        C_hist.insert(0, nu * box.curl_curl(uh_hist[0]))
        g = 1 if n == 0 else 2
        uh_new, ph = velocity_step(box, nu, dt, uh_hist[:g], F_hist[:g], C_hist[:g])
        uh_hist = [uh_new] + uh_hist[:1]
        F_hist, C_hist = F_hist[:1], C_hist[:1]
        kappas.append(box.flat(box.gradient(uh_new)))
        vels.append(np.stack([box.flat(box.ifft(uh_new[i])) for i in range(d)]))
        if eps is None:
            res = _pointwise.run(d, w, lam, De, eta_p, dt, n + 1, np.stack(kappas), X0, extrap=False,
                                 startup=startup, want_modes=True)
        else:
            res = _spatial.run(d, shape, extent, eps, w, lam, De, eta_p, dt, n + 1, np.stack(kappas), X0,
                               extrap=False, want_modes=True, u=np.stack(vels),
                               scheme="exp" if startup == "exp" else "bdf2")
        tau = res["tau"]
        if want_levels:
            levels.append(uh_new)
    uh = uh_hist[0]
    u = np.stack([box.flat(box.ifft(uh[i])) for i in range(d)])
    div = sum(1j * box.xi[j] * uh[j] for j in range(d))
    out = {"u": u, "kappa": kappas[-1], "uh": uh, "p": ph, "tau": tau,
           "X": res["X"] if res else np.stack([X0, X0]), "modes": res["modes"] if res else None,
           "div": float(np.max(np.abs(box.ifft(div)))), "box": box}
    if want_levels:
        out["levels"] = levels
    return out
