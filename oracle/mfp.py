"""Oracle of the spatial form (test infrastructure only: tests, the smoke check and the
benchmark's CPU-baseline leg may use it; the product path never does).

What it computes: the macroscopic Fokker-Planck (MFP) equation of Sec. 4.1 with
centre-of-mass diffusion and, optionally, advection by a given velocity field u(x, t), on a
periodic grid,

    d/dt Phi + L( sum_k (w_k Phi - lam_k Phi_k) ) = 0,   L = u.grad - eps Laplace - A(kappa),
    d/dt Phi_k = -lam_k Phi_k + w_k Phi                  (Sec. 2.2, kernel compression),

in the paper's own variables: at every grid point the vector Phi of Hermite coefficients
of degrees 0 and 2 (mass mode included), with the coupling matrix A(kappa) of the tested
operator taken from the pinned pointwise oracle.  The time scheme is the paper's:

  * first step: Alexander's two-stage SDIRK2 on the augmented linear system (Sec. 5.1
    asks for an SDIRK2 start);
  * then BDF2, eq. FP_discrete:
        (b0 + eta L) Phi^{n+1} = -sum_{j=1,2} b_j (Phi^{n+1-j} + sum_k eta_k L Phi_k^{n+1-j}),
    and the mode push-forward, eq. BDF_Phi_k_n+1.

With scheme="exp" it runs instead the exponential-mode scheme of the pointwise oracle (an
extension, not the paper's scheme) with L in place of -A(kappa): each mode integrates
Phi_k' = -lam_k Phi_k + w_k Phi exactly with Phi linear over the step,
    Phi_k^{n+1} = e_k Phi_k^n + w_k dt (a0_k Phi^n + a1_k Phi^{n+1}),
and since the compressed derivative is sum_k Phi_k', the state takes the increment form
    Phi^{n+1} - Phi^n = -L sum_k (Phi_k^{n+1} - Phi_k^n),
one step from n = 0 with zero modes (no start-up), kappa and u taken at the half step
(3/2 level n - 1/2 level n-1).

Everything is assembled in physical space as dense matrices over (grid point, Hermite
component) and solved directly (numpy.linalg.solve), so only small grids are meant.  The
Laplacian is the spectral one on the periodic grid: its symbol is -|xi|^2 on the discrete
Fourier modes (numpy.fft), the Nyquist mode included.  The advection u.grad acts on every
Hermite coefficient: at each point u_j(x) times the spectral derivative d/dx_j, whose
symbol is i xi_j with the Nyquist wave number taken as zero (an odd derivative of a real
grid field has no Nyquist component).  kappa and u may vary in space and time; both use the
level rule of eq. BDF_and_extrapolation (kappa~ = 2 kappa^n - kappa^{n-1}, likewise u~) or,
without extrapolation, the level n+1.

The stress is tau = (eta_p / De) D^{1-alpha}(C - I) with D^{1-alpha} Phi taken from the
modes of the new level (eq. fractional_modes_fractional_derivative), summed with Neumaier
compensation over k.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as _pointwise

B0, B1, B2 = 1.5, -2.0, 0.5
GS = 1.0 - 1.0 / math.sqrt(2.0)      # SDIRK2 diagonal (Alexander)


def wavenumber_squared(shape, extent):
    """|xi|^2 on the grid of discrete Fourier modes of a periodic box (numpy's fftn order)."""
    axes = [2.0 * math.pi * np.fft.fftfreq(n, d=L / n) for n, L in zip(shape, extent)]
    grids = np.meshgrid(*axes, indexing="ij")
    return sum(g * g for g in grids)


def laplacian_matrix(shape, extent):
    """Dense matrix of the spectral Laplacian on the flattened grid (C order)."""
    P = int(np.prod(shape))
    k2 = wavenumber_squared(shape, extent)
    lap = np.empty((P, P))
    for j in range(P):
        e = np.zeros(P)
        e[j] = 1.0
        col = np.fft.ifftn(-k2 * np.fft.fftn(e.reshape(shape)))
        lap[:, j] = col.real.reshape(P)
    return lap


def derivative_matrix(shape, extent, axis):
    """Dense matrix of the spectral first derivative along `axis` on the flattened grid."""
    P = int(np.prod(shape))
    n, L = shape[axis], extent[axis]
    k = 2.0 * math.pi * np.fft.fftfreq(n, d=L / n)
    if n % 2 == 0:
        k[n // 2] = 0.0
    sym = k.reshape([n if j == axis else 1 for j in range(len(shape))])
    D = np.empty((P, P))
    for j in range(P):
        e = np.zeros(P)
        e[j] = 1.0
        col = np.fft.ifftn(1j * sym * np.fft.fftn(e.reshape(shape)))
        D[:, j] = col.real.reshape(P)
    return D


def hermite_map(d):
    """B with Phi = B [1, X_packed] (mass mode one), from the pointwise oracle's map."""
    c = d * (d + 1) // 2
    n = c + 1
    B = np.empty((n, n))
    h0 = _pointwise.tensor_to_hermite(d, np.zeros(c))
    B[:, 0] = h0
    for j in range(c):
        e = np.zeros(c)
        e[j] = 1.0
        B[:, 1 + j] = _pointwise.tensor_to_hermite(d, e) - h0
    return B


def _kappa_at(kappa, d, P, lev):
    """kappa of level lev as [P][d][d] (steady [d*d][P] or levels [nlev][d*d][P])."""
    k = kappa if kappa.ndim == 2 else kappa[lev]
    return np.asarray(k, dtype=np.float64).reshape(d, d, P).transpose(2, 0, 1)


def _u_at(u, d, P, lev):
    """u of level lev as [d][P] (steady [d][P] or levels [nlev][d][P])."""
    uu = np.asarray(u, dtype=np.float64)
    return uu if uu.ndim == 2 else uu[lev]


def _operator(d, De, eps, lap, kap_pts, adv=None):
    """Dense A(kappa) + eps Laplace - u.grad over [point][component] (= -L); adv is the
    dense u.grad of one scalar field (or None)."""
    P = kap_pts.shape[0]
    n = d * (d + 1) // 2 + 1
    A = eps * np.kron(lap, np.eye(n))
    if adv is not None:
        A -= np.kron(adv, np.eye(n))
    for p in range(P):
        A[p * n:(p + 1) * n, p * n:(p + 1) * n] += _pointwise.coupling_matrix(d, De, kap_pts[p])
    return A


def _neumaier(terms):
    """Compensated sum over the first axis."""
    s = np.zeros_like(terms[0])
    comp = np.zeros_like(terms[0])
    for t in terms:
        u = s + t
        big = np.abs(s) >= np.abs(t)
        comp += np.where(big, (s - u) + t, (t - u) + s)
        s = u
    return s + comp


def run(d, shape, extent, eps, w, lam, De, eta_p, dt, nsteps, kappa, X0, extrap=True,
        want_modes=False, want_traj=False, u=None, scheme="bdf2"):
    """Run the spatial oracle.

    shape, extent: grid points and box length per axis (len d); points in C order.
    kappa: [d*d][P] (steady) or [nlev][d*d][P], nlev >= nsteps + 1; X0: [c][P] (packed,
    X = C - I); u: None (no advection), [d][P] (steady) or [nlev][d][P]; scheme: "bdf2"
    (SDIRK2 start, then BDF2) or "exp".  Returns X [2][c][P] (levels N, N-1), tau [c][P],
    modes [2][m][c][P] (plain, levels N and N-1) or None, traj [N+1][c][P] or None."""
    assert scheme in ("bdf2", "exp")
    w = np.asarray(w, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    m = w.size
    c = d * (d + 1) // 2
    n = c + 1
    P = int(np.prod(shape))
    X0 = np.asarray(X0, dtype=np.float64)
    kappa = np.asarray(kappa, dtype=np.float64)
    assert X0.shape == (c, P) and len(shape) == d
    lap = laplacian_matrix(shape, extent)
    Dm = [derivative_matrix(shape, extent, j) for j in range(d)] if u is not None else None
    B = hermite_map(d)
    Binv = np.linalg.inv(B)
    gamma = eta_p / De

    def to_phi(X):                       # [c][P] -> [P*n]
        ones = np.ones((1, X.shape[1]))
        return (B @ np.vstack([ones, X])).T.reshape(P * n)

    def to_x(Phi):                       # [P*n] -> [c][P]
        return (Binv @ Phi.reshape(P, n).T)[1:]

    phi = [to_phi(X0), None]             # levels n, n-1
    modes = [np.zeros((m, P * n)), np.zeros((m, P * n))]
    traj = [X0.copy()] if want_traj else None
    eta = sum(B0 * w[k] * dt / (B0 + lam[k] * dt) for k in range(m))
    etak = lam * dt / (B0 + lam * dt)

    I = np.eye(P * n)
    # extrapolation to t_{n+1} (BDF2) or to the half step (exponential scheme)
    fa, fb = (2.0, -1.0) if scheme == "bdf2" else (1.5, -0.5)
    if scheme == "exp":
        ew = np.array([_pointwise.exp_weights(lam[k] * dt) for k in range(m)])     # (e, a0, a1) per mode
        q_exp = float(np.sum(w * dt * ew[:, 2]))
    kt_prev, ut_prev, A = None, None, None
    for step in range(nsteps):
        ut = None
        if extrap:
            ka = _kappa_at(kappa, d, P, step)
            kt = ka if step == 0 else fa * ka + fb * _kappa_at(kappa, d, P, step - 1)
            if u is not None:
                ua = _u_at(u, d, P, step)
                ut = ua if step == 0 else fa * ua + fb * _u_at(u, d, P, step - 1)
        else:
            kt = _kappa_at(kappa, d, P, step + 1)
            if u is not None:
                ut = _u_at(u, d, P, step + 1)
        same_u = (ut is None and ut_prev is None) or (
            ut is not None and ut_prev is not None and np.array_equal(ut, ut_prev))
        if kt_prev is None or not np.array_equal(kt, kt_prev) or not same_u:
            adv = None if ut is None else sum(ut[j][:, None] * Dm[j] for j in range(d))
            A = _operator(d, De, eps, lap, kt, adv)
            kt_prev, ut_prev = kt, ut
        if scheme == "exp":
            # (I - q A) Phi^{n+1} = Phi^n + A sum_k ((e_k - 1) Phi_k^n + w_k dt a0_k Phi^n)
            v = np.sum((ew[:, 0] - 1.0)[:, None] * modes[0] + (w * dt * ew[:, 1])[:, None] * phi[0][None, :],
                       axis=0)
            new_phi = np.linalg.solve(I - q_exp * A, phi[0] + A @ v)
            new_modes = ew[:, 0][:, None] * modes[0] + (w * dt)[:, None] * (
                ew[:, 1][:, None] * phi[0][None, :] + ew[:, 2][:, None] * new_phi[None, :])
        elif step == 0:
            hg = dt * GS
            theta = np.sum(w / (1.0 + hg * lam))
            M = I - hg * theta * A
            E, Ek = phi[0], np.zeros((m, P * n))
            F1 = Fk = None
            for stage in range(2):
                if stage == 1:
                    E = phi[0] + dt * (1.0 - GS) * F1
                    Ek = modes[0] + dt * (1.0 - GS) * Fk
                v = np.sum((lam / (1.0 + hg * lam))[:, None] * Ek, axis=0)
                Y = np.linalg.solve(M, E - hg * (A @ v))
                Yk = (Ek + hg * w[:, None] * Y[None, :]) / (1.0 + hg * lam)[:, None]
                if stage == 0:
                    Fk = w[:, None] * Y[None, :] - lam[:, None] * Yk
                    F1 = A @ np.sum(Fk, axis=0)
            new_phi, new_modes = Y, Yk
        else:
            hist = np.sum(etak[:, None] * (B1 * modes[0] + B2 * modes[1]), axis=0)
            rhs = -(B1 * phi[0] + B2 * phi[1]) + A @ hist
            new_phi = np.linalg.solve(B0 * I - eta * A, rhs)
            new_modes = (-(B1 * modes[0] + B2 * modes[1]) + (w * dt)[:, None] * new_phi[None, :]) / \
                (B0 + lam * dt)[:, None]
        phi = [new_phi, phi[0]]
        modes = [new_modes, modes[0]]
        if want_traj:
            traj.append(to_x(new_phi))

    D = _neumaier([w[k] * phi[0] - lam[k] * modes[0][k] for k in range(m)])
    out = {"X": np.stack([to_x(phi[0]), to_x(phi[1]) if phi[1] is not None else X0]),
           "tau": gamma * to_x(D), "modes": None, "traj": np.stack(traj) if want_traj else None}
    if want_modes:
        out["modes"] = np.stack([np.stack([to_x(modes[lv][k]) for k in range(m)]) for lv in range(2)])
    return out
