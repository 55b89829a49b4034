"""Pins of the spatial oracle (oracle/mfp.py): the MFP equation with centre-of-mass
diffusion on a periodic grid (Sec. 4.1 eq. FP_discrete with u = 0).

Each pin ties the oracle to something other than itself:
  * the spectral Laplacian against derivatives of trigonometric polynomials in closed form,
    the Nyquist mode included;
  * eps = 0 against the pinned pointwise oracle (two implementations of the scheme);
  * one Fourier mode with kappa != 0 against the pointwise oracle through the identity
    "eps Laplace acts on exp(i xi.x) like an extra relaxation rate eps |xi|^2", with the
    mean and the mass-mode source carried by a separate pointwise run;
  * the paper's own convergence experiment (Sec. 5.1): the Mittag-Leffler solution
    cos(2 pi x1) cos(4 pi x2) E_alpha(-(r + 20 eps pi^2) t^alpha) on the unit square,
    eps = 1e-2, De = 0.5, T = 1, alpha = 0.5, with an error decaying like dt^{1+alpha} in
    the weighted norm of eq. weighted_Bochner_space_norm (Fig. 2a).  r = 1/De under the
    tested operator (the paper prints 1/(2De) with its block matrix).
The first three (and the uniform-advection pin) run for both time schemes: the paper's
BDF2 and the exponential-mode extension, each against the pointwise oracle's own run of
that scheme."""
import math

import numpy as np
import pytest

from oracle import mfp
from oracle import oracle as O
from oracle import soe
from tests.mlf import mittag_leffler


STARTUP = {"bdf2": "sdirk2", "exp": "exp"}     # the pointwise oracle's name of each scheme


def grid_points(shape, extent):
    axes = [np.arange(n) * (L / n) for n, L in zip(shape, extent)]
    return [g.reshape(-1) for g in np.meshgrid(*axes, indexing="ij")]


@pytest.mark.parametrize("shape,extent", [((6, 8), (1.0, 2.0)), ((4, 6, 8), (1.0, 2.0 * math.pi, 3.0))])
def test_spectral_laplacian_of_trigonometric_polynomials(shape, extent):
    """Laplace of sin(2 pi a x/Lx) cos(2 pi b y/Ly) ... is -(sum (2 pi k_j / L_j)^2) times it,
    for modes up to the Nyquist mode of each axis (where only the cosine survives)."""
    lap = mfp.laplacian_matrix(shape, extent)
    xs = grid_points(shape, extent)
    d = len(shape)
    rng = np.random.default_rng(3)
    for trial in range(6):
        ks = [int(rng.integers(0, n // 2 + 1)) for n in shape]
        f = np.ones_like(xs[0])
        rate = 0.0
        for j in range(d):
            arg = 2 * math.pi * ks[j] * xs[j] / extent[j]
            # sine is zero on the grid at the Nyquist mode; use the cosine there
            f = f * (np.cos(arg) if (trial + j) % 2 == 0 or 2 * ks[j] == shape[j] else np.sin(arg))
            rate += (2 * math.pi * ks[j] / extent[j]) ** 2
        np.testing.assert_allclose(lap @ f, -rate * f, rtol=0, atol=1e-10 * max(1.0, rate))
    # constants are annihilated
    assert np.max(np.abs(lap @ np.ones(lap.shape[0]))) < 1e-12


@pytest.mark.parametrize("scheme", ["bdf2", "exp"])
@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("levels", [False, True])
def test_eps_zero_is_the_pointwise_oracle(d, levels, scheme):
    """Without diffusion the grid points decouple: every output equals the pointwise
    oracle's, for kappa varying in space (and in time), with either time scheme."""
    shape = (3, 4) if d == 2 else (2, 2, 3)
    P = int(np.prod(shape))
    c = d * (d + 1) // 2
    rng = np.random.default_rng(7 + d)
    N = 9
    kap = rng.standard_normal((N + 1, d * d, P)) * 0.3 if levels else rng.standard_normal((d * d, P)) * 0.3
    X0 = rng.standard_normal((c, P)) * 0.05
    w, lam, _ = soe.soe_fit(0.5, 6, 2e-3, 2e-3 * N)
    r = mfp.run(d, shape, (1.0,) * d, 0.0, w, lam, 1.2, 0.1, 2e-3, N, kap, X0, want_modes=True, scheme=scheme)
    o = O.run(d, w, lam, 1.2, 0.1, 2e-3, N, kap, X0, want_modes=True, startup=STARTUP[scheme])
    for k in ("X", "tau", "modes"):
        err = np.max(np.abs(r[k] - o[k])) / np.max(np.abs(o[k]))
        assert err < 1e-13, (k, err)


@pytest.mark.parametrize("scheme", ["bdf2", "exp"])
@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("N", [1, 2, 12])
def test_one_fourier_mode_is_a_shifted_relaxation_rate(d, N, scheme):
    """X0 = F + E cos(xi.x), kappa constant: the mean follows the pointwise scheme from F
    (with the mass-mode source), and the cos(xi.x) part follows the source-free pointwise
    scheme from E with 1/De replaced by 1/De + eps |xi|^2 (a pointwise run from E minus one
    from 0), at the same eta_p/De."""
    shape, extent = ((6, 8), (1.0, 2.0)) if d == 2 else ((4, 4, 6), (1.0, 2.0, 3.0))
    ks = (1, 3) if d == 2 else (1, 2, 2)
    P = int(np.prod(shape))
    c = d * (d + 1) // 2
    xs = grid_points(shape, extent)
    phase = sum(2 * math.pi * ks[j] * xs[j] / extent[j] for j in range(d))
    xi2 = sum((2 * math.pi * ks[j] / extent[j]) ** 2 for j in range(d))
    rng = np.random.default_rng(11 + d)
    kd = rng.standard_normal((d, d)) * 0.4
    kd -= np.trace(kd) / d * np.eye(d)
    kap = np.repeat(kd.reshape(d * d, 1), P, axis=1)
    E = rng.standard_normal(c) * 0.05
    F = rng.standard_normal(c) * 0.05
    X0 = F[:, None] + E[:, None] * np.cos(phase)[None, :]
    De, eta_p, eps, dt = 0.8, 0.1, 0.02, 2e-3
    w, lam, _ = soe.soe_fit(0.6, 8, dt, dt * max(N, 2))
    r = mfp.run(d, shape, extent, eps, w, lam, De, eta_p, dt, N, kap, X0, want_modes=True, scheme=scheme)
    one = kd.reshape(d * d, 1)
    De_x = 1.0 / (1.0 / De + eps * xi2)
    st = STARTUP[scheme]
    mean = O.run(d, w, lam, De, eta_p, dt, N, one, F[:, None], want_modes=True, startup=st)
    withE = O.run(d, w, lam, De_x, eta_p * De_x / De, dt, N, one, E[:, None], want_modes=True, startup=st)
    zero = O.run(d, w, lam, De_x, eta_p * De_x / De, dt, N, one, np.zeros((c, 1)), want_modes=True, startup=st)
    for k in ("X", "tau", "modes"):
        pred = mean[k] + (withE[k] - zero[k]) * np.cos(phase)
        err = np.max(np.abs(r[k] - pred)) / np.max(np.abs(pred))
        assert err < 1e-12, (k, err)


def test_paper_convergence_experiment_sec_5_1():
    """Unit square, cos(2 pi x1) cos(4 pi x2) in every Hermite component, kappa = 0,
    eps = 1e-2, De = 0.5, T = 1, alpha = 0.5, m = 60 modes: the error against the
    Mittag-Leffler solution, in the weighted norm int_0^1 ||u||_L2^2 t^{2(1-alpha)} dt,
    decays like dt^{1.5}.  The grid (8 x 8) resolves the mode exactly, so the error is the
    time discretisation's."""
    d, shape, extent = 2, (8, 8), (1.0, 1.0)
    alpha, De, eps, T = 0.5, 0.5, 1e-2, 1.0
    x1, x2 = grid_points(shape, extent)
    prof = np.cos(2 * math.pi * x1) * np.cos(4 * math.pi * x2)
    # every Hermite component of degree 2 equal to the profile: X_ll = sqrt(2) Phi_2el, X_lm = Phi
    X0 = np.stack([math.sqrt(2) * prof, math.sqrt(2) * prof, prof])
    rate = 1.0 / De + 20 * eps * math.pi ** 2
    P = prof.size
    norms = []
    for dt in (1 / 50, 1 / 100, 1 / 200, 1 / 400):
        N = int(round(T / dt))
        w, lam, _ = soe.soe_fit(alpha, 60, dt, T)
        traj = mfp.run(d, shape, extent, eps, w, lam, De, 0.1, dt, N, np.zeros((4, P)), X0, want_traj=True)["traj"]
        ts = np.arange(1, N + 1) * dt
        ml = np.array([mittag_leffler(alpha, -rate * t ** alpha) for t in ts])
        err = traj[1:] - ml[:, None, None] * X0[None]
        l2 = np.mean(np.sum(err ** 2, axis=1), axis=1)       # ||.||_L2^2 over the unit square
        norms.append(math.sqrt(np.sum(dt * l2 * ts ** (2 * (1 - alpha)))))
    orders = [math.log2(norms[i] / norms[i + 1]) for i in range(len(norms) - 1)]
    assert all(1.3 < o < 1.7 for o in orders), (norms, orders)


@pytest.mark.parametrize("shape,extent", [((6, 8), (1.0, 2.0)), ((4, 6, 8), (1.0, 2.0 * math.pi, 3.0))])
def test_spectral_derivatives_of_trigonometric_polynomials(shape, extent):
    """d/dx_j of sin(2 pi k.x/L) and cos(...) below the Nyquist mode in closed form; the
    Nyquist cosine (the only Nyquist mode a real grid field carries) has derivative zero."""
    d = len(shape)
    xs = grid_points(shape, extent)
    rng = np.random.default_rng(21)
    for axis in range(d):
        Dm = mfp.derivative_matrix(shape, extent, axis)
        for trial in range(4):
            ks = [int(rng.integers(-(n // 2 - 1), n // 2)) for n in shape]
            arg = sum(2 * math.pi * ks[j] * xs[j] / extent[j] for j in range(d))
            dk = 2 * math.pi * ks[axis] / extent[axis]
            np.testing.assert_allclose(Dm @ np.sin(arg), dk * np.cos(arg), rtol=0, atol=1e-10 * max(1.0, abs(dk)))
            np.testing.assert_allclose(Dm @ np.cos(arg), -dk * np.sin(arg), rtol=0, atol=1e-10 * max(1.0, abs(dk)))
        nyq = np.cos(math.pi * shape[axis] * xs[axis] / extent[axis])
        assert np.max(np.abs(Dm @ nyq)) < 1e-10


@pytest.mark.parametrize("scheme", ["bdf2", "exp"])
@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("N", [1, 2, 12])
def test_uniform_advection_of_one_fourier_mode_is_a_complex_rate(d, N, scheme):
    """u uniform, kappa constant, X0 = F + E cos(xi.x): the mean follows the pointwise scheme
    from F, and since u.grad acts on exp(i xi.x) as i xi.u, the cos(xi.x) part is the real
    part of exp(i xi.x) times the source-free pointwise scheme from E with the complex rate
    1/De + eps |xi|^2 + i xi.u in place of 1/De (complex runs of the pointwise oracle, from E
    minus from 0), at the same eta_p/De."""
    shape, extent = ((6, 8), (1.0, 2.0)) if d == 2 else ((4, 4, 6), (1.0, 2.0, 3.0))
    ks = (1, 3) if d == 2 else (1, -1, 2)
    P = int(np.prod(shape))
    c = d * (d + 1) // 2
    xs = grid_points(shape, extent)
    xi = [2 * math.pi * ks[j] / extent[j] for j in range(d)]
    phase = sum(xi[j] * xs[j] for j in range(d))
    rng = np.random.default_rng(31 + d)
    kd = rng.standard_normal((d, d)) * 0.4
    u0 = rng.standard_normal(d) * 0.7
    E = rng.standard_normal(c) * 0.05
    F = rng.standard_normal(c) * 0.05
    X0 = F[:, None] + E[:, None] * np.cos(phase)[None, :]
    De, eta_p, eps, dt = 0.8, 0.1, 0.02, 2e-3
    w, lam, _ = soe.soe_fit(0.6, 8, dt, dt * max(N, 2))
    kap = np.repeat(kd.reshape(d * d, 1), P, axis=1)
    u = np.repeat(u0.reshape(d, 1), P, axis=1)
    r = mfp.run(d, shape, extent, eps, w, lam, De, eta_p, dt, N, kap, X0, want_modes=True, u=u, scheme=scheme)
    one = kd.reshape(d * d, 1)
    rate = 1.0 / De + eps * sum(x * x for x in xi) + 1j * sum(xi[j] * u0[j] for j in range(d))
    De_x = 1.0 / rate
    st = STARTUP[scheme]
    mean = O.run(d, w, lam, De, eta_p, dt, N, one, F[:, None], want_modes=True, startup=st)
    zE = O.run_complex(d, w, lam, De_x, eta_p * De_x / De, dt, N, one.astype(complex), E[:, None].astype(complex),
                       want_modes=True, startup=st)
    z0 = O.run_complex(d, w, lam, De_x, eta_p * De_x / De, dt, N, one.astype(complex), np.zeros((c, 1), complex),
                       want_modes=True, startup=st)
    wave = np.exp(1j * phase)
    for k in ("X", "tau", "modes"):
        pred = mean[k] + np.real((zE[k] - z0[k]) * wave)
        err = np.max(np.abs(r[k] - pred)) / np.max(np.abs(pred))
        assert err < 1e-12, (k, err)
