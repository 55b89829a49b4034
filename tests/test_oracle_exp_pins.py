"""Pins of the oracle's exponential-mode scheme (an extension of the paper's method).

Each mode solves X_k' = -lambda_k X_k + w_k X (Sec. 2.2) exactly over a step on which X is
linear in time, and the state is integrated as X^{n+1} - X^n = A(sum_k (X_k^{n+1} - X_k^n)),
which is exact for a constant kappa because the kernel-compressed derivative equals
sum_k X_k'.  Checked against: quadrature of the step weights, Crank-Nicolson for Oldroyd-B
at alpha = 1 (to rounding), a tight ODE solve with a time-varying kappa (second order), the
Mittag-Leffler closed forms, and the paper's BDF2 scheme at equal step size."""
import math

import numpy as np
import pytest
from scipy.integrate import quad, solve_ivp

from oracle import oracle as O
from oracle import soe
from paper_2411_17294_amd import inputs as I
from tests.mlf import mittag_leffler
from tests.test_oracle_pins import _kappa_t, one_point, packed_operator

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


@pytest.mark.parametrize("z", [0.0, 1e-9, 1e-4, 0.05, 0.5, 0.99, 1.0, 1.7, 12.0, 300.0])
def test_exp_weights_match_quadrature(z):
    """e = exp(-z), a0 = int_0^1 e^{-z(1-u)} (1-u) du, a1 = int_0^1 e^{-z(1-u)} u du."""
    e, a0, a1 = O.exp_weights(z)
    q0 = quad(lambda u: math.exp(-z * (1 - u)) * (1 - u), 0, 1, epsabs=0, epsrel=1e-13, limit=200)[0]
    q1 = quad(lambda u: math.exp(-z * (1 - u)) * u, 0, 1, epsabs=0, epsrel=1e-13, limit=200)[0]
    assert e == pytest.approx(math.exp(-z), rel=1e-15, abs=1e-300)
    assert a0 == pytest.approx(q0, rel=1e-13)
    assert a1 == pytest.approx(q1, rel=1e-13)


@pytest.mark.parametrize("d", [2, 3])
def test_exp_alpha_one_is_crank_nicolson_oldroyd_b(d):
    """alpha = 1 (w = 1, lambda = 0): the mode is the running integral of X, its step update
    the trapezoid rule, so the scheme is Crank-Nicolson for Oldroyd-B:
    (I - dt/2 L) X^{n+1} = (I + dt/2 L) X^n + dt S."""
    rng = np.random.default_rng(40 + d)
    k = rng.standard_normal((d, d)) * 0.8
    De, eta_p, dt, N = 0.8, 0.1, 2e-3, 150
    c = I.ncomp(d)
    X0 = rng.standard_normal(c) * 1e-2
    L, S = packed_operator(d, k, De)
    x = X0.copy()
    for _ in range(N):
        x = np.linalg.solve(np.eye(c) - 0.5 * dt * L, (np.eye(c) + 0.5 * dt * L) @ x + dt * S)
    r = O.run(d, [1.0], [0.0], De, eta_p, dt, N, one_point(k), X0.reshape(-1, 1), startup="exp")
    assert np.max(np.abs(r["X"][0][:, 0] - x)) < 1e-13 * max(1, np.max(np.abs(x)))
    assert np.max(np.abs(r["tau"][:, 0] - eta_p / De * x)) < 1e-13


@pytest.mark.parametrize("extrap", [True, False])
def test_exp_time_varying_kappa_half_step(extrap):
    """alpha = 1 with a time-varying kappa: Crank-Nicolson with kappa~ = 3/2 kappa^n - 1/2
    kappa^{n-1} (kappa^0 at the first step) matches to rounding and converges at second
    order to a tight ODE solve; without extrapolation kappa~ = kappa^{n+1} (first order)."""
    d, De, T = 2, 0.6, 0.4
    X0 = np.array([0.01, -0.02, 0.005])

    def textbook(dt, N):
        ks = [_kappa_t(n * dt) for n in range(N + 1)]
        kt = (lambda n: 1.5 * ks[n] - 0.5 * ks[n - 1] if n >= 1 else ks[0]) if extrap else (lambda n: ks[n + 1])
        x = X0.copy()
        for n in range(N):
            L, S = packed_operator(d, kt(n), De)
            x = np.linalg.solve(np.eye(3) - 0.5 * dt * L, (np.eye(3) + 0.5 * dt * L) @ x + dt * S)
        return x, np.stack([k.reshape(4, 1) for k in ks])

    def rhs(t, x):
        L, S = packed_operator(d, _kappa_t(t), De)
        return L @ x + S
    ref = solve_ivp(rhs, (0, T), X0, rtol=1e-13, atol=1e-15, method="DOP853").y[:, -1]
    errs = []
    for dt in (1e-2, 5e-3, 2.5e-3):
        N = int(round(T / dt))
        xt, kap = textbook(dt, N)
        r = O.run(d, [1.0], [0.0], De, 0.1, dt, N, kap, X0.reshape(-1, 1), extrap=extrap, startup="exp")
        assert np.max(np.abs(r["X"][0][:, 0] - xt)) < 1e-14
        errs.append(np.max(np.abs(r["X"][0][:, 0] - ref)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    lo, hi = (1.7, 2.4) if extrap else (0.8, 1.3)
    assert all(lo < o < hi for o in orders), (errs, orders)


def _relaxation_errors(scheme, dts, alpha=0.5, De=0.5, T=1.0):
    """kappa = 0: X(t) = X0 E_alpha(-t^alpha/De).  Returns the weighted-norm errors
    (||u||^2 = int_0^T ||u||^2 t^{2(1-alpha)} dt, the paper's norm of Fig. 2a) and the
    errors at t = T."""
    X0 = np.array([[0.3], [-0.2], [0.1]])
    norms, ends = [], []
    for dt in dts:
        N = int(round(T / dt))
        w, lam, _ = soe.soe_fit(alpha, 60, dt, T)
        ts = np.arange(1, N + 1) * dt
        ml = np.array([mittag_leffler(alpha, -(t ** alpha) / De) for t in ts])
        Xs = O.run(2, w, lam, De, 0.1, dt, N, np.zeros((4, 1)), X0, want_traj=True, startup=scheme)["traj"][1:, :, 0]
        err = Xs - ml[:, None] * X0[:, 0][None, :]
        norms.append(math.sqrt(np.sum(dt * np.sum(err ** 2, axis=1) * ts ** (2 * (1 - alpha)))))
        ends.append(float(np.max(np.abs(err[-1]))))
    return norms, ends


def test_exp_relaxation_order_and_accuracy_against_bdf2():
    """Both schemes converge like dt^{1+alpha} in the weighted norm (alpha = 0.5).  At equal
    dt the exponential scheme's weighted error is below the paper's BDF2 scheme's (it
    integrates the t^{alpha-1} start of the memory exactly over each step); its error at
    t = T is larger but of the same order.  Both sets of numbers are printed."""
    dts = (1 / 50, 1 / 100, 1 / 200, 1 / 400)
    nb, eb = _relaxation_errors("sdirk2", dts)
    ne, ee = _relaxation_errors("exp", dts)
    ob = [math.log2(nb[i] / nb[i + 1]) for i in range(3)]
    oe = [math.log2(ne[i] / ne[i + 1]) for i in range(3)]
    print("weighted  BDF2", [f"{x:.3e}" for x in nb], ob, " EXP", [f"{x:.3e}" for x in ne], oe)
    print("at t = T  BDF2", [f"{x:.2e}" for x in eb], " EXP", [f"{x:.2e}" for x in ee])
    assert all(1.3 < o < 1.8 for o in oe), oe
    assert all(x < y for x, y in zip(ne, nb)), (ne, nb)
    assert all(x < 10 * y for x, y in zip(ee, eb)), (ee, eb)


def test_exp_general_kappa_closed_form():
    """Constant non-normal kappa (2-D): X(t) = E_alpha(L t^alpha)(X0 + L^{-1} S) - L^{-1} S."""
    alpha, De, T = 0.6, 0.8, 0.3
    k = np.array([[0.2, 0.9], [-0.4, -0.2]])
    X0 = np.array([0.01, -0.01, 0.02])
    L, S = packed_operator(2, k, De)
    lam_, V = np.linalg.eig(L)
    Ea = (V @ np.diag([mittag_leffler(alpha, complex(l * T ** alpha)) for l in lam_]) @ np.linalg.inv(V)).real
    Ls = np.linalg.solve(L, S)
    ex = Ea @ (X0 + Ls) - Ls
    errs = []
    for dt in (1e-3, 5e-4):
        w, lam, _ = soe.soe_fit(alpha, 60, dt, T)
        r = O.run(2, w, lam, De, 0.1, dt, int(round(T / dt)), one_point(k), X0.reshape(-1, 1), startup="exp")
        errs.append(np.max(np.abs(r["X"][0][:, 0] - ex)))
    assert errs[-1] < 2e-5 * np.max(np.abs(ex)) and errs[1] < errs[0], errs


@pytest.mark.parametrize("d", [2, 3])
def test_exp_extensional_flow_closed_form(d):
    """Constant diagonal kappa: X_ll = (X_ll^0 + 2k_ll/mu_l) E_alpha(mu_l t^alpha) - 2k_ll/mu_l,
    mu_l = 2k_ll - 1/De;  X_lm = X_lm^0 E_alpha((k_ll + k_mm - 1/De) t^alpha)."""
    alpha, De, T = 0.5, 1.0, 0.5
    kd = np.array([0.3, -0.1, -0.2])[:d]
    kd = kd - kd.mean()
    X0 = np.array([0.01, -0.02, 0.015, 0.005, -0.01, 0.02])[:I.ncomp(d)]
    ex = []
    for (i, j) in I.packed_pairs(d):
        if i == j:
            mu = 2 * kd[i] - 1 / De
            ex.append((X0[len(ex)] + 2 * kd[i] / mu) * mittag_leffler(alpha, mu * T ** alpha) - 2 * kd[i] / mu)
        else:
            ex.append(X0[len(ex)] * mittag_leffler(alpha, (kd[i] + kd[j] - 1 / De) * T ** alpha))
    ex = np.array(ex)
    w, lam, _ = soe.soe_fit(alpha, 60, 5e-4, T)
    r = O.run(d, w, lam, De, 0.1, 5e-4, 1000, one_point(np.diag(kd)), X0.reshape(-1, 1), startup="exp")
    assert np.max(np.abs(r["X"][0][:, 0] - ex)) < 2e-5 * max(1.0, np.max(np.abs(ex)))


def test_exp_complex_step_matches_real_run():
    """The complex build of the exponential scheme: zero imaginary input reproduces the real
    run, and the imaginary part of a kappa perturbation matches central differences."""
    d, P, N = 3, 4, 12
    kappa, X0 = I.random_symmetric_case(d, P, 3, kscale=0.6, xscale=1e-2)
    w, lam, _ = soe.soe_fit(0.4, 8, 1e-3, N * 1e-3)
    r = O.run(d, w, lam, 1.0, 0.1, 1e-3, N, kappa, X0, startup="exp")
    rc = O.run_complex(d, w, lam, 1.0, 0.1, 1e-3, N, kappa, X0, startup="exp")
    assert np.max(np.abs(rc["tau"].real - r["tau"])) < 1e-15 * np.max(np.abs(r["tau"])) + 1e-300
    dk = np.zeros_like(kappa); dk[1] = 1.0
    h = 1e-6
    cs = O.run_complex(d, w, lam, 1.0, 0.1, 1e-3, N, kappa + 1e-30j * dk, X0, startup="exp")["tau"].imag / 1e-30
    fd = (O.run(d, w, lam, 1.0, 0.1, 1e-3, N, kappa + h * dk, X0, startup="exp")["tau"]
          - O.run(d, w, lam, 1.0, 0.1, 1e-3, N, kappa - h * dk, X0, startup="exp")["tau"]) / (2 * h)
    assert np.max(np.abs(cs - fd)) < 1e-6 * np.max(np.abs(cs))
