"""Pins of the oracle's extended-precision build (orcl_*, x87 long double).

The full-size FP64 parity tests use this build as the reference for the rounding error
of FP64 evaluations of the scheme.  Here it is checked against the same discrete scheme
integrated in 30-digit arithmetic (mpmath) on the augmented linear system of the state
X, its fractional modes X_k and the mass modes mu_k: Alexander's SDIRK2 for the first step,
then BDF2 (Sec. 4.1, eqs. BDF_Phi_k_n+1 and FP_discrete: with kappa steady the scheme is
BDF2 on that system), and tau = gamma sum_k (w_k X - lam_k X_k).  The extended build must
agree far below FP64 rounding, and the FP64 build within its own rounding.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2411_17294_amd import inputs as I


def _packed_operator_mp(mp, d, k, De):
    """Matrix of X -> kappa X + X kappa^T - X/De on packed symmetric X, and S = kappa + kappa^T."""
    pairs = I.packed_pairs(d)
    c = len(pairs)
    K = mp.matrix(d, d)
    for i in range(d):
        for j in range(d):
            K[i, j] = mp.mpf(float(k[i, j]))

    def full(e):
        E = mp.matrix(d, d)
        for s, (i, j) in enumerate(pairs):
            E[i, j] = e[s]
            E[j, i] = e[s]
        return E
    L = mp.matrix(c, c)
    for s in range(c):
        e = [mp.mpf(0)] * c
        e[s] = mp.mpf(1)
        E = full(e)
        Z = K * E + E * K.T - E / De
        for r, (i, j) in enumerate(pairs):
            L[r, s] = Z[i, j]
    S = mp.matrix(c, 1)
    for r, (i, j) in enumerate(pairs):
        S[r] = K[i, j] + K[j, i]
    return L, S


def _augmented_reference(d, w, lam, De, eta_p, dt, N, k, X0):
    """X^N and tau^N of the scheme on the augmented system, in 30-digit arithmetic."""
    import mpmath as mp
    with mp.workdps(30):
        m = len(w)
        c = I.ncomp(d)
        De = mp.mpf(float(De))
        L, S = _packed_operator_mp(mp, d, k, De)
        W = [mp.mpf(float(x)) for x in w]
        Lm = [mp.mpf(float(x)) for x in lam]
        h = mp.mpf(float(dt))
        nu = c + m * c + m
        M = mp.matrix(nu, nu)
        b = mp.matrix(nu, 1)
        for kk in range(m):
            o = c + kk * c
            for r in range(c):
                for s in range(c):
                    M[r, s] += W[kk] * L[r, s]
                    M[r, o + s] += -Lm[kk] * L[r, s]
                M[r, c + m * c + kk] += -Lm[kk] * S[r]
                b[r] += W[kk] * S[r]
                M[o + r, r] += W[kk]
                M[o + r, o + r] += -Lm[kk]
            M[c + m * c + kk, c + m * c + kk] = -Lm[kk]
            b[c + m * c + kk] = W[kk]
        Id = mp.eye(nu)
        y0 = mp.matrix(nu, 1)
        for s in range(c):
            y0[s] = mp.mpf(float(X0[s]))
        gs = 1 - 1 / mp.sqrt(2)
        A = Id - h * gs * M
        Y1 = mp.lu_solve(A, y0 + h * gs * b)
        Y2 = mp.lu_solve(A, y0 + h * (1 - gs) * (M * Y1 + b) + h * gs * b)
        ym, yn = y0, Y2
        B = mp.mpf(3) / 2 * Id - h * M
        for _ in range(1, N):
            yp = mp.lu_solve(B, 2 * yn - ym / 2 + h * b)
            ym, yn = yn, yp
        X = np.array([yn[s] for s in range(c)], dtype=object)
        tau = []
        g = mp.mpf(float(eta_p)) / De
        for s in range(c):
            acc = mp.mpf(0)
            for kk in range(m):
                acc += W[kk] * yn[s] - Lm[kk] * yn[c + kk * c + s]
            tau.append(g * acc)
        return X, np.array(tau, dtype=object)


def _relerr_ref(a, ref):
    num = max(abs(float(x - y)) for x, y in zip(a, ref))
    den = max(abs(float(y)) for y in ref)
    return num / den


@pytest.mark.parametrize("d", [2, 3])
def test_extended_build_matches_30_digit_augmented_scheme(d):
    import mpmath as mp
    rng = np.random.default_rng(70 + d)
    m, dt, N, De, eta_p = 5, 2e-3, 30, 0.8, 0.1
    # a wide pole range, as in the fitted rules: the stress is a near-cancelling sum
    w = rng.uniform(0.1, 3.0, m)
    lam = np.concatenate([[0.0], 10 ** rng.uniform(-1, 5, m - 1)])
    k = rng.standard_normal((d, d)) * 0.7
    X0 = rng.standard_normal(I.ncomp(d)) * 0.05
    Xr, tr = _augmented_reference(d, w, lam, De, eta_p, dt, N, k, X0)
    with mp.workdps(30):
        ld = O.run_long(d, w, lam, De, eta_p, dt, N, k.reshape(-1, 1), X0.reshape(-1, 1))
        db = O.run(d, w, lam, De, eta_p, dt, N, k.reshape(-1, 1), X0.reshape(-1, 1))
        # shortest round-tripping decimal of each element: exact at 30 digits
        to_mp = lambda a: [mp.mpf(np.format_float_scientific(x, unique=True)) for x in a]
        eX_ld = _relerr_ref(to_mp(ld["X"][0][:, 0]), Xr)
        et_ld = _relerr_ref(to_mp(ld["tau"][:, 0]), tr)
        eX_db = _relerr_ref(to_mp(db["X"][0][:, 0]), Xr)
        et_db = _relerr_ref(to_mp(db["tau"][:, 0]), tr)
    print(f"d={d}: extended X {eX_ld:.1e} tau {et_ld:.1e}; FP64 X {eX_db:.1e} tau {et_db:.1e}")
    # x87 extended: 2^-64 = 5.4e-20 per rounding
    assert eX_ld < 1e-16 and et_ld < 1e-15
    assert eX_db < 1e-12 and et_db < 1e-10
    # the extended build is the more accurate reference
    assert et_ld < et_db or et_db < 1e-16


def test_extended_build_agrees_with_fp64_build_on_workload_points():
    """On a sample of the 1024^2 workload (alpha = 0.7, time-varying kappa) the FP64 and the
    extended builds agree to FP64 rounding, so both run the same scheme."""
    from oracle import soe as osoe
    wl = I.WORKLOADS[2]
    ff = I.fourier_field(wl)
    pts = np.arange(0, wl.npoints, 4099)[:64]
    idx = I.grid_multi_index(wl.grid, 2, pts)
    N = 60
    kap = np.stack([ff.kappa_at(idx, wl.grid, n * wl.dt) for n in range(N + 1)])
    X0 = I.initial_state(wl, pts)
    w, lam, _ = osoe.soe_fit(0.7, wl.nmodes, wl.dt, wl.dt * wl.nsteps)
    a = O.run(2, w, lam, wl.De, wl.eta_p, wl.dt, N, kap, X0)
    b = O.run_long(2, w, lam, wl.De, wl.eta_p, wl.dt, N, kap, X0)
    for key, tol in (("X", 1e-13), ("tau", 1e-12)):
        ref = b[key].astype(np.float64)
        e = float(np.max(np.abs(a[key] - ref)) / np.max(np.abs(ref)))
        assert e < tol, (key, e)
    assert math.isfinite(float(b["tau"].max()))
