"""Pins of the coupled-step oracle (oracle/ns.py): the projection method of Sec. 4.1 for the
Navier-Stokes equations of Sec. 2 on a periodic box, coupled to the pointwise stress update.

Each pin ties the oracle to something other than itself:
  * spectral derivatives of trigonometric fields against their closed forms (the index
    convention kappa_ij = d u_i / d x_j and the divergence of a symmetric tensor);
  * the explicit term against the exact product computed on a twice finer grid and cut to
    the 2/3 band, and against the closed form for the Taylor-Green field;
  * exact Navier-Stokes solutions (the 2-D Taylor-Green vortex, the 3-D ABC flow), whose
    advection is a pure gradient: errors of order dt^2 for the BDF2 scheme;
  * a zero divergence at every level from a velocity that starts with a gradient part;
  * a shear wave u = (U(t) sin(k y), 0[, 0]), for which the coupled system reduces exactly
    to a scalar recurrence for U driven by the pointwise stress of one point; with the MFP
    transport terms on, by the pointwise stress at the shifted rate 1/De + eps k^2."""
import math

import numpy as np
import pytest

from oracle import ns
from oracle import oracle as O
from oracle import soe


def coords(shape, extent):
    axes = [np.arange(n) * (L / n) for n, L in zip(shape, extent)]
    return np.meshgrid(*axes, indexing="ij")


@pytest.mark.parametrize("shape,extent", [((8, 10), (2 * math.pi, 3.0)), ((6, 8, 10), (1.0, 2.0, 2 * math.pi))])
def test_derivatives_of_trigonometric_fields(shape, extent):
    d = len(shape)
    box = ns.Box(shape, extent)
    x = coords(shape, extent)
    rng = np.random.default_rng(5 + d)
    terms = []
    for _ in range(3):
        k = np.array([int(rng.integers(-(n // 3 - 1), n // 3)) for n in shape])
        terms.append((k, rng.standard_normal(d), rng.uniform(0, 2 * math.pi)))
    kv = lambda k: [2 * math.pi * k[j] / extent[j] for j in range(d)]
    u = np.stack([sum(A[i] * np.sin(sum(kv(k)[j] * x[j] for j in range(d)) + ph) for k, A, ph in terms)
                  for i in range(d)])
    du = np.stack([sum(A[i] * kv(k)[j] * np.cos(sum(kv(k)[q] * x[q] for q in range(d)) + ph) for k, A, ph in terms)
                   for i in range(d) for j in range(d)])
    kap = box.gradient(box.fft(u))
    np.testing.assert_allclose(kap, du, rtol=0, atol=1e-12 * np.max(np.abs(du)))
    # divergence of a symmetric tensor with one trigonometric term per packed component
    c = d * (d + 1) // 2
    tau = np.empty((c,) + shape)
    div = np.zeros((d,) + shape)
    for s, (i, j) in enumerate(ns.PAIRS[d]):
        k, A, ph = terms[s % 3]
        arg = sum(kv(k)[q] * x[q] for q in range(d)) + ph
        tau[s] = A[0] * np.cos(arg)
        div[i] += -A[0] * kv(k)[j] * np.sin(arg)
        if i != j:
            div[j] += -A[0] * kv(k)[i] * np.sin(arg)
    got = box.ifft(box.div_tensor(box.fft(tau)))
    np.testing.assert_allclose(got, div, rtol=0, atol=1e-12 * np.max(np.abs(div)))


def band_limited_velocity(box, seed, amp=1.0):
    rng = np.random.default_rng(seed)
    u = rng.standard_normal((box.d,) + box.shape)
    return box.ifft(box.fft(u) * box.band) * amp


@pytest.mark.parametrize("shape", [(12, 9), (6, 9, 7)])
def test_explicit_term_is_the_exact_product_cut_to_the_band(shape):
    """-(u.grad)u + div tau for band-limited u and tau equals the exact product (a grid of
    twice the points per axis holds it without aliasing) with its modes outside the band
    removed."""
    d = len(shape)
    extent = (1.0, 2.0, 1.5)[:d]
    box = ns.Box(shape, extent)
    u = band_limited_velocity(box, 3)
    uh = box.fft(u)
    c = d * (d + 1) // 2
    rng = np.random.default_rng(4)
    tau = box.ifft(box.fft(rng.standard_normal((c,) + shape)) * box.band)
    F = ns.explicit_term(box, uh, tau)
    fine = ns.Box(tuple(2 * n for n in shape), extent)

    def up(fh):            # zero-pad coefficients onto the fine grid (same normalisation)
        out = np.zeros(fine.shape, dtype=complex)
        idx = np.meshgrid(*[np.fft.fftfreq(n, 1.0 / n).astype(int) for n in shape], indexing="ij")
        out[tuple(idx)] = fh
        return out

    def down(fh):
        idx = np.meshgrid(*[np.fft.fftfreq(n, 1.0 / n).astype(int) for n in shape], indexing="ij")
        return fh[tuple(idx)]
    uf = np.stack([fine.ifft(up(uh[i])) for i in range(d)])
    duf = [[fine.ifft(1j * fine.xi[j] * up(uh[i])) for j in range(d)] for i in range(d)]
    adv = np.stack([sum(uf[j] * duf[i][j] for j in range(d)) for i in range(d)])
    tauh = box.fft(tau)
    full = {}
    for s, (i, j) in enumerate(ns.PAIRS[d]):
        full[(i, j)] = full[(j, i)] = tauh[s]
    xi = [x for x in box.xi]
    divt = np.stack([sum(1j * xi[j] * full[(i, j)] for j in range(d)) for i in range(d)])
    want = np.stack([(-down(fine.fft(adv[i])) + divt[i]) * box.band for i in range(d)])
    assert np.max(np.abs(F - want)) < 1e-13 * np.max(np.abs(want))
    assert np.max(np.abs(F[:, ~box.band])) == 0.0


def test_explicit_term_of_the_taylor_green_field():
    """u = (sin x cos y, -cos x sin y): (u.grad)u = (sin 2x, sin 2y) / 2."""
    shape, extent = (8, 8), (2 * math.pi, 2 * math.pi)
    box = ns.Box(shape, extent)
    x, y = coords(shape, extent)
    u = np.stack([np.sin(x) * np.cos(y), -np.cos(x) * np.sin(y)])
    F = np.stack([box.ifft(f) for f in ns.explicit_term(box, box.fft(u), np.zeros((3,) + shape))])
    np.testing.assert_allclose(F, -0.5 * np.stack([np.sin(2 * x), np.sin(2 * y)]), rtol=0, atol=1e-14)


def decay_errors(d, nu, T, Ns):
    if d == 2:
        shape, extent = (8, 8), (2 * math.pi,) * 2
        x, y = coords(shape, extent)
        u0 = np.stack([np.sin(x) * np.cos(y), -np.cos(x) * np.sin(y)])
        rate = 2 * nu
    else:
        shape, extent = (8, 8, 8), (2 * math.pi,) * 3
        x, y, z = coords(shape, extent)
        A, B, Cc = 1.0, 0.7, 0.4
        u0 = np.stack([A * np.sin(z) + Cc * np.cos(y), B * np.sin(x) + A * np.cos(z), Cc * np.sin(y) + B * np.cos(x)])
        rate = nu
    P = int(np.prod(shape))
    c = d * (d + 1) // 2
    errs = []
    for N in Ns:
        dt = T / N
        w, lam, _ = soe.soe_fit(0.5, 3, dt, T)
        r = ns.run(d, shape, extent, nu, w, lam, 1.0, 0.0, dt, N, u0.reshape(d, P), np.zeros((c, P)))
        exact = u0.reshape(d, P) * math.exp(-rate * T)
        errs.append(np.max(np.abs(r["u"] - exact)))
    return errs


@pytest.mark.parametrize("d", [2, 3])
def test_exact_solutions_decay_with_second_order(d):
    """Taylor-Green (2-D) and ABC (3-D) flows: advection is a gradient, the pressure takes
    it, and the velocity decays like exp(-nu |k|^2 t); BDF2 (BDF1 first step) errors shrink
    like dt^2.  eta_p = 0, so the stress stays zero."""
    errs = decay_errors(d, 0.1, 0.5, (8, 16, 32))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.85 < o < 2.15 for o in orders), (errs, orders)
    assert errs[-1] < 1e-4


@pytest.mark.parametrize("shape", [(12, 10), (6, 8, 6)])
def test_velocity_stays_divergence_free(shape):
    """A random velocity with a gradient part and a stress driven by it: the initial
    projection and every step leave div u at rounding level."""
    d = len(shape)
    extent = (1.0, 1.3, 0.8)[:d]
    box = ns.Box(shape, extent)
    P = box.P
    c = d * (d + 1) // 2
    u0 = band_limited_velocity(box, 9, amp=0.5).reshape(d, P)
    rng = np.random.default_rng(10)
    X0 = rng.standard_normal((c, P)) * 0.05
    w, lam, _ = soe.soe_fit(0.6, 5, 1e-2, 0.1)
    for N in (0, 1, 6):
        r = ns.run(d, shape, extent, 0.05, w, lam, 0.7, 0.3, 1e-2, N, u0, X0)
        assert r["div"] < 1e-13 * np.max(np.abs(r["u"])), (N, r["div"])
    assert np.max(np.abs(r["tau"])) > 1e-3       # the stress is really coupled in


@pytest.mark.parametrize("d", [2, 3])
def test_shear_wave_reduces_to_a_scalar_recurrence(d):
    """u0 = (U0 sin(k y), 0[, 0]), X0 = 0.  Advection vanishes, only kappa_xy = U k cos(k y) is
    non-zero, the pointwise stress is linear in it with tau_xy = T cos(k y), and only
    d tau_xy / dy drives u (the rest of div tau is a gradient).  So u_x = U^n sin(k y) with
        (b0/dt + nu k^2) U^{n+1} = -sum_j (b_j/dt) U^{n+1-j} + sum_j a_j (-k T^{n+1-j}),
    T^n the xy stress of one point driven by kappa_xy^j = k U^j."""
    shape = (6, 12) if d == 2 else (4, 12, 4)
    extent = (1.0, 1.5) if d == 2 else (1.0, 1.5, 0.7)
    P = int(np.prod(shape))
    c = d * (d + 1) // 2
    x = coords(shape, extent)
    k = 2 * math.pi * 2 / extent[1]
    U0, nu, De, eta_p, dt, N = 0.8, 0.05, 0.6, 0.4, 0.01, 15
    w, lam, _ = soe.soe_fit(0.6, 6, dt, dt * N)
    u0 = np.zeros((d,) + shape)
    u0[0] = U0 * np.sin(k * x[1])
    r = ns.run(d, shape, extent, nu, w, lam, De, eta_p, dt, N, u0.reshape(d, P), np.zeros((c, P)))
    xy = 2 if d == 2 else 3
    U, T = [U0], [0.0]
    for n in range(N):
        if n == 0:
            b, a = (1.0, -1.0), (1.0,)
        else:
            b, a = (1.5, -2.0, 0.5), (2.0, -1.0)
        g = len(a)
        rhs = -sum(b[j] / dt * U[n + 1 - j] for j in range(1, g + 1)) + sum(
            a[j - 1] * (-k * T[n + 1 - j]) for j in range(1, g + 1))
        U.append(rhs / (b[0] / dt + nu * k * k))
        lev = np.zeros((n + 2, d * d, 1))
        lev[:, 1, 0] = k * np.array(U)                  # kappa_xy = d u_x / d y at y = 0
        T.append(O.run(d, w, lam, De, eta_p, dt, n + 1, lev, np.zeros((c, 1)), extrap=False)["tau"][xy, 0])
    ux = U[-1] * np.sin(k * x[1]).reshape(P)
    txy = T[-1] * np.cos(k * x[1]).reshape(P)
    assert abs(T[-1]) > 1e-3 and abs(U[-1]) > 0.1
    np.testing.assert_allclose(r["u"][0], ux, rtol=0, atol=1e-12 * abs(U[-1]))
    assert np.max(np.abs(r["u"][1:])) < 1e-14
    np.testing.assert_allclose(r["tau"][xy], txy, rtol=0, atol=1e-12 * abs(T[-1]))


@pytest.mark.parametrize("d", [2, 3])
def test_shear_wave_with_diffusion_reduces_to_a_scalar_recurrence(d):
    """With the MFP transport terms on: advection of the stress vanishes for the shear wave
    (u depends on y only, X too), and eps Laplace acts on tau_xy = T cos(k y) as the extra
    rate eps k^2, so T^n is the pointwise stress at 1/De + eps k^2 (same eta_p/De)."""
    shape = (4, 12) if d == 2 else (4, 12, 4)
    extent = (1.0, 1.5) if d == 2 else (1.0, 1.5, 0.7)
    P = int(np.prod(shape))
    c = d * (d + 1) // 2
    x = coords(shape, extent)
    k = 2 * math.pi * 2 / extent[1]
    U0, nu, De, eta_p, dt, N, eps = 0.8, 0.05, 0.6, 0.02, 0.01, 6, 0.03
    w, lam, _ = soe.soe_fit(0.6, 5, dt, dt * N)
    u0 = np.zeros((d,) + shape)
    u0[0] = U0 * np.sin(k * x[1])
    r = ns.run(d, shape, extent, nu, w, lam, De, eta_p, dt, N, u0.reshape(d, P), np.zeros((c, P)), eps=eps)
    xy = 2 if d == 2 else 3
    Dx = 1.0 / (1.0 / De + eps * k * k)
    U, T = [U0], [0.0]
    for n in range(N):
        b, a = ((1.0, -1.0), (1.0,)) if n == 0 else ((1.5, -2.0, 0.5), (2.0, -1.0))
        g = len(a)
        rhs = -sum(b[j] / dt * U[n + 1 - j] for j in range(1, g + 1)) + sum(
            a[j - 1] * (-k * T[n + 1 - j]) for j in range(1, g + 1))
        U.append(rhs / (b[0] / dt + nu * k * k))
        lev = np.zeros((n + 2, d * d, 1))
        lev[:, 1, 0] = k * np.array(U)
        T.append(O.run(d, w, lam, Dx, eta_p * Dx / De, dt, n + 1, lev, np.zeros((c, 1)), extrap=False)["tau"][xy, 0])
    assert abs(T[-1]) > 1e-4
    np.testing.assert_allclose(r["u"][0], U[-1] * np.sin(k * x[1]).reshape(P), rtol=0, atol=1e-12 * abs(U[-1]))
    np.testing.assert_allclose(r["tau"][xy], T[-1] * np.cos(k * x[1]).reshape(P), rtol=0, atol=1e-12 * abs(T[-1]))
