"""Sum-of-exponentials approximation of the Riemann-Liouville kernel (oracle side).

Test infrastructure only.  The paper compresses g_alpha(t) = t^(alpha-1)/Gamma(alpha)
into sum_k w_k exp(-lam_k t) with w_k, lam_k >= 0 (Sec. 2.2, eq. tf_approximate_kernel),
which keeps the approximate kernel completely monotone.

Two fits are provided, written independently of the device library's fitter:

* ``soe_gl_log`` -- exactly m modes from the Stieltjes form of the symbol,
      s^(-alpha) = (sin(pi alpha)/pi) * int_R exp((1-alpha) y) / (s + e^y) dy,
  whose inverse Laplace transform is the kernel.  Modes: one lam = 0 mode for the
  lower tail y < y_lo (weight (sin(pi alpha)/pi) e^{(1-alpha) y_lo}/(1-alpha)), an
  (m-2)-point Gauss-Legendre rule on [y_lo, y_hi] (lam = e^y), and one exponential
  for the upper tail y > y_hi that matches the tail's mass and first moment in
  time (lam = e^{y_hi}(1+alpha)/alpha).  Positivity holds by construction.  The
  window minimises the relative error of the Laplace symbol on [0.1/T, 10/dt]:
  the scheme sees the kernel only through that symbol (it is a convolution
  quadrature, Sec. 4.1), and a time-domain fit on [dt, T] leaves O(dt^alpha) of
  the kernel's mass near t = 0 unrepresented.
* ``soe_aaa_duswald`` -- the paper's own recipe (Sec. 2.2, last paragraph):
  AAA rational approximation of s^(1-alpha), divided by s, partial fractions,
  inverse Laplace transform; this gives w_infinity = 0.  The AAA step is scipy's.
"""
from __future__ import annotations

import math

import numpy as np


def kernel(alpha: float, t: np.ndarray) -> np.ndarray:
    return np.asarray(t, dtype=np.float64) ** (alpha - 1.0) / math.gamma(alpha)


def soe_eval(w, lam, t):
    t = np.asarray(t, dtype=np.float64)
    return np.exp(-np.outer(t, lam)) @ w


def kernel_relerr(alpha, w, lam, dt, T, nsample=400):
    t = np.geomspace(dt, T, nsample)
    g = kernel(alpha, t)
    return float(np.max(np.abs(soe_eval(w, lam, t) - g) / g))


def soe_gl_log(alpha: float, m: int, y_lo: float, y_hi: float):
    """Exactly m modes on a fixed window; returns (w, lam, dw/dalpha, dlam/dalpha)."""
    if m < 1:
        raise ValueError("m >= 1")
    if alpha == 1.0:
        w = np.zeros(m); w[0] = 1.0
        return w, np.zeros(m), np.zeros(m), np.zeros(m)
    s = math.sin(math.pi * alpha) / math.pi
    cot = math.pi * math.cos(math.pi * alpha) / math.sin(math.pi * alpha)
    w = np.zeros(m)
    lam = np.zeros(m)
    dw = np.zeros(m)
    dlam = np.zeros(m)
    w[0] = s * math.exp((1.0 - alpha) * y_lo) / (1.0 - alpha)
    dw[0] = w[0] * (cot - y_lo + 1.0 / (1.0 - alpha))
    if m >= 2:
        j = m - 1
        lam[j] = math.exp(y_hi) * (1.0 + alpha) / alpha
        w[j] = s * math.exp((1.0 - alpha) * y_hi) * (1.0 + alpha) / alpha ** 2
        dlam[j] = -math.exp(y_hi) / alpha ** 2
        dw[j] = w[j] * (cot - y_hi + 1.0 / (1.0 + alpha) - 2.0 / alpha)
    if m >= 3:
        x, gw = np.polynomial.legendre.leggauss(m - 2)
        half = 0.5 * (y_hi - y_lo)
        y = 0.5 * (y_hi + y_lo) + half * x
        w[1:m - 1] = s * half * gw * np.exp((1.0 - alpha) * y)
        lam[1:m - 1] = np.exp(y)
        dw[1:m - 1] = w[1:m - 1] * (cot - y)
    return w, lam, dw, dlam


def symbol_relerr(alpha, w, lam, dt, T, nsample=300):
    """max over s in [0.1/T, 10/dt] of |sum_k w_k/(s+lam_k) * s^alpha - 1|."""
    s = np.geomspace(0.1 / T, 10.0 / dt, nsample)
    K = (1.0 / (s[:, None] + np.asarray(lam)[None, :])) @ np.asarray(w)
    return float(np.max(np.abs(K * s ** alpha - 1.0)))


def soe_fit(alpha: float, m: int, dt: float, T: float):
    """GL-log fit with the window found by a coarse-then-fine grid search.

    Returns (w, lam, info) with info = {y_lo, y_hi, symbol_relerr, kernel_relerr}."""
    if alpha == 1.0:
        w, lam, _, _ = soe_gl_log(alpha, m, 0.0, 1.0)
        return w, lam, {"y_lo": 0.0, "y_hi": 1.0, "symbol_relerr": 0.0, "kernel_relerr": 0.0}
    lo0 = math.log(0.1 / T)
    hi0 = math.log(10.0 / dt)
    best = None
    for lo_off in np.arange(-16.0, 1.01, 0.5):
        for hi_off in np.arange(-2.0, 40.01, 1.0):
            ylo, yhi = lo0 + lo_off, hi0 + hi_off
            w, lam, _, _ = soe_gl_log(alpha, m, ylo, yhi)
            e = symbol_relerr(alpha, w, lam, dt, T, 120)
            if best is None or e < best[0]:
                best = (e, ylo, yhi)
    _, ylo_b, yhi_b = best
    for dlo in np.arange(-0.5, 0.501, 0.1):
        for dhi in np.arange(-1.0, 1.001, 0.1):
            ylo, yhi = ylo_b + dlo, yhi_b + dhi
            w, lam, _, _ = soe_gl_log(alpha, m, ylo, yhi)
            e = symbol_relerr(alpha, w, lam, dt, T, 120)
            if e < best[0]:
                best = (e, ylo, yhi)
    _, ylo, yhi = best
    w, lam, _, _ = soe_gl_log(alpha, m, ylo, yhi)
    return w, lam, {"y_lo": ylo, "y_hi": yhi, "symbol_relerr": symbol_relerr(alpha, w, lam, dt, T),
                    "kernel_relerr": kernel_relerr(alpha, w, lam, dt, T)}


def soe_aaa_duswald(alpha: float, dt: float, T: float, rtol: float = 1e-13, max_terms: int = 100):
    """The paper's AAA-on-s^(1-alpha), divide-by-s construction.

    Returns (w, lam) with the lam = 0 pole from the division included, or raises
    if the fit has poles off the negative real axis or negative weights."""
    from scipy.interpolate import AAA

    z = np.geomspace(0.1 / T, 10.0 / dt, 2000)
    r = AAA(z, z ** (1.0 - alpha), rtol=rtol, max_terms=max_terms)
    poles = r.poles()
    res = r.residues()
    # r(s)/s = r(0)/s + sum_j res_j / (p_j (s - p_j))  with r(s) = r_inf + sum_j res_j/(s - p_j)
    r0 = complex(r(np.array([0.0]))[0])
    w = [r0.real]
    lam = [0.0]
    for p, q in zip(poles, res):
        wk = q / p
        lk = -p
        if abs(lk.imag) > 1e-8 * max(1.0, abs(lk)) or abs(wk.imag) > 1e-8 * max(1.0, abs(wk)):
            raise ValueError("complex pole in AAA fit")
        w.append(wk.real)
        lam.append(lk.real)
    w = np.array(w); lam = np.array(lam)
    if np.any(w < 0) or np.any(lam < 0):
        raise ValueError("non-positive weight or pole in AAA fit")
    order = np.argsort(lam)
    return w[order], lam[order]
