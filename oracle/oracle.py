"""ctypes front end of the CPU oracle (test infrastructure only).

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
module.  It loads oracle/liboracle.so (building it with gcc if it is missing)
and exposes:

  run(...)              real FP64 run; returns final X levels, tau, plain modes, diagnostics
  run_complex(...)      the same with complex inputs, for complex-step derivatives
  run_long(...)         the same in x87 extended precision (rounding-error reference)
  coupling_matrix(...)  the Hermite coupling matrix A(kappa) of the tested operator
  tensor_to_hermite(...), hermite_indices(d)
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

from . import build as _build

_lib = None
_lock = threading.Lock()

_dp = C.POINTER(C.c_double)


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_build.LIB):
                _build.build()
            L = C.CDLL(_build.LIB)
            for pre, scal in (("orc_", C.c_double), ("orcz_", None)):
                f = getattr(L, pre + "run")
                f.restype = C.c_int
                if scal is not None:
                    f.argtypes = [C.c_int, C.c_long, C.c_int, _dp, _dp, C.c_double, C.c_double, C.c_double,
                                  C.c_long, _dp, C.c_long, C.c_int, C.c_int, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                  C.c_int]
            _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def ncomp(d):
    return d * (d + 1) // 2


_SCHEME = {"sdirk2": 0, "ghost_bdf2": 1, "exp": 2}


def _mass(mass, P):
    """Per-point mass mode (1 = the normalised density; 0 = no mass mode, hence no source)."""
    if mass is None:
        return None
    return np.ascontiguousarray(np.broadcast_to(np.asarray(mass, dtype=np.float64), (P,)))


def run(d, w, lam, De, eta_p, dt, nsteps, kappa, X0, extrap=True, startup="sdirk2",
        want_modes=False, want_diag=False, want_traj=False, nthreads=0, mass=None):
    """Run the oracle.

    startup: "sdirk2" (the paper's scheme: SDIRK2 first step, BDF2 after), "ghost_bdf2"
    (BDF2 from a ghost level, for the convolution check) or "exp" (the exponential-mode
    scheme: each mode integrated exactly for a state linear over the step, and the state
    equation integrated over the step with kappa at the half step; no start-up step).

    kappa: [d*d][P] (steady) or [nlev][d*d][P] (time-varying, nlev >= nsteps+1)
    X0:    [c][P]
    mass:  None (every point's mass mode is 1), or per point (scalar or [P]) 1 or 0; 0 removes
           the mass mode and its source term (a non-constant spatial coefficient)
    Returns dict with X [2][c][P] (levels N, N-1), tau [c][P], modes [2][m][c][P] or None,
    traj [N+1][c][P] or None, diag [nsteps][6] or None."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    m = w.size
    kappa = np.ascontiguousarray(kappa, dtype=np.float64)
    X0 = np.ascontiguousarray(X0, dtype=np.float64)
    c = ncomp(d)
    P = X0.shape[1]
    nlev = 1 if kappa.ndim == 2 else kappa.shape[0]
    X = np.empty((2, c, P))
    tau = np.empty((c, P))
    modes = np.empty((2, m, c, P)) if want_modes else None
    diag = np.empty((max(nsteps, 1), 6)) if want_diag else None
    traj = np.empty((nsteps + 1, c, P)) if want_traj else None
    st = _SCHEME[startup]
    ms = _mass(mass, P)
    rc = lib().orc_run(d, P, m, _ptr(w), _ptr(lam), float(De), float(eta_p), float(dt), int(nsteps),
                       _ptr(kappa), nlev, int(bool(extrap)), st, _ptr(X0), _ptr(ms), _ptr(X), _ptr(tau),
                       _ptr(modes), _ptr(traj), _ptr(diag), int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle run failed with status {rc}")
    return {"X": X, "tau": tau, "modes": modes, "traj": traj,
            "diag": diag[:nsteps] if diag is not None else None}


def run_complex(d, w, lam, De, eta_p, dt, nsteps, kappa, X0, extrap=True, startup="sdirk2",
                want_modes=False, nthreads=0, mass=None):
    """Complex-step variant: every input may carry an imaginary perturbation."""
    w = np.ascontiguousarray(w, dtype=np.complex128)
    lam = np.ascontiguousarray(lam, dtype=np.complex128)
    m = w.size
    kappa = np.ascontiguousarray(kappa, dtype=np.complex128)
    X0 = np.ascontiguousarray(X0, dtype=np.complex128)
    c = ncomp(d)
    P = X0.shape[1]
    nlev = 1 if kappa.ndim == 2 else kappa.shape[0]
    X = np.empty((2, c, P), dtype=np.complex128)
    tau = np.empty((c, P), dtype=np.complex128)
    modes = np.empty((2, m, c, P), dtype=np.complex128) if want_modes else None
    st = _SCHEME[startup]
    De_c = np.array([De], dtype=np.complex128)
    ep_c = np.array([eta_p], dtype=np.complex128)
    L = lib()
    f = L.orcz_run
    f.restype = C.c_int
    # complex scalars are passed by value: declare them as C structs of two doubles
    class _cd(C.Structure):
        _fields_ = [("re", C.c_double), ("im", C.c_double)]
    f.argtypes = [C.c_int, C.c_long, C.c_int, C.c_void_p, C.c_void_p, _cd, _cd, C.c_double,
                  C.c_long, C.c_void_p, C.c_long, C.c_int, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p,
                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int]
    vp = lambda a: None if a is None else a.ctypes.data
    ms = _mass(mass, P)
    rc = f(d, P, m, vp(w), vp(lam), _cd(De_c[0].real, De_c[0].imag), _cd(ep_c[0].real, ep_c[0].imag),
           float(dt), int(nsteps), vp(kappa), nlev, int(bool(extrap)), st, vp(X0), vp(ms), vp(X), vp(tau),
           vp(modes), None, None, int(nthreads))
    if rc != 0:
        raise RuntimeError(f"oracle complex run failed with status {rc}")
    return {"X": X, "tau": tau, "modes": modes}


def run_long(d, w, lam, De, eta_p, dt, nsteps, kappa, X0, extrap=True, startup="sdirk2", nthreads=0, mass=None):
    """The same scheme in x87 extended precision (64-bit significand), from the same FP64
    inputs (converted exactly): a reference for the rounding error of FP64 evaluations.
    Returns dict with X [2][c][P] (levels N, N-1) and tau [c][P] as np.longdouble."""
    ld = np.longdouble
    w = np.ascontiguousarray(np.asarray(w, dtype=np.float64).astype(ld))
    lam = np.ascontiguousarray(np.asarray(lam, dtype=np.float64).astype(ld))
    m = w.size
    kappa = np.ascontiguousarray(np.asarray(kappa, dtype=np.float64).astype(ld))
    X0 = np.ascontiguousarray(np.asarray(X0, dtype=np.float64).astype(ld))
    c = ncomp(d)
    P = X0.shape[1]
    nlev = 1 if kappa.ndim == 2 else kappa.shape[0]
    X = np.empty((2, c, P), dtype=ld)
    tau = np.empty((c, P), dtype=ld)
    f = lib().orcl_run
    f.restype = C.c_int
    lp = C.c_void_p
    f.argtypes = [C.c_int, C.c_long, C.c_int, lp, lp, C.c_longdouble, C.c_longdouble, C.c_double, C.c_long, lp,
                  C.c_long, C.c_int, C.c_int, lp, lp, lp, lp, lp, lp, lp, C.c_int]
    ms = _mass(mass, P)
    rc = f(d, P, m, w.ctypes.data, lam.ctypes.data, C.c_longdouble(float(De)), C.c_longdouble(float(eta_p)),
           float(dt), int(nsteps), kappa.ctypes.data, nlev, int(bool(extrap)), _SCHEME[startup], X0.ctypes.data,
           None if ms is None else ms.ctypes.data, X.ctypes.data, tau.ctypes.data, None, None, None, int(nthreads))
    if rc != 0:
        raise RuntimeError(f"extended-precision oracle run failed with status {rc}")
    return {"X": X, "tau": tau}


def exp_weights(z):
    """(e, a0, a1) of the exponential mode update at z = lambda * dt (real z)."""
    L = lib()
    out = np.empty(3)
    L.orc_exp_weights_of.argtypes = [C.c_double, _dp]
    L.orc_exp_weights_of.restype = None
    L.orc_exp_weights_of(float(z), _ptr(out))
    return out


def coupling_matrix(d, De, kappa_dd):
    L = lib()
    n = d * (d + 1) // 2 + 1
    A = np.empty((n, n))
    k = np.ascontiguousarray(kappa_dd, dtype=np.float64).reshape(d * d)
    L.orc_coupling_matrix.argtypes = [C.c_int, C.c_double, _dp, _dp]
    L.orc_coupling_matrix(d, float(De), _ptr(k), _ptr(A))
    return A


def tensor_to_hermite(d, Xpacked):
    L = lib()
    n = d * (d + 1) // 2 + 1
    x = np.ascontiguousarray(Xpacked, dtype=np.float64)
    out = np.empty(n)
    L.orc_tensor_to_hermite_packed.argtypes = [C.c_int, _dp, _dp]
    L.orc_tensor_to_hermite_packed(d, _ptr(x), _ptr(out))
    return out


def hermite_indices(d):
    L = lib()
    z = np.zeros((7, 3), dtype=np.int32)
    L.orc_hermite_indices.argtypes = [C.c_int, C.POINTER(C.c_int)]
    L.orc_hermite_indices.restype = C.c_int
    n = L.orc_hermite_indices(d, z.ctypes.data_as(C.POINTER(C.c_int)))
    return z[:n, :d].copy()
