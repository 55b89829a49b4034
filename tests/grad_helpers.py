"""Gradients of the final-stress misfit for the adjoint tests.

Loss: L = 1/2 sum_x ||tau^N(x) - tau*(x)||_F^2 over the full symmetric tensor, so packed
off-diagonal components carry weight 2.

* oracle_gradients: complex-step derivatives of the oracle (exact to rounding), one sweep
  per direction; points are independent, so one sweep per component of a per-point field
  gives that component's gradient at every point.
* gpu_gradients: forward on the GPU keeping every level (tfs_step_levels), then the adjoint
  (tfs_step_adjoint) from level N back to 0, then the host chain (tfs_pbar_to_params).
"""
import numpy as np
import torch

from oracle import oracle as O
from paper_2411_17294_amd import tfs

H_CS = 1e-30


def pack_weights(d):
    c = d * (d + 1) // 2
    return np.array([1.0 if s < d else 2.0 for s in range(c)])


def loss(tau, target, d):
    w = pack_weights(d)[:, None]
    return 0.5 * float(np.sum(w * (tau - target) ** 2))


def oracle_gradients(d, w, lam, De, eta_p, dt, N, kappa, X0, target, dw_da=None, dl_da=None,
                     per_mode=False, extrap=True, scheme="bdf2"):
    """Returns dict: kappa [d*d][P] (derivative w.r.t. an additive steady perturbation of
    kappa at every level), X0 [c][P], De, eta_p, alpha (if dw_da given), w, lam (per_mode)."""
    wts = pack_weights(d)[:, None]
    startup = "exp" if scheme == "exp" else "sdirk2"
    base = O.run(d, w, lam, De, eta_p, dt, N, kappa, X0, extrap=extrap, startup=startup)
    resid = base["tau"] - target

    def run(dk=None, dX0=None, dwv=None, dlv=None, dDe=0.0, dep=0.0):
        kc = kappa.astype(complex) + (1j * H_CS * dk if dk is not None else 0)
        Xc = X0.astype(complex) + (1j * H_CS * dX0 if dX0 is not None else 0)
        wc = np.asarray(w, complex) + (1j * H_CS * dwv if dwv is not None else 0)
        lc = np.asarray(lam, complex) + (1j * H_CS * dlv if dlv is not None else 0)
        r = O.run_complex(d, wc, lc, De + 1j * H_CS * dDe, eta_p + 1j * H_CS * dep, dt, N, kc, Xc, extrap=extrap,
                          startup=startup)
        return r["tau"].imag / H_CS          # dtau along the direction

    out = {"loss": loss(base["tau"], target, d)}
    nk = d * d
    gk = np.zeros((nk,) + kappa.shape[-1:])
    for q in range(nk):
        dk = np.zeros_like(kappa)
        dk[..., q, :] = 1.0
        gk[q] = np.sum(wts * resid * run(dk=dk), axis=0)
    out["kappa"] = gk
    c = X0.shape[0]
    gx = np.zeros_like(X0)
    for s in range(c):
        dX = np.zeros_like(X0)
        dX[s] = 1.0
        gx[s] = np.sum(wts * resid * run(dX0=dX), axis=0)
    out["X0"] = gx
    out["De"] = float(np.sum(wts * resid * run(dDe=1.0)))
    out["eta_p"] = float(np.sum(wts * resid * run(dep=1.0)))
    if dw_da is not None:
        out["alpha"] = float(np.sum(wts * resid * run(dwv=np.asarray(dw_da), dlv=np.asarray(dl_da))))
    if per_mode:
        m = len(w)
        gw, gl = np.zeros(m), np.zeros(m)
        for k in range(m):
            e = np.zeros(m); e[k] = 1.0
            gw[k] = float(np.sum(wts * resid * run(dwv=e)))
            if lam[k] != 0.0 or True:
                gl[k] = float(np.sum(wts * resid * run(dlv=e)))
        out["w"], out["lam"] = gw, gl
    return out


def oracle_spatial_gradients(d, w, lam, De, eta_p, dt, N, kappa, X0, target, rate, source, per_mode=False,
                             extrap=True, scheme="bdf2"):
    """Complex-step gradients of the spatial form in the Fourier layout, from the pointwise
    oracle: a point of rate r follows the pointwise scheme with 1/De -> 1/De + r at the same
    eta_p/De, without the mass mode and its source (mass 0) unless it is the source point or
    no source point is set (source < 0).  Points of equal rate and source flag run together.
    Returns the keys of oracle_gradients (no alpha) plus "rate" = sum_p rate_p dL/drate_p.
    scheme: "bdf2" (SDIRK2 start) or "exp"."""
    wts = pack_weights(d)[:, None]
    startup = "exp" if scheme == "exp" else "sdirk2"
    P = X0.shape[1]
    m = len(w)
    groups = {}
    for p in range(P):
        groups.setdefault((float(rate[p]), source < 0 or p == source), []).append(p)
    out = {"kappa": np.zeros((d * d, P)), "X0": np.zeros_like(X0), "De": 0.0, "eta_p": 0.0, "rate": 0.0,
           "loss": 0.0}
    if per_mode:
        out["w"], out["lam"] = np.zeros(m), np.zeros(m)
    for (r, src), idx in groups.items():
        idx = np.asarray(idx)
        kap, x0, tg = kappa[..., idx], X0[:, idx], target[:, idx]

        def tau(dk=None, dX0=None, dwv=None, dlv=None, dDe=0.0, dep=0.0, drate=0.0):
            Dc = De + 1j * H_CS * dDe
            ec = eta_p + 1j * H_CS * dep
            rc = r + 1j * H_CS * drate
            Dx = 1.0 / (1.0 / Dc + rc)
            ex = ec * Dx / Dc
            kc = kap.astype(complex) + (1j * H_CS * dk if dk is not None else 0)
            xc = x0.astype(complex) + (1j * H_CS * dX0 if dX0 is not None else 0)
            wc = np.asarray(w, complex) + (1j * H_CS * dwv if dwv is not None else 0)
            lc = np.asarray(lam, complex) + (1j * H_CS * dlv if dlv is not None else 0)
            return O.run_complex(d, wc, lc, Dx, ex, dt, N, kc, xc, extrap=extrap, startup=startup,
                                 mass=1.0 if src else 0.0)["tau"]

        base = tau().real
        resid = base - tg
        out["loss"] += loss(base, tg, d)
        dirv = lambda **kw: np.sum(wts * resid * tau(**kw).imag / H_CS, axis=0)
        for q in range(d * d):
            dk = np.zeros_like(kap)
            dk[..., q, :] = 1.0
            out["kappa"][q, idx] = dirv(dk=dk)
        for s in range(x0.shape[0]):
            dX = np.zeros_like(x0)
            dX[s] = 1.0
            out["X0"][s, idx] = dirv(dX0=dX)
        out["De"] += float(np.sum(dirv(dDe=1.0)))
        out["eta_p"] += float(np.sum(dirv(dep=1.0)))
        out["rate"] += float(np.sum(dirv(drate=r)))
        if per_mode:
            for k in range(m):
                e = np.zeros(m)
                e[k] = 1.0
                out["w"][k] += float(np.sum(dirv(dwv=e)))
                out["lam"][k] += float(np.sum(dirv(dlv=e)))
    return out


def gpu_gradients(d, w, lam, alpha, De, eta_p, dt, N, kappa, X0, target, precision="fp64", tile=None,
                  dw_da=None, dl_da=None, extrap=True, tune=None, scheme="bdf2", spatial=None, kappa_prec="fp64",
                  mode_form="auto"):
    """Forward + adjoint on the GPU; kappa steady [d*d][P] or levels [nlev][d*d][P].
    tune: {key: value} passed to tfs_plan_tune (e.g. points per lane).
    spatial: (rate [P], source point) of the spatial form (tfs_plan_set_spatial); the result
    then carries "rate" = sum_p rate_p dL/drate_p.
    kappa_prec: "fp32" stores the velocity gradients in FP32 (FP32-mode plans)."""
    P = X0.shape[1]
    c = d * (d + 1) // 2
    plan = tfs.Plan(d, P, w, lam, alpha, De, eta_p, dt, max(N, 1), precision=precision, tile=tile, scheme=scheme,
                    kappa=kappa_prec, mode_form=mode_form)
    exp = scheme == "exp"
    for key, value in (tune or {}).items():
        plan.tune(key, value)
    st, m = plan.stride, plan.m
    dev = "cuda"
    if spatial is not None:
        rate_t = torch.zeros(st, dtype=torch.float64, device=dev)
        rate_t[:P] = torch.from_numpy(np.ascontiguousarray(spatial[0], dtype=np.float64)).to(dev)
        plan.set_spatial(rate_t, int(spatial[1]))
    mt = plan.mode_dtype
    Xs = [torch.zeros((c, st), dtype=torch.float64, device=dev) for _ in range(N + 1)]
    Ys = [torch.zeros((m * c * st,), dtype=mt, device=dev) for _ in range(N + 1)]
    Xs[0][:, :P] = torch.from_numpy(X0).to(dev)
    steady = kappa.ndim == 2
    if steady:
        kl = [plan.kappa_tensor(kappa)]
        lev = lambda n: (kl[0], kl[0] if extrap else None)
    else:
        kl = [plan.kappa_tensor(kappa[i]) for i in range(kappa.shape[0])]
        lev = (lambda n: (kl[n], kl[n - 1] if n >= 1 else None)) if extrap else (lambda n: (kl[n + 1], None))
    tau = torch.zeros((c, st), dtype=torch.float64, device=dev)
    for n in range(N):
        ka, kb = lev(n)
        if exp:
            plan.step_levels(n, ka, kb, Xs[n], None, Xs[n + 1], Ys[n] if n >= 1 else None, None, Ys[n + 1], tau)
            continue
        plan.step_levels(n, ka, kb, Xs[n], Xs[n - 1] if n >= 1 else None, Xs[n + 1], Ys[n] if n >= 1 else None,
                         Ys[n - 1] if n >= 1 else Ys[0], Ys[n + 1], tau, X_nm2=Xs[n - 2] if n >= 2 else None)
    torch.cuda.synchronize()
    tau_h = tau[:, :P].cpu().numpy()
    wts = pack_weights(d)[:, None]
    taubar = torch.zeros((c, st), dtype=torch.float64, device=dev)
    taubar[:, :P] = torch.from_numpy(wts * (tau_h - target)).to(dev)
    Xbar = torch.zeros((plan.x_levels, c, st), dtype=torch.float64, device=dev)
    Hbar = torch.zeros((plan.mode_levels * m * c * st,), dtype=mt, device=dev)
    pbar = torch.zeros(plan.pbar_size, dtype=torch.float64, device=dev)
    kbar = torch.zeros((d * d, st), dtype=torch.float64, device=dev)
    for n in range(N - 1, -1, -1):
        ka, kb = lev(n)
        if exp:
            plan.step_adjoint(n, ka, kb, Xs[n], None, Xs[n + 1], Ys[n] if n >= 1 else None, None, Xbar, Hbar, pbar,
                              taubar=taubar if n == N - 1 else None, kappabar_a=kbar, kappabar_b=kbar)
            continue
        plan.step_adjoint(n, ka, kb, Xs[n], Xs[n - 1] if n >= 1 else None, Xs[n + 1], Ys[n] if n >= 1 else None,
                          Ys[n - 1] if n >= 1 else None, Xbar, Hbar, pbar,
                          taubar=taubar if n == N - 1 else None, kappabar_a=kbar, kappabar_b=kbar,
                          X_nm2=Xs[n - 2] if n >= 2 else None)
    torch.cuda.synchronize()
    pb = pbar.cpu().numpy()
    gw, gl, gDe, gep, ga = plan.pbar_to_params(pb, dw_da, dl_da)
    out = {"loss": loss(tau_h, target, d), "tau": tau_h, "kappa": kbar[:, :P].cpu().numpy(),
           "X0": Xbar[0, :, :P].cpu().numpy(), "De": gDe, "eta_p": gep, "w": gw, "lam": gl}
    if spatial is not None:
        out["rate"] = plan.pbar_rate_gradient(pb)
    if dw_da is not None:
        out["alpha"] = ga
    return out
