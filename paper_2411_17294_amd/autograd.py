"""Differentiation form: checkpointed forward + adjoint behind torch.autograd.

`fractional_stress(kappa, X0, alpha, De, eta_p, spec)` returns the final stress tau^N
[c][P] of N time steps and back-propagates dL/dtau^N to the velocity gradient kappa
(steady, or an additive steady perturbation of a time-varying field), the initial state
X0, the fractional order alpha, the relaxation time De and eta_p.

alpha enters through the sum-of-exponentials rule at a fixed window (product fitter,
`tfs_soe_gl_log`), whose dw/dalpha and dlambda/dalpha are exact.  Every step of the
forward and of the adjoint runs in the library's HIP kernels; this module only
schedules them and keeps checkpoints:

* forward: the two-slot rings advance N steps; every K steps both ring levels are copied
  into a checkpoint;
* backward, segment by segment from the last: restore the checkpoint, recompute the K
  steps into per-level buffers (tfs_step_levels), then run the adjoint steps back
  through the segment (tfs_step_adjoint).

Memory: N/K checkpoints of two mode levels (one with the exponential-mode scheme) and two or
three X levels, plus K+2 mode levels of one segment.
Points are independent, so `run_slabs` processes a grid in point slabs with the same
code and sums the parameter gradients.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, Optional

import torch

from . import tfs


@dataclasses.dataclass
class Spec:
    dim: int
    nmodes: int
    dt: float
    nsteps: int
    y_lo: float                 # sum-of-exponentials window (fixed while differentiating alpha)
    y_hi: float
    ckpt_every: int = 50
    precision: str = "fp32_modes"
    tile: Optional[int] = None
    extrap: bool = True
    # time-varying base field: kappa_levels(n, out) writes level n into out [d*d][stride];
    # the differentiable kappa input is then an additive steady perturbation
    kappa_levels: Optional[Callable] = None
    # "bdf2" (the paper's scheme) or "exp" (exponential mode update, one mode level)
    scheme: str = "bdf2"
    # storage precision of the velocity-gradient levels the steps read: "fp64", or "fp32"
    # (FP32-mode plans); the differentiable input and its gradient stay FP64
    kappa: str = "fp64"
    # analytic time-varying base field evaluated by the library (tfs_field_eval) in place of
    # kappa_levels: (k [NF][d], phase [NF], omega [NF], coef [NF][d][d], grid, point0)
    field: Optional[tuple] = None


class Checkpointed:
    """Forward with checkpoints and the reverse sweep for one set of points."""

    def __init__(self, spec: Spec, npoints: int, alpha: float, De: float, eta_p: float, device="cuda"):
        self.spec = spec
        self.P = int(npoints)
        self.alpha, self.De, self.eta_p = float(alpha), float(De), float(eta_p)
        w, lam, dw, dl = tfs.soe_gl_log(alpha, spec.nmodes, spec.y_lo, spec.y_hi)
        self.w, self.lam, self.dw, self.dl = w, lam, dw, dl
        self.plan = tfs.Plan(spec.dim, self.P, w, lam, alpha, De, eta_p, spec.dt, spec.nsteps,
                             precision=spec.precision, tile=spec.tile, scheme=spec.scheme, kappa=spec.kappa)
        if spec.field is not None:
            self.plan.set_field(*spec.field)
        self.kdt = self.plan.kappa_dtype
        self.exp = spec.scheme == "exp"
        self.dev = device
        self.c = spec.dim * (spec.dim + 1) // 2
        self.st = self.plan.stride
        self.mt = self.plan.mode_dtype
        self.ys = self.plan.m * self.c * self.st

    # -- velocity gradient of level n ---------------------------------------------------------
    def _time_varying(self):
        return self.spec.kappa_levels is not None or self.spec.field is not None

    def _level_cache(self, nslots):
        """Level buffers of a time-varying base field: slot n % nslots holds level n (+ the
        perturbation) once filled, so consecutive steps and the adjoint sweep over a
        recomputed segment evaluate each level once."""
        st, d2 = self.st, self.spec.dim * self.spec.dim
        return {"buf": [torch.zeros((d2, st), dtype=self.kdt, device=self.dev) for _ in range(nslots)],
                "held": [None] * nslots}

    def _kappa(self, pert, n, cache):
        i = n % len(cache["buf"])
        buf = cache["buf"][i]
        if cache["held"][i] != n:
            if self.spec.field is not None:
                self.plan.field_eval(n * self.spec.dt, buf, add=pert)
            else:
                lev = buf if self.kdt == torch.float64 else self._lev64
                self.spec.kappa_levels(n, lev)
                lev[:, :self.P] += pert[:, :self.P]
                if lev is not buf:
                    buf.copy_(lev)
            cache["held"][i] = n
        return buf

    def _levels(self, pert, n, cache):
        """(kappa_a, kappa_b) of step n."""
        if not self._time_varying():
            k = self.kappa_steady
            return k, (k if self.spec.extrap else None)
        if self.spec.extrap:
            ka = self._kappa(pert, n, cache)
            kb = self._kappa(pert, n - 1, cache) if n >= 1 else None
            return ka, kb
        return self._kappa(pert, n + 1, cache), None

    def forward(self, kappa, X0):
        """kappa: [d*d][P] FP64 device (steady field, or perturbation); X0: [c][P]. Returns tau^N."""
        sp, P, st = self.spec, self.P, self.st
        d2 = sp.dim * sp.dim
        # FP64 perturbation of a time-varying field, or the steady field itself
        self.kappa_pad = torch.zeros((d2, st), dtype=torch.float64, device=self.dev)
        self.kappa_pad[:, :P] = kappa
        if self._time_varying():
            if sp.field is None and self.kdt != torch.float64:
                self._lev64 = torch.zeros((d2, st), dtype=torch.float64, device=self.dev)
        else:
            self.kappa_steady = self.kappa_pad if self.kdt == torch.float64 else self.kappa_pad.to(self.kdt)
        cache = self._level_cache(2) if self._time_varying() else None
        XL = self.plan.x_levels
        X = torch.zeros((XL, self.c, st), dtype=torch.float64, device=self.dev)
        X[0, :, :P] = X0
        Y = torch.zeros((self.plan.mode_levels * self.ys,), dtype=self.mt, device=self.dev)
        tau = torch.zeros((self.c, st), dtype=torch.float64, device=self.dev)
        # a checkpoint of level n: X at levels n, n-1 (and n-2 in the shifted mode form; a level
        # below 0 is not kept) and the mode levels n, n-1 (level n only, exponential scheme)
        self.ckpt = {0: ((X[0].clone(),), ())}
        K, N = sp.ckpt_every, sp.nsteps
        for n in range(N):
            if n > 0 and n % K == 0:
                if self.exp:
                    self.ckpt[n] = ((X[n % XL].clone(),), (Y.clone(),))
                else:
                    xs = tuple(X[(n - j) % XL].clone() for j in range(min(XL, n + 1)))
                    ys = tuple(Y[(l % 2) * self.ys:(l % 2 + 1) * self.ys].clone() for l in (n, n - 1))
                    self.ckpt[n] = (xs, ys)
            ka, kb = self._levels(self.kappa_pad, n, cache)
            self.plan.step(n, ka, kb, X, Y, tau)
        self.X_last = X[N % XL, :, :P].clone()      # the final state, for callers that check it
        return tau[:, :P].clone()

    def backward(self, tau_bar):
        """Returns (dL/dkappa [d*d][P], dL/dX0 [c][P], dL/dalpha, dL/dDe, dL/deta_p)."""
        sp, P, st, c = self.spec, self.P, self.st, self.c
        d2 = sp.dim * sp.dim
        K, N = sp.ckpt_every, sp.nsteps
        taubar = torch.zeros((c, st), dtype=torch.float64, device=self.dev)
        taubar[:, :P] = tau_bar
        Xbar = torch.zeros((self.plan.x_levels, c, st), dtype=torch.float64, device=self.dev)
        Hbar = torch.zeros((self.plan.mode_levels * self.ys,), dtype=self.mt, device=self.dev)
        pbar = torch.zeros(self.plan.pbar_size, dtype=torch.float64, device=self.dev)
        kbar = torch.zeros((d2, st), dtype=torch.float64, device=self.dev)
        starts = sorted(self.ckpt)
        # local index i <-> level s0 - 2 + i: slot 0 = level s0-2 (shifted mode form only),
        # slot 1 = level s0-1, slot 2 = level s0, ..., slot K + 2 = level s0 + K
        Xseg = [torch.zeros((c, st), dtype=torch.float64, device=self.dev) for _ in range(K + 3)]
        Yseg = [torch.zeros((self.ys,), dtype=self.mt, device=self.dev) for _ in range(K + 3)]
        # the levels a segment needs (s0 - 1 .. s1) fit without eviction; the recompute fills
        # them and the adjoint sweep of the same segment reuses them
        cache = self._level_cache(K + 2) if self._time_varying() else None
        lv = lambda n: n - s0 + 2
        for s0 in reversed(starts):
            s1 = min(s0 + K, N)
            xs, ys = self.ckpt[s0]
            for j, x in enumerate(xs):           # levels s0, s0-1, s0-2
                Xseg[lv(s0 - j)].copy_(x)
            for j, y in enumerate(ys):
                Yseg[lv(s0 - j)].copy_(y)
            X2 = lambda n: Xseg[lv(n - 2)] if n >= 2 else None
            for n in range(s0, s1):
                i = lv(n)
                ka, kb = self._levels(self.kappa_pad, n, cache)
                if self.exp:
                    self.plan.step_levels(n, ka, kb, Xseg[i], None, Xseg[i + 1], Yseg[i] if n > 0 else None, None,
                                          Yseg[i + 1], None)
                elif n == 0:
                    self.plan.step_levels(0, ka, kb, Xseg[i], None, Xseg[i + 1], None, Yseg[i], Yseg[i + 1], None)
                else:
                    self.plan.step_levels(n, ka, kb, Xseg[i], Xseg[i - 1], Xseg[i + 1], Yseg[i], Yseg[i - 1],
                                          Yseg[i + 1], None, X_nm2=X2(n))
            for n in range(s1 - 1, s0 - 1, -1):
                i = lv(n)
                ka, kb = self._levels(self.kappa_pad, n, cache)
                tb = taubar if n == N - 1 else None
                if self.exp:
                    self.plan.step_adjoint(n, ka, kb, Xseg[i], None, Xseg[i + 1], Yseg[i] if n > 0 else None, None,
                                           Xbar, Hbar, pbar, taubar=tb, kappabar_a=kbar, kappabar_b=kbar)
                elif n == 0:
                    # the start-up wrote level 0 of the modes into Yseg[i]; its adjoint needs X^0 only
                    self.plan.step_adjoint(0, ka, kb, Xseg[i], None, Xseg[i + 1], None, None, Xbar, Hbar, pbar,
                                           taubar=tb, kappabar_a=kbar, kappabar_b=kbar)
                else:
                    self.plan.step_adjoint(n, ka, kb, Xseg[i], Xseg[i - 1], Xseg[i + 1], Yseg[i], Yseg[i - 1],
                                           Xbar, Hbar, pbar, taubar=tb, kappabar_a=kbar, kappabar_b=kbar,
                                           X_nm2=X2(n))
        gw, gl, gDe, gep, galpha = self.plan.pbar_to_params(pbar.cpu().numpy(), self.dw, self.dl)
        return kbar[:, :P].clone(), Xbar[0, :, :P].clone(), galpha, gDe, gep

    def release(self):
        self.ckpt = {}
        self.plan.close()


class TfsFunction(torch.autograd.Function):
    """tau^N = F(kappa, X0, alpha, De, eta_p); see the module docstring."""

    @staticmethod
    def forward(ctx, kappa, X0, alpha, De, eta_p, spec):
        run = Checkpointed(spec, X0.shape[1], float(alpha), float(De), float(eta_p), device=X0.device)
        tau = run.forward(kappa.detach(), X0.detach())
        ctx.run = run
        return tau

    @staticmethod
    def backward(ctx, tau_bar):
        run = ctx.run
        gk, gx, ga, gD, ge = run.backward(tau_bar.detach().to(torch.float64).contiguous())
        run.release()
        dev, dt = gk.device, torch.float64
        return gk, gx, torch.tensor(ga, dtype=dt, device=dev), torch.tensor(gD, dtype=dt, device=dev), \
            torch.tensor(ge, dtype=dt, device=dev), None


def fractional_stress(kappa, X0, alpha, De, eta_p, spec: Spec):
    """Differentiable final stress; alpha, De, eta_p are 0-d tensors (or floats)."""
    to_t = lambda x: x if torch.is_tensor(x) else torch.tensor(float(x), dtype=torch.float64, device=X0.device)
    return TfsFunction.apply(kappa, X0, to_t(alpha), to_t(De), to_t(eta_p), spec)


def run_slabs(spec: Spec, slabs, alpha, De, eta_p, loss_grad, device="cuda", keep_fields=False):
    """Forward + backward slab by slab (points are independent, so the parameter gradients
    are sums over slabs and the field gradients are slab-local).

    slabs: iterable of (kappa [d*d][P], X0 [c][P]) or (kappa, X0, levels) device
    tensors, or callables returning them; levels is kappa_levels(n, out), which replaces
    spec.kappa_levels for that slab, or a field tuple as Spec.field (with the slab's first
    grid point as point0), which replaces spec.field: a time-varying base field evaluated on
    the slab's points.
    loss_grad(tau [c][P], slab_index) -> (loss_value, dL/dtau).
    Returns dict: loss, alpha, De, eta_p (summed over slabs) and, with keep_fields, the
    per-slab (dL/dkappa, dL/dX0) on the host."""
    total = {"loss": 0.0, "alpha": 0.0, "De": 0.0, "eta_p": 0.0}
    fields = []
    for j, sl in enumerate(slabs):
        item = sl() if callable(sl) else sl
        kappa, X0 = item[0], item[1]
        sp = spec
        if len(item) > 2 and item[2] is not None:
            if isinstance(item[2], tuple):      # the slab's analytic field (tfs_field_eval)
                sp = dataclasses.replace(spec, field=item[2], kappa_levels=None)
            else:
                sp = dataclasses.replace(spec, kappa_levels=item[2])
        run = Checkpointed(sp, X0.shape[1], alpha, De, eta_p, device=device)
        tau = run.forward(kappa, X0)
        lv, tb = loss_grad(tau, j)
        gk, gx, ga, gD, ge = run.backward(tb)
        run.release()
        if keep_fields:
            fields.append((gk.cpu(), gx.cpu()))
        del run, tau, tb, gk, gx
        total["loss"] += lv
        total["alpha"] += ga
        total["De"] += gD
        total["eta_p"] += ge
    if keep_fields:
        total["fields"] = fields
    return total
