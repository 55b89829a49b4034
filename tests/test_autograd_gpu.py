"""Checkpointed forward + adjoint behind torch.autograd (differentiation form)."""
import math

import numpy as np
import pytest
import torch

from oracle import soe as osoe
from paper_2411_17294_amd import inputs as I
from paper_2411_17294_amd.autograd import Checkpointed, Spec, fractional_stress
from oracle import oracle as O
from tests.gpu_helpers import as_fp32, relerr
from tests.grad_helpers import gpu_gradients, oracle_gradients, pack_weights

pytestmark = pytest.mark.gpu


def _case(d, P, seed, m=6, alpha=0.5, dt=2e-3, N=17):
    kappa, X0 = I.random_symmetric_case(d, P, seed, kscale=0.6, xscale=2e-2)
    _, _, info = osoe.soe_fit(alpha, m, dt, dt * N)
    target = np.random.default_rng(seed).standard_normal((d * (d + 1) // 2, P)) * 1e-3
    return kappa, X0, info, target


@pytest.mark.parametrize("scheme", ["bdf2", "exp"])
@pytest.mark.parametrize("prec", ["fp64", "fp32_modes"])
@pytest.mark.parametrize("K", [1, 4, 17, 50])
def test_checkpointed_equals_uncheckpointed_and_oracle(prec, K, scheme):
    d, P, N, m, alpha, De, eta_p, dt = 3, 41, 17, 6, 0.5, 1.2, 0.1, 2e-3
    kappa, X0, info, target = _case(d, P, 5, m=m, alpha=alpha, dt=dt, N=N)
    spec = Spec(dim=d, nmodes=m, dt=dt, nsteps=N, y_lo=info["y_lo"], y_hi=info["y_hi"], ckpt_every=K,
                precision=prec, scheme=scheme)
    kt = torch.from_numpy(kappa).cuda().requires_grad_(True)
    xt = torch.from_numpy(X0).cuda().requires_grad_(True)
    at = torch.tensor(alpha, dtype=torch.float64, device="cuda", requires_grad=True)
    Dt = torch.tensor(De, dtype=torch.float64, device="cuda", requires_grad=True)
    et = torch.tensor(eta_p, dtype=torch.float64, device="cuda", requires_grad=True)
    tau = fractional_stress(kt, xt, at, Dt, et, spec)
    wts = torch.from_numpy(pack_weights(d)[:, None]).cuda()
    L = 0.5 * torch.sum(wts * (tau - torch.from_numpy(target).cuda()) ** 2)
    L.backward()
    w, lam, dw, dl = osoe.soe_gl_log(alpha, m, info["y_lo"], info["y_hi"])
    ref = gpu_gradients(d, w, lam, alpha, De, eta_p, dt, N, kappa, X0, target, precision=prec, dw_da=dw, dl_da=dl,
                        scheme=scheme)
    ek = relerr(kt.grad.cpu().numpy(), ref["kappa"])
    ex = relerr(xt.grad.cpu().numpy(), ref["X0"])
    print(f"checkpointed K={K} {prec} {scheme}: kappa {ek:.2e} X0 {ex:.2e}", flush=True)
    # the same kernels on the same inputs: equal up to the order of the block sums, and in the
    # FP32-mode form up to an FP32 rounding of a recomputed mode tipping the other way
    bar = 1e-13 if prec == "fp64" else 1e-11
    assert ek < bar and ex < bar
    assert at.grad.item() == pytest.approx(ref["alpha"], rel=bar)
    assert Dt.grad.item() == pytest.approx(ref["De"], rel=bar)
    assert et.grad.item() == pytest.approx(ref["eta_p"], rel=bar)
    if prec == "fp64" and K == 4:
        o = oracle_gradients(d, w, lam, De, eta_p, dt, N, kappa, X0, target, dw_da=dw, dl_da=dl, scheme=scheme)
        assert relerr(kt.grad.cpu().numpy(), o["kappa"]) < 1e-12
        assert relerr(xt.grad.cpu().numpy(), o["X0"]) < 1e-12
        assert abs(at.grad.item() - o["alpha"]) < 1e-12 * abs(o["alpha"])
        assert abs(Dt.grad.item() - o["De"]) < 1e-12 * abs(o["De"])


def test_time_varying_perturbation_gradient():
    """kappa^n = f(t_n) + p with p the differentiable steady perturbation."""
    d, P, N, m, dt = 2, 30, 12, 5, 2e-3
    rng = np.random.default_rng(9)
    a, b, om = (rng.standard_normal((d * d, P)) * 0.5 for _ in range(3))
    levels = np.stack([a + b * np.sin(4.0 * n * dt + om) for n in range(N + 1)])
    _, X0, info, target = _case(d, P, 11, m=m, dt=dt, N=N)
    lev_t = torch.from_numpy(levels).cuda()

    def kappa_levels(n, out):
        out.zero_()
        out[:, :P] = lev_t[n]
    spec = Spec(dim=d, nmodes=m, dt=dt, nsteps=N, y_lo=info["y_lo"], y_hi=info["y_hi"], ckpt_every=5,
                precision="fp64", kappa_levels=kappa_levels)
    pert = torch.zeros((d * d, P), dtype=torch.float64, device="cuda", requires_grad=True)
    xt = torch.from_numpy(X0).cuda()
    tau = fractional_stress(pert, xt, 0.5, 1.0, 0.1, spec)
    wts = torch.from_numpy(pack_weights(d)[:, None]).cuda()
    L = 0.5 * torch.sum(wts * (tau - torch.from_numpy(target).cuda()) ** 2)
    L.backward()
    w, lam, dw, dl = osoe.soe_gl_log(0.5, m, info["y_lo"], info["y_hi"])
    o = oracle_gradients(d, w, lam, 1.0, 0.1, dt, N, levels, X0, target)
    assert relerr(pert.grad.cpu().numpy(), o["kappa"]) < 1e-12


def test_workload_128cube_differentiation():
    """128^3, FP32 modes and FP32 kappa, alpha = 0.6, m = 32, 400 steps, dt = 2.5e-4,
    checkpoints every 50.  Loss: misfit of tau^N against a target made with alpha = 0.55 and
    De * 1.05 (same kappa, X0 and fit window).  Checked: dL/dalpha and dL/dDe against central
    differences of the GPU forward (h = 1e-4 relative); on the strided 16^3 subset, dL/dkappa
    and dL/dX0 against the oracle's complex-step derivatives, and dL/dalpha and dL/dDe of the
    subset's own loss (a second backward pass with taubar zero off the subset) against the
    oracle's derivatives of that loss, all at the FP32-rounded kappa the GPU reads."""
    from paper_2411_17294_amd.device_inputs import DeviceKappa
    wl = I.WORKLOADS[4]
    alpha, N, m, dt = wl.alphas[0], wl.nsteps, wl.nmodes, wl.dt
    _, _, info = osoe.soe_fit(alpha, m, dt, dt * N)
    ff = I.fourier_field(wl)
    P = wl.npoints
    kd = torch.zeros((9, P), dtype=torch.float32, device="cuda")
    DeviceKappa(ff, wl.grid, P).fill(kd, 0.0)
    kd = kd.double()                  # FP32 values; the differentiable input is FP64
    X0 = torch.from_numpy(I.initial_state(wl)).cuda()
    spec = Spec(dim=3, nmodes=m, dt=dt, nsteps=N, y_lo=info["y_lo"], y_hi=info["y_hi"],
                ckpt_every=wl.ckpt_every, precision="fp32_modes", kappa="fp32")

    def fwd(al, De):
        r = Checkpointed(spec, P, al, De, wl.eta_p)
        t = r.forward(kd, X0)
        r.release()
        return t
    target = fwd(wl.target_alpha, wl.De * wl.target_De_factor)
    wts = torch.from_numpy(pack_weights(3)[:, None]).cuda()
    lossf = lambda t: 0.5 * float(torch.sum(wts * (t - target) ** 2))
    run = Checkpointed(spec, P, alpha, wl.De, wl.eta_p)
    tau = run.forward(kd, X0)
    L0 = lossf(tau)
    gk, gx, ga, gD, ge = run.backward(wts * (tau - target))
    sub = I.subdomain_points(wl)
    subt = torch.from_numpy(sub).cuda()
    tb_sub = torch.zeros_like(tau)
    tb_sub[:, subt] = (wts * (tau - target))[:, subt]
    _, _, ga_s, gD_s, _ = run.backward(tb_sub)
    run.release()
    torch.cuda.synchronize()
    ha, hD = 1e-4 * alpha, 1e-4 * wl.De
    fd_a = (lossf(fwd(alpha + ha, wl.De)) - lossf(fwd(alpha - ha, wl.De))) / (2 * ha)
    fd_D = (lossf(fwd(alpha, wl.De + hD)) - lossf(fwd(alpha, wl.De - hD))) / (2 * hD)
    print(f"128^3: L={L0:.6e} dL/dalpha adj {ga:.10e} fd {fd_a:.10e}; dL/dDe adj {gD:.10e} fd {fd_D:.10e}",
          flush=True)
    # FP32 mode storage: the finite difference of the FP32-mode forward resolves ~1e-5
    assert abs(ga - fd_a) <= 1e-4 * abs(fd_a)
    assert abs(gD - fd_D) <= 1e-4 * abs(fd_D)
    # the subset against the oracle (each point's gradient depends on that point only)
    w, lam, dw, dl = osoe.soe_gl_log(alpha, m, info["y_lo"], info["y_hi"])
    kap_s = kd[:, subt].cpu().numpy()
    X0_s = X0[:, subt].cpu().numpy()
    tgt_s = target[:, subt].cpu().numpy()
    o = oracle_gradients(3, w, lam, wl.De, wl.eta_p, dt, N, kap_s, X0_s, tgt_s, dw_da=dw, dl_da=dl)
    errs = {"tau": relerr(tau[:, subt].cpu().numpy(), O.run(3, w, lam, wl.De, wl.eta_p, dt, N, kap_s, X0_s)["tau"]),
            "dL/dkappa": relerr(gk[:, subt].cpu().numpy(), o["kappa"]),
            "dL/dX0": relerr(gx[:, subt].cpu().numpy(), o["X0"]),
            "dL/dalpha (subset loss)": abs(ga_s - o["alpha"]) / abs(o["alpha"]),
            "dL/dDe (subset loss)": abs(gD_s - o["De"]) / abs(o["De"])}
    print("128^3 subset vs oracle:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    assert max(errs.values()) < 1e-5, errs


def test_workload_384cube_slab_full_length():
    """The 384^3 configuration at full length on one slab of the grid (884736 consecutive
    points, the slab the whole-grid job runs 64 of): alpha = 0.2, m = 48, 2000 steps,
    dt = 1e-4, the time-varying field, FP32 modes and FP32 kappa, checkpoints every 100.
    Loss: 1/2 sum ||tau^N||_F^2 over a strided subset of 256 points of the slab (taubar zero
    elsewhere), where the GPU reads the host generator's kappa levels.  Against the oracle on
    those points, at the FP32-rounded levels: X^N, tau^N, dL/dkappa (a steady perturbation
    of every level), dL/dX0, dL/dalpha and dL/dDe, each within 1e-5."""
    from paper_2411_17294_amd.device_inputs import DeviceKappa
    wl = I.WORKLOADS[5]
    alpha, m, dt, N, K = wl.alphas[0], wl.nmodes, wl.dt, wl.nsteps, wl.ckpt_every
    S = wl.npoints // 64
    off = 17 * S
    _, _, info = osoe.soe_fit(alpha, m, dt, dt * N)
    ff = I.fourier_field(wl)
    sub = np.arange(0, S, S // 256)[:256]
    subt = torch.from_numpy(sub).cuda()
    idx = I.grid_multi_index(wl.grid, 3, off + sub)
    kap = np.stack([ff.kappa_at(idx, wl.grid, n * dt) for n in range(N + 1)])
    kap_dev = torch.from_numpy(kap).cuda()
    dk = DeviceKappa(ff, wl.grid, S, offset=off)

    def levels(n, out):
        dk.fill(out, n * dt)
        out[:, subt] = kap_dev[n]                # the parity points read the host generator's values
    spec = Spec(dim=3, nmodes=m, dt=dt, nsteps=N, y_lo=info["y_lo"], y_hi=info["y_hi"], ckpt_every=K,
                precision="fp32_modes", kappa="fp32", kappa_levels=levels)
    X0 = torch.from_numpy(I.initial_state(wl, off + np.arange(S))).cuda()
    pert = torch.zeros((9, S), dtype=torch.float64, device="cuda")
    wts = torch.from_numpy(pack_weights(3)[:, None]).cuda()
    print(f"384^3 slab [{off}, {off + S}), {N} steps, checkpoints every {K}", flush=True)
    run = Checkpointed(spec, S, alpha, wl.De, wl.eta_p)
    tau = run.forward(pert, X0)
    X_N = run.X_last
    tb = torch.zeros_like(tau)
    tb[:, subt] = (wts * tau)[:, subt]
    gk, gx, ga, gD, ge = run.backward(tb)
    run.release()
    torch.cuda.synchronize()
    print("GPU done", flush=True)
    w, lam, dw, dl = osoe.soe_gl_log(alpha, m, info["y_lo"], info["y_hi"])
    kin = as_fp32(kap)
    X0_s = X0[:, subt].cpu().numpy()
    base = O.run(3, w, lam, wl.De, wl.eta_p, dt, N, kin, X0_s)
    o = oracle_gradients(3, w, lam, wl.De, wl.eta_p, dt, N, kin, X0_s, np.zeros((6, len(sub))), dw_da=dw, dl_da=dl)
    errs = {"X^N": relerr(X_N[:, subt].cpu().numpy(), base["X"][0]),
            "tau^N": relerr(tau[:, subt].cpu().numpy(), base["tau"]),
            "dL/dkappa": relerr(gk[:, subt].cpu().numpy(), o["kappa"]),
            "dL/dX0": relerr(gx[:, subt].cpu().numpy(), o["X0"]),
            "dL/dalpha": abs(ga - o["alpha"]) / abs(o["alpha"]),
            "dL/dDe": abs(gD - o["De"]) / abs(o["De"])}
    print("384^3 slab, full length, vs oracle:", {k: f"{v:.2e}" for k, v in errs.items()}, flush=True)
    # off the subset taubar is zero, so the field gradients vanish there
    mask = torch.ones(S, dtype=torch.bool, device="cuda")
    mask[subt] = False
    assert float(gk[:, mask].abs().max()) == 0.0 and float(gx[:, mask].abs().max()) == 0.0
    assert max(errs.values()) < 1e-5, errs


def test_slabs_match_one_run_time_varying_384cube_field():
    """Point slabs of the 384^3 configuration's time-varying field (alpha = 0.2, m = 48,
    dt = 1e-4, FP32 modes): three slabs of 20000 consecutive grid points run one after the
    other give the same parameter gradients (up to summation order) and bitwise the same
    field gradients as one run over all 60000 points; dL/dkappa and dL/dX0 at 40 of the
    points match the oracle's complex-step derivatives."""
    from paper_2411_17294_amd.autograd import run_slabs
    from paper_2411_17294_amd.device_inputs import DeviceKappa
    wl = I.WORKLOADS[5]
    alpha, m, dt, N, K = wl.alphas[0], wl.nmodes, wl.dt, 24, 10
    _, _, info = osoe.soe_fit(alpha, m, dt, dt * N)
    ff = I.fourier_field(wl)
    off, S, nslab = 7 * 384 * 384 + 1000, 20000, 3
    P = S * nslab
    pts = np.arange(off, off + P)
    X0 = torch.from_numpy(I.initial_state(wl, pts)).cuda()
    zero_k = torch.zeros((9, P), dtype=torch.float64, device="cuda")
    wts = torch.from_numpy(pack_weights(3)[:, None]).cuda()

    def levels_fn(o, n_pts):
        dk = DeviceKappa(ff, wl.grid, n_pts, offset=o)
        return lambda n, out: dk.fill(out, n * dt)
    spec = Spec(dim=3, nmodes=m, dt=dt, nsteps=N, y_lo=info["y_lo"], y_hi=info["y_hi"], ckpt_every=K,
                precision="fp32_modes")

    def loss_grad(tau, j):
        return 0.5 * float(torch.sum(wts * tau * tau)), (wts * tau).contiguous()
    one = run_slabs(spec, [(zero_k, X0, levels_fn(off, P))], alpha, wl.De, wl.eta_p, loss_grad, keep_fields=True)
    sl = [(zero_k[:, j * S:(j + 1) * S].contiguous(), X0[:, j * S:(j + 1) * S].contiguous(), levels_fn(off + j * S, S))
          for j in range(nslab)]
    many = run_slabs(spec, sl, alpha, wl.De, wl.eta_p, loss_grad, keep_fields=True)
    for key in ("loss", "alpha", "De", "eta_p"):
        print(f"slabs {key}: one {one[key]:.15e} slabs {many[key]:.15e}", flush=True)
        assert many[key] == pytest.approx(one[key], rel=1e-12)
    gk1, gx1 = one["fields"][0]
    gk = torch.cat([f[0] for f in many["fields"]], dim=1)
    gx = torch.cat([f[1] for f in many["fields"]], dim=1)
    assert torch.equal(gk, gk1) and torch.equal(gx, gx1)
    # oracle on a subset of the points (each point's gradient depends on that point only)
    sub = np.random.default_rng(5).choice(P, 40, replace=False)
    idx = I.grid_multi_index(wl.grid, 3, pts[sub])
    kap = np.stack([ff.kappa_at(idx, wl.grid, n * dt) for n in range(N + 1)])
    w, lam, dw, dl = osoe.soe_gl_log(alpha, m, info["y_lo"], info["y_hi"])
    o = oracle_gradients(3, w, lam, wl.De, wl.eta_p, dt, N, kap, X0[:, sub].cpu().numpy(),
                         np.zeros((6, len(sub))))
    ek = relerr(gk1[:, sub].numpy(), o["kappa"])
    ex = relerr(gx1[:, sub].numpy(), o["X0"])
    print(f"slab subset vs oracle: dL/dkappa {ek:.2e}, dL/dX0 {ex:.2e}", flush=True)
    assert ek < 1e-5 and ex < 1e-5
