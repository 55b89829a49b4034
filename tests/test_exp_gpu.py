"""GPU parity of the exponential-mode scheme (TFS_SCHEME_EXP) with the oracle's, through
the C ABI.  Bars as for the paper's scheme: FP64 1e-12 and FP32 modes 1e-5, normwise per
field, for X at the last two levels, tau, the plain modes of the last level and the
diagnostics (the non-finite count exactly)."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import soe as osoe
from paper_2411_17294_amd import inputs as I
from paper_2411_17294_amd import tfs
from tests.gpu_helpers import relerr, run_gpu
from tests.test_parity_gpu import TOL, compare, small_case, _tv_kappa

pytestmark = pytest.mark.gpu


def _compare(g, o, prec, label):
    o1 = dict(o)
    if o.get("modes") is not None:
        o1["modes"] = o["modes"][:1]
    compare(g, o1, prec, modes="modes" in g, diag="diag" in g, label=label)


@pytest.mark.parametrize("prec", ["fp64", "fp32_modes"])
@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("P,nsteps", [(1, 1), (7, 2), (300, 17)])
def test_exp_small_random_cases(d, prec, P, nsteps):
    kappa, X0, w, lam = small_case(d, P, 100 + 10 * d + P)
    print(f"exp case d={d} prec={prec} P={P} N={nsteps}", flush=True)
    g = run_gpu(d, w, lam, 1.0, 0.1, 1e-3, nsteps, kappa, X0, precision=prec, want_modes=True, want_diag=True,
                scheme="exp")
    o = O.run(d, w, lam, 1.0, 0.1, 1e-3, nsteps, kappa, X0, want_modes=True, want_diag=True, startup="exp")
    _compare(g, o, prec, f"exp d={d} {prec} P={P} N={nsteps}")


@pytest.mark.parametrize("prec", ["fp64", "fp32_modes"])
@pytest.mark.parametrize("layout", ["untiled_padded", "tile4", "tile1024", "unaligned", "vec1", "vec2", "vec4"])
@pytest.mark.parametrize("d", [2, 3])
def test_exp_layouts_and_vector_widths(d, prec, layout):
    P, N = 1021, 9
    if layout == "vec4" and prec == "fp64":
        pytest.skip("4 points per lane exists for FP32 modes only")
    kappa, X0, w, lam = small_case(d, P, 70 + d)
    kw = {"untiled_padded": dict(tile=0, stride=1100), "tile4": dict(tile=4), "tile1024": dict(tile=1024),
          "unaligned": dict(offset=1)}.get(layout)
    if kw is None:
        kw = dict(vec=int(layout[-1]), stride=1024, tile=1024)
    print(f"exp layout {layout} d={d} {prec}", flush=True)
    g = run_gpu(d, w, lam, 0.8, 0.2, 1e-3, N, kappa, X0, precision=prec, want_modes=True, want_diag=True,
                scheme="exp", **kw)
    o = O.run(d, w, lam, 0.8, 0.2, 1e-3, N, kappa, X0, want_modes=True, want_diag=True, startup="exp")
    _compare(g, o, prec, f"exp {layout} d={d} {prec}")


@pytest.mark.parametrize("prec", ["fp64", "fp32_modes"])
@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("extrap", [True, False])
def test_exp_time_varying_kappa(d, prec, extrap):
    P, N, dt = 777, 30, 2e-3
    kap = _tv_kappa(d, P, N + 1, dt, 15 + d)
    _, X0 = I.random_symmetric_case(d, P, 19, xscale=1e-2)
    w, lam, _ = osoe.soe_fit(0.35, 9, dt, N * dt)
    print(f"exp time-varying d={d} {prec} extrap={extrap}", flush=True)
    g = run_gpu(d, w, lam, 1.3, 0.1, dt, N, kap, X0, precision=prec, extrap=extrap, want_modes=True,
                want_diag=True, scheme="exp")
    o = O.run(d, w, lam, 1.3, 0.1, dt, N, kap, X0, extrap=extrap, want_modes=True, want_diag=True, startup="exp")
    _compare(g, o, prec, f"exp tv d={d} {prec} extrap={extrap}")


@pytest.mark.parametrize("prec", ["fp64", "fp32_modes"])
def test_exp_workload_64sq_full_grid(prec):
    """64x64, alpha = 0.5, m = 20, 200 steps, dt = 1e-3 with the exponential-mode scheme."""
    wl = I.WORKLOADS[1]
    ff = I.fourier_field(wl)
    kap = ff.kappa_at(I.grid_multi_index(wl.grid, 2, np.arange(wl.npoints)), wl.grid, 0.0)
    X0 = I.initial_state(wl)
    w, lam, _ = osoe.soe_fit(wl.alphas[0], wl.nmodes, wl.dt, wl.dt * wl.nsteps)
    g = run_gpu(2, w, lam, wl.De, wl.eta_p, wl.dt, wl.nsteps, kap, X0, precision=prec, want_modes=True,
                want_diag=True, alpha=wl.alphas[0], scheme="exp")
    o = O.run(2, w, lam, wl.De, wl.eta_p, wl.dt, wl.nsteps, kap, X0, want_modes=True, want_diag=True,
              startup="exp")
    _compare(g, o, prec, f"exp 64^2 {prec}")


def test_exp_256cube_fp32_modes_subdomain():
    """256^3, alpha = 0.4, m = 40, 500 steps, dt = 2e-4, FP32 modes and FP32 kappa,
    exponential-mode scheme, full grid in the benchmark's launch configuration; the strided
    32^3 subset, where the GPU reads the host generator's kappa (FP32-rounded, as the oracle
    gets it), against the oracle (1e-5)."""
    from paper_2411_17294_amd.device_inputs import x0_ring
    wl = I.WORKLOADS[3]
    N, alpha = wl.nsteps, wl.alphas[0]
    ff = I.fourier_field(wl)
    w, lam, _ = osoe.soe_fit(alpha, wl.nmodes, wl.dt, wl.dt * N)
    plan = tfs.Plan(3, wl.npoints, w, lam, alpha, wl.De, wl.eta_p, wl.dt, N, precision="fp32_modes", scheme="exp",
                    kappa="fp32")
    plan.set_field(*ff.table(wl.grid))
    sub = I.subdomain_points(wl)
    subt = torch.from_numpy(sub).cuda()
    kap = ff.kappa_at(I.grid_multi_index(wl.grid, 3, sub), wl.grid, 0.0).astype(np.float32)
    k0 = plan.kappa_tensor()
    plan.field_eval(0.0, k0)
    k0[:, subt] = torch.from_numpy(kap).cuda()
    X = x0_ring(wl, plan.stride, levels=plan.x_levels)
    _, Y, tau, _ = plan.alloc()
    for n in range(N):
        plan.step(n, k0, k0 if n >= 1 else None, X, Y, tau)
    torch.cuda.synchronize()
    o = O.run(3, w, lam, wl.De, wl.eta_p, wl.dt, N, kap.astype(np.float64), I.initial_state(wl, sub),
              startup="exp")
    g = {"X": np.stack([X[N % 2][:, subt].cpu().numpy(), X[(N - 1) % 2][:, subt].cpu().numpy()]),
         "tau": tau[:, subt].cpu().numpy()}
    compare(g, o, "fp32_modes", modes=False, diag=False, label="exp 256^3 fp32 vs oracle on 32^3")


def test_exp_step_levels_in_place_equals_ring_step():
    """tfs_step_levels with Y_out aliasing Y_n gives bitwise the ring step's result."""
    d, P, N = 3, 2000, 6
    kappa, X0, w, lam = small_case(d, P, 5)
    a = run_gpu(d, w, lam, 1.0, 0.1, 1e-3, N, kappa, X0, scheme="exp")
    plan = tfs.Plan(d, P, w, lam, 0.5, 1.0, 0.1, 1e-3, N, scheme="exp")
    st, c = plan.stride, plan.c
    Xs = [torch.zeros((c, st), dtype=torch.float64, device="cuda") for _ in range(N + 1)]
    Xs[0][:, :P] = torch.from_numpy(X0).cuda()
    Y = torch.zeros((plan.m * c * st,), dtype=torch.float64, device="cuda")
    kd = plan.kappa_tensor(kappa)
    tau = torch.zeros((c, st), dtype=torch.float64, device="cuda")
    for n in range(N):
        plan.step_levels(n, kd, kd if n >= 1 else None, Xs[n], None, Xs[n + 1], Y, None, Y, tau)
    torch.cuda.synchronize()
    assert np.array_equal(Xs[N][:, :P].cpu().numpy(), a["X"][0])
    assert np.array_equal(tau[:, :P].cpu().numpy(), a["tau"])


# ---------------------------------------------------------------- adjoint of the exponential scheme
from tests.grad_helpers import gpu_gradients, oracle_gradients   # noqa: E402
from tests.test_adjoint_gpu import BAR, compare as compare_grads, setup as grad_setup   # noqa: E402


@pytest.mark.parametrize("prec", ["fp64", "fp32_modes"])
@pytest.mark.parametrize("d", [2, 3])
@pytest.mark.parametrize("P,N", [(1, 1), (5, 2), (37, 12)])
def test_exp_adjoint_matches_oracle(d, prec, P, N):
    """dL/dkappa, dL/dX0, dL/dDe, dL/deta_p, dL/dalpha and the per-mode dL/dw_k, dL/dlambda_k
    against the oracle's complex-step derivatives of the exponential scheme."""
    m = 5
    kappa, X0, w, lam, dw, dl, target = grad_setup(d, P, m, 600 + 10 * d + P)
    print(f"exp adjoint d={d} {prec} P={P} N={N}", flush=True)
    o = oracle_gradients(d, w, lam, 1.1, 0.1, 2e-3, N, kappa, X0, target, dw_da=dw, dl_da=dl, per_mode=True,
                         scheme="exp")
    g = gpu_gradients(d, w, lam, 0.45, 1.1, 0.1, 2e-3, N, kappa, X0, target, precision=prec, dw_da=dw, dl_da=dl,
                      scheme="exp")
    compare_grads(g, o, prec, label=f"exp adj d={d} {prec} P={P} N={N}")


@pytest.mark.parametrize("tile", [None, 64])
@pytest.mark.parametrize("adj_vec", [1, 2])
@pytest.mark.parametrize("prec", ["fp64", "fp32_modes"])
@pytest.mark.parametrize("d", [2, 3])
def test_exp_adjoint_whole_waves_and_tail(d, prec, adj_vec, tile):
    P, N, m = 389, 6, 7
    kappa, X0, w, lam, dw, dl, target = grad_setup(d, P, m, 700 + d)
    print(f"exp adjoint waves d={d} {prec} adj_vec={adj_vec} tile={tile}", flush=True)
    o = oracle_gradients(d, w, lam, 1.1, 0.1, 2e-3, N, kappa, X0, target, dw_da=dw, dl_da=dl, scheme="exp")
    g = gpu_gradients(d, w, lam, 0.45, 1.1, 0.1, 2e-3, N, kappa, X0, target, precision=prec, tile=tile,
                      dw_da=dw, dl_da=dl, tune={"adj_vec": adj_vec}, scheme="exp")
    compare_grads(g, o, prec, per_mode=False, label=f"exp adj waves d={d} {prec} V={adj_vec} tile={tile}")


@pytest.mark.parametrize("extrap", [True, False])
@pytest.mark.parametrize("d", [2, 3])
def test_exp_adjoint_time_varying_kappa(d, extrap):
    P, N, m, dt = 23, 15, 6, 2e-3
    rng = np.random.default_rng(80 + d)
    a, b, om = (rng.standard_normal((d * d, P)) * 0.6 for _ in range(3))
    t = np.arange(N + 1)[:, None, None] * dt
    kap = np.ascontiguousarray(a[None] + b[None] * np.sin(3.0 * t + om[None]))
    _, X0, w, lam, dw, dl, target = grad_setup(d, P, m, 90 + d)
    print(f"exp adjoint tv d={d} extrap={extrap}", flush=True)
    o = oracle_gradients(d, w, lam, 0.9, 0.2, dt, N, kap, X0, target, dw_da=dw, dl_da=dl, extrap=extrap,
                         scheme="exp")
    g = gpu_gradients(d, w, lam, 0.45, 0.9, 0.2, dt, N, kap, X0, target, dw_da=dw, dl_da=dl, extrap=extrap,
                      scheme="exp")
    compare_grads(g, o, "fp64", per_mode=False, label=f"exp adj tv d={d} extrap={extrap}")


def test_exp_adjoint_alpha_against_gpu_finite_differences():
    d, P, N, m = 3, 200, 20, 8
    kappa, X0, w, lam, dw, dl, target = grad_setup(d, P, m, 177)
    alpha, dt, T = 0.45, 2e-3, 0.05
    _, _, info = osoe.soe_fit(alpha, m, dt, T)
    g = gpu_gradients(d, w, lam, alpha, 1.1, 0.1, dt, N, kappa, X0, target, dw_da=dw, dl_da=dl, scheme="exp")

    def L(al, De):
        wa, la, _, _ = osoe.soe_gl_log(al, m, info["y_lo"], info["y_hi"])
        return gpu_gradients(d, wa, la, al, De, 0.1, dt, N, kappa, X0, target, scheme="exp")["loss"]
    h = 1e-4 * alpha
    fd_a = (L(alpha + h, 1.1) - L(alpha - h, 1.1)) / (2 * h)
    hD = 1e-4 * 1.1
    fd_D = (L(alpha, 1.1 + hD) - L(alpha, 1.1 - hD)) / (2 * hD)
    print("exp FD alpha", fd_a, g["alpha"], "De", fd_D, g["De"], flush=True)
    assert abs(fd_a - g["alpha"]) <= 1e-6 * abs(fd_a)
    assert abs(fd_D - g["De"]) <= 1e-6 * abs(fd_D)
