"""Temporally fused exponential-mode steps (tfs_run_fused): K time levels per launch with
kappa evaluated from the analytic Fourier field inside the kernel, against the oracle
(kappa levels from the same field definition in numpy) and against the step-by-step GPU
path fed with those levels, for the exponential scheme and for the paper's BDF2 scheme
(after its SDIRK2 start).  Launches of 69 and more steps pass the points where the kernel
re-evaluates the rotated field terms with a fresh sincos."""
import numpy as np
import pytest
import torch

from oracle import oracle as O
from oracle import soe as osoe
from paper_2411_17294_amd import inputs as I
from paper_2411_17294_amd import tfs
from tests.gpu_helpers import relerr

pytestmark = pytest.mark.gpu


def field_of(wl_id, steady):
    ff = I.fourier_field(I.WORKLOADS[wl_id])
    if steady:
        ff.omega = np.zeros_like(ff.omega)
    return ff


def make_plan(d, P, m, prec, dt, N, alpha=0.5, De=1.0, eta_p=0.1, scheme="exp"):
    w, lam, _ = osoe.soe_fit(alpha, m, dt, dt * N * 10)
    # fused launches keep the modes in the Y form
    plan = tfs.Plan(d, P, w, lam, alpha, De, eta_p, dt, N, precision=prec, scheme=scheme, mode_form="y")
    return plan, w, lam


def levels(ff, grid, points, dt, N):
    idx = I.grid_multi_index(grid, ff.dim, points)
    return np.stack([ff.kappa_at(idx, grid, n * dt) for n in range(N + 1)])      # [N+1][d*d][P]


def fused_run(plan, ff, grid, point0, X0, chunks, kap0=None):
    """Fused launches of the given step counts from level 0; returns X ring, Y, tau.  For
    BDF2 plans the first level comes from tfs_step (the SDIRK2 start) with kappa level kap0."""
    d, c, st, P = plan.dim, plan.c, plan.stride, plan.npoints
    plan.set_field(ff.k, ff.phase, ff.omega, ff.coef(), grid, point0)
    X, Y, tau, _ = plan.alloc()
    X[0, :, :P] = torch.from_numpy(X0).cuda()
    n0 = 0
    if kap0 is not None:
        k0 = torch.zeros((d * d, st), dtype=torch.float64, device="cuda")
        k0[:, :P] = torch.from_numpy(kap0).cuda()
        plan.step(0, k0, None, X, Y, tau)
        n0 = 1
    for K in chunks:
        plan.run_fused(n0, K, X, Y, tau)
        n0 += K
    torch.cuda.synchronize()
    return X, Y, tau, n0


def stepwise_run(plan, kap_levels, X0, N):
    d, c, st, P = plan.dim, plan.c, plan.stride, plan.npoints
    X, Y, tau, _ = plan.alloc()
    X[0, :, :P] = torch.from_numpy(X0).cuda()
    lv = []
    for n in range(N + 1):
        t = torch.zeros((d * d, st), dtype=torch.float64, device="cuda")
        t[:, :P] = torch.from_numpy(kap_levels[n]).cuda()
        lv.append(t)
    for n in range(N):
        plan.step(n, lv[n], lv[n - 1] if n >= 1 else None, X, Y, tau)
    torch.cuda.synchronize()
    return X, Y, tau


def plain_modes(plan, X, Y, level):
    o = torch.zeros((plan.m, plan.c, plan.stride), dtype=torch.float64, device="cuda")
    plan.modes_to_plain(level, X, Y, o)
    torch.cuda.synchronize()
    return o[:, :, :plan.npoints].cpu().numpy()


CASES = [(2, "fp64", 16, 32, False), (2, "fp64", 32, 32, False), (2, "fp32_modes", 32, 32, False),
         (2, "fp32_modes", 16, 32, True), (3, "fp32_modes", 32, 12, False), (3, "fp32_modes", 16, 12, True)]


@pytest.mark.parametrize("d,prec,m,grid,steady", CASES)
@pytest.mark.parametrize("chunks", [(1,), (13,), (4, 1, 8), (70,), (33, 31)])
def test_fused_matches_oracle_and_stepwise_path(d, prec, m, grid, steady, chunks):
    wl_id = 2 if d == 2 else 5
    ff = field_of(wl_id, steady)
    P = grid ** d - 7                                   # not a multiple of the block or the pair
    point0 = 5
    N = sum(chunks)
    dt = 2e-3
    plan, w, lam = make_plan(d, P, m, prec, dt, N)
    X0 = I.random_symmetric_case(d, P, 41, kscale=0.6, xscale=2e-2)[1]
    points = np.arange(point0, point0 + P)
    kl = levels(ff, grid, points, dt, N)
    X, Y, tau, n_end = fused_run(plan, ff, grid, point0, X0, chunks)
    Xs, Ys, taus = stepwise_run(plan, kl, X0, N)
    o = O.run(d, w, lam, 1.0, 0.1, dt, N, kl, X0, startup="exp", want_modes=True)
    bar = 1e-12 if prec == "fp64" else 1e-5
    got = {"X": np.stack([X[N % 2, :, :P].cpu().numpy(), X[(N - 1) % 2, :, :P].cpu().numpy()]),
           "tau": tau[:, :P].cpu().numpy(), "modes": plain_modes(plan, X, Y, N)}
    step = {"X": np.stack([Xs[N % 2, :, :P].cpu().numpy(), Xs[(N - 1) % 2, :, :P].cpu().numpy()]),
            "tau": taus[:, :P].cpu().numpy(), "modes": plain_modes(plan, Xs, Ys, N)}
    errs = {k: relerr(got[k], o[k][0] if k == "modes" else o[k]) for k in got}
    errs_step = {k: relerr(got[k], step[k]) for k in got}
    print(d, prec, m, steady, chunks, "oracle", errs, "stepwise", errs_step, flush=True)
    assert all(e < bar for e in errs.values()), errs
    assert all(e < bar for e in errs_step.values()), errs_step


def test_fused_full_size_128cube_sampled():
    """The 128^3, m = 32, FP32-mode configuration with a time-varying field, 40 steps in two
    launches, in the benchmark's launch configuration: 48 sampled points against the oracle."""
    wl = I.WORKLOADS[4]
    ff = field_of(5, False)
    g, d, m, dt, N = 128, 3, 32, 2.5e-4, 40
    P = g ** 3
    plan, w, lam = make_plan(d, P, m, "fp32_modes", dt, N, alpha=wl.alphas[0], De=wl.De, eta_p=wl.eta_p)
    X0 = I.initial_state(wl)
    X, Y, tau, _ = fused_run(plan, ff, g, 0, X0, (25, 15))
    rng = np.random.default_rng(4)
    sample = np.unique(np.concatenate([[0, P - 1], rng.choice(P, 46, replace=False)]))
    kl = levels(ff, g, sample, dt, N)
    o = O.run(d, w, lam, wl.De, wl.eta_p, dt, N, kl, X0[:, sample], startup="exp", want_modes=True)
    sel = torch.from_numpy(sample).cuda()
    ex = relerr(X[N % 2][:, sel].cpu().numpy(), o["X"][0])
    et = relerr(tau[:, sel].cpu().numpy(), o["tau"])
    em = relerr(plain_modes(plan, X, Y, N)[:, :, sample], o["modes"][0])
    print("128^3 fused sample", ex, et, em, flush=True)
    assert ex < 1e-5 and et < 1e-5 and em < 1e-5


def test_fused_errors_and_noop():
    ff = field_of(2, False)
    plan, _, _ = make_plan(2, 100, 16, "fp64", 1e-3, 10)
    X, Y, tau, _ = plan.alloc()
    with pytest.raises(tfs.TfsError):              # no field yet
        plan.run_fused(0, 1, X, Y, tau)
    plan.set_field(ff.k, ff.phase, ff.omega, ff.coef(), 32, 0)
    with pytest.raises(tfs.TfsError):              # past max_steps
        plan.run_fused(5, 6, X, Y, tau)
    with pytest.raises(tfs.TfsError):              # points outside the grid
        plan.set_field(ff.k, ff.phase, ff.omega, ff.coef(), 32, 32 * 32 - 50)
    X[0].fill_(0.25)
    before = X.clone()
    plan.run_fused(3, 0, X, Y, tau)                # nothing to do
    torch.cuda.synchronize()
    assert torch.equal(X, before)
    bad, _, _ = make_plan(2, 100, 20, "fp64", 1e-3, 10)
    bad.set_field(ff.k, ff.phase, ff.omega, ff.coef(), 32, 0)
    with pytest.raises(tfs.TfsError):              # m = 20 has no fused variant
        bad.run_fused(0, 1, *bad.alloc()[:3])
    w, lam, _ = osoe.soe_fit(0.5, 16, 1e-3, 1e-2)
    bdf = tfs.Plan(2, 100, w, lam, 0.5, 1.0, 0.1, 1e-3, 10)
    bdf.set_field(ff.k, ff.phase, ff.omega, ff.coef(), 32, 0)
    with pytest.raises(tfs.TfsError):              # BDF2 fused launches start after the SDIRK2 step
        bdf.run_fused(0, 1, *bdf.alloc()[:3])


BDF2_CASES = [(2, "fp64", 32, 32, False), (2, "fp32_modes", 16, 32, True), (2, "fp64", 16, 32, True),
              (3, "fp32_modes", 32, 12, False), (3, "fp32_modes", 16, 12, True)]


@pytest.mark.parametrize("d,prec,m,grid,steady", BDF2_CASES)
@pytest.mark.parametrize("chunks", [(1,), (12,), (4, 1, 7), (69,)])
def test_fused_bdf2_matches_oracle_and_stepwise_path(d, prec, m, grid, steady, chunks):
    """The paper's scheme fused: the SDIRK2 start by tfs_step, then levels 1 -> N in fused
    launches, against the oracle (SDIRK2 + BDF2 with the extrapolated kappa levels) and the
    step-by-step GPU path."""
    ff = field_of(2 if d == 2 else 5, steady)
    P = grid ** d - 7
    point0 = 5
    N = 1 + sum(chunks)
    dt = 2e-3
    plan, w, lam = make_plan(d, P, m, prec, dt, N, scheme="bdf2")
    X0 = I.random_symmetric_case(d, P, 43, kscale=0.6, xscale=2e-2)[1]
    kl = levels(ff, grid, np.arange(point0, point0 + P), dt, N)
    X, Y, tau, _ = fused_run(plan, ff, grid, point0, X0, chunks, kap0=kl[0])
    Xs, Ys, taus = stepwise_run(plan, kl, X0, N)
    o = O.run(d, w, lam, 1.0, 0.1, dt, N, kl, X0, startup="sdirk2", want_modes=True)
    bar = 1e-12 if prec == "fp64" else 1e-5
    got = {"X": np.stack([X[N % 2, :, :P].cpu().numpy(), X[(N - 1) % 2, :, :P].cpu().numpy()]),
           "tau": tau[:, :P].cpu().numpy(),
           "modes": np.stack([plain_modes(plan, X, Y, N), plain_modes(plan, X, Y, N - 1)])}
    step = {"X": np.stack([Xs[N % 2, :, :P].cpu().numpy(), Xs[(N - 1) % 2, :, :P].cpu().numpy()]),
            "tau": taus[:, :P].cpu().numpy(),
            "modes": np.stack([plain_modes(plan, Xs, Ys, N), plain_modes(plan, Xs, Ys, N - 1)])}
    errs = {k: relerr(got[k], o[k]) for k in got}
    errs_step = {k: relerr(got[k], step[k]) for k in got}
    print("bdf2", d, prec, m, steady, chunks, "oracle", errs, "stepwise", errs_step, flush=True)
    assert all(e < bar for e in errs.values()), errs
    assert all(e < bar for e in errs_step.values()), errs_step


def test_fused_bdf2_needs_the_start_step():
    ff = field_of(2, False)
    plan, _, _ = make_plan(2, 100, 16, "fp64", 1e-3, 10, scheme="bdf2")
    plan.set_field(ff.k, ff.phase, ff.omega, ff.coef(), 32, 0)
    with pytest.raises(tfs.TfsError):
        plan.run_fused(0, 3, *plan.alloc()[:3])


def many_terms_field(d, nterms, seed, steady):
    """A field of nterms terms (the workload's terms repeated at new phases and rates): its
    table is too large for the fused kernels' LDS copy, so they read it from global memory."""
    base = I.fourier_field(I.WORKLOADS[2 if d == 2 else 5])
    rng = np.random.default_rng(seed)
    reps = -(-nterms // len(base.amp))
    k = np.tile(base.k, (reps, 1))[:nterms]
    e = np.tile(base.e, (reps, 1))[:nterms]
    amp = np.tile(base.amp, reps)[:nterms] / reps
    phase = rng.uniform(0.0, 2.0 * np.pi, nterms)
    omega = np.zeros(nterms) if steady else rng.uniform(0.5, 2.0, nterms)
    return I.FourierField(d, k, e, amp, phase, omega)


@pytest.mark.parametrize("scheme", ["exp", "bdf2"])
@pytest.mark.parametrize("d,prec,nterms", [(3, "fp32_modes", 300), (2, "fp64", 450)])
@pytest.mark.parametrize("steady", [True, False])
def test_fused_large_field_table(d, prec, nterms, steady, scheme):
    """A field table larger than the LDS copy (300 terms in 3-D, 450 in 2-D): the same results
    against the oracle and the step-by-step path."""
    ff = many_terms_field(d, nterms, 7 + d, steady)
    grid = 12 if d == 3 else 32
    P = grid ** d - 7
    point0 = 5
    chunks = (3, 4)
    N = sum(chunks) + (1 if scheme == "bdf2" else 0)
    dt = 2e-3
    plan, w, lam = make_plan(d, P, 16, prec, dt, N, scheme=scheme)
    X0 = I.random_symmetric_case(d, P, 47, kscale=0.6, xscale=2e-2)[1]
    kl = levels(ff, grid, np.arange(point0, point0 + P), dt, N)
    X, Y, tau, _ = fused_run(plan, ff, grid, point0, X0, chunks, kap0=kl[0] if scheme == "bdf2" else None)
    Xs, Ys, taus = stepwise_run(plan, kl, X0, N)
    o = O.run(d, w, lam, 1.0, 0.1, dt, N, kl, X0, startup="sdirk2" if scheme == "bdf2" else "exp")
    bar = 1e-12 if prec == "fp64" else 1e-5
    got = {"X": X[N % 2, :, :P].cpu().numpy(), "tau": tau[:, :P].cpu().numpy()}
    step = {"X": Xs[N % 2, :, :P].cpu().numpy(), "tau": taus[:, :P].cpu().numpy()}
    errs = {k: relerr(got[k], o["X"][0] if k == "X" else o[k]) for k in got}
    errs_step = {k: relerr(got[k], step[k]) for k in got}
    print("large table", d, prec, nterms, steady, scheme, "oracle", errs, "stepwise", errs_step, flush=True)
    assert all(e < bar for e in errs.values()), errs
    assert all(e < bar for e in errs_step.values()), errs_step


@pytest.mark.parametrize("scheme,nterms", [("bdf2", 227), ("bdf2", 228), ("exp", 128), ("bdf2", 257)])
def test_fused_lds_limits(scheme, nterms):
    """The LDS a fused launch asks for at its limits in 3-D (table rows of 18 doubles): the BDF2
    kernel with 227 time-varying terms copies a 32 688-byte table, just under the 32 KB limit,
    and rotates 57 terms a lane (117 KB), 149 KB per block; with 228 the table stays in global
    memory; with 257 (65 a lane) the terms are evaluated directly; the exponential kernel with
    128 terms rotates 64 a lane (128 KB) next to an 18 KB table."""
    d, grid, prec = 3, 10, "fp32_modes"
    ff = many_terms_field(d, nterms, 11 + nterms, False)
    P = grid ** d - 3
    point0 = 2
    chunks = (5, 33)                              # passes a re-seed of the rotated terms
    N = sum(chunks) + (1 if scheme == "bdf2" else 0)
    dt = 2e-3
    plan, w, lam = make_plan(d, P, 16, prec, dt, N, scheme=scheme)
    X0 = I.random_symmetric_case(d, P, 53, kscale=0.6, xscale=2e-2)[1]
    kl = levels(ff, grid, np.arange(point0, point0 + P), dt, N)
    X, Y, tau, _ = fused_run(plan, ff, grid, point0, X0, chunks, kap0=kl[0] if scheme == "bdf2" else None)
    Xs, Ys, taus = stepwise_run(plan, kl, X0, N)
    o = O.run(d, w, lam, 1.0, 0.1, dt, N, kl, X0, startup="sdirk2" if scheme == "bdf2" else "exp")
    got = {"X": X[N % 2, :, :P].cpu().numpy(), "tau": tau[:, :P].cpu().numpy()}
    step = {"X": Xs[N % 2, :, :P].cpu().numpy(), "tau": taus[:, :P].cpu().numpy()}
    errs = {k: relerr(got[k], o["X"][0] if k == "X" else o[k]) for k in got}
    errs_step = {k: relerr(got[k], step[k]) for k in got}
    print("lds limits", scheme, nterms, "oracle", errs, "stepwise", errs_step, flush=True)
    assert all(e < 1e-5 for e in errs.values()), errs
    assert all(e < 1e-5 for e in errs_step.values()), errs_step


@pytest.mark.parametrize("scheme", ["exp", "bdf2"])
def test_fused_with_row_exchanges(scheme):
    """The 3-D field's amplitudes scaled until b max|kappa~| = 1.5 a in the local operator
    a I - b K of the scheme's steps: the local solves exchange rows at some points (the
    exchange selects run for those waves), against the step-by-step path and the oracle."""
    d, grid, prec, m = 3, 10, "fp32_modes", 16
    P = grid ** d - 3
    point0 = 2
    chunks = (4, 5)
    N = sum(chunks) + (1 if scheme == "bdf2" else 0)
    dt = 2e-3
    plan, w, lam = make_plan(d, P, m, prec, dt, N, scheme=scheme)
    t = plan.tables()
    a, b = t["a_diag"], t["eta"]      # the operator's a and b (for the exponential scheme 1 + q/De and q)
    ff = field_of(5, False)
    kl = levels(ff, grid, np.arange(point0, point0 + P), dt, N)
    ff.amp = ff.amp * (1.5 * a / (b * np.abs(kl).max()))
    kl = levels(ff, grid, np.arange(point0, point0 + P), dt, N)
    from tests.test_parity_gpu import local_matrix, partial_pivot_exchanges
    kt = 2.0 * kl[2] - kl[1] if scheme == "bdf2" else 1.5 * kl[2] - 0.5 * kl[1]    # kappa~ of step 2
    nsw = sum(partial_pivot_exchanges(local_matrix(d, kt[:, p], a, b)) > 0 for p in range(P))
    assert 0.05 * P < nsw < 0.95 * P, nsw
    X0 = I.random_symmetric_case(d, P, 57, kscale=0.6, xscale=2e-2)[1]
    X, Y, tau, _ = fused_run(plan, ff, grid, point0, X0, chunks, kap0=kl[0] if scheme == "bdf2" else None)
    Xs, Ys, taus = stepwise_run(plan, kl, X0, N)
    o = O.run(d, w, lam, 1.0, 0.1, dt, N, kl, X0, startup="sdirk2" if scheme == "bdf2" else "exp")
    got = {"X": X[N % 2, :, :P].cpu().numpy(), "tau": tau[:, :P].cpu().numpy()}
    step = {"X": Xs[N % 2, :, :P].cpu().numpy(), "tau": taus[:, :P].cpu().numpy()}
    errs = {k: relerr(got[k], o["X"][0] if k == "X" else o[k]) for k in got}
    errs_step = {k: relerr(got[k], step[k]) for k in got}
    print("fused row exchanges", scheme, "points exchanging at step 2", nsw, "oracle", errs, "stepwise",
          errs_step, flush=True)
    assert all(e < 1e-5 for e in errs.values()), errs
    assert all(e < 1e-5 for e in errs_step.values()), errs_step
