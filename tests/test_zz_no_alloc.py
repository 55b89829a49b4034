"""tfs_step_noalloc (the step with its diagnostics block partials in the library's static
device scratch) against tfs_step, through the C ABI: two runs in a row on one device, the
first filling every partial slot a launch can use on the device, the second with a much
smaller input; X, the modes, the stress and the diagnostics after every step must equal
tfs_step's bit for bit (same kernels, same fixed-order fold).  Also the refusal of a plan
whose launches would write more partials than the scratch holds."""
import numpy as np
import pytest
import torch

from oracle import soe as osoe
from paper_2411_17294_amd import inputs as I
from paper_2411_17294_amd import tfs

pytestmark = pytest.mark.gpu


def make_plan(d, P, m, prec, scheme, steps, kappa="fp64"):
    w, lam, _ = osoe.soe_fit(0.45, m, 1e-3, 1e-3 * steps * 10)
    return tfs.Plan(d, P, w, lam, 0.45, 1.0, 0.1, 1e-3, steps, precision=prec, scheme=scheme, kappa=kappa)


def inputs(plan, seed):
    """Seeded kappa levels and X0 (identity plus noise) on the device."""
    d, c, st, P = plan.dim, plan.c, plan.stride, plan.npoints
    g = torch.Generator(device="cuda").manual_seed(seed)
    ka = torch.zeros((d * d, st), dtype=plan.kappa_dtype, device="cuda")
    kb = torch.zeros_like(ka)
    ka[:, :P] = (torch.randn((d * d, P), generator=g, device="cuda", dtype=torch.float64) * 0.6).to(ka.dtype)
    kb[:, :P] = (torch.randn((d * d, P), generator=g, device="cuda", dtype=torch.float64) * 0.6).to(kb.dtype)
    X0 = torch.randn((c, P), generator=g, device="cuda", dtype=torch.float64) * 1e-2
    for s, (i, j) in enumerate(I.packed_pairs(d)):
        if i == j:
            X0[s] += 1.0
    return ka, kb, X0


def run(plan, ka, kb, X0, steps, noalloc):
    X, Y, tau, diag = plan.alloc()
    X[0, :, :plan.npoints] = X0
    step = plan.step_noalloc if noalloc else plan.step
    diags = []
    for n in range(steps):
        step(n, ka, kb if n >= 1 else None, X, Y, tau, diag)
        diags.append(diag.clone())
    torch.cuda.synchronize()
    return X, Y, tau, torch.stack(diags)


CASES = [(3, "fp32_modes", "bdf2", "fp32"), (2, "fp64", "bdf2", "fp64"), (3, "fp32_modes", "exp", "fp64")]


@pytest.mark.parametrize("d,prec,scheme,kappa", CASES)
def test_noalloc_step_matches_step_twice_second_smaller(d, prec, scheme, kappa):
    steps, m = 4, 6
    # first run: enough points that the V-wide launch uses every block the device allows
    # (num_cus * 16) and a tail launch follows; second run: a few hundred points
    for P, seed in ((4 * 256 * 256 * 16 + 13, 5), (389, 6)):
        plan = make_plan(d, P, m, prec, scheme, steps, kappa)
        plan.tune("grid_per_cu", 16)              # the largest grid the static scratch allows
        print(f"noalloc d={d} {prec} {scheme} kappa {kappa} P={P}", flush=True)
        ka, kb, X0 = inputs(plan, seed)
        ref = run(plan, ka, kb, X0, steps, noalloc=False)
        got = run(plan, ka, kb, X0, steps, noalloc=True)
        for name, a, b in zip(("X", "Y", "tau", "diag"), got, ref):
            assert torch.equal(a, b), f"{name} differs at P={P}"
        assert float(ref[3][-1][5]) == 0.0          # no non-finite entries
        del plan, ka, kb, X0, ref, got
        torch.cuda.empty_cache()


def test_noalloc_refuses_more_partials_than_the_scratch_holds():
    plan = make_plan(2, 1000, 5, "fp64", "bdf2", 3)
    ka, kb, X0 = inputs(plan, 7)
    X, Y, tau, diag = plan.alloc()
    X[0, :, :plan.npoints] = X0
    plan.tune("grid_per_cu", 17)
    with pytest.raises(tfs.TfsError, match="static scratch"):
        plan.step_noalloc(0, ka, None, X, Y, tau, diag)
    # without diagnostics the call needs no scratch and equals tfs_step
    plan.step_noalloc(0, ka, None, X, Y, tau, None)
    X2, Y2, tau2, _ = plan.alloc()
    X2[0, :, :plan.npoints] = X0
    plan.step(0, ka, None, X2, Y2, tau2, None)
    torch.cuda.synchronize()
    assert torch.equal(X, X2) and torch.equal(Y, Y2) and torch.equal(tau, tau2)
