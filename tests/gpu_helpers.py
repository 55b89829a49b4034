"""Helpers of the GPU parity tests: drive the C ABI through the thin binding and compare
with the oracle, normwise per output field (max |a - b| / max |b|)."""
import numpy as np
import torch

from paper_2411_17294_amd import tfs


def relerr(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b))
    if den == 0.0:
        return float(np.max(np.abs(a)))
    return float(np.max(np.abs(a - b)) / den)


def run_gpu(d, w, lam, De, eta_p, dt, nsteps, kappa, X0, precision="fp64", extrap=True, stride=0,
            offset=0, want_modes=False, want_diag=False, alpha=0.5, vec=None, flags=0, max_steps=None,
            tile=None, scheme="bdf2"):
    """Run nsteps steps on the GPU for small host inputs.

    kappa: [d*d][P] steady or [nlev][d*d][P]; X0: [c][P].  offset shifts every field base
    by that many elements (to exercise unaligned starts)."""
    c = d * (d + 1) // 2
    P = X0.shape[1]
    plan = tfs.Plan(d, P, w, lam, alpha, De, eta_p, dt, max_steps or max(nsteps, 1), precision=precision,
                    stride=stride, tile=tile, flags=flags, scheme=scheme)
    if vec is not None:
        plan.tune("vec", vec)
    st = plan.stride
    dev = "cuda"
    m = plan.m

    def field(shape, dtype):
        n = int(np.prod(shape))
        buf = torch.zeros(n + offset, dtype=dtype, device=dev)
        return buf[offset:].view(*shape)

    X = field((2, c, st), torch.float64)
    Y = field((plan.mode_levels * m * c * st,), plan.mode_dtype)
    tau = field((c, st), torch.float64)
    diag = field((6,), torch.float64)
    X[0, :, :P] = torch.from_numpy(np.ascontiguousarray(X0)).to(dev)
    steady = kappa.ndim == 2
    if steady:
        kd = field((d * d, st), torch.float64)
        kd[:, :P] = torch.from_numpy(np.ascontiguousarray(kappa)).to(dev)
        levels = None
    else:
        levels = []
        for lv in range(kappa.shape[0]):
            t = field((d * d, st), torch.float64)
            t[:, :P] = torch.from_numpy(np.ascontiguousarray(kappa[lv])).to(dev)
            levels.append(t)
    for n in range(nsteps):
        if steady:
            ka, kb = kd, (kd if extrap else None)
        elif extrap:
            ka, kb = levels[n], (levels[n - 1] if n >= 1 else None)
        else:
            ka, kb = levels[n + 1], None
        plan.step(n, ka, kb, X, Y, tau, diag if want_diag else None)
    torch.cuda.synchronize()
    N = nsteps
    out = {"X": np.stack([X[N % 2, :, :P].cpu().numpy(), X[(N - 1) % 2, :, :P].cpu().numpy()]),
           "tau": tau[:, :P].cpu().numpy()}
    if want_modes:
        mods = []
        for lv in ((N, N - 1) if plan.mode_levels == 2 else (N,)):
            o = torch.zeros((m, c, st), dtype=torch.float64, device=dev)
            plan.modes_to_plain(lv % 2, X, Y, o)
            mods.append(o[:, :, :P].cpu().numpy())
        torch.cuda.synchronize()
        out["modes"] = np.stack(mods)
    if want_diag:
        out["diag"] = diag.cpu().numpy()
    out["plan"] = plan
    return out
