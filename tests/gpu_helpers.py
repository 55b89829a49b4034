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


def as_fp32(a):
    """FP64 array rounded to FP32 and back: the values an FP32-kappa plan reads."""
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


def relerr_ref(a, ref):
    """Normwise relative error of a against a reference that may be extended precision."""
    ref = np.asarray(ref)
    a = np.asarray(a).astype(ref.dtype)
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(a - ref)) / den) if den != 0 else float(np.max(np.abs(a)))


FP64_TOL = 1e-12


def check_fp64_bar(label, g, o, ol):
    """FP64 bar of a full-size run, on inputs identical for the GPU and the oracle.

    g, o, ol: GPU, FP64-oracle and extended-precision-oracle results, dicts of same-shaped
    arrays per field.  The reference is the extended-precision run of the oracle (the same
    scheme with a 64-bit significand).  Each field of the GPU must be within
    max(1e-12, 4 e_o) of it, e_o being the FP64 oracle's own error there: 1e-12 for a
    well-conditioned field (e_o ~ 1e-14), and for the stress, a near-cancelling sum over the
    modes whose FP64 evaluations are a few 1e-12 apart, no worse than a plain FP64
    evaluation of the scheme within a factor 4.  Returns the error table."""
    rows = {}
    bad = {}
    for k in g:
        eg = relerr_ref(g[k], ol[k])
        eo = relerr_ref(o[k], ol[k])
        e64 = relerr(g[k], o[k])
        bar = max(FP64_TOL, 4.0 * eo)
        rows[k] = (eg, eo, e64, bar)
        if not eg <= bar:
            bad[k] = (eg, bar)
    print(label, {k: f"gpu {v[0]:.2e} fp64-oracle {v[1]:.2e} (gpu vs fp64-oracle {v[2]:.2e}) bar {v[3]:.1e}"
                  for k, v in rows.items()}, flush=True)
    assert not bad, f"{label}: {bad}"
    return rows


def run_gpu(d, w, lam, De, eta_p, dt, nsteps, kappa, X0, precision="fp64", extrap=True, stride=0,
            offset=0, want_modes=False, want_diag=False, alpha=0.5, vec=None, flags=0, max_steps=None,
            tile=None, scheme="bdf2", kappa_prec="fp64", mode_form="auto"):
    """Run nsteps steps on the GPU for small host inputs.

    kappa: [d*d][P] steady or [nlev][d*d][P]; X0: [c][P].  offset shifts every field base
    by that many elements (to exercise unaligned starts).  kappa_prec "fp32" stores the
    velocity gradients in FP32 (rounded from the given FP64 values)."""
    c = d * (d + 1) // 2
    P = X0.shape[1]
    plan = tfs.Plan(d, P, w, lam, alpha, De, eta_p, dt, max_steps or max(nsteps, 1), precision=precision,
                    stride=stride, tile=tile, flags=flags, scheme=scheme, kappa=kappa_prec, mode_form=mode_form)
    if vec is not None:
        plan.tune("vec", vec)
    st = plan.stride
    dev = "cuda"
    m = plan.m

    def field(shape, dtype):
        n = int(np.prod(shape))
        buf = torch.zeros(n + offset, dtype=dtype, device=dev)
        return buf[offset:].view(*shape)

    XL = plan.x_levels
    X = field((XL, c, st), torch.float64)
    Y = field((plan.mode_levels * m * c * st,), plan.mode_dtype)
    tau = field((c, st), torch.float64)
    diag = field((6,), torch.float64)
    X[0, :, :P] = torch.from_numpy(np.ascontiguousarray(X0)).to(dev)
    steady = kappa.ndim == 2
    kdt = plan.kappa_dtype
    if steady:
        kd = field((d * d, st), kdt)
        kd[:, :P] = torch.from_numpy(np.ascontiguousarray(kappa)).to(dev).to(kdt)
        levels = None
    else:
        levels = []
        for lv in range(kappa.shape[0]):
            t = field((d * d, st), kdt)
            t[:, :P] = torch.from_numpy(np.ascontiguousarray(kappa[lv])).to(dev).to(kdt)
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
    out = {"X": np.stack([X[N % XL, :, :P].cpu().numpy(), X[(N - 1) % XL, :, :P].cpu().numpy()]),
           "tau": tau[:, :P].cpu().numpy()}
    if want_modes:
        mods = []
        for lv in ((N, N - 1) if plan.mode_levels == 2 else (N,)):
            o = torch.zeros((m, c, st), dtype=torch.float64, device=dev)
            plan.modes_to_plain(lv, X, Y, o)
            mods.append(o[:, :, :P].cpu().numpy())
        torch.cuda.synchronize()
        out["modes"] = np.stack(mods)
    if want_diag:
        out["diag"] = diag.cpu().numpy()
    out["plan"] = plan
    return out
