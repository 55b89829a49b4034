#!/usr/bin/env python3
"""Benchmark of the time-fractional extra-stress update on one MI355X.

Default workload (the headline): the 384^3 differentiation configuration -- alpha = 0.2,
m = 48 exponential modes, dt = 1e-4, FP32 mode storage with FP64 recombination and local
solve, FP32 velocity gradients of the time-varying seeded field -- on one point slab of the
grid (884736 consecutive points; the whole grid is 64 such slabs, which is how the
checkpointed job fits one device).  One benchmark step is one time level of that job: a
forward step with the fused diagnostics, the recomputed step of the backward sweep and the
adjoint step.  All kappa levels, the state and mode rings and the adjoint buffers are
resident in HBM before the timed region.

Prints one JSON line: point-mode updates/s (points x modes per time level / time), the
roofline of the dominant kernel (its algorithmic bytes per launch / its average launch
duration from HIP events on the plan's stream inside the timed loop), and the CPU oracle
timed on the same slab's kappa and X0.  --workload 2 or 3 times the forward step of the 2-D
FP64 or the 256^3 configuration instead.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def algorithmic_bytes_per_point(dim, m, mode_bytes, kappa_reads, kappa_bytes=8, x_levels=2):
    """Minimum HBM traffic of one step per point: two mode levels read and one written,
    X at x_levels levels read (2; 3 in the shifted mode form) and one written, tau written,
    kappa read (1 or 2 levels)."""
    c = dim * (dim + 1) // 2
    return 3 * m * c * mode_bytes + (x_levels + 1) * c * 8 + c * 8 + kappa_reads * dim * dim * kappa_bytes


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def profiled_traffic(profile_name):
    """HBM traffic per launch from the committed rocprofv3 counter summary, or None when
    there is none or the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", profile_name + ".md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#", "rocprofv3")):
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip()
    names = fields.get("sources", "tfs_kernels.hip,tfs_device.h,tfs_internal.h").split(",")
    src = b"".join(open(os.path.join(ROOT, "paper_2411_17294_amd", "csrc", f), "rb").read() for f in names)
    if fields.get("source_sha256") != hashlib.sha256(src).hexdigest():
        return None
    try:
        return float(fields["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def exp_bytes_per_point(dim, m, mode_bytes, kappa_reads, kappa_bytes=8):
    """Minimum HBM traffic of one exponential-mode step per point: the single mode level read
    and written in place, X^n read and X^{n+1} written, tau written, kappa read."""
    c = dim * (dim + 1) // 2
    return 2 * m * c * mode_bytes + 2 * c * 8 + c * 8 + kappa_reads * dim * dim * kappa_bytes


def exp_adjoint_bytes_per_point(dim, m, mode_bytes, kappa_bytes=8):
    """Minimum HBM traffic of one adjoint step of the exponential-mode scheme per point: the
    forward mode level read, the adjoint mode level read and written in place; X^n and
    X^{n+1} read, Xbar^{n+1} read and Xbar^n written; kappa at two levels read and its FP64
    adjoint read and written."""
    c = dim * (dim + 1) // 2
    return 3 * m * c * mode_bytes + 2 * c * 8 + 2 * c * 8 + 2 * dim * dim * kappa_bytes + 2 * dim * dim * 8


def adjoint_bytes_per_point(dim, m, mode_bytes, kappa_bytes=8, x_levels=2):
    """Minimum HBM traffic of one adjoint step per point: four mode streams read (H^(n+1),
    H^(n+2), Y^n, Y^(n-1)) and one written (H^(n)); X at x_levels + 1 levels read (n+1, n,
    n-1 and, in the shifted mode form, n-2), the x_levels adjoint X slots read and written;
    kappa at two levels read and its FP64 adjoint read and written."""
    c = dim * (dim + 1) // 2
    return (5 * m * c * mode_bytes + (x_levels + 1) * c * 8 + 2 * x_levels * c * 8 + 2 * dim * dim * kappa_bytes
            + 2 * dim * dim * 8)


def _timed(stream, fn, first, count):
    """Average ms per call of fn(n), n = first .. first + count - 1, by HIP events on stream."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for n in range(first, first + count):
        fn(n)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / count


def copy_rate_gbs(stream):
    """A plain device-to-device copy of 2 GiB (read + write) on the stream: the reference
    for the counter scale factors and a measured bandwidth ceiling."""
    import torch
    csrc = torch.empty(1 << 28, dtype=torch.float64, device="cuda")
    cdst = torch.empty_like(csrc)
    cdst.copy_(csrc)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record(stream)
    for _ in range(10):
        cdst.copy_(csrc)
    c1.record(stream)
    torch.cuda.synchronize()
    gbs = 10 * 2 * csrc.numel() * 8 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del csrc, cdst
    torch.cuda.empty_cache()
    return gbs


def measure_forms(stream, steps=20, which="all"):
    """The two 3-D forms next to the headline workload.

    * FP32 modes vs FP64: one forward step of the 256^3, m = 40 configuration in each form
      (same seeded inputs), the speedup, and the relative difference of the two stresses
      after the same steps.
    * Forward + adjoint, 128^3, m = 32, FP32 modes and FP64: per time level the
      differentiation pass runs one forward step (ring), one recomputed step into per-level
      buffers and one adjoint step; each is timed and priced at its algorithmic bytes, and
      the FP32-mode time level is compared with the FP64 one.
    """
    import torch
    from paper_2411_17294_amd import inputs as I
    from paper_2411_17294_amd import tfs
    from paper_2411_17294_amd.device_inputs import DeviceKappa, x0_ring
    out = {}
    if which in ("all", "fp32_vs_fp64"):
        out["fp32_vs_fp64_3d"] = _fp32_vs_fp64(stream, steps)
    if which in ("all", "fwd_adjoint"):
        out["fwd_adjoint_3d"] = _fwd_adjoint(stream, steps)
        out["fwd_adjoint_3d_fp64"] = _fwd_adjoint(stream, steps, precision="fp64")
        out["fwd_adjoint_3d"]["speedup_vs_fp64"] = (out["fwd_adjoint_3d_fp64"]["ms_per_time_level"]
                                                    / out["fwd_adjoint_3d"]["ms_per_time_level"])
    if which in ("all", "exp_vs_bdf2"):
        out["exp_vs_bdf2_3d"] = _exp_vs_bdf2(stream, steps)
    if which in ("all", "fwd_adjoint_exp"):
        out["fwd_adjoint_3d_exp"] = _fwd_adjoint(stream, steps, scheme="exp")
    if which in ("all", "slab384"):
        out["fwd_adjoint_384cube_slab"] = _fwd_adjoint(stream, steps, workload=5, npoints=SLAB_384)
        out["fwd_adjoint_384cube_slab_fp64"] = _fwd_adjoint(stream, steps, workload=5, npoints=SLAB_384,
                                                            precision="fp64")
        out["fwd_adjoint_384cube_slab"]["speedup_vs_fp64"] = (
            out["fwd_adjoint_384cube_slab_fp64"]["ms_per_time_level"]
            / out["fwd_adjoint_384cube_slab"]["ms_per_time_level"])
    if which in ("all", "mfp_2d"):
        out["mfp_spectral_2d"] = _mfp_2d(stream, steps)
    if which in ("all", "fused"):
        out["fused_exp"] = _fused(stream)
    if which in ("all", "ns"):
        out["ns_coupled"] = _ns_coupled(stream, steps)
    if which in ("all", "transport"):
        out["transport_2d"] = _transport(stream, 10)
    return out


# The 384^3 configuration runs as 64 point slabs of 884736 points (checkpoints of a whole
# slab, 2000 steps every 100, fit in one device's HBM).
SLAB_384 = 384 ** 3 // 64


def _fp32_vs_fp64(stream, steps):
    import torch
    from paper_2411_17294_amd import inputs as I
    from paper_2411_17294_amd import tfs
    from paper_2411_17294_amd.device_inputs import DeviceKappa, x0_ring
    wl = I.WORKLOADS[3]
    alpha = wl.alphas[0]
    w, lam, _, _, _ = tfs.soe_fit(alpha, wl.nmodes, wl.dt, wl.dt * wl.nsteps)
    res = {}
    taus = {}
    for form in ("fp64", "fp32_modes"):
        # the FP32-mode form reads FP32 velocity gradients
        p = tfs.Plan(wl.dim, wl.npoints, w, lam, alpha, wl.De, wl.eta_p, wl.dt, wl.nsteps, precision=form,
                     kappa="fp64" if form == "fp64" else "fp32")
        # the steady field at two levels in two buffers, as a time-varying one would be read
        ka, kb = p.kappa_tensor(), p.kappa_tensor()
        DeviceKappa(I.fourier_field(wl), wl.grid, wl.npoints).fill(ka, 0.0)
        kb.copy_(ka)
        X = x0_ring(wl, p.stride, levels=p.x_levels)
        _, Y, tau, _ = p.alloc()
        p.step(0, ka, None, X, Y, tau)
        for n in range(1, 4):
            p.step(n, ka, kb, X, Y, tau)
        ms = _timed(stream, lambda n: p.step(n, ka, kb, X, Y, tau), 4, steps)
        mb = 8 if form == "fp64" else 4
        nbytes = algorithmic_bytes_per_point(wl.dim, wl.nmodes, mb, 2, mb, p.x_levels) * wl.npoints
        gbs = nbytes / (ms * 1e-3) / 1e9
        prof = "bdf2_kernel_" + ("fp64_3d_256cube_m40" if form == "fp64" else wl.name)
        res[form] = {"ms_per_step": ms, "point_mode_updates_per_s": wl.npoints * wl.nmodes / (ms * 1e-3),
                     "bytes_per_launch": nbytes, "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS,
                     "traffic": profiled_traffic(prof)}
        taus[form] = tau[:, :wl.npoints].clone()
        del p, ka, kb, X, Y, tau
        torch.cuda.empty_cache()
    diff = float((taus["fp32_modes"] - taus["fp64"]).abs().max() / taus["fp64"].abs().max())
    del taus
    torch.cuda.empty_cache()
    return {"workload": wl.name, "steps": 4 + steps, **{f: res[f] for f in res},
            "speedup_fp32_modes": res["fp64"]["ms_per_step"] / res["fp32_modes"]["ms_per_step"],
            "tau_rel_diff_fp32_vs_fp64": diff}


def _exp_vs_bdf2(stream, steps):
    """The 256^3, m = 40, FP32-mode forward step with the exponential-mode scheme (one mode
    level, two accesses per mode-component) next to the paper's BDF2 scheme, and the
    relative difference of their stresses after the same steps (the two discretisations,
    not rounding)."""
    import torch
    from paper_2411_17294_amd import inputs as I
    from paper_2411_17294_amd import tfs
    from paper_2411_17294_amd.device_inputs import DeviceKappa, x0_ring
    wl = I.WORKLOADS[3]
    alpha = wl.alphas[0]
    w, lam, _, _, _ = tfs.soe_fit(alpha, wl.nmodes, wl.dt, wl.dt * wl.nsteps)
    res, taus = {}, {}
    for scheme in ("bdf2", "exp"):
        p = tfs.Plan(wl.dim, wl.npoints, w, lam, alpha, wl.De, wl.eta_p, wl.dt, wl.nsteps,
                     precision=wl.precision, scheme=scheme, kappa="fp32")
        ka, kb = p.kappa_tensor(), p.kappa_tensor()
        DeviceKappa(I.fourier_field(wl), wl.grid, wl.npoints).fill(ka, 0.0)
        kb.copy_(ka)
        X = x0_ring(wl, p.stride, levels=p.x_levels)
        _, Y, tau, _ = p.alloc()
        p.step(0, ka, None, X, Y, tau)
        for n in range(1, 4):
            p.step(n, ka, kb, X, Y, tau)
        ms = _timed(stream, lambda n: p.step(n, ka, kb, X, Y, tau), 4, steps)
        bpp = (exp_bytes_per_point(wl.dim, wl.nmodes, 4, 2, 4) if scheme == "exp"
               else algorithmic_bytes_per_point(wl.dim, wl.nmodes, 4, 2, 4, p.x_levels))
        nbytes = bpp * wl.npoints
        gbs = nbytes / (ms * 1e-3) / 1e9
        kern = "exp_kernel_" if scheme == "exp" else "bdf2_kernel_"
        res[scheme] = {"ms_per_step": ms, "point_mode_updates_per_s": wl.npoints * wl.nmodes / (ms * 1e-3),
                       "bytes_per_launch": nbytes, "achieved_GBs": gbs, "frac": gbs / HBM_PEAK_GBS,
                       "mode_memory_GB": p.mode_levels * wl.npoints * wl.nmodes * p.c * 4 / 1e9,
                       "traffic": profiled_traffic(kern + wl.name)}
        taus[scheme] = tau[:, :wl.npoints].clone()
        del p, ka, kb, X, Y, tau
        torch.cuda.empty_cache()
    diff = float((taus["exp"] - taus["bdf2"]).abs().max() / taus["bdf2"].abs().max())
    return {"workload": wl.name, "form": wl.precision, "steps": 4 + steps, **res,
            "speedup_exp": res["bdf2"]["ms_per_step"] / res["exp"]["ms_per_step"],
            "tau_rel_diff_exp_vs_bdf2": diff}


def _mfp_2d(stream, steps):
    """The spatial form (centre-of-mass diffusion, u = 0) at the parameters of the paper's
    convergence experiment (Sec. 5.1: unit square, eps = 1e-2, De = 0.5, alpha = 0.5,
    kappa = 0, initial profile cos(2 pi x1) cos(4 pi x2)) on a 1024 x 1024 periodic grid in
    the Fourier layout (1 050 624 coefficients), m = 32, FP64, dt = 1e-3: one BDF2 step,
    priced at the pointwise step's algorithmic bytes plus the rate field (8 B per point)."""
    import math
    import torch
    from paper_2411_17294_amd import tfs
    from paper_2411_17294_amd.spectral import PeriodicGrid
    n, m, alpha, De, eps, dt, T = 1024, 32, 0.5, 0.5, 1e-2, 1e-3, 1.0
    grid = PeriodicGrid((n, n), (1.0, 1.0))
    P = grid.npoints
    w, lam, _, _, _ = tfs.soe_fit(alpha, m, dt, T)
    p = tfs.Plan(2, P, w, lam, alpha, De, 0.1, dt, steps + 8, precision="fp64")
    p.set_spatial(grid.rate(eps, p.stride), grid.source_point)
    X, Y, tau, _ = p.alloc()
    x = torch.arange(n, dtype=torch.float64, device="cuda") / n
    prof = torch.cos(2 * math.pi * x)[:, None] * torch.cos(4 * math.pi * x)[None, :]
    X[0, :, :P] = grid.to_points(torch.stack([math.sqrt(2) * prof, math.sqrt(2) * prof, prof]))
    ka = p.kappa_tensor()
    p.step(0, ka, None, X, Y, tau)
    for k in range(1, 4):
        p.step(k, ka, ka, X, Y, tau)
    ms = _timed(stream, lambda k: p.step(k, ka, ka, X, Y, tau), 4, steps)
    nbytes = (algorithmic_bytes_per_point(2, m, 8, 2) + 8) * P
    gbs = nbytes / (ms * 1e-3) / 1e9
    name = "mfp_spectral_fp64_2d_1024sq_m32"
    return {"workload": name, "grid": [n, n], "coefficients": P, "ms_per_step": ms,
            "point_mode_updates_per_s": P * m / (ms * 1e-3), "bytes_per_launch": nbytes, "achieved_GBs": gbs,
            "frac": gbs / HBM_PEAK_GBS, "traffic": profiled_traffic("bdf2_kernel_" + name)}


def _ns_coupled(stream, steps):
    """The coupled step (tfs_ns_step: the velocity by the projection method, then the stress
    update with the new gradient) on [0, 2 pi)^d from device_inputs.synthetic_velocity, beta = 0.9 at
    Re = 1000 (nu = 9e-4, eta_p = 1e-4), De = 1, alpha = 0.5, dt = 1e-3: 1024^2 with m = 32
    FP64 modes and 128^3 with m = 32 FP32 modes.  Per configuration the ms of a coupled step,
    of the stress update alone (tfs_step with the same kappa, timed after the coupled steps)
    and of the velocity part (the difference)."""
    import math
    import torch
    from paper_2411_17294_amd import ns, tfs
    from paper_2411_17294_amd.device_inputs import synthetic_velocity
    res = {}
    for name, d, n, prec in (("ns_coupled_2d_1024sq_m32_fp64", 2, 1024, "fp64"),
                             ("ns_coupled_3d_128cube_m32_fp32modes", 3, 128, "fp32_modes")):
        P, m, alpha, De, beta, Re, dt = n ** d, 32, 0.5, 1.0, 0.9, 1000.0, 1e-3
        w, lam, _, _, _ = tfs.soe_fit(alpha, m, dt, 1.0)
        p = tfs.Plan(d, P, w, lam, alpha, De, (1 - beta) / Re, dt, 3 * steps + 16, precision=prec)
        sol = ns.Solver(p, (n,) * d, (2 * math.pi,) * d, beta / Re, dt)
        u, kappa, uh, fh = sol.alloc()
        X, Y, tau, _ = p.alloc()
        u[:, :P] = synthetic_velocity(d, n, 11 + d)
        sol.init(u, uh, kappa)
        for k in range(4):
            sol.step(k, u, uh, fh, kappa, X, Y, tau)
        ms = _timed(stream, lambda k: sol.step(k, u, uh, fh, kappa, X, Y, tau), 4, steps)
        ms_stress = _timed(stream, lambda k: p.step(k, kappa, None, X, Y, tau), 4 + steps, steps)
        if not bool(torch.isfinite(u[:, :P]).all()) or not bool(torch.isfinite(tau[:, :P]).all()):
            raise SystemExit("non-finite field in the coupled-step benchmark")
        res[name] = {"grid": [n] * d, "modes": m, "precision": prec, "ms_per_coupled_step": ms,
                     "ms_stress_update": ms_stress, "ms_velocity_part": ms - ms_stress,
                     "point_mode_updates_per_s": P * m / (ms * 1e-3), "u_rms": float(u[:, :P].pow(2).mean().sqrt())}
        if d == 2:
            # the same with the MFP transport terms (eps = 0.1, 20 splitting iterations)
            from paper_2411_17294_amd.transport import Transport
            tr = Transport(p, (n,) * d, (2 * math.pi,) * d, 0.1, 20)
            sol.set_transport(tr)
            base = 4 + 2 * steps if 4 + 2 * steps + steps < p.max_steps else 0
            ms_t = _timed(stream, lambda k: sol.step(k, u, uh, fh, kappa, X, Y, tau), base, min(steps, 4))
            res[name]["ms_per_coupled_step_with_transport"] = ms_t
            sol.set_transport(None)
            del tr
        del sol, p
    return res


def _transport(stream, steps):
    """The stress update with the MFP transport terms (tfs_transport_step: advection by u and
    centre-of-mass diffusion eps = 0.1 inside the implicit operator) on [0, 2 pi)^2, 1024^2,
    m = 32 FP64 modes, with u from device_inputs.synthetic_velocity and kappa = grad u (steady levels),
    De = 1, alpha = 0.5, eta_p = 1e-4, dt = 1e-3: ms per step with 10 and 20 splitting
    iterations and 10 and 20 GMRES steps per solve, the relative difference of X from the
    20-step GMRES result after the same steps (the solvers' convergence), and the pointwise
    step on the same fields for comparison; then the exponential-mode scheme with 10
    splitting iterations and its pointwise step."""
    import math
    import torch
    from paper_2411_17294_amd import ns, tfs
    from paper_2411_17294_amd.device_inputs import synthetic_velocity
    from paper_2411_17294_amd.transport import Transport
    n, m, alpha, De, dt, eps = 1024, 32, 0.5, 1.0, 1e-3, 0.1
    P = n * n
    w, lam, _, _, _ = tfs.soe_fit(alpha, m, dt, 1.0)
    out = {"grid": [n, n], "modes": m, "eps": eps}
    Xs = {}
    for method, iters, scheme in (("splitting", 10, "bdf2"), ("splitting", 20, "bdf2"), ("gmres", 10, "bdf2"),
                                  ("gmres", 20, "bdf2"), ("splitting", 10, "exp")):
        p = tfs.Plan(2, P, w, lam, alpha, De, 1e-4, dt, 2 * steps + 16, precision="fp64", scheme=scheme)
        sol = ns.Solver(p, (n, n), (2 * math.pi,) * 2, 9e-4, dt)
        u, kappa, uh, fh = sol.alloc()
        u[:, :P] = synthetic_velocity(2, n, 13)
        sol.init(u, uh, kappa)
        tr = Transport(p, (n, n), (2 * math.pi,) * 2, eps, iters)
        tr.set_method(method)
        X, Y, tau, _ = p.alloc()
        for k in range(4):
            tr.step(k, kappa, kappa, u, u, X, Y, tau)
        ms = _timed(stream, lambda k: tr.step(k, kappa, kappa, u, u, X, Y, tau), 4, steps)
        torch.cuda.synchronize()
        if scheme == "exp":
            out["ms_per_step_exp_splitting_10"] = ms
            ms_pt = _timed(stream, lambda k: p.step(k, kappa, kappa, X, Y, tau), 4 + steps, steps)
            out["ms_pointwise_exp_step_same_fields"] = ms_pt
            del tr, sol, p
            continue
        Xs[(method, iters)] = X[(4 + steps) % 2, :, :P].clone()
        out[f"ms_per_step_{method}_{iters}"] = ms
        if (method, iters) == ("splitting", 10):
            ms_pt = _timed(stream, lambda k: p.step(k, kappa, kappa, X, Y, tau), 4 + steps, steps)
            out["ms_pointwise_step_same_fields"] = ms_pt
        del tr, sol, p
    ref = Xs[("gmres", 20)]
    for key, X in Xs.items():
        out[f"x_rel_diff_{key[0]}_{key[1]}_vs_gmres_20"] = float((X - ref).abs().max() / ref.abs().max())
    out["point_mode_updates_per_s_gmres_20"] = P * m / (out["ms_per_step_gmres_20"] * 1e-3)
    return out


FP64_VECTOR_PEAK_TFLOPS = 78.6   # MI355X


def fused_flops_per_point_step(dim, m, nterms, scheme="exp"):
    """Floating-point operations of one fused step per point: the mode update (7 per
    mode-component: e y + f X, (1 - e) y into H, lambda dt Y into G for the exponential
    scheme; 2 Y^n - Y^{n-1}/2, d h + dc P, eta h into G for BDF2), the field (per term:
    rotation 6, extrapolation weight 6, the d x d accumulation 2 d^2) and the local system
    (assembly, elimination 2c^3/3, A(.), tau: taken as 2c^3/3 + 8c^2)."""
    c = dim * (dim + 1) // 2
    return 7 * m * c + nterms * (12 + 2 * dim * dim) + (2 * c ** 3) // 3 + 8 * c * c


def _fused(stream, K=50):
    """Temporally fused steps (tfs_run_fused): K = 50 levels per launch with kappa evaluated
    in the kernel from the analytic field, next to the step-by-step path (one step kernel per
    level plus the synthesis of that level's kappa on the device), for the exponential scheme
    and the paper's BDF2 scheme (after its SDIRK2 start), time-varying and steady fields:
    128^3, m = 32, FP32 modes with the 384^3 configuration's field; 1024^2, m = 32, FP64 with
    the 1024^2 workload's field."""
    import numpy as np
    import torch
    from paper_2411_17294_amd import inputs as I
    from paper_2411_17294_amd import tfs
    from paper_2411_17294_amd.device_inputs import DeviceKappa
    res = {}
    for name, d, g, wl_id, ff_id, prec, scheme in (
            ("exp_3d_128cube_m32_fp32modes", 3, 128, 4, 5, "fp32_modes", "exp"),
            ("bdf2_3d_128cube_m32_fp32modes", 3, 128, 4, 5, "fp32_modes", "bdf2"),
            ("exp_2d_1024sq_m32_fp64", 2, 1024, 2, 2, "fp64", "exp"),
            ("bdf2_2d_1024sq_m32_fp64", 2, 1024, 2, 2, "fp64", "bdf2")):
        wl = I.WORKLOADS[wl_id]
        P, m, dt = g ** d, 32, wl.dt
        w, lam, _, _, _ = tfs.soe_fit(wl.alphas[0], m, dt, dt * wl.nsteps)
        for steady in (False, True):
            ff = I.fourier_field(I.WORKLOADS[ff_id])
            if steady:
                ff.omega = np.zeros_like(ff.omega)
            p = tfs.Plan(d, P, w, lam, wl.alphas[0], wl.De, wl.eta_p, dt, 3 * K + 16, precision=prec,
                         scheme=scheme, mode_form="y")
            p.set_field(ff.k, ff.phase, ff.omega, ff.coef(), g, 0)
            X, Y, tau, _ = p.alloc()
            ka, kb = p.kappa_tensor(), p.kappa_tensor()
            dk = DeviceKappa(ff, g, P)
            first = 0
            if scheme == "bdf2":       # level 0 -> 1 is the SDIRK2 start (tfs_step)
                dk.fill(ka, 0.0)
                p.step(0, ka, None, X, Y, tau)
                first = 1
            p.run_fused(first, K, X, Y, tau)
            ms = _timed(stream, lambda n: p.run_fused(first + K + n * K, K, X, Y, tau), 0, 2) / K
            n0 = 3 * K
            for n in range(n0, n0 + 3):
                p.step(n, ka, kb, X, Y, tau)
            ms_step = _timed(stream, lambda n: p.step(n, ka, kb, X, Y, tau), n0 + 3, 10)
            dk.fill(ka, 0.0)
            # a steady field is synthesised once, not per step
            ms_fill = 0.0 if steady else _timed(stream, lambda n: dk.fill(ka, n * dt), 1, 5)
            flops = fused_flops_per_point_step(d, m, 0 if steady else len(ff.amp), scheme) * P
            tf = flops / (ms * 1e-3) / 1e12
            res[name + ("_steady" if steady else "_time_varying")] = {
                "ms_per_step": ms, "point_mode_updates_per_s": P * m / (ms * 1e-3), "steps_per_launch": K,
                "stepwise_kernel_ms": ms_step, "kappa_synthesis_ms_per_step": ms_fill,
                "speedup_vs_stepwise_with_synthesis": (ms_step + ms_fill) / ms,
                "speedup_vs_step_kernel_alone": ms_step / ms,
                "roofline": {"bound": "alu", "achieved": tf, "peak": FP64_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                             "frac": tf / FP64_VECTOR_PEAK_TFLOPS}}
            del p, X, Y, tau, ka, kb, dk
            torch.cuda.empty_cache()
    return res


def _fwd_adjoint(stream, steps, workload=4, npoints=None, scheme="bdf2", precision=None):
    """Forward (ring), recompute (levels) and adjoint steps of a differentiation workload on
    npoints points (default: the whole grid; a slab of the grid for the 384^3 case), in the
    workload's precision form or the one given (FP64 plans read FP64 velocity gradients)."""
    import numpy as np
    import torch
    from paper_2411_17294_amd import inputs as I
    from paper_2411_17294_amd import tfs
    from paper_2411_17294_amd.device_inputs import DeviceKappa
    wl = I.WORKLOADS[workload]
    P = wl.npoints if npoints is None else npoints
    alpha = wl.alphas[0]
    prec = precision or wl.precision
    f32 = prec == "fp32_modes"
    mb = kb_ = 4 if f32 else 8                # mode and velocity-gradient bytes
    w, lam, _, _, _ = tfs.soe_fit(alpha, wl.nmodes, wl.dt, wl.dt * wl.nsteps)
    # the library's mode-ring tile (32 KB planes: 8192 FP32 points), measured best for the
    # current kernels at both the 128^3 grid and the 384^3 slab
    tile = None
    p = tfs.Plan(wl.dim, P, w, lam, alpha, wl.De, wl.eta_p, wl.dt, wl.nsteps, precision=prec,
                 scheme=scheme, tile=tile, kappa="fp32" if f32 else "fp64")
    exp = scheme == "exp"
    ka, kb = p.kappa_tensor(), p.kappa_tensor()
    dk = DeviceKappa(I.fourier_field(wl), wl.grid, P)
    dk.fill(ka, wl.dt if wl.time_varying else 0.0)
    dk.fill(kb, 0.0)
    st, c, m = p.stride, p.c, p.m
    X, Y, tau, _ = p.alloc()
    X[0, :, :P] = torch.from_numpy(I.initial_state(wl, np.arange(P))).cuda()
    # levels n-1, n, n+1 and (read by the shifted mode form) n-2 of the recomputed steps
    Xs = [torch.zeros((c, st), dtype=torch.float64, device="cuda") for _ in range(4)]
    Ys = [torch.zeros((m * c * st,), dtype=p.mode_dtype, device="cuda") for _ in range(3)]
    Xs[0].copy_(X[0])
    Xs[3].copy_(X[0])
    if exp:
        p.step_levels(0, ka, None, Xs[0], None, Xs[1], None, None, Ys[1], tau)
        p.step_levels(1, ka, kb, Xs[1], None, Xs[2], Ys[1], None, Ys[2], tau)
    else:
        p.step_levels(0, ka, None, Xs[0], None, Xs[1], None, Ys[0], Ys[1], tau)
        p.step_levels(1, ka, kb, Xs[1], Xs[0], Xs[2], Ys[1], Ys[0], Ys[2], tau)
    Xbar = torch.zeros((p.x_levels, c, st), dtype=torch.float64, device="cuda")
    Xbar[0, :, :P].normal_()
    Hbar = torch.zeros((p.mode_levels * m * c * st,), dtype=p.mode_dtype, device="cuda")
    pbar = torch.zeros(p.pbar_size, dtype=torch.float64, device="cuda")
    kbar = torch.zeros(ka.shape, dtype=torch.float64, device="cuda")
    p.step(0, ka, None, X, Y, tau)

    def fwd(n):
        p.step(n, ka, kb, X, Y, tau)

    def rec(n):
        if exp:
            p.step_levels(n, ka, kb, Xs[1], None, Xs[2], Ys[1], None, Ys[2], tau)
        else:
            p.step_levels(n, ka, kb, Xs[1], Xs[0], Xs[2], Ys[1], Ys[0], Ys[2], None, X_nm2=Xs[3])

    def adj(n):
        if exp:
            p.step_adjoint(n, ka, kb, Xs[1], None, Xs[2], Ys[1], None, Xbar, Hbar, pbar, kappabar_a=kbar,
                           kappabar_b=kbar)
        else:
            p.step_adjoint(n, ka, kb, Xs[1], Xs[0], Xs[2], Ys[1], Ys[0], Xbar, Hbar, pbar, kappabar_a=kbar,
                           kappabar_b=kbar, X_nm2=Xs[3])
    if exp:
        fb = exp_bytes_per_point(wl.dim, m, mb, 2, kb_) * P
        rb = fb - c * 8 * P
        ab = exp_adjoint_bytes_per_point(wl.dim, m, mb, kb_) * P
    else:
        fb = algorithmic_bytes_per_point(wl.dim, m, mb, 2, kb_, p.x_levels) * P
        rb = fb - c * 8 * P            # the recomputation writes no stress
        ab = adjoint_bytes_per_point(wl.dim, m, mb, kb_, p.x_levels) * P
    tag = ("fp32modes" if f32 else "fp64") + ("_3d_128cube_m32" if workload == 4 else "_3d_384cube_m48_slab")
    kf, ka_ = ("exp_kernel_", "exp_adj_kernel_") if exp else ("bdf2_kernel_", "adj_kernel_")
    parts = {}
    for name, fn, nbytes, prof in (("forward", fwd, fb, kf + tag),
                                   ("recompute", rec, rb, kf + tag),
                                   ("adjoint", adj, ab, ka_ + tag)):
        for n in range(1, 4):
            fn(n)
        ms = _timed(stream, fn, 4, steps)
        gbs = nbytes / (ms * 1e-3) / 1e9
        parts[name] = {"ms_per_step": ms, "bytes_per_launch": nbytes, "achieved_GBs": gbs,
                       "frac": gbs / HBM_PEAK_GBS, "traffic": profiled_traffic(prof)}
    total = sum(v["ms_per_step"] for v in parts.values())
    out = {"workload": wl.name, "form": prec, "scheme": scheme, "points": P, **parts,
           "ms_per_time_level": total,
           "point_mode_updates_per_s": P * m / (total * 1e-3),
           "mode_form": "shifted (Z)" if p.x_levels == 3 else "Y",
           "frac_all": (fb + rb + ab) / (total * 1e-3) / 1e9 / HBM_PEAK_GBS}
    if P != wl.npoints:
        # kernels only: every slab runs the same three kernels per time level
        out["kernel_seconds_whole_grid_all_steps"] = total * 1e-3 * (wl.npoints / P) * wl.nsteps
    return out


def differentiation_job(steps, slabs_to_run):
    """The 384^3 differentiation workload end to end: 64 slabs of 884736 points, each a
    checkpointed forward (checkpoints every 100 steps) and backward through
    autograd.run_slabs, with the time-varying field evaluated per level on the slab's points
    by the library (FP32 levels).
    Loss: 1/2 sum ||tau^N||_F^2.  Wall time includes the field synthesis and the checkpoint
    copies; the kernels alone are measured by the slab384 form."""
    import numpy as np
    import torch
    from paper_2411_17294_amd import inputs as I
    from paper_2411_17294_amd import tfs
    from paper_2411_17294_amd.autograd import Spec, run_slabs
    from paper_2411_17294_amd.device_inputs import DeviceKappa
    wl = I.WORKLOADS[5]
    alpha, m, dt = wl.alphas[0], wl.nmodes, wl.dt
    _, _, _, _, info = tfs.soe_fit(alpha, m, dt, dt * wl.nsteps)
    spec = Spec(dim=3, nmodes=m, dt=dt, nsteps=steps, y_lo=info["y_lo"], y_hi=info["y_hi"],
                ckpt_every=wl.ckpt_every, precision=wl.precision, kappa="fp32")
    S, nslab = SLAB_384, wl.npoints // SLAB_384
    X0_all = I.initial_state(wl)
    ff = I.fourier_field(wl)
    wts = torch.tensor([1.0, 1.0, 1.0, 2.0, 2.0, 2.0], dtype=torch.float64, device="cuda")[:, None]
    zero_k = torch.zeros((9, S), dtype=torch.float64, device="cuda")
    t_slab = []

    def slab(j):
        def make():
            t_slab.append(time.perf_counter())
            log(f"slab {j}/{slabs_to_run}: points [{j * S}, {(j + 1) * S})")
            X0 = torch.from_numpy(np.ascontiguousarray(X0_all[:, j * S:(j + 1) * S])).cuda()
            return zero_k, X0, ff.table(wl.grid, j * S)      # the slab's levels from tfs_field_eval
        return make

    def loss_grad(tau, j):
        return 0.5 * float(torch.sum(wts * tau * tau)), (wts * tau).contiguous()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = run_slabs(spec, [slab(j) for j in range(slabs_to_run)], alpha, wl.De, wl.eta_p, loss_grad)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    t_slab.append(time.perf_counter())
    per = [b - a for a, b in zip(t_slab[:-1], t_slab[1:])]
    pts = S * slabs_to_run
    return {"workload": wl.name, "steps": steps, "checkpoint_every": wl.ckpt_every, "slab_points": S,
            "slabs_run": slabs_to_run, "slabs_whole_grid": nslab, "wall_s": wall,
            "slab_wall_s": {"min": min(per), "max": max(per), "mean": sum(per) / len(per)},
            "point_mode_updates_per_s": pts * m * steps / wall,
            "whole_grid_projected_s": wall * nslab / slabs_to_run,
            "loss": res["loss"], "dL_dalpha": res["alpha"], "dL_dDe": res["De"], "dL_deta_p": res["eta_p"],
            "note": "forward + checkpointed backward per time level and point, wall clock incl. field synthesis"}


def host_threads():
    """Threads for the CPU baseline: the process's CPU share (OMP_NUM_THREADS when the
    environment sets it, as the GPU hosts do), else the CPUs it may run on."""
    vis = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS", "")
    return (int(env) if env.isdigit() and int(env) > 0 else vis), vis


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            return next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "unknown")
    except OSError:
        return "unknown"


def cpu_baseline(wl, alpha, w, lam, nthreads):
    """Oracle on a bounded sample of a forward workload: every 2nd point of the grid for all
    time levels, kappa frozen at t = 0 (the oracle's per-step work does not depend on it)."""
    import numpy as np
    from oracle import oracle as O
    from paper_2411_17294_amd import inputs as I
    pts = np.arange(0, wl.npoints, 2)
    ff = I.fourier_field(wl)
    kap = ff.kappa_at(I.grid_multi_index(wl.grid, wl.dim, pts), wl.grid, 0.0)
    X0 = I.initial_state(wl, pts)
    O.run(wl.dim, w, lam, wl.De, wl.eta_p, wl.dt, 2, kap, X0, nthreads=nthreads)  # load + warm
    t0 = time.perf_counter()
    O.run(wl.dim, w, lam, wl.De, wl.eta_p, wl.dt, wl.nsteps, kap, X0, nthreads=nthreads)
    el = time.perf_counter() - t0
    rate = len(pts) * len(w) * wl.nsteps / el
    return {"value": rate, "unit": "point-mode updates/s", "cores": nthreads, "kind": "oracle",
            "sample": f"{len(pts)} points (every 2nd of {wl.grid}^{wl.dim}), {wl.nsteps} steps, alpha={alpha}, "
                      f"m={len(w)}, FP64, {el:.1f} s", "cpu_model": cpu_model()}


def cpu_baseline_slab(wl, w, lam, kap_dev, X0, nsteps=24, single_points=65536):
    """The FP64 oracle on the benchmark's own slab inputs: the kappa levels 0..nsteps the GPU
    read (FP32 values, copied to the host) and the same X0, forward from level 0 (the SDIRK2
    start, then BDF2): all points with the process's CPU share of threads, and the first
    single_points points with one thread.  The oracle has no reverse mode, so its rate is that
    of the forward sweep; the GPU's rate counts a forward, a recomputed and an adjoint step per
    time level."""
    import numpy as np
    from oracle import oracle as O
    P = X0.shape[1]
    kap = kap_dev[:nsteps + 1, :, :P].double().cpu().numpy()
    nth, vis = host_threads()
    m = len(w)
    O.run(3, w, lam, wl.De, wl.eta_p, wl.dt, 1, kap[:2, :, :1024], X0[:, :1024], nthreads=nth)  # load + warm
    t0 = time.perf_counter()
    O.run(3, w, lam, wl.De, wl.eta_p, wl.dt, nsteps, kap, X0, nthreads=nth)
    el = time.perf_counter() - t0
    Ps = min(single_points, P)
    t0 = time.perf_counter()
    O.run(3, w, lam, wl.De, wl.eta_p, wl.dt, nsteps, np.ascontiguousarray(kap[:, :, :Ps]),
          np.ascontiguousarray(X0[:, :Ps]), nthreads=1)
    el1 = time.perf_counter() - t0
    return {"value": P * m * nsteps / el, "unit": "point-mode updates/s", "cores": nth, "kind": "oracle",
            "sample": f"forward only (the oracle has no reverse mode): the benchmark slab's {P} points, "
                      f"levels 0..{nsteps} of its kappa (the GPU's FP32 values) and X0, alpha={wl.alphas[0]}, "
                      f"m={m}, FP64, {el:.1f} s with {nth} threads",
            "single_thread": {"value": Ps * m * nsteps / el1, "points": Ps, "steps": nsteps, "seconds": el1},
            "host_cpus_visible": vis, "cpu_model": cpu_model()}


def headline_differentiation(args, stream, wl_id=5):
    """One time level of the checkpointed differentiation job, timed: the forward step (with
    the fused diagnostics), the recomputed step and the adjoint step of the 384^3
    configuration on its first point slab (wl_id 5), or of the 128^3 configuration on the
    whole grid (wl_id 4).  FP32 modes, FP32 velocity gradients of the seeded field."""
    import numpy as np
    import torch
    from paper_2411_17294_amd import inputs as I
    from paper_2411_17294_amd import tfs
    wl = I.WORKLOADS[wl_id]
    P = SLAB_384 if wl_id == 5 else wl.npoints
    point0 = 0
    alpha, m = wl.alphas[0], wl.nmodes
    W, K = args.warmup, args.steps
    if W < 1:
        raise SystemExit("warmup must include the start-up step (>= 1)")
    if W + K + 1 > wl.nsteps:
        raise SystemExit(f"warmup + steps must stay below the workload's {wl.nsteps} time levels")
    w, lam, _, _, info = tfs.soe_fit(alpha, m, wl.dt, wl.dt * wl.nsteps)
    log(f"{wl.name}: SOE symbol rel err {info['symbol_relerr']:.2e}, kernel rel err {info['kernel_relerr']:.2e}")
    tile = None if args.tile < 0 else args.tile
    p = tfs.Plan(3, P, w, lam, alpha, wl.De, wl.eta_p, wl.dt, wl.nsteps, precision="fp32_modes", kappa="fp32",
                 tile=tile)
    if args.grid_per_cu:
        p.tune("grid_per_cu", args.grid_per_cu)
    ff = I.fourier_field(wl)
    p.set_field(*ff.table(wl.grid, point0))
    st, c = p.stride, p.c
    nlev = max(W + K + 1, 25)
    t0 = time.perf_counter()
    kap = torch.zeros((nlev, 9, st), dtype=torch.float32, device="cuda")
    for n in range(nlev):
        p.field_eval(n * wl.dt, kap[n])
    X0 = I.initial_state(wl, point0 + np.arange(P))
    X, Y, tau, diag = p.alloc()
    X[0, :, :P] = torch.from_numpy(X0).cuda()
    # levels n-1, n, n+1 and (read by the shifted mode form) n-2 of the recomputed steps
    Xs = [torch.zeros((c, st), dtype=torch.float64, device="cuda") for _ in range(4)]
    Ys = [torch.zeros((m * c * st,), dtype=torch.float32, device="cuda") for _ in range(3)]
    Xs[0].copy_(X[0])
    Xs[3].copy_(X[0])
    Xbar = torch.zeros((p.x_levels, c, st), dtype=torch.float64, device="cuda")
    Xbar[0, :, :P].normal_()
    Hbar = torch.zeros((2 * m * c * st,), dtype=torch.float32, device="cuda")
    pbar = torch.zeros(p.pbar_size, dtype=torch.float64, device="cuda")
    kbar = torch.zeros((9, st), dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s ({P} points, stride {st}, tile {p.tile})")
    level = lambda n: (kap[n], kap[n - 1] if n >= 1 else None)

    def fwd(n):
        p.step(n, *level(n), X, Y, tau, diag)

    def rec(n):
        # the backward sweep recomputes the state and the modes; it needs no stress
        p.step_levels(n, *level(n), Xs[1], Xs[0], Xs[2], Ys[1], Ys[0], Ys[2], None, X_nm2=Xs[3])

    def adj(n):
        p.step_adjoint(n, *level(n), Xs[1], Xs[0], Xs[2], Ys[1], Ys[0], Xbar, Hbar, pbar,
                       kappabar_a=kbar, kappabar_b=kbar, X_nm2=Xs[3])
    p.step_levels(0, kap[0], None, Xs[0], None, Xs[1], None, Ys[0], Ys[1], None)
    for n in range(W):
        fwd(n)
        rec(max(n, 1))
        adj(max(n, 1))
    torch.cuda.synchronize()
    E = lambda: torch.cuda.Event(enable_timing=True)
    evs = {"forward": [], "recompute": [], "adjoint": []}
    e0, e1 = E(), E()
    w0 = time.perf_counter()
    e0.record(stream)
    for n in range(W, W + K):
        for name, fn in (("forward", fwd), ("recompute", rec), ("adjoint", adj)):
            a, b = E(), E()
            a.record(stream)
            fn(n)
            b.record(stream)
            evs[name].append((a, b))
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = e0.elapsed_time(e1)
    d = diag.cpu().numpy()
    if not bool(torch.isfinite(tau[:, :P]).all()) or d[5] != 0 or not d[2] > 0:
        raise SystemExit(f"non-finite or non-positive-definite state in the benchmark run (diag {d})")
    kb = 4
    xl = p.x_levels
    nbytes = {"forward": algorithmic_bytes_per_point(3, m, 4, 2, kb, xl) * P,
              # no stress written by the recomputation
              "recompute": (algorithmic_bytes_per_point(3, m, 4, 2, kb, xl) - c * 8) * P,
              "adjoint": adjoint_bytes_per_point(3, m, 4, kb, xl) * P}
    kern = {"forward": "bdf2_kernel", "recompute": "bdf2_kernel", "adjoint": "adj_kernel"}
    parts = {}
    for name, lst in evs.items():
        t = sum(a.elapsed_time(b) for a, b in lst) / K
        gbs = nbytes[name] / (t * 1e-3) / 1e9
        parts[name] = {"ms_per_launch": t, "bytes_per_launch": nbytes[name], "achieved_GBs": gbs,
                       "frac": gbs / HBM_PEAK_GBS, "kernel": kern[name]}
    dom = max(parts, key=lambda k: parts[k]["ms_per_launch"])
    tag = "fp32modes_3d_384cube_m48_slab" if wl_id == 5 else "fp32modes_3d_128cube_m32"
    prof = {"forward": "bdf2_kernel_diag_", "recompute": "bdf2_kernel_", "adjoint": "adj_kernel_"}[dom] + tag
    ms_level = ms / K
    total_bytes = sum(nbytes.values())
    out = {
        "metric": "point-mode updates/s + % HBM roofline, FP64 vs FP32-mode fwd+adjoint",
        "value": P * m / (ms_level * 1e-3),
        "unit": "point-mode updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_level,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 modes / f64",
        "data": "synthetic",
        "config": {"workload": wl.name + ("_slab" if wl_id == 5 else ""), "grid": f"{wl.grid}^3",
                   "points": P, "point0": point0, "alpha": alpha, "modes": m, "dt": wl.dt,
                   "time_levels": wl.nsteps, "checkpoint_every": wl.ckpt_every,
                   "form": "fp32 modes, fp32 kappa; fp64 recombination, solve, X, tau",
                   "kappa": "time-varying, extrapolated" if wl.time_varying else "steady",
                   "step": "forward (with diagnostics) + recomputed forward + adjoint, per time level",
                   "mode_form": "shifted (Z)" if p.x_levels == 3 else "Y",
                   "mode_tile": p.tile},
        "roofline": {"bound": "hbm", "achieved": parts[dom]["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": parts[dom]["frac"], "traffic": profiled_traffic(prof),
                     "kernel": parts[dom]["kernel"] + f" ({dom})", "bytes_per_launch": nbytes[dom],
                     "avg_launch_us": parts[dom]["ms_per_launch"] * 1e3},
        "parts": parts,
        "frac_all": total_bytes / (ms_level * 1e-3) / 1e9 / HBM_PEAK_GBS,
        "wall_s": wall,
        "diag_last_step": d.tolist(),
    }
    state = {"wl": wl, "w": w, "lam": lam, "kap": kap, "X0": X0}
    del X, Y, tau, Xs, Ys, Xbar, Hbar, pbar, kbar
    return out, state


def forward_line(stream, wl_id, steps, warmup, form="default", tile=-1, vec=0, grid_per_cu=0, keep_plans=False):
    """The forward step of a forward workload (1024^2 FP64 with both alphas, or 256^3) timed on
    its whole grid: all kappa levels resident, one benchmark step advances every field by one
    time level.  The FP32-mode form reads FP32 velocity gradients."""
    import torch
    from paper_2411_17294_amd import inputs as I
    from paper_2411_17294_amd import tfs
    from paper_2411_17294_amd.device_inputs import DeviceKappa, x0_ring
    wl = I.WORKLOADS[wl_id]
    form = wl.precision if form == "default" else form
    kp = "fp64" if form == "fp64" else "fp32"
    N = wl.nsteps
    if warmup < 1:
        raise SystemExit("warmup must include the start-up step (>= 1)")
    if warmup + steps > N:
        raise SystemExit(f"warmup + steps must not exceed the workload's {N} time levels")
    dev = "cuda"
    ff = I.fourier_field(wl)
    dk = DeviceKappa(ff, wl.grid, wl.npoints)
    plans, states = [], []
    for alpha in wl.alphas:
        w, lam, _, _, info = tfs.soe_fit(alpha, wl.nmodes, wl.dt, wl.dt * N)
        log(f"alpha={alpha}: SOE symbol rel err {info['symbol_relerr']:.2e}")
        p = tfs.Plan(wl.dim, wl.npoints, w, lam, alpha, wl.De, wl.eta_p, wl.dt, N, precision=form,
                     tile=None if tile < 0 else tile, kappa=kp)
        if vec:
            p.tune("vec", vec)
        if grid_per_cu:
            p.tune("grid_per_cu", grid_per_cu)
        X = x0_ring(wl, p.stride, levels=p.x_levels)
        _, Y, tau, _ = p.alloc()
        plans.append((alpha, w, lam, p))
        states.append((X, Y, tau))
    st = plans[0][3].stride
    kdt = plans[0][3].kappa_dtype
    t0 = time.perf_counter()
    if wl.time_varying:
        nlev = warmup + steps
        kap = torch.zeros((nlev, wl.dim * wl.dim, st), dtype=kdt, device=dev)
        for n in range(nlev):
            dk.fill(kap[n], n * wl.dt)
        level = lambda n: (kap[n], kap[n - 1] if n >= 1 else None)
    else:
        k0 = torch.zeros((wl.dim * wl.dim, st), dtype=kdt, device=dev)
        dk.fill(k0, 0.0)
        level = lambda n: (k0, k0)
    torch.cuda.synchronize()
    log(f"inputs ready in {time.perf_counter() - t0:.1f} s")

    def step(n):
        ka, kb = level(n)
        for (_, _, _, p), (X, Y, tau) in zip(plans, states):
            p.step(n, ka, kb, X, Y, tau)

    for n in range(warmup):
        step(n)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    ev0.record(stream)
    for n in range(warmup, warmup + steps):
        step(n)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms = ev0.elapsed_time(ev1)
    for (X, Y, tau) in states:
        if not bool(torch.isfinite(tau[:, :wl.npoints]).all()):
            raise SystemExit("non-finite stress in the benchmark run")
    nfields = len(wl.alphas)
    mode_bytes = 8 if form == "fp64" else 4
    bytes_per_launch = algorithmic_bytes_per_point(wl.dim, wl.nmodes, mode_bytes, 2, 8 if kp == "fp64" else 4,
                                                   plans[0][3].x_levels) * wl.npoints
    avg_launch_s = ms * 1e-3 / (nfields * steps)
    achieved = bytes_per_launch / avg_launch_s / 1e9
    profile = "bdf2_kernel_" + wl.name + ("" if form == wl.precision else "_" + form)
    out = {
        "metric": "point-mode updates/s + % HBM roofline, FP64 vs FP32-mode fwd+adjoint",
        "value": nfields * wl.npoints * wl.nmodes * steps / (ms * 1e-3),
        "unit": "point-mode updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": ms / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if form == "fp64" else "f32 modes / f64",
        "data": "synthetic",
        "config": {"workload": wl.name, "grid": f"{wl.grid}^{wl.dim}", "alphas": list(wl.alphas),
                   "modes": wl.nmodes, "dt": wl.dt, "time_levels": N, "form": form, "kappa_storage": kp,
                   "kappa": "time-varying, extrapolated" if wl.time_varying else "steady",
                   "fields_per_step": nfields, "mode_tile": plans[0][3].tile},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": profiled_traffic(profile),
                     "kernel": "bdf2_kernel", "bytes_per_launch": bytes_per_launch,
                     "avg_launch_us": avg_launch_s * 1e6},
        "wall_s": wall,
    }
    keep = [(a, w, lam) for (a, w, lam, _) in plans]
    del states, plans
    if wl.time_varying:
        del kap
    torch.cuda.empty_cache()
    return (out, keep) if keep_plans else out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", type=int, default=5,
                    help="5 (default): one time level of the 384^3 differentiation job on a slab; 4: the same "
                         "on the 128^3 grid; 2, 3: the forward step of the 2-D FP64 / 256^3 configuration")
    ap.add_argument("--form", choices=["default", "fp64", "fp32_modes"], default="default")
    ap.add_argument("--vec", type=int, default=0)
    ap.add_argument("--tile", type=int, default=-1, help="mode-ring tile (points); -1 = library default")
    ap.add_argument("--grid-per-cu", type=int, default=0, help="blocks per CU cap; 0 = library default")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the 3-D FP32/FP64 and forward+adjoint lines")
    ap.add_argument("--job", type=int, default=0, metavar="STEPS",
                    help="run the 384^3 differentiation workload end to end with STEPS time levels")
    ap.add_argument("--job-slabs", type=int, default=64, help="slabs of the --job run (64 = whole grid)")
    ap.add_argument("--only-forms", choices=["all", "fp32_vs_fp64", "fwd_adjoint", "slab384", "exp_vs_bdf2",
                                             "fwd_adjoint_exp", "mfp_2d", "fused", "ns", "transport"],
                    default=None,
                    help="only the 3-D form measurements (for profiling)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU; the update is pointwise and would shard by "
                                   "point slabs with no exchange, but multi-GPU runs are not part of it",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2411_17294_amd import inputs as I
    from paper_2411_17294_amd import tfs
    from paper_2411_17294_amd.device_inputs import DeviceKappa, x0_ring

    if args.job:
        torch.cuda.set_device(0)
        print(json.dumps({"job": differentiation_job(args.job, args.job_slabs)}), flush=True)
        return

    if args.only_forms:
        torch.cuda.set_device(0)
        stream = torch.cuda.current_stream()
        forms = measure_forms(stream, which=args.only_forms)
        print(json.dumps({"forms": forms, "measured_copy_GBs": copy_rate_gbs(stream)}), flush=True)
        return

    if args.workload in (4, 5):
        torch.cuda.set_device(0)
        stream = torch.cuda.current_stream()
        out, st = headline_differentiation(args, stream, args.workload)
        out["roofline"]["measured_copy_GBs"] = copy_rate_gbs(stream)
        if not args.no_cpu_baseline and args.workload == 5:
            t0 = time.perf_counter()
            out["cpu_baseline"] = cpu_baseline_slab(st["wl"], st["w"], st["lam"], st["kap"], st["X0"])
            log(f"CPU baseline in {time.perf_counter() - t0:.1f} s")
        del st
        torch.cuda.empty_cache()
        if not args.no_forms:
            t0 = time.perf_counter()
            out["forms"] = {"forward_2d_1024sq_fp64": forward_line(stream, 2, 20, 5)}
            out["forms"].update(measure_forms(stream))
            log(f"form measurements in {time.perf_counter() - t0:.1f} s")
        print(json.dumps(out), flush=True)
        return
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    out, plans = forward_line(stream, args.workload, args.steps, args.warmup, form=args.form, tile=args.tile,
                              vec=args.vec, grid_per_cu=args.grid_per_cu, keep_plans=True)
    out["roofline"]["measured_copy_GBs"] = copy_rate_gbs(stream)
    if not args.no_forms:
        torch.cuda.empty_cache()
        t0 = time.perf_counter()
        out["forms"] = measure_forms(stream)
        log(f"3-D form measurements in {time.perf_counter() - t0:.1f} s")
    if not args.no_cpu_baseline:
        nthreads, _ = host_threads()
        alpha, w, lam = plans[0]
        out["cpu_baseline"] = cpu_baseline(I.WORKLOADS[args.workload], alpha, w, lam, nthreads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
