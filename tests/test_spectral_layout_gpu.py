"""The Fourier layout of the spatial form (tfs_spectral_*, Sec. 4.1 with L = -eps Laplace -
A(kappa~)) on the GPU: the rate field against the spatial oracle's |xi|^2, the change of
basis against the discrete Fourier transform summed directly on tiny grids and against
numpy's FFT on larger ones, the way back, and the argument checks."""
import ctypes as C

import numpy as np
import pytest
import torch

from oracle import mfp
from paper_2411_17294_amd import tfs
from paper_2411_17294_amd.spectral import PeriodicGrid

pytestmark = pytest.mark.gpu

# even and odd axes, unequal extents; 2-D and 3-D
TINY = [((6, 8), (1.0, 2.0)), ((7, 5), (0.5, 3.0)), ((4, 4, 6), (1.0, 2.0, 3.0)), ((5, 6, 3), (2.0, 1.0, 0.7))]


def half_spectrum_dft(f, shape):
    """F_q = (1/N) sum_x f(x) exp(-2 pi i sum_j k_j x_j / n_j) for every q of the half
    spectrum, summed directly (tiny grids only)."""
    d = len(shape)
    half = shape[:-1] + (shape[-1] // 2 + 1,)
    x = np.indices(shape).reshape(d, -1)
    k = np.indices(half).reshape(d, -1)
    ph = sum(np.outer(k[j], x[j]) / shape[j] for j in range(d))
    return (np.exp(-2j * np.pi * ph) @ f.reshape(-1)) / f.size


def interleave(F):
    """Complex half spectrum (any shape) -> the layout's points (re, im per coefficient)."""
    return np.stack([F.real.reshape(-1), F.imag.reshape(-1)], axis=1).reshape(-1)


@pytest.mark.parametrize("shape,extent", TINY)
def test_rate_matches_oracle_wavenumbers(shape, extent):
    """rate[2q] = rate[2q+1] = eps |xi_q|^2 with the spatial oracle's wave vectors (numpy's
    full-spectrum order cut to the half spectrum: |xi|^2 is even in the last wave number),
    zero on the padding."""
    g = PeriodicGrid(shape, extent)
    eps = 0.37
    st = g.npoints + 13
    r = g.rate(eps, st).cpu().numpy()
    h = shape[-1] // 2 + 1
    k2 = mfp.wavenumber_squared(shape, extent)[..., :h]
    want = eps * np.repeat(k2.reshape(-1), 2)
    assert np.all(np.abs(r[:g.npoints] - want) <= 2e-15 * np.abs(want))
    assert np.all(r[g.npoints:] == 0.0)
    assert r[0] == 0.0 and r[1] == 0.0 and g.source_point == 0


@pytest.mark.parametrize("shape,extent", TINY)
def test_to_points_matches_direct_dft(shape, extent):
    """Three fields with padded planes on both sides: every coefficient against the
    directly summed transform, the padding and the input untouched."""
    rng = np.random.default_rng(5)
    g = PeriodicGrid(shape, extent)
    N = int(np.prod(shape))
    f = rng.standard_normal((3, N))
    gs, ps = N + 5, g.npoints + 6
    src = torch.full((3, gs), 11.0, dtype=torch.float64, device="cuda")
    src[:, :N] = torch.from_numpy(f).cuda()
    dst = torch.full((3, ps), -3.0, dtype=torch.float64, device="cuda")
    s = tfs.lib().tfs_spectral_to_points(g._handle(), src.data_ptr(), 3, gs, dst.data_ptr(), ps,
                                         torch.cuda.current_stream().cuda_stream)
    tfs.check(s)
    out = dst.cpu().numpy()
    for i in range(3):
        want = interleave(half_spectrum_dft(f[i].reshape(shape), shape))
        err = np.max(np.abs(out[i, :g.npoints] - want)) / np.max(np.abs(want))
        assert err <= 1e-14, (shape, i, err)
    assert np.all(out[:, g.npoints:] == -3.0)
    assert np.array_equal(src[:, :N].cpu().numpy(), f) and np.all(src[:, N:].cpu().numpy() == 11.0)


@pytest.mark.parametrize("shape,extent", TINY)
def test_to_grid_inverts_to_points(shape, extent):
    """The way back: against numpy's inverse real transform of the same coefficients, the
    round trip to the starting field, the coefficients and the padding untouched."""
    rng = np.random.default_rng(6)
    g = PeriodicGrid(shape, extent)
    f = torch.from_numpy(rng.standard_normal((2, 3) + shape)).cuda()
    pts = g.to_points(f)
    keep = pts.clone()
    back = g.to_grid(pts).cpu().numpy()
    assert torch.equal(pts, keep)
    assert np.max(np.abs(back - f.cpu().numpy())) <= 1e-14 * np.max(np.abs(f.cpu().numpy()))
    P = pts.cpu().numpy().reshape(2, 3, -1, 2)
    Fc = (P[..., 0] + 1j * P[..., 1]).reshape((2, 3) + g.half)
    ref = np.fft.irfftn(Fc * np.prod(shape), s=shape, axes=tuple(range(-len(shape), 0)))
    assert np.max(np.abs(back - ref)) <= 1e-14 * np.max(np.abs(ref))
    N = int(np.prod(shape))
    gs = N + 3
    dst = torch.full((2, gs), 5.0, dtype=torch.float64, device="cuda")
    flat = pts.reshape(6, -1)[:2].contiguous()
    tfs.check(tfs.lib().tfs_spectral_to_grid(g._handle(), flat.data_ptr(), 2, g.npoints, dst.data_ptr(), gs,
                                             torch.cuda.current_stream().cuda_stream))
    d = dst.cpu().numpy()
    assert np.all(d[:, N:] == 5.0)
    assert np.max(np.abs(d[:, :N] - f.cpu().numpy().reshape(6, N)[:2])) <= 1e-14 * np.max(np.abs(d[:, :N]))


def test_to_grid_of_a_strided_state_view():
    """The binding passes the plane stride of a plan-shaped view ([c][stride], first npoints
    used) instead of copying it."""
    g = PeriodicGrid((8, 6), (1.0, 1.0))
    st = g.npoints + 64
    rng = np.random.default_rng(8)
    f = torch.from_numpy(rng.standard_normal((3, 8, 6))).cuda()
    X = torch.zeros((2, 3, st), dtype=torch.float64, device="cuda")
    X[1, :, :g.npoints] = g.to_points(f)
    back = g.to_grid(X[1, :, :g.npoints])
    assert torch.max(torch.abs(back - f)).item() <= 1e-14 * torch.max(torch.abs(f)).item()


@pytest.mark.parametrize("shape", [(1024, 1024), (128, 128, 128), (96, 80, 50)])
def test_large_grids_against_numpy_fft(shape):
    """Workload sizes: the coefficients against numpy's real transform (scaled by 1/N), and
    the round trip."""
    rng = np.random.default_rng(9)
    g = PeriodicGrid(shape, (1.0,) * len(shape))
    f = rng.standard_normal((2,) + shape)
    pts = g.to_points(torch.from_numpy(f).cuda())
    F = np.fft.rfftn(f, axes=tuple(range(-len(shape), 0))) / np.prod(shape)
    want = np.stack([interleave(F[i]) for i in range(2)])
    got = pts.cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-14 * np.max(np.abs(want))
    back = g.to_grid(pts).cpu().numpy()
    assert np.max(np.abs(back - f)) <= 1e-13 * np.max(np.abs(f))
    r = g.rate(1.0).cpu().numpy()
    h = shape[-1] // 2 + 1
    want_r = np.repeat(mfp.wavenumber_squared(shape, (1.0,) * len(shape))[..., :h].reshape(-1), 2)
    assert np.all(np.abs(r - want_r) <= 2e-15 * want_r)


def test_layout_errors_and_empty_calls():
    L = tfs.lib()
    h = C.c_void_p()
    sh2 = (C.c_int64 * 2)(8, 6)
    ex2 = (C.c_double * 2)(1.0, 1.0)
    assert L.tfs_spectral_create(4, sh2, ex2, C.byref(h)) == tfs.TFS_EINVAL and not h.value
    assert L.tfs_spectral_create(2, (C.c_int64 * 2)(1, 6), ex2, C.byref(h)) == tfs.TFS_EINVAL
    assert L.tfs_spectral_create(2, sh2, (C.c_double * 2)(1.0, float("nan")), C.byref(h)) == tfs.TFS_EINVAL
    assert L.tfs_spectral_create(2, sh2, (C.c_double * 2)(1.0, -1.0), C.byref(h)) == tfs.TFS_EINVAL
    assert L.tfs_spectral_create(2, None, ex2, C.byref(h)) == tfs.TFS_EINVAL
    assert L.tfs_spectral_create(2, sh2, ex2, None) == tfs.TFS_EINVAL
    assert L.tfs_spectral_npoints(None) == -1
    assert L.tfs_spectral_destroy(None) == tfs.TFS_OK
    g = PeriodicGrid((8, 6), (1.0, 1.0))
    s = g._handle()
    assert L.tfs_spectral_npoints(s) == 2 * 8 * 4
    buf = torch.zeros((2, 256), dtype=torch.float64, device="cuda")
    p = buf.data_ptr()
    assert L.tfs_spectral_rate(s, -1.0, p, 256, None) == tfs.TFS_EINVAL
    assert L.tfs_spectral_rate(s, float("inf"), p, 256, None) == tfs.TFS_EINVAL
    assert L.tfs_spectral_rate(s, 1.0, p, 63, None) == tfs.TFS_EINVAL
    assert L.tfs_spectral_rate(s, 1.0, None, 256, None) == tfs.TFS_EINVAL
    assert L.tfs_spectral_rate(None, 1.0, p, 256, None) == tfs.TFS_EINVAL
    for fn in (L.tfs_spectral_to_points, L.tfs_spectral_to_grid):
        assert fn(s, p, -1, 256, p + 2048, 256, None) == tfs.TFS_EINVAL
        assert fn(s, None, 1, 256, p, 256, None) == tfs.TFS_EINVAL
        assert fn(s, p, 1, 256, None, 256, None) == tfs.TFS_EINVAL
        assert fn(None, p, 1, 256, p + 2048, 256, None) == tfs.TFS_EINVAL
    assert L.tfs_spectral_to_points(s, p, 1, 47, p + 2048, 256, None) == tfs.TFS_EINVAL
    assert L.tfs_spectral_to_points(s, p, 1, 48, p + 2048, 63, None) == tfs.TFS_EINVAL
    assert L.tfs_spectral_to_grid(s, p, 1, 63, p + 2048, 48, None) == tfs.TFS_EINVAL
    assert L.tfs_spectral_to_grid(s, p, 1, 64, p + 2048, 47, None) == tfs.TFS_EINVAL
    buf.fill_(2.0)
    assert L.tfs_spectral_to_points(s, None, 0, 48, None, 64, None) == tfs.TFS_OK
    assert L.tfs_spectral_to_grid(s, p, 0, 64, p + 2048, 48, None) == tfs.TFS_OK
    torch.cuda.synchronize()
    assert torch.all(buf == 2.0)
    g.close()
