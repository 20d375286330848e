"""GPU parity on degenerate and limiting inputs: one-pixel, one-row and
one-column grids, the widest stencil this build accepts (3 sigma s = 25
lattice points, lag D = 10), grids with sides of 400 to 4096 pixels, a
single valid pixel, non-finite data entries, and PSFs beyond the limits
(rejected at creation)."""
import sys
import zlib

import numpy as np
import pytest
import torch

import workloads as W
from oracle import model as M

pytestmark = pytest.mark.gpu

from bounds import LOGL_ATOL, MAP_RTOL, logl_tol
GRAD_RTOL, GRAD_NORM_TOL = 1e-3, 1e-4


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_06819_amd as gk
    return gk


def bound(spec, data, err, th):
    return logl_tol(spec, data, err, th, "far")


def check_grad(got, ref, tag):
    tol = GRAD_RTOL * np.abs(ref) + GRAD_NORM_TOL * np.linalg.norm(ref)
    assert np.isfinite(got).all(), f"{tag}: non-finite gradient"
    bad = ~(np.abs(got - ref) <= tol)
    assert not bad.any(), f"{tag}: params {np.nonzero(bad)[0]}: gpu {got[bad]} oracle {ref[bad]}"


SPECS = {
    "one_pixel": W.GridSpec(1, 1, 0.3, 3, 1.0, 1, 1, W.HALO_NFW),
    "one_row": W.GridSpec(17, 1, 0.2, 3, 0.8, 1, 2, W.HALO_NFW),
    "one_column": W.GridSpec(1, 13, 0.2, 1, 1.2, 0, 1, W.HALO_HERNQUIST),
    "widest_stencil": W.GridSpec(12, 9, 0.15, 5, W.SIGMA_FWHM_4, 1, 2, W.HALO_NFW),
    # extreme aspect ratios: many ragged column bands of three rows, one
    # column band of many rows (forward bands and adjoint lattice blocks)
    "long_strip": W.GridSpec(257, 3, 0.2, 3, W.SIGMA_FWHM_2P5, 1, 2, W.HALO_NFW),
    "tall_strip": W.GridSpec(2, 263, 0.15, 1, 1.5, W.BULGE_JAFFE, 1, W.HALO_HERNQUIST),
}


@pytest.mark.parametrize("name", list(SPECS))
def test_degenerate_and_limit_grids(gk, name):
    spec = SPECS[name]
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    truth = W.draw_thetas(spec, 1, rng)[0]
    data, err = M.synthetic_data(spec, truth, np.ones((spec.ny, spec.nx), bool), rng)
    thetas = np.vstack([truth[None], W.draw_thetas(spec, 3, rng)])
    say(f"[edge] {name}: {spec.nx}x{spec.ny} s={spec.supersample} sigma={spec.psf_sigma_px:.4f}")
    grid = gk.Grid(spec, max_batch=8)
    grid.set_data(data, err)
    th = torch.tensor(thetas, device="cuda")
    maps = grid.maps(th).cpu().numpy().astype(np.float64)
    logl = grid.loglike(th).cpu().numpy()
    _, g = grid.loglike_grad(th[:2])
    g = g.cpu().numpy()
    for k, t in enumerate(thetas):
        F = M.psf_maps(spec, t)
        ref = np.stack([F[0], F[1], F[2], 1.0 / F[3]])
        for m in (0, 2, 3):
            assert np.max(np.abs(maps[k, m] / ref[m] - 1.0)) < MAP_RTOL, (k, m)
        assert np.max(np.abs(maps[k, 1] - ref[1])) <= MAP_RTOL * np.max(np.abs(ref[1])) + 1e-6
        lo = M.loglike(spec, data, err, t)
        tol = LOGL_ATOL if k == 0 else bound(spec, data, err, t)
        assert abs(logl[k] - lo) <= tol, (k, logl[k], lo)
        if k < 2:
            check_grad(g[k], M.grad_complex_step(spec, data, err, t), f"{name}[{k}]")
    grid.close()


def test_single_valid_pixel_and_non_finite_data(gk):
    spec = W.GridSpec(15, 11, 0.2, 3, 1.0, 1, 1, W.HALO_NFW)
    rng = np.random.default_rng(99)
    truth = W.draw_thetas(spec, 1, rng)[0]
    data, err = M.synthetic_data(spec, truth, np.ones((spec.ny, spec.nx), bool), rng)
    thetas = np.vstack([truth[None], W.draw_thetas(spec, 3, rng)])
    th = torch.tensor(thetas, device="cuda")
    # non-finite data values and errors mark their pixels invalid
    d2, e2 = data.copy(), err.copy()
    d2[0, 3, 4] = np.nan
    d2[1, 5, 5] = np.inf
    e2[2, 7, 2] = np.nan
    e2[3, 1, 1] = -1.0
    # a single valid pixel (of one map)
    e1 = np.zeros_like(err)
    e1[2, 6, 9] = err[2, 6, 9]
    for tag, (d, e) in {"non-finite": (d2, e2), "one pixel": (data, e1)}.items():
        grid = gk.Grid(spec, max_batch=8)
        grid.set_data(d, e)
        logl = grid.loglike(th).cpu().numpy()
        _, g = grid.loglike_grad(th[:2])
        for k, t in enumerate(thetas):
            lo = M.loglike(spec, d, e, t)
            tol = LOGL_ATOL if k == 0 else bound(spec, d, e, t)
            assert abs(logl[k] - lo) <= tol, (tag, k, logl[k], lo)
        check_grad(g.cpu().numpy()[0], M.grad_complex_step(spec, d, e, thetas[0]), tag)
        say(f"  {tag}: truth logL gpu {logl[0]:.6f} oracle {M.loglike(spec, d, e, thetas[0]):.6f}")
        grid.close()


def test_psf_beyond_the_limits_is_rejected(gk):
    import ctypes
    h = ctypes.c_void_p()
    for spec in (W.GridSpec(10, 10, 0.1, 5, 2.0, 1, 1, W.HALO_NFW),     # 3 sigma s = 30 > 25
                 W.GridSpec(10, 10, 0.1, 1, 3.7, 1, 1, W.HALO_NFW)):    # lag 2 pad / s = 22 > 10
        desc = gk.make_desc(spec)
        assert gk._lib.create_grid(ctypes.byref(desc), 2, ctypes.byref(h)) == gk.GK_EINVAL
        assert "PSF too wide" in gk.last_error()


@pytest.mark.parametrize("bulge", [W.BULGE_HERNQUIST, W.BULGE_JAFFE])
def test_tail_branches(gk, bulge):
    """A bulge of R_b = 5e-4 kpc and a disc of R_d = 1e-3 kpc on a 0.3 kpc/px
    grid: the lattice reaches s = R / R_b > 4096 and y = r / (2 R_d) > 1024, so
    the special functions run on their large-argument tails (cubics in 1/s and
    1/y whose slopes the adjoint takes analytically)."""
    spec = W.GridSpec(24, 20, 0.3, 3, 1.0, bulge, 1, W.HALO_NFW)
    names = W.param_names(spec)
    rng = np.random.default_rng(zlib.crc32(f"tails-{bulge}".encode()))
    truth = W.draw_thetas(spec, 1, rng)[0]
    truth[names.index("logMb")], truth[names.index("Rb")] = 9.0, 5e-4
    truth[names.index("Rd1")] = 1e-3
    # largest s and y on the lattice: every point is >= 0.3/3 kpc from the centre
    # only near it, the far corners are ~3.6 kpc out
    rmax = 0.3 * np.hypot(12, 10)
    assert rmax / 5e-4 > 4096 and rmax / (2 * 1e-3) > 1024
    data, err = M.synthetic_data(spec, truth, np.ones((spec.ny, spec.nx), bool), rng)
    other = truth.copy()
    other[names.index("incl")] += 3.0
    other[names.index("Rb")] = 8e-4
    thetas = np.vstack([truth[None], other[None]])
    say(f"[edge] tails, bulge kind {bulge}")
    grid = gk.Grid(spec, max_batch=4)
    grid.set_data(data, err)
    th = torch.tensor(thetas, device="cuda")
    maps = grid.maps(th).cpu().numpy().astype(np.float64)
    logl = grid.loglike(th).cpu().numpy()
    _, g = grid.loglike_grad(th)
    g = g.cpu().numpy()
    for k, t in enumerate(thetas):
        F = M.psf_maps(spec, t)
        ref = np.stack([F[0], F[1], F[2], 1.0 / F[3]])
        for m in (0, 2, 3):
            assert np.max(np.abs(maps[k, m] / ref[m] - 1.0)) < MAP_RTOL, (k, m)
        assert np.max(np.abs(maps[k, 1] - ref[1])) <= MAP_RTOL * np.max(np.abs(ref[1])) + 1e-6
        lo = M.loglike(spec, data, err, t)
        tol = LOGL_ATOL if k == 0 else bound(spec, data, err, t)
        assert abs(logl[k] - lo) <= tol, (k, logl[k], lo)
        check_grad(g[k], M.grad_complex_step(spec, data, err, t), f"tails[{k}]")
    grid.close()


LARGE = {
    # sides past the 384 pixels that an earlier adjoint layout capped, and the
    # 4096-pixel maximum in each direction (forward bands and adjoint blocks
    # of the library's default shapes)
    "wide_square": W.GridSpec(420, 400, 0.05, 1, 0.8, 1, 1, W.HALO_NFW),
    "widest_row": W.GridSpec(4096, 2, 0.02, 1, 1.2, 2, 1, W.HALO_HERNQUIST),
    "tallest_column": W.GridSpec(3, 4096, 0.02, 1, 1.0, 1, 1, W.HALO_NONE),
}


@pytest.mark.parametrize("name", list(LARGE))
def test_large_sides(gk, name):
    spec = LARGE[name]
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    truth = W.draw_thetas(spec, 1, rng)[0]
    data, err = M.synthetic_data(spec, truth, np.ones((spec.ny, spec.nx), bool), rng)
    thetas = np.vstack([truth[None], W.draw_thetas(spec, 1, rng)])
    say(f"[edge] {name}: {spec.nx}x{spec.ny} s={spec.supersample} sigma={spec.psf_sigma_px:.4f}")
    grid = gk.Grid(spec, max_batch=4)
    grid.set_data(data, err)
    say(f"[edge] {name}: launch shape {grid.launch_shape(2)}, adjoint shape {grid.adjoint_shape()}")
    th = torch.tensor(thetas, device="cuda")
    maps = grid.maps(th).cpu().numpy().astype(np.float64)
    logl = grid.loglike(th).cpu().numpy()
    _, g = grid.loglike_grad(th[:1])
    g = g.cpu().numpy()
    for k, t in enumerate(thetas):
        F = M.psf_maps(spec, t)
        ref = np.stack([F[0], F[1], F[2], 1.0 / F[3]])
        for m in (0, 2, 3):
            assert np.max(np.abs(maps[k, m] / ref[m] - 1.0)) < MAP_RTOL, (k, m)
        assert np.max(np.abs(maps[k, 1] - ref[1])) <= MAP_RTOL * np.max(np.abs(ref[1])) + 1e-6
        lo = M.loglike(spec, data, err, t)
        # the truth row: LOGL_ATOL up to 4e4 residuals, beyond that the FP32
        # random-walk bound (the 420 x 400 grid has 6.7e5)
        tol = logl_tol(spec, data, err, t, "truth") if k == 0 else bound(spec, data, err, t)
        assert abs(logl[k] - lo) <= tol, (k, logl[k], lo)
    check_grad(g[0], M.grad_complex_step(spec, data, err, truth), f"{name}[0]")
    grid.close()
