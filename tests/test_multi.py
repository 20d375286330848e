"""GPU parity of the many-grid launch (loglike_multi): galaxies of different
sizes and component sets in one launch give the single-grid
results (to FP64 summation order) and the oracle's at each galaxy's truth."""
import sys
import zlib

import numpy as np
import pytest
import torch

import workloads as W
from oracle import model as M

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_06819_amd as gk
    return gk


SPECS = [
    # spec, rows
    (W.GridSpec(40, 40, W.PK_50MPC, 1, 1.5, 1, 1, W.HALO_NFW), 5),
    (W.GridSpec(37, 23, 0.2, 3, 1.2, 1, 2, W.HALO_HERNQUIST), 0),
    (W.GridSpec(29, 31, 0.15, 3, 0.9, 0, 1, W.HALO_NFW), 3),
    (W.GridSpec(24, 18, 0.25, 1, 1.6, 0, 2, W.HALO_NONE), 7),
    (W.GridSpec(17, 19, 0.3, 5, 0.7, 1, 0, W.HALO_NONE), 2),
    (W.GridSpec(21, 20, 0.2, 3, 0.0, 1, 1, W.HALO_NFW), 4),
    (W.GridSpec(70, 66, 0.12, 3, 1.06, 1, 2, W.HALO_NFW), 3),   # wider than one band
    (W.GridSpec(26, 28, 0.2, 3, 1.06, W.BULGE_JAFFE, 2, W.HALO_NFW), 4),
    (W.GridSpec(30, 24, 0.15, 3, 1.1, 1, 2, W.HALO_NFW, psf_mode=W.PSF_LUMINOSITY), 3),
    (W.GridSpec(22, 26, 0.1, 1, 1.4, 1, 1, W.HALO_HERNQUIST, frame_px_kpc=0.2, frame_dx=0.5), 2),
]


def build(gk, specs):
    grids, truths, datas = [], [], []
    for k, (spec, rows) in enumerate(specs):
        rng = np.random.default_rng(zlib.crc32(f"multi{k}".encode()))
        truth = W.draw_thetas(spec, 1, rng)[0]
        mask = np.ones((spec.ny, spec.nx), bool)
        if k % 2 == 0:
            mask = W.elliptical_mask(spec.nx, spec.ny, 0.45 * spec.nx, 0.4 * spec.ny)
        data, err = M.synthetic_data(spec, truth, mask, rng)
        g = gk.Grid(spec, max_batch=16)
        g.set_data(data, err)
        grids.append(g)
        truths.append(truth)
        datas.append((data, err))
    return grids, truths, datas


def stacked_thetas(specs, truths, stride, seed=7):
    rng = np.random.default_rng(seed)
    rows, offs = [], [0]
    for (spec, n), truth in zip(specs, truths):
        th = np.zeros((n, stride))
        if n:
            th[:, :spec.n_params] = np.vstack([truth[None], W.draw_thetas(spec, n - 1, rng)])[:n]
            th[:, spec.n_params:] = 1e300      # padding columns are never read
        rows.append(th)
        offs.append(offs[-1] + n)
    return np.vstack(rows), offs


def test_multi_matches_single_grid_and_oracle(gk):
    say(f"[multi] {len(SPECS)} grids, uneven sizes and component sets")
    grids, truths, datas = build(gk, SPECS)
    stride = max(s.n_params for s, _ in SPECS) + 2
    th_np, offs = stacked_thetas(SPECS, truths, stride)
    th_np[offs[3] + 2, 2] = np.nan                      # one invalid row
    th = torch.tensor(th_np, device="cuda")
    handles = [g.handle for g in grids]
    got = gk.loglike_multi(handles, th, offs).cpu().numpy()
    again = gk.loglike_multi(handles, th, offs).cpu().numpy()
    assert np.array_equal(got, again, equal_nan=True)   # cached plan, same order
    for k, ((spec, n), g) in enumerate(zip(SPECS, grids)):
        if n == 0:
            continue
        sl = slice(offs[k], offs[k + 1])
        ref = g.loglike(th[sl, :spec.n_params].contiguous()).cpu().numpy()
        np.testing.assert_allclose(got[sl], ref, rtol=1e-12, atol=1e-9, err_msg=f"grid {k}")
        data, err = datas[k]
        lo = M.loglike(spec, data, err, th_np[offs[k]][:spec.n_params])
        assert abs(got[offs[k]] - lo) <= 1e-3, (k, got[offs[k]], lo)
        say(f"  grid {k} {spec.nx}x{spec.ny} s={spec.supersample}: truth logL {got[offs[k]]:.5f} oracle {lo:.5f}")
    assert got[offs[3] + 2] == -np.inf
    for g in grids:
        g.close()


def test_multi_new_offsets_grad_and_eviction(gk):
    say("[multi] offsets change, gradient path, destroyed grid")
    specs = SPECS[:4] + SPECS[5:6]
    grids, truths, _ = build(gk, specs)
    stride = max(s.n_params for s, _ in specs)
    th_np, offs = stacked_thetas(specs, truths, stride, seed=11)
    th = torch.tensor(th_np, device="cuda")
    handles = [g.handle for g in grids]
    a = gk.loglike_multi(handles, th, offs).cpu().numpy()
    # fewer rows per galaxy: a different plan on the same grids
    offs2 = [0]
    for (spec, n) in specs:
        offs2.append(offs2[-1] + max(0, n - 1))
    rows2 = np.concatenate([np.arange(offs[k], offs[k] + max(0, n - 1)) for k, (_, n) in enumerate(specs)])
    th2 = th[torch.tensor(rows2, device="cuda", dtype=torch.long)].contiguous()
    b = gk.loglike_multi(handles, th2, offs2).cpu().numpy()
    np.testing.assert_allclose(b, a[rows2], rtol=1e-12, atol=1e-9)
    # gradient through the same entry point equals the single-grid gradient
    grad = torch.zeros_like(th)
    c = gk.loglike_multi(handles, th, offs, grad=grad).cpu().numpy()
    np.testing.assert_allclose(c, a, rtol=1e-12, atol=1e-9)
    for k, ((spec, n), g) in enumerate(zip(specs, grids)):
        if n == 0:
            continue
        sl = slice(offs[k], offs[k + 1])
        _, gref = g.loglike_grad(th[sl, :spec.n_params].contiguous())
        assert torch.equal(grad[sl, :spec.n_params], gref), k
    # destroying a grid drops its cached plans; a new grid set still works
    grids[1].close()
    keep = [0, 2, 3, 4]
    offs3 = [0]
    for k in keep:
        offs3.append(offs3[-1] + specs[k][1])
    th3 = torch.cat([th[offs[k]:offs[k + 1]] for k in keep]).contiguous()
    d = gk.loglike_multi([handles[k] for k in keep], th3, offs3).cpu().numpy()
    np.testing.assert_allclose(d, np.concatenate([a[offs[k]:offs[k + 1]] for k in keep]), rtol=1e-12, atol=1e-9)
    for k in keep:
        grids[k].close()


def test_multi_argument_errors(gk):
    spec = SPECS[0][0]
    g = gk.Grid(spec, max_batch=2)
    th = torch.zeros(3, spec.n_params, dtype=torch.float64, device="cuda")
    with pytest.raises(gk.GalkinError) as e:                 # no data yet
        gk.loglike_multi([g.handle], th, [0, 1])
    assert e.value.code == gk.GK_ESTATE
    rng = np.random.default_rng(0)
    truth = W.draw_thetas(spec, 1, rng)[0]
    data, err = M.synthetic_data(spec, truth, np.ones((spec.ny, spec.nx), bool), rng)
    g.set_data(data, err)
    with pytest.raises(gk.GalkinError) as e:                 # rows > max_batch
        gk.loglike_multi([g.handle], th, [0, 3])
    assert e.value.code == gk.GK_EINVAL
    with pytest.raises(gk.GalkinError) as e:                 # the same grid twice
        gk.loglike_multi([g.handle, g.handle], th, [0, 1, 2])
    assert e.value.code == gk.GK_EINVAL
    out = gk.loglike_multi([], th, [0])
    assert out.numel() == 0
    g.close()


def test_multi_follows_new_data_with_fewer_maps(gk):
    """set_data that drops maps (zero errors) changes which maps a grid
    convolves; a cached many-grid plan must follow."""
    say("[multi] data with fewer maps after a cached plan")
    specs = SPECS[:3]
    grids, truths, datas = build(gk, specs)
    stride = max(s.n_params for s, _ in specs)
    th_np, offs = stacked_thetas(specs, truths, stride, seed=5)
    th = torch.tensor(th_np, device="cuda")
    handles = [g.handle for g in grids]
    gk.loglike_multi(handles, th, offs)
    data, err = datas[0]
    err = err.copy()
    err[1:] = 0.0                     # B only
    grids[0].set_data(data, err)
    got = gk.loglike_multi(handles, th, offs).cpu().numpy()
    for k, ((spec, n), g) in enumerate(zip(specs, grids)):
        if n == 0:
            continue
        sl = slice(offs[k], offs[k + 1])
        ref = g.loglike(th[sl, :spec.n_params].contiguous()).cpu().numpy()
        np.testing.assert_allclose(got[sl], ref, rtol=1e-12, atol=1e-9, err_msg=f"grid {k}")
    lo = M.loglike(specs[0][0], data, err, th_np[0][:specs[0][0].n_params])
    assert abs(got[0] - lo) <= 1e-3, (got[0], lo)
    for g in grids:
        g.close()
