"""GPU parity: the HIP path against the FP64 oracle on the same seeded inputs.

Tolerances (see the derivation in the design notes):
* maps: per-pixel relative 1e-4 for surface brightness, dispersion and M/L;
  |dv| <= 1e-4 max|v| for the velocity, which crosses zero;
* log-likelihood: absolute 1e-3 at the truth of noisy synthetic data; away
  from it |dlogL| <= 1e-3 + eps * sum_i |r_i| |F_i| / e_i with eps = 1e-5, the
  first-order effect of a relative map error eps on the chi^2.
"""
import math
import sys
import zlib

import numpy as np
import pytest
import torch

import workloads as W
from oracle import model as M

pytestmark = pytest.mark.gpu

MAP_RTOL = 1e-4
LOGL_ATOL = 1e-3
MAP_EPS = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gk():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_06819_amd as gk
    return gk


def oracle_maps(spec, th):
    F = M.psf_maps(spec, th)
    return np.stack([F[0], F[1], F[2], 1.0 / F[3]])


def check_maps(got, ref, tag):
    got = np.asarray(got, dtype=np.float64)
    for m in (0, 2, 3):
        rel = np.max(np.abs(got[m] / ref[m] - 1.0))
        assert rel < MAP_RTOL, f"{tag} map {m}: rel err {rel:.3e}"
    vmax = np.max(np.abs(ref[1]))
    dv = np.max(np.abs(got[1] - ref[1]))
    assert dv <= MAP_RTOL * vmax + 1e-6, f"{tag} velocity: {dv:.3e} vs max {vmax:.3e}"
    return max(np.max(np.abs(got[m] / ref[m] - 1.0)) for m in (0, 2, 3)), dv / max(vmax, 1e-30)


def logl_bound(spec, data, err, th):
    F = oracle_maps(spec, th)
    ok = M.valid_masks(data, err)
    tot = 0.0
    for m in range(4):
        r = (F[m][ok[m]] - data[m][ok[m]]) / err[m][ok[m]]
        tot += np.sum(np.abs(r) * np.abs(F[m][ok[m]]) / err[m][ok[m]])
    return LOGL_ATOL + MAP_EPS * tot


CASES = {
    # name: (spec, mask axes or None, n_random_theta)
    "tiny": (W.workload("tiny").spec, None, 12),
    "realistic": (W.workload("realistic").spec, (38.0, 33.6), 3),
    "ragged_s3_2d_hq": (W.GridSpec(37, 23, 0.2, 3, 1.2, 1, 2, W.HALO_HERNQUIST), (15.0, 9.0), 6),
    "nobulge_1d": (W.GridSpec(29, 31, 0.15, 3, 0.9, 0, 1, W.HALO_NFW), None, 6),
    "nobulge_2d_nohalo": (W.GridSpec(24, 18, 0.25, 1, 1.6, 0, 2, W.HALO_NONE), None, 6),
    "bulge_only_s5": (W.GridSpec(17, 19, 0.3, 5, 0.7, 1, 0, W.HALO_NONE), (7.0, 8.0), 4),
    "no_psf": (W.GridSpec(21, 20, 0.2, 3, 0.0, 1, 1, W.HALO_NFW), None, 4),
}


def make_case(name):
    spec, axes, n = CASES[name]
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    truth = W.draw_thetas(spec, 1, rng)[0]
    mask = (W.elliptical_mask(spec.nx, spec.ny, *axes) if axes
            else np.ones((spec.ny, spec.nx), bool))
    data, err = M.synthetic_data(spec, truth, mask, rng)
    thetas = np.vstack([truth[None], W.draw_thetas(spec, n, rng)])
    return spec, data, err, thetas


@pytest.mark.parametrize("name", list(CASES))
def test_maps_and_loglike_match_oracle(gk, name):
    spec, data, err, thetas = make_case(name)
    say(f"[parity] case={name} nx={spec.nx} ny={spec.ny} s={spec.supersample} "
        f"B={len(thetas)} P={spec.n_params}")
    grid = gk.Grid(spec, max_batch=64)
    grid.set_data(data, err)
    th = torch.tensor(thetas, dtype=torch.float64, device="cuda")
    maps = grid.maps(th).cpu().numpy()
    logl = grid.loglike(th).cpu().numpy()
    torch.cuda.synchronize()
    worst_map = 0.0
    for k, t in enumerate(thetas):
        ref = oracle_maps(spec, t)
        e, ev = check_maps(maps[k], ref, f"{name}[{k}]")
        worst_map = max(worst_map, e, ev)
        lo = M.loglike(spec, data, err, t)
        tol = LOGL_ATOL if k == 0 else logl_bound(spec, data, err, t)
        assert abs(logl[k] - lo) <= tol, f"{name}[{k}] logL {logl[k]!r} vs {lo!r} (tol {tol:.3g})"
        if k == 0:
            say(f"  truth: logL gpu={logl[k]:.6f} oracle={lo:.6f} diff={logl[k]-lo:.2e}")
    say(f"  worst map error {worst_map:.2e}")
    grid.close()


def test_band_shapes_do_not_change_results(gk):
    spec, data, err, thetas = make_case("ragged_s3_2d_hq")
    say("[parity] band shapes on ragged_s3_2d_hq")
    th = torch.tensor(thetas, dtype=torch.float64, device="cuda")
    grid = gk.Grid(spec, max_batch=64)
    grid.set_data(data, err)
    grid.set_launch_shape(1, spec.ny, spec.nx)
    ref_maps = grid.maps(th).cpu()
    ref_l = grid.loglike(th).cpu()
    for bh, bw in [(1, 1), (5, 7), (8, 37), (23, 4), (3, 16)]:
        grid.set_launch_shape(1, bh, bw)
        mp = grid.maps(th).cpu()
        ll = grid.loglike(th).cpu()
        assert torch.equal(mp, ref_maps), (bh, bw)
        np.testing.assert_allclose(ll.numpy(), ref_l.numpy(), rtol=1e-12, atol=1e-9)
    grid.close()


def test_determinism_and_edge_cases(gk):
    spec, data, err, thetas = make_case("tiny")
    say("[parity] determinism and edge cases")
    grid = gk.Grid(spec, max_batch=64)
    grid.set_data(data, err)
    th = torch.tensor(thetas, dtype=torch.float64, device="cuda")
    a = grid.loglike(th)
    b = grid.loglike(th)
    assert torch.equal(a, b)
    # invalid rows give -inf, valid rows are unaffected
    bad = th.clone()
    names = W.param_names(spec)
    bad[1, names.index("Rb")] = -1.0
    bad[2, names.index("incl")] = 95.0
    bad[3, names.index("k1")] = 1.5
    bad[4, 0] = float("nan")
    out = grid.loglike(bad).cpu()
    assert torch.all(torch.isinf(out[1:5])) and torch.all(out[1:5] < 0)
    assert torch.equal(out[5:], a.cpu()[5:])
    mp = grid.maps(bad).cpu()
    assert torch.all(torch.isnan(mp[1:5]))
    # B = 0 enqueues nothing; padded stride
    empty = torch.empty(0, spec.n_params, dtype=torch.float64, device="cuda")
    assert grid.loglike(empty).numel() == 0
    wide = torch.zeros(th.shape[0], spec.n_params + 5, dtype=torch.float64, device="cuda")
    wide[:, :spec.n_params] = th
    assert torch.equal(grid.loglike(wide), a)
    # a fully masked data set gives the pure normalisation (0)
    grid2 = gk.Grid(spec, max_batch=4)
    grid2.set_data(data, np.zeros_like(err))
    assert torch.all(grid2.loglike(th[:4]).cpu() == 0.0)
    grid2.close()
    grid.close()


def test_errors_on_device(gk):
    spec = W.workload("tiny").spec
    grid = gk.Grid(spec, max_batch=4)
    th = torch.zeros(2, spec.n_params, dtype=torch.float64, device="cuda")
    with pytest.raises(gk.GalkinError) as e:
        grid.loglike(th)
    assert e.value.code == gk.GK_ESTATE
    grid.set_data(np.ones((4, spec.ny, spec.nx)), np.ones((4, spec.ny, spec.nx)))
    with pytest.raises(gk.GalkinError):
        grid.loglike(torch.zeros(5, spec.n_params, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        grid.loglike(torch.zeros(2, spec.n_params - 1, dtype=torch.float64, device="cuda"))
    grid.close()
