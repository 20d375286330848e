"""The autotuner on small grids: the shapes it installs give the same maps
bit for bit and the same log-likelihoods to 1e-12 (only the FP64 band sums
regroup), the many-grid policy search leaves loglike_multi equal to the
per-grid calls, the adjoint search leaves the gradient within FP32 rounding
of the default shape's, and a cached shape the library rejects is re-tuned."""
import json
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


def _grid(gk, spec, mask, B, seed):
    rng = np.random.default_rng(seed)
    truth = W.draw_thetas(spec, 1, rng)[0]
    data, err = M.synthetic_data(spec, truth, mask, rng)
    g = gk.Grid(spec, max_batch=B)
    g.set_data(data, err)
    th = np.vstack([truth[None], W.draw_thetas(spec, B - 1, rng)])
    return g, torch.tensor(th, dtype=torch.float64, device="cuda")


def test_tune_keeps_results(gk, tmp_path, monkeypatch):
    from paper_2205_06819_amd import autotune
    monkeypatch.setattr(autotune, "CACHE", str(tmp_path / "cache.json"))
    spec = W.GridSpec(37, 23, 0.2, 3, 1.2, 1, 2, W.HALO_HERNQUIST)
    say("[tune] 37x23 s=3 B=96: tune() vs the default shape")
    g, th = _grid(gk, spec, W.elliptical_mask(37, 23, 15.0, 9.0), 96, zlib.crc32(b"tune"))
    maps0, ll0 = g.maps(th).cpu(), g.loglike(th).cpu().numpy()
    h, w, st, ms = autotune.tune(g, th, reps=1, use_cache=True)
    assert g.launch_shape(96) == (h, w, st)
    assert torch.equal(g.maps(th).cpu(), maps0)
    np.testing.assert_allclose(g.loglike(th).cpu().numpy(), ll0, rtol=1e-12, atol=0)
    key = autotune._key(g, 96)
    cache = json.load(open(autotune.CACHE))
    assert cache[key][:3] == [h, w, st]
    # a cached shape this build rejects (9 pixel rows per model phase > 4)
    # falls through to tuning
    cache[key] = [4, 16, 9, 0.01]
    json.dump(cache, open(autotune.CACHE, "w"))
    h2, w2, st2, _ = autotune.tune(g, th, reps=1, use_cache=True)
    assert st2 <= 4 and g.launch_shape(96) == (h2, w2, st2)
    np.testing.assert_allclose(g.loglike(th).cpu().numpy(), ll0, rtol=1e-12, atol=0)
    g.close()


def test_cache_key_separates_psf_mode_and_frame(gk):
    from paper_2205_06819_amd import autotune
    a = W.GridSpec(21, 20, 0.2, 3, 1.0, 1, 1, W.HALO_NFW)
    b = W.GridSpec(21, 20, 0.2, 3, 1.0, 1, 1, W.HALO_NFW, psf_mode=W.PSF_LUMINOSITY)
    c = W.GridSpec(21, 20, 0.2, 3, 1.0, 1, 1, W.HALO_NFW, frame_px_kpc=0.4, frame_dx=1.0)
    ga, gb, gc = (gk.Grid(s, max_batch=4) for s in (a, b, c))
    keys = {autotune._key(x, 4) for x in (ga, gb, gc)}
    assert len(keys) == 3
    for x in (ga, gb, gc):
        x.close()


def test_tune_multi_keeps_results(gk):
    from paper_2205_06819_amd import autotune
    say("[tune] tune_multi over 5 grids of sides 23..70")
    specs = [W.GridSpec(n, n, W.PK_50MPC, 3, W.SIGMA_FWHM_2P5, *cs)
             for n, cs in zip((23, 41, 70, 33, 52), [(1, 1, 0), (1, 1, 2), (1, 2, 2), (1, 2, 2), (1, 1, 2)])]
    grids, ths = [], []
    for k, s in enumerate(specs):
        g, th = _grid(gk, s, np.ones((s.ny, s.nx), bool), 24, 100 + k)
        grids.append(g)
        ths.append(th)
    stride = max(s.n_params for s in specs)
    big = torch.zeros(24 * len(specs), stride, dtype=torch.float64, device="cuda")
    for k, th in enumerate(ths):
        big[24 * k:24 * (k + 1), :th.shape[1]] = th
    offs = np.arange(0, 24 * len(specs) + 1, 24, dtype=np.int32)
    handles = [g.handle for g in grids]
    ref = gk.loglike_multi(handles, big, offs).cpu().numpy()
    pol, st, ms = autotune.tune_multi(grids, big, offs, reps=1)
    assert 0 <= pol < 4 and st in (0, 1, 2)
    got = gk.loglike_multi(handles, big, offs).cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=0)
    for k, g in enumerate(grids):
        one = g.loglike(big[24 * k:24 * (k + 1), :specs[k].n_params].contiguous()).cpu().numpy()
        np.testing.assert_allclose(got[24 * k:24 * (k + 1)], one, rtol=1e-12, atol=0)
        g.close()


def test_tune_adjoint_keeps_gradients(gk):
    from paper_2205_06819_amd import autotune
    spec = W.workload("realistic").spec
    say("[tune] tune_adjoint on the realistic cube, B=64")
    g, th = _grid(gk, spec, W.elliptical_mask(80, 80, 38.0, 33.6), 64, zlib.crc32(b"tune-adj"))
    l0, g0 = (x.cpu().numpy() for x in g.loglike_grad(th))
    shapes = [(40, 80, 2), (80, 40, 3), (27, 27, 0), (40, 40, 5)]
    h, w, r, ms = autotune.tune_adjoint(g, th, reps=1, shapes=shapes)
    assert g.adjoint_shape() == (h, w, r)
    l1, g1 = (x.cpu().numpy() for x in g.loglike_grad(th))
    assert np.array_equal(l1, l0)          # the forward pass is unchanged
    # only the FP32 order of the per-point adjoint sums within bands changes
    for a, b in zip(g1, g0):
        assert np.all(np.abs(a - b) <= 1e-5 * np.linalg.norm(b) + 1e-5 * np.abs(b)), (a, b)
    # every candidate shape gives the same gradient to that precision
    for sh in shapes:
        g.set_adjoint_shape(*sh)
        gs = g.loglike_grad(th)[1].cpu().numpy()
        for a, b in zip(gs, g0):
            assert np.all(np.abs(a - b) <= 1e-5 * np.linalg.norm(b) + 1e-5 * np.abs(b)), sh
    g.close()
