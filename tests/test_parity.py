"""GPU parity: the HIP path against the FP64 oracle on the same seeded inputs.

Tolerances (tests/bounds.py):
* maps: per-pixel relative 1e-4 for surface brightness, dispersion and M/L;
  |dv| <= 1e-4 max|v| for the velocity, which crosses zero;
* log-likelihood: absolute 1e-3 at the truth of noisy synthetic data; at two
  perturbations of it with chi^2/N <= 4 (the posterior bulk) 1e-3 plus the
  coherent term 2e-7 sqrt(chi^2 - chi^2_truth) ||F/e||; far from it
  |dlogL| <= 1e-3 + sum_i |r_i| dF_i / e_i with dF_i = 1e-6 |F_i|, the
  first-order effect of the worst relative map error on the chi^2.
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

from bounds import LOGL_ATOL, LW_SIGMA_EPS, MAP_RTOL, bulk_rows, chi2_of, logl_tol

N_BULK = 2      # posterior-bulk rows after the truth in every case


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


def check_maps(got, ref, tag, lw=False):
    got = np.asarray(got, dtype=np.float64)
    for m in (0, 2, 3):
        if lw and m == 2:
            # sigma^2 = F2/F0 - v^2 from FP32 moment sums: |d sigma| <=
            # LW_SIGMA_EPS (sigma^2 + v^2) / (2 sigma)
            sg, v = ref[2], ref[1]
            bound = MAP_RTOL * sg + LW_SIGMA_EPS * (sg * sg + v * v) / (2.0 * np.maximum(sg, 1e-30))
            bad = np.abs(got[2] - sg) > bound
            assert not bad.any(), f"{tag} LW dispersion: {np.abs(got[2] - sg)[bad][:4]} > {bound[bad][:4]}"
            continue
        rel = np.max(np.abs(got[m] / ref[m] - 1.0))
        assert rel < MAP_RTOL, f"{tag} map {m}: rel err {rel:.3e}"
    vmax = np.max(np.abs(ref[1]))
    dv = np.max(np.abs(got[1] - ref[1]))
    assert dv <= MAP_RTOL * vmax + 1e-6, f"{tag} velocity: {dv:.3e} vs max {vmax:.3e}"
    return max(np.max(np.abs(got[m] / ref[m] - 1.0)) for m in (0, 2, 3)), dv / max(vmax, 1e-30)


CASES = {
    # name: (spec, mask axes or None, n_random_theta)
    "tiny": (W.workload("tiny").spec, None, 12),
    "realistic": (W.workload("realistic").spec, (38.0, 33.6), 3),
    "ragged_s3_2d_hq": (W.GridSpec(37, 23, 0.2, 3, 1.2, 1, 2, W.HALO_HERNQUIST), (15.0, 9.0), 6),
    "nobulge_1d": (W.GridSpec(29, 31, 0.15, 3, 0.9, 0, 1, W.HALO_NFW), None, 6),
    "nobulge_2d_nohalo": (W.GridSpec(24, 18, 0.25, 1, 1.6, 0, 2, W.HALO_NONE), None, 6),
    "bulge_only_s5": (W.GridSpec(17, 19, 0.3, 5, 0.7, 1, 0, W.HALO_NONE), (7.0, 8.0), 4),
    "no_psf": (W.GridSpec(21, 20, 0.2, 3, 0.0, 1, 1, W.HALO_NFW), None, 4),
    # Jaffe bulge (Appendix B)
    "jaffe_2d_nfw": (W.GridSpec(33, 29, 0.15, 3, 1.06, W.BULGE_JAFFE, 2, W.HALO_NFW), (14.0, 12.0), 6),
    "jaffe_only_s5": (W.GridSpec(19, 17, 0.25, 5, 0.7, W.BULGE_JAFFE, 0, W.HALO_NONE), None, 4),
    "jaffe_1d_hq_s1": (W.GridSpec(30, 26, 0.3, 1, 1.3, W.BULGE_JAFFE, 1, W.HALO_HERNQUIST), None, 6),
    # luminosity-weighted PSF moments instead of averaged maps
    "lw_2d_nfw": (W.GridSpec(33, 29, 0.15, 3, 1.06, 1, 2, W.HALO_NFW, psf_mode=W.PSF_LUMINOSITY),
                  (14.0, 12.0), 6),
    "lw_jaffe_1d_hq_s1": (W.GridSpec(30, 26, 0.3, 1, 1.3, W.BULGE_JAFFE, 1, W.HALO_HERNQUIST,
                                     psf_mode=W.PSF_LUMINOSITY), None, 4),
    "lw_nobulge_s5": (W.GridSpec(19, 21, 0.25, 5, 0.8, 0, 2, W.HALO_NONE, psf_mode=W.PSF_LUMINOSITY),
                      None, 4),
    # centre parameters in a shared frame of 2.5x larger pixels, offset
    "frame_scaled": (W.GridSpec(31, 27, 0.1, 3, 1.0, 1, 1, W.HALO_NFW, frame_px_kpc=0.25, frame_dx=1.5,
                                frame_dy=-2.0), (12.0, 10.0), 4),
}


def make_case(name):
    spec, axes, n = CASES[name]
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    truth = W.draw_thetas(spec, 1, rng)[0]
    mask = (W.elliptical_mask(spec.nx, spec.ny, *axes) if axes
            else np.ones((spec.ny, spec.nx), bool))
    data, err = M.synthetic_data(spec, truth, mask, rng)
    thetas = np.vstack([truth[None], bulk_rows(spec, data, err, truth, rng, N_BULK),
                        W.draw_thetas(spec, n, rng)])
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
    c2t = chi2_of(spec, data, err, thetas[0])
    for k, t in enumerate(thetas):
        ref = oracle_maps(spec, t)
        e, ev = check_maps(maps[k], ref, f"{name}[{k}]", lw=spec.psf_mode == W.PSF_LUMINOSITY)
        worst_map = max(worst_map, e, ev)
        lo = M.loglike(spec, data, err, t)
        kind = "truth" if k == 0 else "bulk" if k <= N_BULK else "far"
        tol = logl_tol(spec, data, err, t, kind, c2t)
        assert abs(logl[k] - lo) <= tol, f"{name}[{k}] logL {logl[k]!r} vs {lo!r} (tol {tol:.3g})"
        if kind != "far":
            say(f"  {kind}: logL gpu={logl[k]:.6f} oracle={lo:.6f} diff={logl[k]-lo:.2e} (tol {tol:.2e})")
    say(f"  worst map error {worst_map:.2e}")
    grid.close()


@pytest.mark.parametrize("name", ["ragged_s3_2d_hq", "lw_2d_nfw", "no_psf", "jaffe_1d_hq_s1", "bulge_only_s5"])
def test_band_shapes_do_not_change_results(gk, name):
    spec, data, err, thetas = make_case(name)
    say(f"[parity] band shapes on {name}")
    th = torch.tensor(thetas, dtype=torch.float64, device="cuda")
    grid = gk.Grid(spec, max_batch=64)
    grid.set_data(data, err)
    grid.set_launch_shape(1, spec.ny, spec.nx)
    ref_maps = grid.maps(th).cpu()
    ref_l = grid.loglike(th).cpu()
    for bh, bw in [(1, 1), (5, 7), (8, 37), (23, 4), (3, 16)]:
        for steps in (0, 1, 2):            # pixel rows per model phase (0: default)
            grid.set_launch_shape(1, bh, bw, steps)
            assert grid.launch_shape(th.shape[0]) == (min(bh, spec.ny), min(bw, spec.nx), steps)
            mp = grid.maps(th).cpu()
            ll = grid.loglike(th).cpu()
            assert torch.equal(mp, ref_maps), (bh, bw, steps)
            np.testing.assert_allclose(ll.numpy(), ref_l.numpy(), rtol=1e-12, atol=1e-9)
    grid.close()


def test_luminosity_weighting_without_psf_equals_plain_maps(gk):
    """With no PSF every pixel is one lattice point, so the moment ratios give
    back the point model: both modes agree up to FP32 rounding."""
    base = W.GridSpec(21, 20, 0.2, 3, 0.0, 1, 1, W.HALO_NFW)
    lw = W.GridSpec(21, 20, 0.2, 3, 0.0, 1, 1, W.HALO_NFW, psf_mode=W.PSF_LUMINOSITY)
    rng = np.random.default_rng(zlib.crc32(b"lw-nopsf"))
    th = torch.tensor(W.draw_thetas(base, 6, rng), dtype=torch.float64, device="cuda")
    ga, gb = gk.Grid(base, max_batch=8), gk.Grid(lw, max_batch=8)
    a, b = ga.maps(th).cpu().numpy(), gb.maps(th).cpu().numpy()
    for m in (0, 3):
        np.testing.assert_allclose(b[:, m], a[:, m], rtol=1e-6)
    vmax = np.abs(a[:, 1]).max()
    assert np.abs(b[:, 1] - a[:, 1]).max() <= 1e-6 * vmax
    # sigma through sqrt(F2/F0 - v^2): absolute error ~ eps (sigma^2 + v^2) / sigma
    bound = 1e-6 * a[:, 2] + 1e-6 * (a[:, 2] ** 2 + a[:, 1] ** 2) / a[:, 2]
    assert (np.abs(b[:, 2] - a[:, 2]) <= bound).all()
    ga.close()
    gb.close()


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


# --- gradient (hand-written adjoint) -------------------------------------------
GRAD_RTOL, GRAD_NORM_TOL = 1e-3, 1e-4


def check_grad(got, ref, tag):
    tol = GRAD_RTOL * np.abs(ref) + GRAD_NORM_TOL * np.linalg.norm(ref)
    assert np.isfinite(got).all() and np.isfinite(ref).all(), f"{tag}: non-finite gradient {got}"
    bad = ~(np.abs(got - ref) <= tol)
    assert not bad.any(), f"{tag}: params {np.nonzero(bad)[0]}: gpu {got[bad]} oracle {ref[bad]}"
    return float(np.max(np.abs(got - ref) / (np.abs(ref) + np.linalg.norm(ref))))


@pytest.mark.parametrize("name,n", [("tiny", 4), ("ragged_s3_2d_hq", 3), ("nobulge_1d", 3),
                                    ("nobulge_2d_nohalo", 3), ("bulge_only_s5", 3), ("no_psf", 3),
                                    ("realistic", 2), ("jaffe_2d_nfw", 3), ("jaffe_only_s5", 2),
                                    ("jaffe_1d_hq_s1", 2), ("lw_2d_nfw", 3), ("lw_jaffe_1d_hq_s1", 2),
                                    ("lw_nobulge_s5", 2), ("frame_scaled", 3)])
def test_gradient_matches_oracle(gk, name, n):
    spec, data, err, thetas = make_case(name)
    # the truth, one posterior-bulk row and prior draws
    thetas = np.vstack([thetas[:2], thetas[N_BULK + 1:N_BULK + n - 1]])
    say(f"[grad] case={name} B={n} P={spec.n_params}")
    grid = gk.Grid(spec, max_batch=16)
    grid.set_data(data, err)
    th = torch.tensor(thetas, dtype=torch.float64, device="cuda")
    lg, g = grid.loglike_grad(th)
    ll = grid.loglike(th)
    assert torch.equal(lg, ll), "log-likelihood of the gradient call differs from loglike_batch"
    g = g.cpu().numpy()
    worst = 0.0
    for k, t in enumerate(thetas):
        ref = M.grad_complex_step(spec, data, err, t)
        worst = max(worst, check_grad(g[k], ref, f"{name}[{k}]"))
    say(f"  worst relative gradient error {worst:.2e}")
    grid.close()


ADJ_SHAPES = {
    # case: adjoint shapes (band_h, band_w, lattice rows per phase; 0 = automatic)
    "ragged_s3_2d_hq": [(1, 1, 1), (5, 4, 3), (23, 37, 8), (7, 37, 2), (3, 2, 7)],
    "bulge_only_s5": [(4, 3, 1), (19, 17, 5), (2, 17, 2), (1, 17, 0)],
    "jaffe_1d_hq_s1": [(6, 5, 4), (1, 30, 16), (26, 1, 1)],
    "lw_2d_nfw": [(8, 8, 3), (29, 10, 2), (2, 33, 1)],
    "no_psf": [(3, 3, 2), (20, 21, 1)],
}


@pytest.mark.parametrize("name", list(ADJ_SHAPES))
def test_adjoint_shapes_match_oracle(gk, name):
    """Every adjoint block shape (lattice blocks of one pixel, one row or one
    column of bands, up to 16 lattice rows per phase, masked grids, s = 1, 3,
    5, luminosity-weighted moments, no PSF) gives the oracle's gradient; the
    log-likelihood of the gradient call does not depend on it."""
    spec, data, err, thetas = make_case(name)
    thetas = thetas[:2]                                 # the truth and a posterior-bulk row
    refs = [M.grad_complex_step(spec, data, err, t) for t in thetas]
    grid = gk.Grid(spec, max_batch=8)
    grid.set_data(data, err)
    th = torch.tensor(thetas, dtype=torch.float64, device="cuda")
    ll = grid.loglike(th)
    for sh in ADJ_SHAPES[name]:
        say(f"[adjoint shape] case={name} shape={sh}")
        grid.set_adjoint_shape(*sh)
        lg, g = grid.loglike_grad(th)
        assert torch.equal(lg, ll), f"{name} {sh}: log-likelihood of the gradient call differs"
        g = g.cpu().numpy()
        for k, ref in enumerate(refs):
            check_grad(g[k], ref, f"{name}{sh}[{k}]")
    grid.close()


def test_gradient_invalid_rows_and_padding(gk):
    spec, data, err, thetas = make_case("tiny")
    grid = gk.Grid(spec, max_batch=16)
    grid.set_data(data, err)
    th = torch.zeros(3, spec.n_params + 3, dtype=torch.float64, device="cuda")
    th[:, :spec.n_params] = torch.tensor(thetas[:3])
    th[1, W.param_names(spec).index("Rb")] = -1.0
    out = torch.empty(3, dtype=torch.float64, device="cuda")
    grad = torch.full((3, spec.n_params + 3), 7.0, dtype=torch.float64, device="cuda")
    gk.loglike_grad_batch(grid.handle, th, out, grad)
    grad = grad.cpu()
    assert torch.all(grad[1] == 0.0) and torch.isinf(out[1]).item()
    assert torch.all(grad[:, spec.n_params:] == 0.0)
    ref = M.grad_complex_step(spec, data, err, thetas[0])
    check_grad(grad[0, :spec.n_params].numpy(), ref, "padded stride")
    grid.close()


def test_autograd_function(gk):
    spec, data, err, thetas = make_case("ragged_s3_2d_hq")
    grid = gk.Grid(spec, max_batch=8)
    grid.set_data(data, err)
    th = torch.tensor(thetas[:3], dtype=torch.float64, device="cuda", requires_grad=True)
    w = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device="cuda")
    (gk.LogLike.apply(th, grid) * w).sum().backward()
    _, g = grid.loglike_grad(th.detach())
    torch.testing.assert_close(th.grad, w[:, None] * g, rtol=0, atol=0)
    grid.close()


# --- HMC trajectory and HIP-graph capture ---------------------------------------
def _hmc_setup(gk, B=4):
    spec, data, err, thetas = make_case("ragged_s3_2d_hq")
    grid = gk.Grid(spec, max_batch=16)
    grid.set_data(data, err)
    P = spec.n_params
    th = torch.tensor(np.repeat(thetas[:1], B, axis=0), dtype=torch.float64, device="cuda")
    th += 1e-3 * torch.randn(th.shape, dtype=torch.float64, device="cuda",
                             generator=torch.Generator("cuda").manual_seed(5))
    # unit-ish scales: a diagonal mass from the curvature scale of each parameter
    scale = torch.tensor([0.05, 0.05, 0.5, 0.5, 0.01, 0.01, 0.01] + [0.01, 0.01, 0.01, 0.01] * 2
                         + [0.01, 0.1], dtype=torch.float64, device="cuda")[:P]
    inv_mass = scale ** 2
    mom = torch.randn(th.shape, dtype=torch.float64, device="cuda",
                      generator=torch.Generator("cuda").manual_seed(6)) / scale
    return grid, spec, th, mom, inv_mass


def test_hmc_energy_and_reversibility(gk):
    grid, spec, th, mom, inv_mass = _hmc_setup(gk)
    say("[hmc] leapfrog trajectory on ragged_s3_2d_hq")
    B, P = th.shape
    logL0 = grid.loglike(th)
    H0 = -logL0 + 0.5 * (mom ** 2 * inv_mass).sum(1)
    th1, mom1 = th.clone(), mom.clone()
    logL = torch.empty(B, dtype=torch.float64, device="cuda")
    grad = torch.empty(B, P, dtype=torch.float64, device="cuda")
    eps, n = 2e-3, 8
    gk.hmc_leapfrog(grid.handle, th1, mom1, inv_mass, eps, n, logL, grad)
    H1 = -logL + 0.5 * (mom1 ** 2 * inv_mass).sum(1)
    torch.testing.assert_close(logL, grid.loglike(th1), rtol=0, atol=0)
    dH = (H1 - H0).abs().max().item()
    say(f"  max |dH| = {dH:.3e} over {n} steps (|H| ~ {H0.abs().max().item():.3e})")
    assert dH < 1.0, dH
    # reversibility: flip the momentum and integrate back
    th2, mom2 = th1.clone(), -mom1.clone()
    gk.hmc_leapfrog(grid.handle, th2, mom2, inv_mass, eps, n, logL, grad)
    torch.testing.assert_close(th2, th, rtol=0, atol=1e-6)
    grid.close()


def test_hmc_graph_capture_replays(gk):
    grid, spec, th, mom, inv_mass = _hmc_setup(gk)
    say("[hmc] HIP-graph capture of one trajectory")
    B, P = th.shape
    logL = torch.empty(B, dtype=torch.float64, device="cuda")
    grad = torch.empty(B, P, dtype=torch.float64, device="cuda")
    th_s, mom_s = th.clone(), mom.clone()
    # eager reference: three trajectories in a row
    ref = []
    te, me = th.clone(), mom.clone()
    for _ in range(3):
        gk.hmc_leapfrog(grid.handle, te, me, inv_mass, 1e-3, 4, logL, grad)
        ref.append((te.clone(), logL.clone()))
    # captured: the same calls replayed from a graph, with eager work between replays
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        gk.hmc_leapfrog(grid.handle, th.clone(), mom.clone(), inv_mass, 1e-3, 4, logL, grad)
    torch.cuda.current_stream().wait_stream(side)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gk.hmc_leapfrog(grid.handle, th_s, mom_s, inv_mass, 1e-3, 4, logL, grad)
    th_s.copy_(th)
    mom_s.copy_(mom)
    torch.cuda.synchronize()
    for k in range(3):
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(th_s, ref[k][0]), k
        assert torch.equal(logL, ref[k][1]), k
        grid.loglike(th_s[:1])        # eager work between replays
        torch.cuda.synchronize()
    del g
    grid.close()
