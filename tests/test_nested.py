"""Batched nested sampling (paper Sec. 2.5) pinned on likelihoods whose
evidence is known in closed form (CPU), and on a two-parameter galaxy problem
whose evidence the oracle integrates by brute-force quadrature (GPU)."""
import math
import zlib

import numpy as np
import pytest
import torch
from scipy.special import erf

import workloads as W
from oracle import model as M


def gaussian_case(d, sigma, mu):
    mu = torch.tensor(mu, dtype=torch.float64)

    def loglike(th):
        r2 = ((th - mu) ** 2).sum(1)
        return -0.5 * r2 / sigma ** 2 - 0.5 * d * math.log(2 * math.pi * sigma ** 2)

    # Z = (1 / 2^d) prod_i P(-1 < x_i < 1) for x_i ~ N(mu_i, sigma^2)
    mass = [0.5 * (erf((1 - m) / (sigma * math.sqrt(2))) - erf((-1 - m) / (sigma * math.sqrt(2))))
            for m in mu.tolist()]
    log_z = -d * math.log(2.0) + sum(math.log(p) for p in mass)
    return loglike, log_z


@pytest.mark.parametrize("d,sigma,mu", [(2, 0.1, [0.3, -0.2]), (5, 0.2, [0.0, 0.5, -0.3, 0.1, 0.9])])
def test_gaussian_evidence(d, sigma, mu):
    from paper_2205_06819_amd.nested import nested_sampling
    loglike, truth = gaussian_case(d, sigma, mu)
    g = torch.Generator().manual_seed(zlib.crc32(f"ns{d}".encode()))
    res = nested_sampling(loglike, [-1.0] * d, [1.0] * d, n_live=400, k=40, f=1e-4,
                          walk_steps=20, generator=g)
    assert abs(res.log_z - truth) < 4 * res.log_z_err + 0.05, (res.log_z, truth, res.log_z_err)
    # the posterior mean is the Gaussian's mean (truncation included for the last axis)
    post = res.posterior_mean().numpy()
    assert np.allclose(post[: d - 1], np.array(mu[: d - 1]), atol=4 * sigma / math.sqrt(400) + 0.01)
    # information of a Gaussian inside a box: H = log(vol fraction^-1) - d / 2 (untruncated)
    if d == 2:
        h_true = -truth - 0.5 * d - 0.5 * d * math.log(2 * math.pi * sigma ** 2)
        assert res.information == pytest.approx(h_true, abs=0.3)


def test_flat_likelihood_has_unit_evidence_ratio():
    # L = const: Z = L exactly, whatever the shrinkage bookkeeping
    from paper_2205_06819_amd.nested import nested_sampling
    res = nested_sampling(lambda th: torch.full((th.shape[0],), -3.0, dtype=torch.float64),
                          [0.0, 0.0], [1.0, 1.0], n_live=100, k=10, f=1e-2, walk_steps=2,
                          generator=torch.Generator().manual_seed(1))
    assert res.log_z == pytest.approx(-3.0, abs=1e-9)


@pytest.mark.gpu
def test_galaxy_two_parameter_evidence_against_oracle_quadrature():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_06819_amd as gk
    from paper_2205_06819_amd.nested import nested_sampling
    # a small grid with large errors (a broad posterior), two free parameters
    spec = W.GridSpec(16, 16, 0.25, 1, 1.0, W.BULGE_HERNQUIST, 1, W.HALO_NONE)
    rng = np.random.default_rng(zlib.crc32(b"ns-galaxy"))
    truth = W.draw_thetas(spec, 1, rng)[0]
    names = W.param_names(spec)
    data, err = M.synthetic_data(spec, truth, np.ones((spec.ny, spec.nx), bool), rng)
    err = err * 20.0
    free = [names.index("logMb"), names.index("logMd1")]
    lo = np.array([truth[free[0]] - 0.5, truth[free[1]] - 0.5])
    hi = lo + 1.0
    grid = gk.Grid(spec, max_batch=512)
    grid.set_data(data, err)
    base = torch.tensor(truth, dtype=torch.float64, device="cuda")

    def loglike(th2):
        th = base.repeat(th2.shape[0], 1)
        th[:, free] = th2
        return grid.loglike(th.contiguous())

    res = nested_sampling(loglike, lo, hi, n_live=300, k=30, f=1e-4, walk_steps=20, device="cuda",
                          generator=torch.Generator(device="cuda").manual_seed(3))
    # oracle: midpoint-rule quadrature of L over the prior box (uniform prior density 1)
    n = 48
    xs = lo[0] + (np.arange(n) + 0.5) / n
    ys = lo[1] + (np.arange(n) + 0.5) / n
    ll = np.empty((n, n))
    for a, x in enumerate(xs):
        for b, y in enumerate(ys):
            t = truth.copy()
            t[free[0]], t[free[1]] = x, y
            ll[a, b] = M.loglike(spec, data, err, t)
    m = ll.max()
    log_z_ref = m + math.log(np.exp(ll - m).mean())
    print(f"[ns] logZ GPU nested {res.log_z:.3f} +- {res.log_z_err:.3f}, oracle quadrature {log_z_ref:.3f}, "
          f"{res.n_like} likelihood calls", flush=True)
    assert abs(res.log_z - log_z_ref) < 4 * res.log_z_err + 0.1
    grid.close()


def _two_param_galaxy(gk):
    spec = W.GridSpec(16, 16, 0.25, 1, 1.0, W.BULGE_HERNQUIST, 1, W.HALO_NONE)
    rng = np.random.default_rng(zlib.crc32(b"ns-galaxy"))
    truth = W.draw_thetas(spec, 1, rng)[0]
    names = W.param_names(spec)
    data, err = M.synthetic_data(spec, truth, np.ones((spec.ny, spec.nx), bool), rng)
    err = err * 20.0
    free = [names.index("logMb"), names.index("logMd1")]
    lo = np.array([truth[free[0]] - 0.5, truth[free[1]] - 0.5])
    hi = lo + 1.0
    grid = gk.Grid(spec, max_batch=512)
    grid.set_data(data, err)
    base = torch.tensor(truth, dtype=torch.float64, device="cuda")
    free_t = torch.tensor(free, device="cuda")   # a device index: no host copy inside a graph capture

    def loglike(th2):
        th = base.repeat(th2.shape[0], 1)
        th.index_copy_(1, free_t, th2)
        return grid.loglike(th)
    return spec, truth, data, err, free, lo, hi, grid, loglike


@pytest.mark.gpu
def test_graph_iteration_replays_equal_eager_iteration():
    """One nested-sampling iteration captured in a HIP graph, replayed three
    times from the same restored state and generator seed, with eager work and
    synchronisations in between: every replay equals the eager iteration."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_06819_amd as gk
    from paper_2205_06819_amd.nested import _State
    print("case: two-parameter galaxy, 64 live points, 8 replaced, 5 walk steps", flush=True)
    _, _, _, _, _, lo, hi, grid, loglike = _two_param_galaxy(gk)
    gen = torch.Generator(device="cuda").manual_seed(11)
    lo_t = torch.tensor(lo, dtype=torch.float64, device="cuda")
    hi_t = torch.tensor(hi, dtype=torch.float64, device="cuda")
    st = _State(loglike, lo_t, hi_t, 64, 8, 1e-3, 5, gen)
    names = ("live", "live_l", "log_x", "log_z", "stop", "dead_x", "dead_l", "dead_lw")
    st.iteration()                      # a first iteration so that log_z is finite
    saved = {n: getattr(st, n).clone() for n in names}

    def restore():
        for n in names:
            getattr(st, n).copy_(saved[n])

    gen.manual_seed(99)
    st.iteration()
    ref = {n: getattr(st, n).clone() for n in names}
    restore()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        gen.manual_seed(5)
        st.iteration()                  # warm-up on the side stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    g.register_generator_state(gen)
    with torch.cuda.graph(g):
        st.iteration()
    for rep in range(3):
        restore()
        junk = torch.randn(1000, device="cuda").sum()      # eager work between replays
        torch.cuda.synchronize()
        gen.manual_seed(99)
        g.replay()
        torch.cuda.synchronize()
        for n in names:
            assert torch.equal(getattr(st, n), ref[n]), (rep, n)
        assert float(junk) == float(junk)
    del g
    grid.close()


@pytest.mark.gpu
def test_graph_mode_evidence_against_oracle_quadrature():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_06819_amd as gk
    from paper_2205_06819_amd.nested import nested_sampling
    spec, truth, data, err, free, lo, hi, grid, loglike = _two_param_galaxy(gk)
    res = nested_sampling(loglike, lo, hi, n_live=300, k=30, f=1e-4, walk_steps=20, device="cuda",
                          generator=torch.Generator(device="cuda").manual_seed(4), graph=True,
                          check_every=4)
    n = 48
    xs = lo[0] + (np.arange(n) + 0.5) / n
    ys = lo[1] + (np.arange(n) + 0.5) / n
    ll = np.empty((n, n))
    for a, x in enumerate(xs):
        for b, y in enumerate(ys):
            t = truth.copy()
            t[free[0]], t[free[1]] = x, y
            ll[a, b] = M.loglike(spec, data, err, t)
    m = ll.max()
    log_z_ref = m + math.log(np.exp(ll - m).mean())
    print(f"[ns graph] logZ {res.log_z:.3f} +- {res.log_z_err:.3f} ({res.n_iter} iterations), "
          f"oracle quadrature {log_z_ref:.3f}", flush=True)
    assert abs(res.log_z - log_z_ref) < 4 * res.log_z_err + 0.1
    grid.close()


@pytest.mark.gpu
def test_bayes_factor_prefers_the_generating_model():
    """Model comparison in the style of the paper's Table 3 on synthetic data:
    data made by a bulge + one disc and by a bulge + two distinct discs, each
    fitted with both component sets by the batched nested sampler (all
    parameters free over the benchmark priors, graph-captured iterations); the
    log Bayes factor must favour the generating model by more than four
    combined standard deviations."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_06819_amd as gk
    from paper_2205_06819_amd.nested import log_bayes_factor, nested_sampling
    common = dict(nx=20, ny=20, pixel_kpc=0.4, supersample=1, psf_sigma_px=1.0,
                  bulge=W.BULGE_HERNQUIST, halo=W.HALO_NONE)
    s1, s2 = W.GridSpec(n_discs=1, **common), W.GridSpec(n_discs=2, **common)
    # x0, y0, PA, i | log Mb, Rb, M/L_b | discs: log Md, Rd, M/L, k
    t1 = np.array([0.3, -0.4, 35.0, 55.0, 9.2, 0.6, 3.0, 9.6, 2.0, 2.0, 0.7])
    t2 = np.array([0.3, -0.4, 35.0, 55.0, 9.2, 0.6, 3.0, 9.9, 0.9, 1.5, 0.95, 10.6, 4.5, 4.0, 0.2])
    rng = np.random.default_rng(zlib.crc32(b"bayes-factor"))
    mask = np.ones((20, 20), bool)

    def data_of(spec, t):
        # the benchmark noise recipe with 3 km/s instead of 10 km/s on v and
        # sigma: precise kinematics leave no room for a faint, extended
        # second disc (its mass is at least 1e9 Msun under the prior)
        F = M.psf_maps(spec, t)
        maps = np.stack([F[0], F[1], F[2], 1.0 / F[3]])
        err = W.error_maps(maps, mask)
        err[1:3] *= 0.3
        return W.noisy_data(maps, err, rng), err
    datasets = {"B+D": data_of(s1, t1), "B+D1+D2": data_of(s2, t2)}
    results = {}
    for dname, (data, err) in datasets.items():
        for mname, spec in (("B+D", s1), ("B+D1+D2", s2)):
            grid = gk.Grid(spec, max_batch=512)
            grid.set_data(data, err)
            b = W.prior_bounds(spec)
            res = nested_sampling(lambda th: grid.loglike(th), b[:, 0], b[:, 1], n_live=400, k=40, f=1e-3,
                                  walk_steps=25, max_iter=6000, device="cuda", graph=True, check_every=8,
                                  generator=torch.Generator(device="cuda").manual_seed(
                                      zlib.crc32(f"{dname}/{mname}".encode())))
            results[dname, mname] = res
            print(f"[ns model] data {dname}, model {mname}: logZ {res.log_z:.2f} +- {res.log_z_err:.2f} "
                  f"(H {res.information:.1f}, {res.n_iter} iterations, {res.n_like} likelihoods)", flush=True)
            grid.close()
    lb1, e1 = log_bayes_factor(results["B+D", "B+D"], results["B+D", "B+D1+D2"])
    lb2, e2 = log_bayes_factor(results["B+D1+D2", "B+D1+D2"], results["B+D1+D2", "B+D"])
    print(f"[ns model] ln B(B+D : B+D1+D2 | B+D data) = {lb1:.2f} +- {e1:.2f}; "
          f"ln B(B+D1+D2 : B+D | B+D1+D2 data) = {lb2:.2f} +- {e2:.2f}", flush=True)
    assert lb1 > 4 * e1, (lb1, e1)
    assert lb2 > 4 * e2, (lb2, e2)
