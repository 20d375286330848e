"""Model-level pins of the oracle: invariants, limits, Algorithm-1 equivalence,
zero chi^2 at a noiseless truth, gradient consistency (no GPU)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import model as M
from oracle import special as S


def spec_small(**kw):
    base = dict(nx=12, ny=10, pixel_kpc=0.3, supersample=3, psf_sigma_px=0.8,
                bulge=W.BULGE_HERNQUIST, n_discs=2, halo=W.HALO_NFW)
    base.update(kw)
    return W.GridSpec(**base)


def theta_for(spec, **over):
    vals = dict(x0=0.3, y0=-0.4, PA=35.0, incl=55.0, logMb=10.2, Rb=0.7, MLb=4.0,
                logMd1=10.4, Rd1=1.2, MLd1=2.0, k1=0.4, logMd2=10.8, Rd2=3.0, MLd2=2.5,
                k2=0.8, logMh=12.0, c=9.0, Rh=30.0)
    vals.update(over)
    return np.array([vals[n] for n in W.param_names(spec)])


def sky_from_disc_frame(spec, th, xp, yp):
    """Sky pixel coordinates of points given in the rotated (major-axis) frame."""
    p = M.unpack(spec, th)
    pa = math.radians(p["PA"])
    dx = xp * math.cos(pa) - yp * math.sin(pa)
    dy = xp * math.sin(pa) + yp * math.cos(pa)
    x = dx / spec.pixel_kpc + 0.5 * (spec.nx - 1) + p["x0"]
    y = dy / spec.pixel_kpc + 0.5 * (spec.ny - 1) + p["y0"]
    return x, y


RNG = np.random.default_rng(7)
XP = RNG.uniform(-4, 4, 200)
YP = RNG.uniform(-4, 4, 200)


def test_face_on_gives_zero_velocity():
    spec = spec_small()
    th = theta_for(spec, incl=1e-9)
    x, y = sky_from_disc_frame(spec, th, XP, YP)
    out = M.point_model(spec, th, x, y)
    # |v| <= sin(i) v_int; v_int is bounded by sqrt(3) times the dispersion here
    assert np.max(np.abs(out[1])) < math.sin(math.radians(1e-9)) * 5 * np.max(out[2])


def test_minor_axis_antisymmetry_and_major_axis_symmetry():
    spec = spec_small()
    th = theta_for(spec)
    a = M.point_model(spec, th, *sky_from_disc_frame(spec, th, XP, YP))
    b = M.point_model(spec, th, *sky_from_disc_frame(spec, th, -XP, YP))
    c = M.point_model(spec, th, *sky_from_disc_frame(spec, th, XP, -YP))
    np.testing.assert_allclose(b[1], -a[1], rtol=1e-10, atol=1e-10)
    np.testing.assert_allclose(c[1], a[1], rtol=1e-10, atol=1e-10)
    for m in (0, 2, 3):
        np.testing.assert_allclose(b[m], a[m], rtol=1e-10)
        np.testing.assert_allclose(c[m], a[m], rtol=1e-10)


def test_velocity_sign_and_position_angle_convention():
    # On the +x' major axis cos(phi) = 1, so v = -k sin i v_int < 0 for k > 0,
    # and |v| along the PA direction exceeds |v| along the minor axis.
    spec = spec_small(n_discs=1, halo=W.HALO_NONE)
    th = theta_for(spec, PA=30.0)
    R = np.array([1.5])
    x, y = sky_from_disc_frame(spec, th, R, np.zeros(1))
    # sky direction of the major axis must be 30 deg counter-clockwise from +x
    p = M.unpack(spec, th)
    ang = math.degrees(math.atan2(y[0] - (0.5 * (spec.ny - 1) + p["y0"]),
                                  x[0] - (0.5 * (spec.nx - 1) + p["x0"])))
    assert ang == pytest.approx(30.0)
    v_major = M.point_model(spec, th, x, y)[1][0]
    assert v_major < 0
    xm, ym = sky_from_disc_frame(spec, th, np.zeros(1), R)
    assert abs(M.point_model(spec, th, xm, ym)[1][0]) < 1e-12


def test_k_limits():
    spec = spec_small(n_discs=1, bulge=W.BULGE_NONE)
    x, y = sky_from_disc_frame(spec, theta_for(spec), XP, YP)
    out0 = M.point_model(spec, theta_for(spec, k1=0.0), x, y)
    assert np.max(np.abs(out0[1])) == 0.0
    out1 = M.point_model(spec, theta_for(spec, k1=1.0), x, y)
    assert np.max(np.abs(out1[2])) < 1e-12 * np.max(np.abs(out1[1]))
    # intermediate k: v^2 / (k^2 sin^2 i cos^2 phi) + 3 sigma^2 / (1 - k^2) = 2 v_int^2
    k = 0.6
    th = theta_for(spec, k1=k)
    out = M.point_model(spec, th, x, y)
    p = M.unpack(spec, th)
    si = math.sin(math.radians(p["incl"]))
    pa = math.radians(p["PA"])
    cosphi = XP / np.sqrt(XP ** 2 + (YP / math.cos(math.radians(p["incl"]))) ** 2)
    vint2_a = out[1] ** 2 / (k * si * cosphi) ** 2
    vint2_b = 3 * out[2] ** 2 / (1 - k * k)
    np.testing.assert_allclose(vint2_a, vint2_b, rtol=1e-9)


def test_bulge_only_dispersion_and_ml():
    spec = spec_small(n_discs=0, halo=W.HALO_NONE)
    th = theta_for(spec)
    x, y = sky_from_disc_frame(spec, th, XP, YP)
    out = M.point_model(spec, th, x, y)
    p = M.unpack(spec, th)
    Mb, Rb = 10 ** p["logMb"], p["Rb"]
    s = np.sqrt(XP ** 2 + YP ** 2) / Rb
    sig2 = M.G_KPC * Mb / Rb * S.hq_h(s) / (6.0 * S.hq_g(s))
    assert np.max(np.abs(out[1])) == 0.0
    np.testing.assert_allclose(out[2] ** 2, sig2, rtol=1e-12)
    np.testing.assert_allclose(out[3], 1.0 / p["MLb"], rtol=1e-14)
    # surface brightness in Lsun/pc^2
    np.testing.assert_allclose(out[0], 1e-6 * Mb * S.hq_g(s) / (2 * math.pi * Rb ** 2) / p["MLb"],
                               rtol=1e-14)


def test_light_weighted_ml_two_components():
    spec = spec_small(n_discs=1, halo=W.HALO_NONE)
    th = theta_for(spec)
    x, y = sky_from_disc_frame(spec, th, XP, YP)
    out = M.point_model(spec, th, x, y)
    p = M.unpack(spec, th)
    # <L/M> lies between the component values
    lo, hi = sorted([1 / p["MLb"], 1 / p["MLd1"]])
    assert np.all(out[3] >= lo - 1e-15) and np.all(out[3] <= hi + 1e-15)


def test_psf_partition_of_unity_and_delta_limit():
    spec = spec_small()
    taps, Wsum, pad = M.stencil(spec)
    assert len(taps) == sum(1 for a in range(-pad, pad + 1) for b in range(-pad, pad + 1)
                            if a * a + b * b <= (3 * spec.psf_sigma_px * 3) ** 2)
    nfy, nfx = spec.ny * 3 + 2 * pad, spec.nx * 3 + 2 * pad
    f = np.full((nfy, nfx), 2.5)
    np.testing.assert_allclose(M.convolve_lattice(spec, f), 2.5, rtol=1e-14)
    # sigma -> 0: a single tap, F = f at pixel centres
    spec0 = spec_small(psf_sigma_px=0.05)
    assert len(M.stencil(spec0)[0]) == 1
    th = theta_for(spec0)
    jj, ii = np.mgrid[0:spec0.ny, 0:spec0.nx]
    direct = M.point_model(spec0, th, ii.astype(float), jj.astype(float))
    np.testing.assert_allclose(M.psf_maps(spec0, th), direct, rtol=1e-14)


def test_known_stencil_tap_counts():
    # 3 sigma circular stencils of the benchmark workloads
    assert len(M.stencil(W.workload("tiny").spec)[0]) == 69
    assert len(M.stencil(W.workload("realistic").spec)[0]) == 293
    assert len(M.stencil(W.workload("stress").spec)[0]) == 2029


def test_flux_conservation_s1():
    # With s = 1 the PSF average preserves total flux when the source is
    # negligible in the pad band.
    spec = W.GridSpec(41, 41, 0.2, 1, 1.3, W.BULGE_NONE, 1, W.HALO_NONE)
    th = np.array([0.2, -0.1, 20.0, 40.0, 10.0, 0.15, 1.0, 0.5])
    f = M.model_lattice(spec, th)[0]
    _, _, pad = M.stencil(spec)
    F = M.psf_maps(spec, th)[0]
    inner = f[pad:pad + spec.ny, pad:pad + spec.nx]
    assert F.sum() == pytest.approx(inner.sum(), rel=1e-9)


def test_disc_sky_mass_and_bulge_projected_mass():
    # Summing Sigma over the sky recovers M_d (the 1/cos i of the projected
    # density is cancelled by the foreshortened area).
    spec = W.GridSpec(161, 161, 0.05, 1, 0.1, W.BULGE_NONE, 1, W.HALO_NONE)
    th = np.array([0.0, 0.0, 20.0, 60.0, 10.0, 0.4, 1.0, 0.5])
    jj, ii = np.mgrid[0:spec.ny, 0:spec.nx]
    out = M.point_model(spec, th, ii.astype(float), jj.astype(float))
    sigma = out[0] / out[3] * 1e6                      # Msun / kpc^2
    assert sigma.sum() * spec.pixel_kpc ** 2 == pytest.approx(1e10, rel=2e-3)


def test_alg1_equals_shared_lattice():
    spec = spec_small(nx=7, ny=6)
    th = theta_for(spec)
    np.testing.assert_allclose(M.psf_maps_alg1(spec, th), M.psf_maps(spec, th), rtol=1e-12)


def test_noiseless_truth_has_zero_chi2_and_zero_gradient():
    spec = spec_small()
    th = theta_for(spec)
    F = M.psf_maps(spec, th)
    data = np.stack([F[0], F[1], F[2], 1 / F[3]])
    err = W.error_maps(data)
    chi2, norm = M.loglike_terms(spec, data, err, th)
    assert max(chi2) < 1e-20
    assert M.loglike(spec, data, err, th) == pytest.approx(-0.5 * norm, rel=1e-15)
    g = M.grad_complex_step(spec, data, err, th)
    assert np.max(np.abs(g)) < 1e-8


def test_gradient_complex_step_matches_central_fd():
    spec = spec_small()
    th = theta_for(spec)
    rng = np.random.default_rng(3)
    data, err = M.synthetic_data(spec, th, np.ones((spec.ny, spec.nx), bool), rng)
    th2 = th * (1 + 0.01 * rng.standard_normal(th.shape))
    g = M.grad_complex_step(spec, data, err, th2)
    fd = M.grad_central_fd(spec, data, err, th2)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-6 * np.max(np.abs(g)))


def test_invalid_parameters_give_minus_inf():
    spec = spec_small()
    th = theta_for(spec)
    data = np.ones((4, spec.ny, spec.nx))
    err = np.ones((4, spec.ny, spec.nx))
    names = W.param_names(spec)
    for name, bad in [("Rb", -1.0), ("MLb", 0.0), ("incl", 90.0), ("incl", 0.0),
                      ("k1", 1.5), ("Rd2", 0.0), ("c", -2.0)]:
        t = th.copy()
        t[names.index(name)] = bad
        assert M.loglike(spec, data, err, t) == -math.inf


def test_masks_drop_pixels():
    spec = spec_small()
    th = theta_for(spec)
    rng = np.random.default_rng(5)
    mask = W.elliptical_mask(spec.nx, spec.ny, 4.5, 3.5)
    data, err = M.synthetic_data(spec, th, mask, rng)
    chi2, norm = M.loglike_terms(spec, data, err, th)
    ok = err > 0
    assert ok[0].sum() == mask.sum()
    e = err[ok]
    assert norm == pytest.approx(np.sum(np.log(2 * math.pi * e * e)))


def test_paper_table_masses_bookkeeping():
    """Sum of the visible masses of the paper's best fits (Table 2 and the
    colour-M/L table of Appendix C) against the totals quoted in the text."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "paper_masses.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    for tag, lb, ld1, ld2, total in rows:
        s = sum(10 ** float(v) for v in (lb, ld1, ld2))
        assert s == pytest.approx(float(total), rel=0.02), tag


def test_jaffe_bulge_only_dispersion_ml_and_sky_mass():
    spec = spec_small(bulge=W.BULGE_JAFFE, n_discs=0, halo=W.HALO_NONE)
    th = theta_for(spec)
    x, y = sky_from_disc_frame(spec, th, XP, YP)
    out = M.point_model(spec, th, x, y)
    p = M.unpack(spec, th)
    Mb, Rb = 10 ** p["logMb"], p["Rb"]
    s = np.sqrt(XP ** 2 + YP ** 2) / Rb
    # Appendix B: sigma^2 = G Mb^2 h / (4 pi Rb^3 Sigma), Sigma = Mb g / Rb^2
    np.testing.assert_allclose(out[2] ** 2, M.G_KPC * Mb / Rb * S.jf_h(s) / (4 * math.pi * S.jf_g(s)),
                               rtol=1e-12)
    np.testing.assert_allclose(out[3], 1.0 / p["MLb"], rtol=1e-14)
    assert np.max(np.abs(out[1])) == 0.0
    # the sky-integrated bulge mass on a grid of 5 R_b half-width (centre on a
    # pixel corner) against the 2-D quadrature of the projected density over
    # the same square (a units, one quadrant times four)
    big = W.GridSpec(200, 200, 0.01, 1, 0.1, W.BULGE_JAFFE, 0, W.HALO_NONE)
    thb = np.array([0.0, 0.0, 0.0, 45.0, 10.0, 0.2, 1.0])
    jj, ii = np.mgrid[0:big.ny, 0:big.nx]
    ob = M.point_model(big, thb, ii.astype(float), jj.astype(float))
    # the cusp (Sigma ~ 1/R) defeats the midpoint rule in the central cells, so
    # the central 20 x 20 pixels are left out of both sides
    keep = (np.abs(ii - 99.5) > 10) | (np.abs(jj - 99.5) > 10)
    sky = (ob[0] / ob[3] * 1e6)[keep].sum() * big.pixel_kpc ** 2 / 1e10
    from scipy import integrate
    half, core = 100 * big.pixel_kpc / 0.2, 10 * big.pixel_kpc / 0.2
    f = lambda v, u: S.jf_g(np.array([math.hypot(u, v)]))[0]
    q_all, _ = integrate.dblquad(f, 0, half, 0, half, epsrel=1e-9)
    q_core, _ = integrate.dblquad(f, 0, core, 0, core, epsrel=1e-9)
    assert sky == pytest.approx(4 * (q_all - q_core), rel=1e-3)   # midpoint rule, h = R_b / 20


def test_jaffe_bulge_circular_velocity_enters_vint():
    spec = spec_small(bulge=W.BULGE_JAFFE, n_discs=1, halo=W.HALO_NONE)
    th = theta_for(spec, k1=0.0)
    x, y = sky_from_disc_frame(spec, th, XP, YP)
    out = M.point_model(spec, th, x, y)
    p = M.unpack(spec, th)
    incl = math.radians(p["incl"])
    r = np.sqrt(XP ** 2 + (YP / math.cos(incl)) ** 2)
    vb2 = M.G_KPC * 10 ** p["logMb"] / (r + p["Rb"])
    vd2 = 2 * M.G_KPC * 10 ** p["logMd1"] / p["Rd1"] * S.freeman_phi(r / (2 * p["Rd1"]))
    # k = 0: the disc's sigma^2 = (vb2 + vd2) / 3, light-weighted with the bulge's
    Md, Rd, MLd = 10 ** p["logMd1"], p["Rd1"], p["MLd1"]
    Bd = 1e-6 * Md * np.exp(-r / Rd) / (2 * math.pi * Rd ** 2 * math.cos(incl)) / MLd
    Mb, Rb = 10 ** p["logMb"], p["Rb"]
    s = np.sqrt(XP ** 2 + YP ** 2) / Rb
    Bb = 1e-6 * Mb * S.jf_g(s) / Rb ** 2 / p["MLb"]
    BbS2 = 1e-6 * M.G_KPC * Mb ** 2 * S.jf_h(s) / (4 * math.pi * Rb ** 3 * p["MLb"])
    np.testing.assert_allclose(out[2] ** 2, (BbS2 + Bd * (vb2 + vd2) / 3) / (Bb + Bd), rtol=1e-11)


# --- luminosity-weighted PSF moments (psf_mode 1) ------------------------------
def _lw(spec):
    import dataclasses
    return dataclasses.replace(spec, psf_mode=W.PSF_LUMINOSITY)


def test_lw_moments_reduce_to_maps_without_psf():
    spec = spec_small(psf_sigma_px=0.0)
    th = theta_for(spec)
    np.testing.assert_allclose(M.psf_maps(_lw(spec), th), M.psf_maps(spec, th), rtol=1e-12, atol=1e-12)


def test_lw_moments_conserve_light_momentum_energy_and_mass():
    # s = 1 and a source negligible in the pad band: the PSF moves light around
    # but conserves the totals of B, B v, B (sigma^2 + v^2) and the mass
    spec = _lw(W.GridSpec(41, 41, 0.2, 1, 1.3, W.BULGE_NONE, 1, W.HALO_NFW))
    th = np.array([0.2, -0.1, 20.0, 40.0, 10.0, 0.15, 1.0, 0.5, 11.5, 8.0])
    f = M.model_lattice(spec, th)
    _, _, pad = M.stencil(spec)
    B, V, S, LM = (x[pad:pad + spec.ny, pad:pad + spec.nx] for x in f)
    F = M.psf_maps(spec, th)
    assert F[0].sum() == pytest.approx(B.sum(), rel=1e-9)
    assert (F[0] * F[1]).sum() == pytest.approx((B * V).sum(), rel=1e-8, abs=1e-9 * np.abs(B * V).sum())
    assert (F[0] * (F[2] ** 2 + F[1] ** 2)).sum() == pytest.approx((B * (S * S + V * V)).sum(), rel=1e-9)
    assert (F[0] / F[3]).sum() == pytest.approx((B / LM).sum(), rel=1e-9)


def test_lw_alg1_equals_shared_lattice():
    spec = _lw(spec_small(nx=7, ny=6))
    th = theta_for(spec)
    np.testing.assert_allclose(M.psf_maps_alg1(spec, th), M.psf_maps(spec, th), rtol=1e-11, atol=1e-12)


def test_lw_dispersion_includes_unresolved_rotation():
    # under a PSF the luminosity-weighted dispersion exceeds the light-weighted
    # average of sigma where the velocity field has a gradient
    spec = spec_small(nx=15, ny=15, psf_sigma_px=1.5)
    th = theta_for(spec, k1=0.9, k2=0.9)
    F0, F1 = M.psf_maps(spec, th), M.psf_maps(_lw(spec), th)
    assert np.median(F1[2] - F0[2]) > 0


# --- per-map pixelisation: a shared frame for the centre parameters --------
def test_frame_of_own_pixel_size_changes_nothing():
    spec = spec_small()
    same = spec_small(frame_px_kpc=spec.pixel_kpc)
    th = theta_for(spec)
    assert M.frame_scale(same) == 1.0
    np.testing.assert_array_equal(M.psf_maps(same, th), M.psf_maps(spec, th))


def test_frame_scale_samples_the_same_sky_on_a_finer_grid():
    """Without PSF and supersampling a map is the model at the pixel centres:
    a grid of half the pixel size, its centre parameters given in the coarse
    grid's pixels, holds the coarse map at every second pixel."""
    coarse = spec_small(nx=15, ny=11, pixel_kpc=0.2, supersample=1, psf_sigma_px=0.0)
    fine = spec_small(nx=29, ny=21, pixel_kpc=0.1, supersample=1, psf_sigma_px=0.0, frame_px_kpc=0.2)
    th = theta_for(coarse, x0=0.37, y0=-0.61)
    assert M.frame_scale(fine) == 2.0
    a = M.psf_maps(coarse, th)
    b = M.psf_maps(fine, th)[:, ::2, ::2]
    for m in (0, 2, 3):
        np.testing.assert_allclose(b[m], a[m], rtol=1e-12)
    np.testing.assert_allclose(b[1], a[1], atol=1e-10 * np.abs(a[1]).max())


def test_frame_offset_cuts_a_window_out_of_a_larger_grid():
    """A small grid that covers columns 7..17 and rows 2..10 of a larger grid
    of the same pixels, PSF and lattice holds the larger grid's maps there,
    PSF included: its frame centre (the larger grid's centre) sits at
    (10 - 7, 8 - 2) of its own pixels, i.e. (-2, +2) from its own centre."""
    big = spec_small(nx=21, ny=17)
    win = spec_small(nx=11, ny=9, frame_dx=-2.0, frame_dy=2.0)
    th = theta_for(big)
    a = M.psf_maps(big, th)[:, 2:11, 7:18]
    b = M.psf_maps(win, th)
    for m in (0, 2, 3):
        np.testing.assert_allclose(b[m], a[m], rtol=1e-12)
    np.testing.assert_allclose(b[1], a[1], atol=1e-10 * np.abs(a[1]).max())


def test_joint_likelihood_of_maps_split_over_grids_equals_one_grid():
    """The four Gaussian terms are independent: one grid carrying B and
    another carrying v, sigma and M/L (zero errors elsewhere) give the
    likelihood of one grid carrying all four."""
    spec = spec_small()
    th = theta_for(spec)
    rng = np.random.default_rng(11)
    data, err = M.synthetic_data(spec, th, np.ones((spec.ny, spec.nx), bool), rng)
    ea, eb = err.copy(), err.copy()
    ea[1:] = 0.0
    eb[0] = 0.0
    t2 = theta_for(spec, Rd1=1.5, incl=48.0)
    one = M.loglike(spec, data, err, t2)
    two = M.loglike_joint([spec, spec], [data, data], [ea, eb], t2)
    assert two == pytest.approx(one, rel=1e-13)
    assert M.loglike(spec, data, ea, t2) != pytest.approx(one, rel=1e-3)
