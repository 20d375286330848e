"""Pins of the oracle's circular-velocity terms and cosmological constants
against independent definitions (no GPU).

The model's v_int (Sec. 2.3, the intrinsic rotation curve that the Satoh
decomposition splits into rotation and dispersion) is the quadrature sum of
the circular velocities of the bulge (Sec. 2.2, bulge circular-velocity
equation: the Hernquist sphere), the discs (Sec. 2.3, Freeman) and the halo
(Hernquist as in the paper, or NFW as in the benchmark workloads).  Each
term is checked here against G M(<r) / r with M(<r) integrated by
quadrature from that component's own density, the halo's r200 against the
critical density computed in SI units from CODATA / IAU constants, and the
whole sum against the model's dispersion map through the Satoh relation.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle import model as M
from oracle import special as S

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")

# SI constants independent of the oracle's G in kpc (km/s)^2 / Msun
G_SI = 6.67430e-11                    # m^3 kg^-1 s^-2 (CODATA 2018)
GM_SUN_SI = 1.32712440018e20          # m^3 s^-2 (IAU 2015 nominal)
MSUN_KG = GM_SUN_SI / G_SI            # kg (the IAU nominal solar mass)
KPC_M = 3.0856775814913673e19         # m
MPC_M = 1e3 * KPC_M


def rho_crit_si(h: float) -> float:
    """3 H0^2 / (8 pi G) in Msun / kpc^3, H0 = 100 h km/s/Mpc, all in SI."""
    H0 = 100.0 * h * 1e3 / MPC_M                      # s^-1
    rho = 3.0 * H0 * H0 / (8.0 * math.pi * G_SI)      # kg / m^3
    return rho * KPC_M ** 3 / MSUN_KG


def r200_from_definition(M200: float, h: float) -> float:
    """Radius inside which the mean density is 200 rho_crit."""
    return (M200 / (200.0 * rho_crit_si(h) * 4.0 / 3.0 * math.pi)) ** (1.0 / 3.0)


def test_rho_crit_matches_si_and_the_textbook_value():
    # PDG: rho_c = 1.87834(4) e-26 h^2 kg m^-3
    H0 = 100.0e3 / MPC_M
    assert 3.0 * H0 * H0 / (8.0 * math.pi * G_SI) == pytest.approx(1.87834e-26, rel=5e-5)
    assert M.rho_crit(0.7) == pytest.approx(rho_crit_si(0.7), rel=1e-9)
    assert M.rho_crit(0.7) == pytest.approx(135.99, abs=0.01)
    assert M.rho_crit(1.0) == pytest.approx(M.rho_crit(0.7) / 0.49, rel=1e-14)


@pytest.mark.parametrize("logM, r200", [(11.0, 95.7), (12.0, 206.3), (13.0, 444.4)])
def test_r200_values(logM, r200):
    assert r200_from_definition(10.0 ** logM, 0.7) == pytest.approx(r200, abs=0.06)


def hernquist_mass_quad(M_tot: float, a: float, r: float) -> float:
    """M(<r) of the Hernquist density M a / (2 pi r (r + a)^3) by quadrature."""
    rho = lambda x: M_tot * a / (2.0 * math.pi * x * (x + a) ** 3)
    m, _ = integrate.quad(lambda x: 4.0 * math.pi * x * x * rho(x), 0.0, r, epsabs=0, epsrel=1e-12,
                          limit=200)
    return m


def nfw_mass_quad(M200: float, c: float, h: float, r: float) -> float:
    """M(<r) of the NFW density rho_s / (x (1 + x)^2), x = r / r_s, r_s = r200 / c,
    normalised so that the mass inside r200 is M200 (quadrature for both)."""
    shape = lambda t: t / (1.0 + t) ** 2
    rs = r200_from_definition(M200, h) / c
    inner, _ = integrate.quad(shape, 0.0, r / rs, epsabs=0, epsrel=1e-12, limit=200)
    whole, _ = integrate.quad(shape, 0.0, c, epsabs=0, epsrel=1e-12, limit=200)
    return M200 * inner / whole


def freeman_v2_hankel(G: float, Md: float, Rd: float, r: float) -> float:
    """Razor-thin exponential disc, from the Hankel transform of its density
    (independent of the Bessel-product formula): v^2 = (G M / R_d) u
    int_0^inf k J1(k u) / (1 + k^2)^(3/2) dk with u = r / R_d."""
    import mpmath as mp
    u = r / Rd
    with mp.workdps(25):
        f = lambda k: k * mp.besselj(1, k * u) / (1 + k * k) ** 1.5
        val = float(u * mp.quadosc(f, [0, mp.inf], omega=u))
    return G * Md / Rd * val


def _spec(halo):
    return W.GridSpec(nx=9, ny=9, pixel_kpc=0.25, supersample=1, psf_sigma_px=0.0,
                      bulge=W.BULGE_HERNQUIST, n_discs=1, halo=halo)


def _theta(spec, k=0.0, MLb=1.0e12):
    vals = dict(x0=0.0, y0=0.0, PA=0.0, incl=40.0, logMb=10.3, Rb=0.8, MLb=MLb,
                logMd1=10.6, Rd1=2.2, MLd1=3.0, k1=k, logMh=12.2, c=8.0, Rh=25.0)
    return np.array([vals[n] for n in W.param_names(spec)])


RADII = np.array([0.05, 0.4, 1.3, 3.7, 9.0])      # kpc, on the major axis


@pytest.mark.parametrize("halo", [W.HALO_NFW, W.HALO_HERNQUIST])
def test_vint_through_point_model_is_the_sum_of_enclosed_mass_terms(halo):
    # On the major axis (PA = 0, y = 0) the disc-plane radius is r = R = x'.
    # With k = 0 the disc carries sigma_d^2 = v_int^2 / 3, and with a bulge
    # M/L of 1e12 the bulge light is negligible (its mass still enters v_int),
    # so the model dispersion map gives v_int^2 = 3 sigma^2.
    spec = _spec(halo)
    th = _theta(spec)
    p = M.unpack(spec, th)
    xc = 0.5 * (spec.nx - 1)
    out = M.point_model(spec, th, xc + RADII / spec.pixel_kpc, np.full(RADII.shape, 0.5 * (spec.ny - 1)))
    vint2_model = 3.0 * out[2] ** 2
    Mb, Md = 10.0 ** p["logMb"], 10.0 ** p["logMd1"]
    for r, v2 in zip(RADII, vint2_model):
        ref = M.G_KPC * hernquist_mass_quad(Mb, p["Rb"], r) / r
        ref += freeman_v2_hankel(M.G_KPC, Md, p["Rd1"], r)
        if halo == W.HALO_NFW:
            ref += M.G_KPC * nfw_mass_quad(10.0 ** p["logMh"], p["c"], spec.hubble_h, r) / r
        else:
            ref += M.G_KPC * hernquist_mass_quad(10.0 ** p["logMh"], p["Rh"], r) / r
        assert v2 == pytest.approx(ref, rel=1e-8)


def test_vint_enters_rotation_with_the_satoh_factor():
    # k = 1 on the major axis (cos phi = 1): v_los = -sin(i) v_int, sigma_d = 0,
    # with the same v_int^2 as the dispersion route (k = 0) gives
    spec = _spec(W.HALO_NFW)
    xc, yc = 0.5 * (spec.nx - 1), 0.5 * (spec.ny - 1)
    x, y = xc + RADII / spec.pixel_kpc, np.full(RADII.shape, yc)
    out0 = M.point_model(spec, _theta(spec, k=0.0), x, y)
    out1 = M.point_model(spec, _theta(spec, k=1.0), x, y)
    si = math.sin(math.radians(40.0))
    np.testing.assert_allclose(out1[1], -si * np.sqrt(3.0) * out0[2], rtol=1e-9)
    assert np.all(out1[1] < 0.0)
    # the bulge (M/L 1e12) is dark but does not rotate: half-way k gives
    # sigma^2 = (1 - k^2) v_int^2 / 3 and v = -k sin i v_int
    out5 = M.point_model(spec, _theta(spec, k=0.5), x, y)
    np.testing.assert_allclose(out5[2] ** 2, 0.75 * out0[2] ** 2, rtol=1e-9)
    np.testing.assert_allclose(out5[1], 0.5 * out1[1], rtol=1e-10)


def test_bulge_light_weights_the_dispersion():
    # With a luminous bulge the dispersion is the light-weighted mean of the
    # bulge's own sigma_b^2 (Sec. 2.2) and the disc's v_int^2 / 3:
    # sigma^2 (B_b + B_d) = B_b sigma_b^2 + B_d v_int^2 / 3
    spec = _spec(W.HALO_NFW)
    th_dark = _theta(spec)
    th = _theta(spec, MLb=2.0)
    p = M.unpack(spec, th)
    xc, yc = 0.5 * (spec.nx - 1), 0.5 * (spec.ny - 1)
    x, y = xc + RADII / spec.pixel_kpc, np.full(RADII.shape, yc)
    vint2 = 3.0 * M.point_model(spec, th_dark, x, y)[2] ** 2
    out = M.point_model(spec, th, x, y)
    Mb, Rb = 10.0 ** p["logMb"], p["Rb"]
    s = RADII / Rb
    Bb = 1e-6 * Mb * S.hq_g(s) / (2.0 * math.pi * Rb * Rb) / p["MLb"]
    sig_b2 = M.G_KPC * Mb / Rb * S.hq_h(s) / (6.0 * S.hq_g(s))
    Bd = out[0] - Bb
    np.testing.assert_allclose(out[2] ** 2 * out[0], Bb * sig_b2 + Bd * vint2 / 3.0, rtol=1e-10)
