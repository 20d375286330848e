"""Pins of the oracle's special functions against closed forms, brute-force
quadrature and independent high-precision evaluations (no GPU)."""
import math

import mpmath as mp
import numpy as np
import pytest
from scipy import integrate

from oracle import special as S
from oracle import model as M

pytestmark = pytest.mark.filterwarnings("ignore::scipy.integrate.IntegrationWarning")


# --- Hernquist (G = M = a = 1 units) ---------------------------------------
def rho_hq(r):
    """Hernquist density, paper Sec. 2.2 (first equation)."""
    return 1.0 / (2.0 * math.pi * r * (r + 1.0) ** 3)


def mass_hq(r):
    return r * r / (r + 1.0) ** 2


def sigma_r2_closed(r):
    """The paper's isotropic-Jeans radial dispersion (Sec. 2.2, bulge_sigma_r)."""
    return (1.0 / 12.0) * (12.0 * r * (r + 1.0) ** 3 * math.log((r + 1.0) / r)
                           - r / (r + 1.0) * (25.0 + 52.0 * r + 42.0 * r * r + 12.0 * r ** 3))


def sigma_r2_jeans(r):
    """Isotropic Jeans equation by quadrature: (1/rho) int_r^inf rho G M / r'^2 dr'."""
    # substitute x = r e^u; the integrand decays like x^-5, so u <= 60 is enough
    val, _ = integrate.quad(lambda u: rho_hq(r * math.exp(u)) * mass_hq(r * math.exp(u))
                            / (r * math.exp(u)) * 1.0, 0.0, 60.0,
                            epsabs=0, epsrel=1e-13, limit=400)
    return val / rho_hq(r)


def abel(f, R):
    """2 int_R^inf f(r) r / sqrt(r^2 - R^2) dr with r = R cosh(u)."""
    # the integrands decay at least like r^-3, so cosh(u) <= e^40 / 2 is enough
    val, _ = integrate.quad(lambda u: 2.0 * f(R * math.cosh(u)) * R * math.cosh(u), 0.0, 40.0,
                            epsabs=0, epsrel=1e-12, limit=400)
    return val


S_GRID = [0.05, 0.3, 0.5, 0.7, 0.9, 0.99, 1.01, 1.1, 1.3, 2.0, 3.0, 8.0]


@pytest.mark.parametrize("s", S_GRID)
def test_surface_density_is_abel_projection_of_rho(s):
    # Sigma_b = M g(s) / (2 pi a^2): must equal the Abel projection of rho
    sig = abel(rho_hq, s)
    assert S.hq_g(np.array([s]))[0] / (2.0 * math.pi) == pytest.approx(sig, rel=1e-9)


def test_literal_second_form_of_X_is_rejected():
    # The printed logarithmic form log[1 + sqrt(1-s^2)/s] / sqrt(1-s^2) gives a
    # projected density that disagrees with the Abel projection (reading noted
    # in the oracle); the arcsech form agrees.
    s = 0.3
    q = math.sqrt(1 - s * s)
    X_lit = math.log(1 + q / s) / q
    g_lit = ((2 + s * s) * X_lit - 3) / (1 - s * s) ** 2
    sig = abel(rho_hq, s) * 2 * math.pi
    assert abs(g_lit / sig - 1) > 0.5
    assert S.hq_g(np.array([s]))[0] == pytest.approx(sig, rel=1e-9)


@pytest.mark.parametrize("r", [0.05, 0.3, 1.0, 3.0, 10.0])
def test_paper_radial_dispersion_matches_jeans_quadrature(r):
    assert sigma_r2_closed(r) == pytest.approx(sigma_r2_jeans(r), rel=1e-8)


@pytest.mark.parametrize("s", [0.05, 0.3, 0.7, 0.99, 1.01, 1.3, 3.0, 8.0, 30.0])
def test_projected_dispersion_matches_jeans_projection(s):
    # Sigma sigma_p^2 = 2 int rho sigma_r^2 r / sqrt(r^2 - R^2) dr, sigma_r^2 from
    # brute-force Jeans quadrature, against h(s) / (12 pi).
    if s < 20:
        jeans = abel(lambda r: rho_hq(r) * sigma_r2_jeans(r), s)
    else:   # at large radii use the closed-form sigma_r^2 in extended precision
        mp.mp.dps = 90          # the closed form cancels ~ r^4 at large r
        f = lambda r: (1 / (2 * mp.pi * r * (r + 1) ** 3)) * (1 / mp.mpf(12)) * (
            12 * r * (r + 1) ** 3 * mp.log((r + 1) / r)
            - r / (r + 1) * (25 + 52 * r + 42 * r * r + 12 * r ** 3))
        jeans = float(2 * mp.quad(lambda u: f(s * mp.cosh(u)) * s * mp.cosh(u), [0, 1, 4, 12, 24]))
    assert S.hq_h(np.array([s]))[0] / (12.0 * math.pi) == pytest.approx(jeans, rel=2e-7)


def test_hernquist_special_values():
    g1 = S.hq_g(np.array([1.0]))[0]
    assert g1 == pytest.approx(4.0 / 15.0, rel=1e-14)
    # h -> 3 as s -> 0; s^4 h -> 8/5 and s^3 g -> pi/2 as s -> infinity
    assert S.hq_h(np.array([1e-9]))[0] == pytest.approx(3.0, rel=1e-6)
    s = 1e5
    assert S.hq_h(np.array([s]))[0] * s ** 4 == pytest.approx(1.6, rel=1e-4)
    assert S.hq_g(np.array([s]))[0] * s ** 3 == pytest.approx(math.pi / 2, rel=1e-4)
    # series and direct branches agree across the split points
    for edge in [math.sqrt(1 - S.T_SERIES_MAX), math.sqrt(1 + S.T_SERIES_MAX), S.W_SERIES_MIN_S]:
        lo, hi = edge * (1 - 1e-12), edge * (1 + 1e-12)
        for f in (S.hq_g, S.hq_h, S.hq_X):
            a, b = f(np.array([lo, hi]))
            assert a == pytest.approx(b, rel=1e-11)


@pytest.mark.parametrize("s", [0.1, 0.5, 0.999, 1.5, 4.0])
def test_projected_mass_closed_form(s):
    # int_0^s 2 pi s' Sigma ds' = M s^2 (X - 1) / (1 - s^2)  (Hernquist 1990)
    val, _ = integrate.quad(lambda x: x * S.hq_g(np.array([x]))[0], 0, s, epsrel=1e-12, limit=200)
    X = S.hq_X(np.array([s]))[0]
    assert val == pytest.approx(s * s * (X - 1) / (1 - s * s), rel=1e-9)


def test_total_projected_mass_is_one():
    val1, _ = integrate.quad(lambda x: x * S.hq_g(np.array([x]))[0], 0, 1, limit=200)
    val2, _ = integrate.quad(lambda x: x * S.hq_g(np.array([x]))[0], 1, np.inf, limit=400)
    assert val1 + val2 == pytest.approx(1.0, rel=1e-8)


def test_hernquist_mpmath_agreement_dense():
    mp.mp.dps = 60

    def X(s):
        s = mp.mpf(s)
        return mp.acosh(1 / s) / mp.sqrt(1 - s * s) if s < 1 else mp.asec(s) / mp.sqrt(s * s - 1)

    def h(s):
        s = mp.mpf(s)
        s2 = s * s
        return ((-3 * s2 * X(s) * (8 * s2 ** 3 - 28 * s2 ** 2 + 35 * s2 - 20) - 24 * s2 ** 3
                 + 68 * s2 ** 2 - 65 * s2 + 6) / (2 * (1 - s2) ** 3) - 6 * mp.pi * s)

    ss = np.concatenate([np.logspace(-6, 4, 80), [0.999999, 1.000001, 1.2649, 0.6325]])
    ref = np.array([float(h(x)) for x in ss])
    assert np.max(np.abs(S.hq_h(ss) / ref - 1)) < 1e-12


# --- Freeman disc ------------------------------------------------------------
def freeman_v2_hankel(R):
    """v^2 of a razor-thin exponential disc (G = M = R_d = 1) from the Hankel
    transform of its density: v^2(R) = R int_0^inf k J1(kR) / (1 + k^2)^(3/2) dk.
    Independent of the Bessel-product formula used by the oracle."""
    mp.mp.dps = 25
    f = lambda k: k * mp.besselj(1, k * R) / (1 + k * k) ** 1.5
    return float(R * mp.quadosc(f, [0, mp.inf], omega=R))


@pytest.mark.parametrize("R", [0.1, 1.0, 2.0, 5.0, 10.0])
def test_freeman_curve_matches_hankel_transform(R):
    # model: v^2 = (2 G M / R_d) y^2 [I0K0 - I1K1](y), y = R / (2 R_d)
    v2 = 2.0 * S.freeman_phi(np.array([R / 2.0]))[0]
    assert v2 == pytest.approx(freeman_v2_hankel(R), rel=1e-8)


def test_freeman_peak_and_kepler_limit():
    from scipy.optimize import minimize_scalar
    res = minimize_scalar(lambda R: -2.0 * S.freeman_phi(np.array([R / 2]))[0],
                          bounds=(1, 4), method="bounded", options={"xatol": 1e-10})
    assert res.x == pytest.approx(2.1500, abs=2e-3)       # peak near 2.15 R_d
    # Kepler: v^2 r / (G M) -> 1
    R = 400.0
    assert 2.0 * S.freeman_phi(np.array([R / 2]))[0] * R == pytest.approx(1.0, abs=1e-4)


def test_freeman_F_library_special_case():
    mp.mp.dps = 40
    for y in [1e-3, 0.1, 1.0, 5.0, 30.0, 150.0]:
        ref = (mp.besseli(0, y) * mp.besselk(0, y) - mp.besseli(1, y) * mp.besselk(1, y))
        assert S.freeman_F(np.array([y]))[0] == pytest.approx(float(ref), rel=1e-9)


# --- NFW and constants ----------------------------------------------------
def test_nfw_mu_small_x_series():
    # mu(x) = ln(1 + x) - x / (1 + x) = sum_n>=2 (-1)^n (n - 1) x^n / n
    #       = x^2/2 (1 - 4x/3 + 3x^2/2 - 8x^3/5 + ...)
    for x in (1e-4, 1e-3):
        series = x * x / 2.0 * (1.0 - 4.0 * x / 3.0 + 1.5 * x * x - 1.6 * x ** 3)
        assert S.nfw_mu(np.array([x]))[0] == pytest.approx(series, rel=1e-9, abs=0)


def test_nfw_mu_is_the_enclosed_mass_of_the_nfw_density():
    # NFW density rho ~ 1 / (x (1 + x)^2), x = r / r_s: the mass inside x is
    # 4 pi r_s^3 rho_s int_0^x t / (1 + t)^2 dt, which must be mu(x)
    for x in (0.01, 0.3, 1.0, 4.0, 25.0):
        m, _ = integrate.quad(lambda t: t / (1.0 + t) ** 2, 0.0, x, epsabs=0, epsrel=1e-13, limit=200)
        assert S.nfw_mu(np.array([x]))[0] == pytest.approx(m, rel=1e-11)
def test_gravitational_constant_in_kpc_units():
    GM_sun = 1.32712440018e20            # m^3 s^-2 (IAU)
    kpc = 3.0856775814913673e19          # m
    assert M.G_KPC == pytest.approx(GM_sun / (kpc * 1e6), rel=1e-9)
    # 0.5 arcsec at 50 Mpc
    import workloads as W
    assert W.PK_50MPC == pytest.approx(50e3 * 0.5 / 206264.806247, rel=1e-9)


# --- Jaffe (Appendix B; G = M = a = 1 units) ---------------------------------
def rho_jf(r):
    """Jaffe density (Appendix B, first equation)."""
    return 1.0 / (4.0 * math.pi * r * r * (r + 1.0) ** 2)


def mass_jf(r):
    return r / (r + 1.0)


def sigma_r2_jf_jeans(r):
    """Isotropic Jeans equation by quadrature for the Jaffe sphere."""
    val, _ = integrate.quad(lambda u: rho_jf(r * math.exp(u)) * mass_jf(r * math.exp(u))
                            / (r * math.exp(u)), 0.0, 60.0, epsabs=0, epsrel=1e-13, limit=400)
    return val / rho_jf(r)


@pytest.mark.parametrize("s", S_GRID)
def test_jaffe_surface_density_is_abel_projection_of_rho(s):
    # Sigma_b = M g(s) / a^2
    assert S.jf_g(np.array([s]))[0] == pytest.approx(abel(rho_jf, s), rel=1e-9)


@pytest.mark.parametrize("s", [0.05, 0.3, 0.7, 0.99, 1.01, 1.3, 3.0, 8.0])
def test_jaffe_projected_dispersion_matches_jeans_projection(s):
    # Sigma sigma_p^2 = G M^2 h / (4 pi a^3), from brute-force Jeans quadrature
    jeans = abel(lambda r: rho_jf(r) * sigma_r2_jf_jeans(r), s)
    assert S.jf_h(np.array([s]))[0] / (4.0 * math.pi) == pytest.approx(jeans, rel=2e-7)


def test_jaffe_circular_velocity_is_enclosed_mass():
    # v_c^2 = G M(r) / r with M(r) from the density by quadrature equals G M / (r + a)
    for r in (0.01, 0.5, 2.0, 40.0):
        m, _ = integrate.quad(lambda x: 4.0 * math.pi * x * x * rho_jf(x), 0.0, r, epsrel=1e-12, limit=200)
        assert m / r == pytest.approx(1.0 / (r + 1.0), rel=1e-9)


def test_jaffe_total_projected_mass_is_one():
    f = lambda x: 2.0 * math.pi * x * S.jf_g(np.array([x]))[0]
    v1, _ = integrate.quad(f, 0, 1, limit=200)
    v2, _ = integrate.quad(f, 1, np.inf, limit=400)
    assert v1 + v2 == pytest.approx(1.0, rel=1e-8)


def test_jaffe_limits_and_series_continuity():
    # small s: Sigma -> 1/(4s) (the 1/r^2 cusp) and h -> pi/(2s); large s: both fall
    # as the r^-4 density tail: s^3 g -> 1/4 ... checked against the Abel tail
    s = 1e-6
    assert S.jf_g(np.array([s]))[0] * s == pytest.approx(0.25, rel=1e-4)
    assert S.jf_h(np.array([s]))[0] * s == pytest.approx(math.pi / 2, rel=1e-4)
    big = 200.0
    assert S.jf_g(np.array([big]))[0] == pytest.approx(abel(rho_jf, big), rel=1e-8)
    for edge in [math.sqrt(1 - S.T_SERIES_MAX), math.sqrt(1 + S.T_SERIES_MAX), S.W_SERIES_MIN_S]:
        lo, hi = edge * (1 - 1e-12), edge * (1 + 1e-12)
        for f in (S.jf_g, S.jf_h):
            a, b = f(np.array([lo, hi]))
            assert a == pytest.approx(b, rel=1e-11)


def test_jaffe_mpmath_agreement_dense():
    mp.mp.dps = 60

    def X(s):
        return mp.acosh(1 / s) / mp.sqrt(1 - s * s) if s < 1 else mp.asec(s) / mp.sqrt(s * s - 1)

    def g(s):
        return 1 / (4 * s) + (1 - (2 - s * s) * X(s)) / (2 * mp.pi * (1 - s * s))

    def h(s):
        return (mp.pi / (2 * s) + 11 - mp.mpf(13) / 2 * mp.pi * s - 12 * s ** 2 + 6 * mp.pi * s ** 3
                - X(s) * (6 - 19 * s ** 2 + 12 * s ** 4)) / (1 - s * s)

    ss = np.concatenate([np.geomspace(1e-5, 0.99, 40), np.geomspace(1.01, 1e4, 40)])
    with mp.workdps(200):
        ref_g = np.array([float(g(mp.mpf(float(x)))) for x in ss])
        ref_h = np.array([float(h(mp.mpf(float(x)))) for x in ss])
    assert np.max(np.abs(S.jf_g(ss) / ref_g - 1)) < 1e-12
    assert np.max(np.abs(S.jf_h(ss) / ref_h - 1)) < 1e-12
