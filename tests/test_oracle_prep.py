"""Pins of the data-preparation oracle (no GPU): limits of the colour-M/L
relation, its error propagation against a Monte Carlo of the magnitudes, and
the paper's worked numbers for the surface-brightness floor."""
import math

import numpy as np
import pytest

from oracle import prep as P


def test_colour_relation_limits():
    a, b, s = -0.70, 0.89, 0.07           # Appendix C's calibration for the g-i colour
    m = np.array([17.0, 18.5])
    ml, err = P.ml_from_colour(m, m, [0.0, 0.0], [0.0, 0.0], a, b, s)
    np.testing.assert_allclose(ml, 10 ** a)                      # zero colour
    np.testing.assert_allclose(err, 10 ** a * math.log(10) * s)  # only the scatter
    ml, err = P.ml_from_colour([19.0], [18.0], [0.0], [0.0], a, 0.0, 0.0)
    assert ml[0] == pytest.approx(10 ** a) and err[0] == 0.0
    # one magnitude unit of colour multiplies M/L by 10^b
    ml1, _ = P.ml_from_colour([19.0], [18.0], [0.0], [0.0], a, b, s)
    ml0, _ = P.ml_from_colour([18.0], [18.0], [0.0], [0.0], a, b, s)
    assert ml1[0] / ml0[0] == pytest.approx(10 ** b)


def test_colour_error_propagation_matches_monte_carlo():
    rng = np.random.default_rng(3)
    a, b, s = -0.70, 0.89, 0.07
    mb, mg, eb, eg = 18.3, 17.4, 0.04, 0.03
    n = 400000
    logml = a + b * ((mb + eb * rng.standard_normal(n)) - (mg + eg * rng.standard_normal(n))) \
        + s * rng.standard_normal(n)
    ml, err = P.ml_from_colour([mb], [mg], [eb], [eg], a, b, s)
    # linear propagation: sigma(M/L) = M/L ln10 sigma(log10 M/L)
    assert err[0] / (ml[0] * math.log(10)) == pytest.approx(np.std(logml), rel=5e-3)


def test_masked_pixels():
    ml, err = P.ml_from_colour([np.nan, 1.0, 1.0], [1.0, np.inf, 1.0], [0.1, 0.1, np.nan], [0.1] * 3, 0, 1, 0)
    assert np.all(np.isnan(ml)) and np.all(err == 0)
    e = P.brightness_errors([np.nan, -1.0, 0.0, 10.0])
    assert list(e[:3]) == [0.0, 0.0, 0.0] and e[3] > 0


def test_brightness_floor_paper_numbers():
    # Sec. 3: 5 % of B plus a systematic 10 % of the faintest B (~5 Lsun/pc^2 for
    # a faintest pixel of ~50 Lsun/pc^2); the relative error grows outwards
    B = np.array([50.0, 200.0, 5000.0])
    e = P.brightness_errors(B)
    assert e[0] == pytest.approx(math.hypot(2.5, 5.0))
    assert e[2] == pytest.approx(math.hypot(250.0, 5.0))
    rel = e / B
    assert rel[0] > rel[1] > rel[2] > 0.05
