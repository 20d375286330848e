"""FP64 data-preparation formulas (oracle; test infrastructure only: used by
the tests, never by the product path).

* ``ml_from_colour``: the colour-M/L relation of Sec. 2.5.1
  (log10 (M/L)_alpha = a_alpha + b_alpha (m_beta - m_gamma)), with the error
  of Appendix C: the magnitude errors propagated through the relation and
  the relation's tabulated scatter sigma_alpha added in quadrature (in dex).
* ``brightness_errors``: the surface-brightness error model of Sec. 3 (data):
  a relative error (5 %) and a constant systematic term of 10 % of the
  faintest surface brightness, combined in quadrature (the text says the
  systematic error is "added"; quadrature is the reading taken).

Pixels with non-finite inputs are masked: M/L = NaN, error 0.
"""
from __future__ import annotations

import math

import numpy as np

LN10 = math.log(10.0)


def ml_from_colour(m_beta, m_gamma, dm_beta, dm_gamma, a: float, b: float, sigma_a: float):
    mb, mg = np.asarray(m_beta, np.float64), np.asarray(m_gamma, np.float64)
    eb, eg = np.asarray(dm_beta, np.float64), np.asarray(dm_gamma, np.float64)
    ok = np.isfinite(mb) & np.isfinite(mg) & np.isfinite(eb) & np.isfinite(eg)
    with np.errstate(invalid="ignore", over="ignore"):
        log_ml = a + b * (mb - mg)
        ml = 10.0 ** log_ml
        sig_log = np.sqrt(b * b * (eb * eb + eg * eg) + sigma_a * sigma_a)
        err = ml * LN10 * sig_log
    return np.where(ok, ml, np.nan), np.where(ok, err, 0.0)


def brightness_errors(B, rel: float = 0.05, floor_frac: float = 0.1):
    B = np.asarray(B, np.float64)
    good = np.isfinite(B) & (B > 0)
    sys = floor_frac * B[good].min() if good.any() else 0.0
    with np.errstate(invalid="ignore"):
        err = np.sqrt((rel * B) ** 2 + sys * sys)
    return np.where(good, err, 0.0)
