"""Tolerances of the GPU parity tests against the FP64 oracle, in one place.

* Maps: per-pixel relative MAP_RTOL for surface brightness, dispersion and
  M/L; |dv| <= MAP_RTOL max|v| for the velocity, which crosses zero.
* Log-likelihood at the truth of noisy synthetic data: absolute LOGL_ATOL up
  to 4e4 residuals.  The error there is sum_i r_i dF_i / e_i with random
  unit-variance residuals r_i and map errors dF_i dominated by the FP32
  rounding of each vector's constants, which is coherent over a map: a random
  walk of standard deviation ~EPS_COH ||F / e||_2, growing as sqrt(N).  Beyond
  4e4 residuals the bound is three of those standard deviations (the 300x300,
  5x5 stress grid, 3.6e5 residuals, ||F/e|| ~ 9.5e3: measured 1.2e-3 to
  2.9e-3 against 5.7e-3; the error stays the same when the PSF sums are
  accumulated in FP64, so it is the FP32 model itself).
* In the posterior bulk (perturbations of the truth with chi^2/N <= 4) the
  residuals r_i gain a part coherent with the model, and the FP32 rounding of
  each vector's constants (amplitudes, scale radii, ~6e-8 relative) shifts
  whole maps coherently, so the error gains a first-order term
  sum_i r_i dF_i / e_i that does not average out.  With dF_i <= EPS_COH F_i
  and the coherent residual of norm sqrt(chi^2 - chi^2_truth), Cauchy-Schwarz
  bounds it by EPS_COH sqrt(dchi2) ||F / e||_2; the bulk tolerance is the
  truth's plus that term (EPS_COH = 2e-7: the constants' rounding plus the
  special-function tables' fit error, 9e-8; it is also the measured standard
  deviation of the truth-row error over ||F/e||).  Measured on the realistic cube:
  5e-5 at dchi2 = 702 and 1.8e-3 at dchi2 = 370 (different directions).
* Log-likelihood far from the truth (prior draws, chi^2/N up to ~1e3): the
  first-order change of chi^2 / 2 under the worst per-pixel map error,
  LOGL_ATOL + sum_i |r_i| dF_i / e_i with dF_i = MAP_EPS |F_i| (MAP_EPS max|v|
  for the velocity, and the FP32 moment-cancellation bound for the
  dispersion of luminosity-weighted grids).  MAP_EPS = 1e-6 is twice the
  largest per-pixel map error measured on any case (5e-7).
"""
import numpy as np

import workloads as W
from oracle import model as M

MAP_RTOL = 1e-4
LOGL_ATOL = 1e-3
MAP_EPS = 1e-6
EPS_COH = 2e-7
LW_SIGMA_EPS = 1e-5        # |d sigma| <= LW_SIGMA_EPS (sigma^2 + v^2) / (2 sigma) for moment maps
BULK_CHI2N = 4.0
N_RES_REF = 4.0e4


def oracle_model_maps(spec, th):
    """Oracle maps as compared: B, v, sigma and M/L = 1 / <L/M>."""
    F = M.psf_maps(spec, th)
    return np.stack([F[0], F[1], F[2], 1.0 / F[3]])


def _map_error(spec, F):
    dF = MAP_EPS * np.abs(F)
    dF[1] = MAP_EPS * np.max(np.abs(F[1]))
    if spec.psf_mode == W.PSF_LUMINOSITY:
        sg, v = F[2], F[1]
        dF[2] = MAP_EPS * sg + LW_SIGMA_EPS * (sg * sg + v * v) / (2.0 * np.maximum(sg, 1e-30))
    return dF


def residual_stats(spec, data, err, th, F=None):
    """(chi^2 / N, first-order far-row bound sum_i |r_i| dF_i / e_i, N,
    chi^2, ||F / e||_2), all over the valid pixels of each map."""
    F = oracle_model_maps(spec, th) if F is None else F
    dF = _map_error(spec, F)
    ok = M.valid_masks(data, err)
    chi2, tot, n, fe2 = 0.0, 0.0, 0, 0.0
    for m in range(4):
        e = err[m][ok[m]]
        r = (F[m][ok[m]] - data[m][ok[m]]) / e
        chi2 += float(np.sum(r * r))
        tot += float(np.sum(np.abs(r) * dF[m][ok[m]] / e))
        fe2 += float(np.sum((F[m][ok[m]] / e) ** 2))
        n += int(ok[m].sum())
    return chi2 / max(n, 1), tot, n, chi2, fe2 ** 0.5


def truth_tol(n_res, fe):
    """The truth row: LOGL_ATOL up to N_RES_REF residuals, beyond that three
    standard deviations of the FP32 random walk."""
    return LOGL_ATOL if n_res <= N_RES_REF else max(LOGL_ATOL, 3.0 * EPS_COH * fe)


def logl_tol(spec, data, err, th, kind, chi2_truth=None):
    """kind: 'truth', 'bulk' (chi^2/N <= 4, asserted; needs the truth's chi^2)
    or 'far'."""
    chi2n, tot, n, chi2, fe = residual_stats(spec, data, err, th)
    if kind == "truth":
        return truth_tol(n, fe)
    if kind == "bulk":
        assert chi2n <= BULK_CHI2N, f"row meant for the posterior bulk has chi^2/N = {chi2n:.2f}"
        return truth_tol(n, fe) + EPS_COH * max(chi2 - chi2_truth, 0.0) ** 0.5 * fe
    return LOGL_ATOL + tot


def chi2_of(spec, data, err, th):
    return residual_stats(spec, data, err, th)[3]


def bulk_rows(spec, data, err, truth, rng, n, scale=1e-3, min_scale=1e-7):
    """n perturbations truth + scale * (prior width) * N(0, 1), the scale cut
    by 10 until chi^2/N <= BULK_CHI2N (checked with the oracle's maps)."""
    width = np.diff(W.prior_bounds(spec), axis=1)[:, 0]
    out = []
    for _ in range(n):
        z = rng.standard_normal(len(truth))
        sc = scale
        while True:
            t = truth + sc * width * z
            if M.is_valid(spec, t) and residual_stats(spec, data, err, t)[0] <= BULK_CHI2N:
                out.append(t)
                break
            sc *= 0.1
            assert sc >= min_scale, "no posterior-bulk perturbation found"
    return np.array(out)
