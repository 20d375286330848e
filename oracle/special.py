"""FP64 special functions of the model (oracle; test infrastructure only).

Every function accepts real or complex numpy arrays (complex inputs are used
for complex-step differentiation; branches are selected on the real part).

Hernquist bulge, paper Sec. 2.2 (projected density and projected dispersion
equations, with the auxiliary function X(s) of the same section):

* ``hq_X(s)``: X(s) in its first (inverse hyperbolic secant / inverse secant)
  form.  The second, logarithmic form printed for s <= 1 drops a factor and
  gives negative densities for s >= 0.5, so it is not used.
* ``hq_g(s)`` = [(2 + s^2) X(s) - 3] / (1 - s^2)^2, so that the projected
  density is M_b g(s) / (2 pi R_b^2).
* ``hq_h(s)``: the curly bracket of the projected-dispersion equation,
  {[-3 s^2 X (8s^6 - 28s^4 + 35s^2 - 20) - 24s^6 + 68s^4 - 65s^2 + 6]
  / (2 (1-s^2)^3) - 6 pi s}, so that Sigma_b sigma_b^2 = G M_b^2 h / (12 pi R_b^3).

The printed closed forms cancel catastrophically near s = 1 (removable
singularity) and, for h, at large s (h ~ 1.6 s^-4 while each term grows like
s).  There the oracle evaluates exact power series of the same closed forms:

* in t = 1 - s^2, where X = sum_n t^n / (2n+1) on both sides of s = 1
  (artanh(q)/q for s < 1, arctan(q)/q for s > 1);
* for h at large s, in w = 1/s, with X = w arccos(w) / sqrt(1 - w^2).

Their coefficients are computed exactly (``fractions.Fraction``, pi carried
as a separate basis element) from the printed formula itself; the vanishing
of the low-order coefficients that must cancel is asserted when the module is
imported, which checks the transcription of the formula.

Jaffe bulge, Appendix B (projected density and projected dispersion
equations; same X(s)):

* ``jf_g(s)`` = 1/(4s) + [1 - (2 - s^2) X(s)] / (2 pi (1 - s^2)), so that the
  projected density is M_b g / R_b^2;
* ``jf_h(s)`` = [pi/(2s) + 11 - (13/2) pi s - 12 s^2 + 6 pi s^3
  - X(s)(6 - 19 s^2 + 12 s^4)] / (1 - s^2), so that
  Sigma_b sigma_b^2 = G M_b^2 h / (4 pi R_b^3).

Both cancel at s = 1 (removable) and at large s (g ~ s^-3, h ~ s^-4 while
the printed terms grow); the same exact-series treatment applies, with the
series kept in a (rational, pi) or (rational, 1/pi) basis.

Exponential (Freeman) disc, paper Sec. 2.3, circular-velocity equation: the
printed form is dimensionally garbled; the oracle uses the form of the cited
Binney & Tremaine text, v^2 = (2 G M_d / R_d) y^2 [I0 K0 - I1 K1](y) with
y = r / (2 R_d).  ``freeman_phi(y)`` returns y^2 [I0 K0 - I1 K1](y) using
scipy's exponentially scaled Bessel functions.

NFW halo: ``nfw_mu(x)`` = ln(1 + x) - x / (1 + x).
"""
from __future__ import annotations

from fractions import Fraction
from typing import List, Tuple

import numpy as np
import scipy.special as sp

# ---------------------------------------------------------------------------
# exact truncated power series (coefficient lists, index = power)
# ---------------------------------------------------------------------------
NTERMS = 100

# pi to 60 significant digits (enough to round any coefficient to FP64)
PI_FRACTION = Fraction("3.14159265358979323846264338327950288419716939937510582097494459")


def _mul(a: List[Fraction], b: List[Fraction], n: int = NTERMS) -> List[Fraction]:
    out = [Fraction(0)] * n
    for i, ai in enumerate(a[:n]):
        if ai == 0:
            continue
        for j, bj in enumerate(b[: n - i]):
            out[i + j] += ai * bj
    return out


def _add(*series: List[Fraction], n: int = NTERMS) -> List[Fraction]:
    out = [Fraction(0)] * n
    for s in series:
        for i, c in enumerate(s[:n]):
            out[i] += c
    return out


def _scale(a: List[Fraction], c) -> List[Fraction]:
    return [c * x for x in a]


def _poly(coeffs: dict, n: int = NTERMS) -> List[Fraction]:
    out = [Fraction(0)] * n
    for p, c in coeffs.items():
        out[p] += Fraction(c)
    return out


def _pow(a: List[Fraction], k: int) -> List[Fraction]:
    out = _poly({0: 1})
    for _ in range(k):
        out = _mul(out, a)
    return out


def _series_t() -> Tuple[List[Fraction], List[Fraction], List[Fraction]]:
    """Series in t = 1 - s^2 of X, g and A = N / (2 t^3) (so h = A - 6 pi s)."""
    X = [Fraction(1, 2 * n + 1) for n in range(NTERMS + 3)]
    s2 = _poly({0: 1, 1: -1}, NTERMS + 3)             # s^2 = 1 - t
    s4 = _mul(s2, s2, NTERMS + 3)
    s6 = _mul(s4, s2, NTERMS + 3)
    # g: [(2 + s^2) X - 3] / t^2
    num_g = _add(_mul(_add(_poly({0: 2}, NTERMS + 3), s2, n=NTERMS + 3), X, NTERMS + 3),
                 _poly({0: -3}, NTERMS + 3), n=NTERMS + 3)
    assert num_g[0] == 0 and num_g[1] == 0, "g numerator must vanish to O(t^2)"
    g = num_g[2:NTERMS + 2]
    # N = -3 s^2 X (8 s^6 - 28 s^4 + 35 s^2 - 20) - 24 s^6 + 68 s^4 - 65 s^2 + 6
    P = _add(_scale(s6, 8), _scale(s4, -28), _scale(s2, 35), _poly({0: -20}, NTERMS + 3),
             n=NTERMS + 3)
    N = _add(_scale(_mul(_mul(s2, X, NTERMS + 3), P, NTERMS + 3), -3),
             _scale(s6, -24), _scale(s4, 68), _scale(s2, -65), _poly({0: 6}, NTERMS + 3),
             n=NTERMS + 3)
    assert N[0] == 0 and N[1] == 0 and N[2] == 0, "h numerator must vanish to O(t^3)"
    A = [c / 2 for c in N[3:NTERMS + 3]]
    return X[:NTERMS], g, A


NTERMS_W = 230


def _series_w() -> List[Fraction]:
    """Series of h(s) in w = 1/s (s > 1), as exact (rational, pi-coefficient) pairs.

    With Y = (pi/2 - arcsin w) / sqrt(1 - w^2) (so X = w Y),
    Z = [3 Y (8 - 28w^2 + 35w^4 - 20w^6) + w (24 - 68w^2 + 65w^4 - 6w^6)] / (2 (1-w^2)^3)
    and h = (Z - 6 pi) / w.
    """
    n = NTERMS_W + 2
    # (1 - w^2)^(-1/2) = sum C(2k, k) / 4^k w^(2k)
    inv_sqrt = [Fraction(0)] * n
    # arcsin(w) = sum (2k)! / (4^k (k!)^2 (2k+1)) w^(2k+1)
    asin = [Fraction(0)] * n
    from math import comb
    for k in range(n // 2 + 1):
        if 2 * k < n:
            inv_sqrt[2 * k] = Fraction(comb(2 * k, k), 4 ** k)
        if 2 * k + 1 < n:
            asin[2 * k + 1] = Fraction(comb(2 * k, k), 4 ** k * (2 * k + 1))
    # Y = (pi/2) inv_sqrt - asin * inv_sqrt : keep pi part and rational part apart
    Y_pi = _scale(inv_sqrt, Fraction(1, 2))
    Y_q = _scale(_mul(asin, inv_sqrt, n), -1)
    Pw = _poly({0: 8, 2: -28, 4: 35, 6: -20}, n)
    Qw = _poly({1: 24, 3: -68, 5: 65, 7: -6}, n)       # w * (24 - 68 w^2 + ...)
    inv_cube = [Fraction(0)] * n                        # (1 - w^2)^(-3)
    for k in range(n // 2 + 1):
        if 2 * k < n:
            inv_cube[2 * k] = Fraction(comb(k + 2, 2))
    Z_pi = _scale(_mul(_mul(Y_pi, Pw, n), inv_cube, n), Fraction(3, 2))
    Z_q = _add(_scale(_mul(_mul(Y_q, Pw, n), inv_cube, n), Fraction(3, 2)),
               _scale(_mul(Qw, inv_cube, n), Fraction(1, 2)), n=n)
    assert Z_pi[0] == 6 and Z_q[0] == 0, "the 6 pi s term must cancel the leading order"
    coeffs = [Z_q[k] + Z_pi[k] * PI_FRACTION for k in range(1, n)]  # h = sum c_k w^k
    return coeffs[:NTERMS_W]


_X_T, _G_T, _A_T = _series_t()
_H_W = _series_w()

X_T = np.array([float(c) for c in _X_T])
G_T = np.array([float(c) for c in _G_T])
A_T = np.array([float(c) for c in _A_T])
H_W = np.array([float(c) for c in _H_W])

# the first non-zero term of h at large s is (8/5) w^4, i.e. sigma_b^2 -> (8/15pi) G M_b / R
assert all(abs(c) < 1e-12 for c in H_W[:4]), H_W[:5]
assert abs(H_W[4] - 1.6) < 1e-12, H_W[4]

# ---------------------------------------------------------------------------
# Jaffe series
# ---------------------------------------------------------------------------
def _binom_half(n: int, a: Fraction) -> List[Fraction]:
    """(1 - t)^a = sum_k binom(a, k) (-t)^k, a rational."""
    out = [Fraction(0)] * n
    c = Fraction(1)
    for k in range(n):
        out[k] = c if k % 2 == 0 else -c
        c = c * (a - k) / (k + 1)
    return out


def _jaffe_series_t():
    """Series in t = 1 - s^2: g = 1/(4s) + Gq(t) / (2 pi); h = Hq(t) + pi Hp(t)."""
    n = NTERMS + 2
    X = [Fraction(1, 2 * k + 1) for k in range(n)]
    s2 = _poly({0: 1, 1: -1}, n)
    s4 = _mul(s2, s2, n)
    # g: [1 - (2 - s^2) X] / t
    num = _add(_poly({0: 1}, n), _scale(_mul(_add(_poly({0: 2}, n), _scale(s2, -1), n=n), X, n), -1), n=n)
    assert num[0] == 0, "Jaffe g numerator must vanish at s = 1"
    Gq = num[1:NTERMS + 1]
    # h bracket, pi part: (1/2) s^-1 - (13/2) s + 6 s^3 ; rational part: 11 - 12 s^2 - X (6 - 19 s^2 + 12 s^4)
    s_m1 = _binom_half(n, Fraction(-1, 2))
    s_p1 = _binom_half(n, Fraction(1, 2))
    s_p3 = _binom_half(n, Fraction(3, 2))
    Bp = _add(_scale(s_m1, Fraction(1, 2)), _scale(s_p1, Fraction(-13, 2)), _scale(s_p3, 6), n=n)
    Bq = _add(_poly({0: 11}, n), _scale(s2, -12),
              _scale(_mul(X, _add(_poly({0: 6}, n), _scale(s2, -19), _scale(s4, 12), n=n), n), -1), n=n)
    assert Bp[0] == 0 and Bq[0] == 0, "Jaffe h bracket must vanish at s = 1"
    return Gq, Bq[1:NTERMS + 1], Bp[1:NTERMS + 1]


def _jaffe_series_w():
    """Series in w = 1/s (s > 1): g = Gr(w) + Gi(w) / pi, h = Hq(w) + pi Hp(w)."""
    from math import comb
    n = NTERMS_W + 4
    inv_sqrt = [Fraction(0)] * n
    asin = [Fraction(0)] * n
    for k in range(n // 2 + 1):
        if 2 * k < n:
            inv_sqrt[2 * k] = Fraction(comb(2 * k, k), 4 ** k)
        if 2 * k + 1 < n:
            asin[2 * k + 1] = Fraction(comb(2 * k, k), 4 ** k * (2 * k + 1))
    Y_pi = _scale(inv_sqrt, Fraction(1, 2))             # X = w (Y_q + pi Y_pi)
    Y_q = _scale(_mul(asin, inv_sqrt, n), -1)
    geo = [Fraction(1) if k % 2 == 0 else Fraction(0) for k in range(n)]   # 1 / (1 - w^2)
    # g = w/4 - (w - 2 w^3) Y_pi / (2 (1 - w^2)) - [w^2 + (w - 2 w^3) Y_q] / (2 pi (1 - w^2))
    a = _poly({1: 1, 3: -2}, n)
    Gr = _add(_poly({1: Fraction(1, 4)}, n), _scale(_mul(_mul(a, Y_pi, n), geo, n), Fraction(-1, 2)), n=n)
    Gi = _scale(_mul(_add(_poly({2: 1}, n), _mul(a, Y_q, n), n=n), geo, n), Fraction(-1, 2))
    assert Gr[0] == Gr[1] == Gr[2] == 0 and Gi[0] == Gi[1] == Gi[2] == 0, "Jaffe g must fall as s^-3"
    # h = -B3 / (w (1 - w^2)), B3 = w^3 x bracket
    P = _poly({0: 12, 2: -19, 4: 6}, n)
    B3p = _add(_poly({4: Fraction(1, 2), 2: Fraction(-13, 2), 0: 6}, n), _scale(_mul(Y_pi, P, n), -1), n=n)
    B3q = _add(_poly({3: 11, 1: -12}, n), _scale(_mul(Y_q, P, n), -1), n=n)
    assert B3p[0] == 0 and B3q[0] == 0, "Jaffe h: leading terms must cancel"
    Hp = _scale(_mul(B3p[1:] + [Fraction(0)], geo, n), -1)
    Hq = _scale(_mul(B3q[1:] + [Fraction(0)], geo, n), -1)
    for k in range(4):
        assert Hp[k] == 0 and Hq[k] == 0, ("Jaffe h must fall as s^-4", k)
    return Gr[:NTERMS_W], Gi[:NTERMS_W], Hq[:NTERMS_W], Hp[:NTERMS_W]


_JG_T, _JHq_T, _JHp_T = _jaffe_series_t()
_JGr_W, _JGi_W, _JHq_W, _JHp_W = _jaffe_series_w()
JG_T = np.array([float(c) for c in _JG_T])
JH_T = np.array([float(q + p * PI_FRACTION) for q, p in zip(_JHq_T, _JHp_T)])
JG_W = np.array([float(r + i / PI_FRACTION) for r, i in zip(_JGr_W, _JGi_W)])
JH_W = np.array([float(q + p * PI_FRACTION) for q, p in zip(_JHq_W, _JHp_W)])

# domain split (on the real part of s)
T_SERIES_MAX = 0.6          # |1 - s^2| <= 0.6, i.e. 0.632 <= s <= 1.265
W_SERIES_MIN_S = 1.2649     # h at s >= 1.2649 from the w series (w <= 0.7906)


def _horner(c: np.ndarray, x):
    acc = np.zeros_like(x) + c[-1]
    for k in range(len(c) - 2, -1, -1):
        acc = acc * x + c[k]
    return acc


def _as_array(s):
    s = np.asarray(s)
    if not np.iscomplexobj(s):
        s = s.astype(np.float64)
    return s


def hq_X(s):
    """X(s) of the Hernquist projection; s > 0."""
    s = _as_array(s)
    out = np.empty_like(s)
    t = 1.0 - s * s
    near = np.abs(t.real) <= T_SERIES_MAX
    lo = (~near) & (s.real < 1.0)
    hi = (~near) & (s.real > 1.0)
    out[near] = _horner(X_T, t[near])
    q = np.sqrt(t[lo])
    out[lo] = np.log((1.0 + q) / s[lo]) / q                 # arcsech(s) / sqrt(1 - s^2)
    q = np.sqrt(-t[hi])
    out[hi] = np.arctan(q) / q                              # arcsec(s) / sqrt(s^2 - 1)
    return out


def hq_g(s):
    """g(s) = [(2 + s^2) X(s) - 3] / (1 - s^2)^2; Sigma_b = M_b g / (2 pi R_b^2)."""
    s = _as_array(s)
    out = np.empty_like(s)
    t = 1.0 - s * s
    near = np.abs(t.real) <= T_SERIES_MAX
    out[near] = _horner(G_T, t[near])
    far = ~near
    sf, tf = s[far], t[far]
    out[far] = ((2.0 + sf * sf) * hq_X(sf) - 3.0) / (tf * tf)
    return out


def hq_h(s):
    """Bracket of the projected Hernquist dispersion: Sigma_b sigma_b^2 = G M_b^2 h / (12 pi R_b^3)."""
    s = _as_array(s)
    out = np.empty_like(s)
    t = 1.0 - s * s
    near = np.abs(t.real) <= T_SERIES_MAX
    big = (~near) & (s.real >= W_SERIES_MIN_S)
    direct = ~(near | big)
    out[near] = _horner(A_T, t[near]) - 6.0 * np.pi * s[near]
    w = 1.0 / s[big]
    out[big] = _horner(H_W, w)
    sd, td = s[direct], t[direct]
    s2 = sd * sd
    s4 = s2 * s2
    s6 = s4 * s2
    num = (-3.0 * s2 * hq_X(sd) * (8.0 * s6 - 28.0 * s4 + 35.0 * s2 - 20.0)
           - 24.0 * s6 + 68.0 * s4 - 65.0 * s2 + 6.0)
    out[direct] = num / (2.0 * td ** 3) - 6.0 * np.pi * sd
    return out


def jf_g(s):
    """Jaffe projected density: Sigma_b = M_b g / R_b^2 (Appendix B); s > 0."""
    s = _as_array(s)
    out = np.empty_like(s)
    t = 1.0 - s * s
    near = np.abs(t.real) <= T_SERIES_MAX
    big = (~near) & (s.real >= W_SERIES_MIN_S)
    direct = ~(near | big)
    out[near] = 0.25 / s[near] + _horner(JG_T, t[near]) / (2.0 * np.pi)
    out[big] = _horner(JG_W, 1.0 / s[big])
    sd, td = s[direct], t[direct]
    out[direct] = 0.25 / sd + (1.0 - (2.0 - sd * sd) * hq_X(sd)) / (2.0 * np.pi * td)
    return out


def jf_h(s):
    """Jaffe projected dispersion: Sigma_b sigma_b^2 = G M_b^2 h / (4 pi R_b^3) (Appendix B)."""
    s = _as_array(s)
    out = np.empty_like(s)
    t = 1.0 - s * s
    near = np.abs(t.real) <= T_SERIES_MAX
    big = (~near) & (s.real >= W_SERIES_MIN_S)
    direct = ~(near | big)
    out[near] = _horner(JH_T, t[near])
    out[big] = _horner(JH_W, 1.0 / s[big])
    sd, td = s[direct], t[direct]
    s2 = sd * sd
    br = (np.pi / (2.0 * sd) + 11.0 - 6.5 * np.pi * sd - 12.0 * s2 + 6.0 * np.pi * s2 * sd
          - hq_X(sd) * (6.0 - 19.0 * s2 + 12.0 * s2 * s2))
    out[direct] = br / td
    return out


def freeman_F(y):
    """I0(y) K0(y) - I1(y) K1(y) for y > 0 (real or complex)."""
    y = _as_array(y)
    prod = sp.ive(0, y) * sp.kve(0, y) - sp.ive(1, y) * sp.kve(1, y)
    if np.iscomplexobj(y):
        # ive * kve = I K exp(z - |Re z|) = I K exp(i Im z) for complex z
        prod = prod * np.exp(-1j * y.imag)
    return prod


def freeman_phi(y):
    """y^2 [I0 K0 - I1 K1](y), with the limit 0 at y = 0."""
    y = _as_array(y)
    out = np.zeros_like(y)
    nz = y.real > 0.0
    yn = y[nz]
    out[nz] = yn * yn * freeman_F(yn)
    return out


def nfw_mu(x):
    """mu(x) = ln(1 + x) - x / (1 + x), the NFW enclosed-mass shape."""
    x = _as_array(x)
    return np.log1p(x) - x / (1.0 + x)
