"""Generate the FP32 piecewise-polynomial tables used by the HIP kernels.

Run:  python paper_2205_06819_amd/csrc/gen_tables.py   (writes gk_tables.h)

The kernels evaluate four universal functions of one argument:

* g(s) and h(s) of the projected Hernquist bulge (paper Sec. 2.2: projected
  density M g / (2 pi R_b^2) and Sigma sigma^2 = G M^2 h / (12 pi R_b^3));
* the same pair for the Jaffe bulge (Appendix B: M g / R_b^2 and
  G M^2 h / (4 pi R_b^3));
* phi(y) = y^2 [I0 K0 - I1 K1](y) of the exponential-disc rotation curve
  (paper Sec. 2.3, read as in Binney & Tremaine: v^2 = (2 G M / R_d) phi(r / 2R_d));
* m(x) = [ln(1 + x) - x / (1 + x)] / x of the NFW halo (v^2 = G M200 m(r/r_s) / (r_s mu(c))).

The printed closed forms lose all FP32 accuracy near s = 1 and, for h, at
large s.  Each function is therefore tabulated as a polynomial of degree 7
on quarter-octave pieces: piece k covers [2^e (1 + q/4), 2^e (1 + (q+1)/4))
with k = 4 (e - e_lo) + q, so the kernel finds k and the local coordinate
from the bits of the FP32 argument (exponent and the top two mantissa bits)
with integer operations only.  Coefficients are Chebyshev interpolants computed with
mpmath at 80 digits from the closed forms, converted to the monomial basis in
u in [-1, 1] and rounded to FP32.  Outside the tabulated range a short
expansion in w = 1/arg is used (also fitted here).

This generator is part of the GPU implementation; it is independent of the
CPU oracle and shares no code with it.
"""
from __future__ import annotations

import math
import os
import sys

import mpmath as mp
import numpy as np

mp.mp.dps = 80
DEG = 7
NCOEF = DEG + 1


def X(s):
    s = mp.mpf(s)
    if s < 1:
        return mp.acosh(1 / s) / mp.sqrt(1 - s * s)
    if s > 1:
        return mp.asec(s) / mp.sqrt(s * s - 1)
    return mp.mpf(1)


def _near_one(f, s):
    """Evaluate a closed form with a removable singularity at s = 1 (the
    cancellation there costs ~3 log10(1/|s-1|) digits): raise the precision
    and step off s = 1 by far less than FP64 resolution."""
    with mp.workdps(400):
        s = mp.mpf(s)
        if s == 1:
            s = s + mp.mpf(10) ** -40
        return +f(s)


def g_hq(s):
    if abs(mp.mpf(s) - 1) < mp.mpf(10) ** -6:
        return _near_one(g_hq_raw, s)
    return g_hq_raw(s)


def g_hq_raw(s):
    s = mp.mpf(s)
    return ((2 + s * s) * X(s) - 3) / (1 - s * s) ** 2


def h_hq(s):
    if abs(mp.mpf(s) - 1) < mp.mpf(10) ** -6:
        return _near_one(h_hq_raw, s)
    return h_hq_raw(s)


def h_hq_raw(s):
    s = mp.mpf(s)
    s2 = s * s
    return ((-3 * s2 * X(s) * (8 * s2 ** 3 - 28 * s2 ** 2 + 35 * s2 - 20) - 24 * s2 ** 3
             + 68 * s2 ** 2 - 65 * s2 + 6) / (2 * (1 - s2) ** 3) - 6 * mp.pi * s)


def g_jf_raw(s):
    s = mp.mpf(s)
    return 1 / (4 * s) + (1 - (2 - s * s) * X(s)) / (2 * mp.pi * (1 - s * s))


def h_jf_raw(s):
    s = mp.mpf(s)
    s2 = s * s
    return (mp.pi / (2 * s) + 11 - mp.mpf(13) / 2 * mp.pi * s - 12 * s2 + 6 * mp.pi * s2 * s
            - X(s) * (6 - 19 * s2 + 12 * s2 * s2)) / (1 - s2)


def g_jf(s):
    """Jaffe projected density / (M / R_b^2) (Appendix B)."""
    if abs(mp.mpf(s) - 1) < mp.mpf(10) ** -6:
        return _near_one(g_jf_raw, s)
    if mp.mpf(s) > 8:                       # the printed form cancels ~ s^4 at large s
        with mp.workdps(80 + int(4 * mp.log10(mp.mpf(s)))):
            return +g_jf_raw(s)
    return g_jf_raw(s)


def h_jf(s):
    """Jaffe Sigma sigma^2 / (G M^2 / (4 pi R_b^3)) (Appendix B)."""
    if abs(mp.mpf(s) - 1) < mp.mpf(10) ** -6:
        return _near_one(h_jf_raw, s)
    if mp.mpf(s) > 8:
        with mp.workdps(80 + int(5 * mp.log10(mp.mpf(s)))):
            return +h_jf_raw(s)
    return h_jf_raw(s)


def phi_disc(y):
    y = mp.mpf(y)
    return y * y * (mp.besseli(0, y) * mp.besselk(0, y) - mp.besseli(1, y) * mp.besselk(1, y))


def m_nfw(x):
    x = mp.mpf(x)
    return (mp.log(1 + x) - x / (1 + x)) / x


def cheb_fit(f, a, b, deg=DEG):
    """Monomial coefficients in u in [-1, 1] (x = mid + half u) of the Chebyshev
    interpolant of f at the deg+1 first-kind nodes."""
    n = deg + 1
    nodes = [mp.cos(mp.pi * (k + mp.mpf(1) / 2) / n) for k in range(n)]
    mid, half = (mp.mpf(a) + b) / 2, (mp.mpf(b) - a) / 2
    vals = [f(mid + half * u) for u in nodes]
    # Chebyshev coefficients
    c = []
    for j in range(n):
        sj = sum(vals[k] * mp.cos(mp.pi * j * (k + mp.mpf(1) / 2) / n) for k in range(n))
        c.append(sj * (1 if j == 0 else 2) / n)
    # convert sum c_j T_j(u) to monomials
    T = [[mp.mpf(0)] * n for _ in range(n)]
    T[0][0] = mp.mpf(1)
    if n > 1:
        T[1][1] = mp.mpf(1)
    for j in range(2, n):
        for k in range(n):
            T[j][k] = (2 * T[j - 1][k - 1] if k > 0 else 0) - T[j - 2][k]
    mono = [sum(c[j] * T[j][k] for j in range(n)) for k in range(n)]
    return mono


def horner_f32(coef32, u):
    acc = np.float32(coef32[-1])
    u = np.float32(u)
    for k in range(len(coef32) - 2, -1, -1):
        acc = np.float32(np.float32(acc * u) + np.float32(coef32[k]))
    return acc


PPO = 4          # pieces per octave (top two mantissa bits)


def build_table(f, e_lo, e_hi, name, check=12):
    """Quarter-octave pieces over [2^e_lo, 2^e_hi)."""
    rows = []
    worst = 0.0
    for e in range(e_lo, e_hi):
        for q in range(PPO):
            a = mp.mpf(2) ** e * (1 + mp.mpf(q) / PPO)
            b = mp.mpf(2) ** e * (1 + mp.mpf(q + 1) / PPO)
            mono = cheb_fit(f, a, b)
            c32 = np.array([float(x) for x in mono], dtype=np.float32)
            rows.append(c32)
            mid, half = (a + b) / 2, (b - a) / 2
            for u in np.linspace(-1, 1, check):
                ref = f(mid + half * mp.mpf(float(u)))
                val = float(np.polyval(c32[::-1].astype(np.float64), u))
                worst = max(worst, abs(val / float(ref) - 1))
    print(f"{name}: {len(rows)} pieces over [2^{e_lo}, 2^{e_hi}), max rel fit error {worst:.2e}",
          file=sys.stderr)
    return np.array(rows, dtype=np.float32), worst


def asym_fit(f_scaled, wmax, deg=3):
    """Polynomial in w on [0, wmax] fitting f_scaled(w) (Chebyshev interpolant)."""
    mono = cheb_fit(f_scaled, 0, wmax, deg)
    # re-expand from u = (w - wmax/2) / (wmax/2) to powers of w
    half = mp.mpf(wmax) / 2
    n = deg + 1
    out = [mp.mpf(0)] * n
    # u = (w - half)/half = w/half - 1
    for k, ck in enumerate(mono):
        # (w/half - 1)^k
        for j in range(k + 1):
            out[j] += ck * mp.binomial(k, j) * (1 / half) ** j * (-1) ** (k - j)
    return [float(x) for x in out]


# ranges (argument exponents)
S_LO, S_HI = -20, 12        # bulge s = R / R_b   (s is clamped to >= 1e-6 > 2^-20)
Y_LO, Y_HI = -24, 10        # disc y = r / (2 R_d)
X_LO, X_HI = -24, 8         # NFW x = r / r_s


def main(out_path):
    g_tab, eg = build_table(g_hq, S_LO, S_HI, "g")
    h_tab, eh = build_table(h_hq, S_LO, S_HI, "h")
    jg_tab, ejg = build_table(g_jf, S_LO, S_HI, "jaffe g")
    jh_tab, ejh = build_table(h_jf, S_LO, S_HI, "jaffe h")
    p_tab, ep = build_table(phi_disc, Y_LO, Y_HI, "phi")
    m_tab, em = build_table(m_nfw, X_LO, X_HI, "m")
    # asymptotic tails: s^3 g, s^4 h in w = 1/s on [0, 2^-S_HI]; 4 y phi in 1/y on [0, 2^-Y_HI]
    wg = 2.0 ** -S_HI
    tg = asym_fit(lambda w: g_hq(1 / w) / w ** 3 if w > 0 else mp.pi / 2, wg)
    th = asym_fit(lambda w: h_hq(1 / w) / w ** 4 if w > 0 else mp.mpf(8) / 5, wg)
    # Jaffe tails: s^3 g and s^4 h in w = 1/s (limits from the closed forms at s = 1e30)
    jg_inf = g_jf(mp.mpf(10) ** 30) * mp.mpf(10) ** 90
    jh_inf = h_jf(mp.mpf(10) ** 30) * mp.mpf(10) ** 120
    tjg = asym_fit(lambda w: g_jf(1 / w) / w ** 3 if w > 0 else jg_inf, wg)
    tjh = asym_fit(lambda w: h_jf(1 / w) / w ** 4 if w > 0 else jh_inf, wg)
    wy = 2.0 ** -Y_HI
    tp = asym_fit(lambda w: 4 * phi_disc(1 / w) / w if w > 0 else mp.mpf(1), wy)
    for nm, cf, ff, sc, wm in [("g", tg, g_hq, 3, wg), ("h", th, h_hq, 4, wg),
                               ("jaffe g", tjg, g_jf, 3, wg), ("jaffe h", tjh, h_jf, 4, wg),
                               ("phi", tp, phi_disc, None, wy)]:
        worst = 0.0
        for w in np.linspace(wm / 100, wm, 7):
            ref = ff(1 / mp.mpf(w))
            if sc is not None:
                val = np.polyval(cf[::-1], w) * w ** sc
            else:
                val = np.polyval(cf[::-1], w) * w / 4
            worst = max(worst, abs(val / float(ref) - 1))
        print(f"tail {nm}: {cf}  max rel {worst:.2e}", file=sys.stderr)

    gh = np.concatenate([g_tab, h_tab], axis=1)          # [npiece, 16]
    jgh = np.concatenate([jg_tab, jh_tab], axis=1)

    def arr(a):
        flat = a.reshape(-1)
        lines = []
        for i in range(0, len(flat), 4):
            lines.append("  " + ", ".join(f"{float(v):.9e}f" for v in flat[i:i + 4]) + ",")
        return "\n".join(lines)

    with open(out_path, "w") as fh:
        fh.write("// Generated by gen_tables.py; do not edit.\n")
        fh.write("// Degree-7 polynomials in u in [-1,1] on quarter-octave pieces; see gen_tables.py.\n")
        fh.write(f"// max relative fit errors: g {eg:.1e}, h {eh:.1e}, Jaffe g {ejg:.1e}, Jaffe h {ejh:.1e}, "
                 f"phi {ep:.1e}, m {em:.1e}\n")
        fh.write("#pragma once\n\n")
        fh.write("#ifndef GK_TABLE_QUAL\n#define GK_TABLE_QUAL static const\n#endif\n\n")
        fh.write(f"#define GK_S_ELO ({S_LO})\n#define GK_S_EHI ({S_HI})\n")
        fh.write(f"#define GK_Y_ELO ({Y_LO})\n#define GK_Y_EHI ({Y_HI})\n")
        fh.write(f"#define GK_X_ELO ({X_LO})\n#define GK_X_EHI ({X_HI})\n")
        fh.write(f"#define GK_GH_NPIECE {gh.shape[0]}\n#define GK_PHI_NPIECE {p_tab.shape[0]}\n")
        fh.write(f"#define GK_M_NPIECE {m_tab.shape[0]}\n\n")
        fh.write("// g coefficients c0..c7 then h coefficients c0..c7, per piece\n")
        fh.write(f"GK_TABLE_QUAL float gk_tab_gh[{gh.size}] = {{\n{arr(gh)}\n}};\n\n")
        fh.write("// Jaffe bulge (Appendix B): g then h coefficients per piece, same pieces as gk_tab_gh\n")
        fh.write(f"GK_TABLE_QUAL float gk_tab_jgh[{jgh.size}] = {{\n{arr(jgh)}\n}};\n\n")
        fh.write(f"GK_TABLE_QUAL float gk_tab_phi[{p_tab.size}] = {{\n{arr(p_tab)}\n}};\n\n")
        fh.write(f"GK_TABLE_QUAL float gk_tab_m[{m_tab.size}] = {{\n{arr(m_tab)}\n}};\n\n")
        fh.write("// tails: s^3 g(s), s^4 h(s) as cubics in w = 1/s for s >= 2^GK_S_EHI;\n")
        fh.write("// 4 y phi(y) as a cubic in w = 1/y for y >= 2^GK_Y_EHI\n")
        for nm, cf in [("g", tg), ("h", th), ("jg", tjg), ("jh", tjh), ("phi", tp)]:
            fh.write(f"#define GK_TAIL_{nm.upper()}(w) ({cf[0]:.9e}f + (w) * ({cf[1]:.9e}f + (w) * "
                     f"({cf[2]:.9e}f + (w) * {cf[3]:.9e}f)))\n")


if __name__ == "__main__":
    here = os.path.dirname(os.path.abspath(__file__))
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(here, "gk_tables.h"))
