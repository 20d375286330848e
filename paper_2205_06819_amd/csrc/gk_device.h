// Device-side building blocks of the galkin kernels (gfx950 / CDNA4).
//
// Per-theta constants (computed in FP64, stored as FP32), the FP32
// special functions of the model (piecewise polynomials in constant memory), and
// the per-lattice-point model of the paper's Sec. 2.1-2.4 with its
// reverse-mode derivative.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define GK_TABLE_QUAL __constant__
#include "gk_tables.h"

namespace gk {

constexpr double G_KPC = 4.300917270e-6;     // kpc (km/s)^2 / Msun
constexpr double PI = 3.14159265358979323846;
constexpr float S_MIN = 1.0e-6f;             // clamp of s = R / R_b at the centre

// FP32 table sizes in floats
constexpr int TAB_GH = GK_GH_NPIECE * 16;
constexpr int TAB_PHI = GK_PHI_NPIECE * 8;
constexpr int TAB_M = GK_M_NPIECE * 8;
constexpr int TAB_ALL = TAB_GH + TAB_PHI + TAB_M;

// ---------------------------------------------------------------------------
// per-theta constants
// ---------------------------------------------------------------------------
struct TC {
    int valid;
    int Ui, Vi;          // integer part of the model centre in lattice units
    float Uf, Vf;        // fractional part
    float ca, sa;        // (pixel_kpc / s) cos PA, (pixel_kpc / s) sin PA
    float sec2i;         // 1 / cos^2 i
    // bulge: B_b = Ab g(s), B_b sigma_b^2 = Cb h(s), v_c^2 = GMb r / (r + Rb)^2
    float invRb, Ab, Cb, GMb, Rb, MLb;
    // discs: B_d = Ad 2^(r nl2Rd), v_c^2 = Kd phi(r inv2Rd); v = kf cos(phi) v_int; sigma^2 = sf v_int^2
    float nl2Rd[2], Ad[2], inv2Rd[2], Kd[2], kf[2], sf[2], MLd[2];
    // halo: NFW v^2 = H1 m(r H0) with H0 = 1/r_s, H1 = G M200 / (r_s mu(c));
    //       Hernquist v^2 = H1 r / (r + H0)^2 with H0 = Rh, H1 = G Mh
    float H0, H1;
};

struct GridGeom {
    int nx, ny, s, hs, pad;
    float pk_over_s;
    double pk;
    double rho_crit;     // Msun / kpc^3
    int bulge, ndisc, halo;
    int lw;              // 1: luminosity-weighted PSF moments instead of averaged maps
    double fscale;       // this grid's pixels per pixel of the centre parameters' frame
    double fdx, fdy;     // that frame's centre, in this grid's pixels from its centre
};

__device__ __forceinline__ bool gk_finite(double x) { return x == x && fabs(x) <= 1.7e308; }

// theta (sampling coordinates) -> FP32 constants, all arithmetic in FP64.
__device__ inline TC make_tc(const double* th, const GridGeom& g) {
    TC c;
    bool ok = true;
    int P = 4 + 3 * (g.bulge != 0) + 4 * g.ndisc + 2 * (g.halo != 0);
    for (int k = 0; k < P; ++k) ok = ok && gk_finite(th[k]);
    const double x0 = th[0], y0 = th[1], pa = th[2] * (PI / 180.0), inc = th[3] * (PI / 180.0);
    ok = ok && th[3] > 0.0 && th[3] < 90.0;
    const double Uc = (0.5 * (g.nx - 1) + g.fdx + g.fscale * x0) * g.s + g.hs + g.pad;
    const double Vc = (0.5 * (g.ny - 1) + g.fdy + g.fscale * y0) * g.s + g.hs + g.pad;
    const double Uflo = floor(Uc), Vflo = floor(Vc);
    c.Ui = ok ? (int)Uflo : 0;
    c.Vi = ok ? (int)Vflo : 0;
    c.Uf = (float)(Uc - Uflo);
    c.Vf = (float)(Vc - Vflo);
    double spa, cpa, si, ci;
    sincos(pa, &spa, &cpa);
    sincos(inc, &si, &ci);
    const double pks = g.pk / g.s;
    c.ca = (float)(pks * cpa);
    c.sa = (float)(pks * spa);
    c.sec2i = (float)(1.0 / (ci * ci));
    int k = 4;
    c.invRb = c.Ab = c.Cb = c.GMb = c.Rb = c.MLb = 0.f;
    if (g.bulge) {
        const double Mb = exp10(th[k]), Rb = th[k + 1], ML = th[k + 2];
        ok = ok && Rb > 0.0 && ML > 0.0;
        c.invRb = (float)(1.0 / Rb);
        // Hernquist (Sec. 2.2): Sigma = M g / (2 pi Rb^2), Sigma sigma^2 = G M^2 h / (12 pi Rb^3);
        // Jaffe (Appendix B): Sigma = M g / Rb^2, Sigma sigma^2 = G M^2 h / (4 pi Rb^3)
        const double fa = g.bulge == 2 ? 1.0 : 2.0 * PI, fc = g.bulge == 2 ? 4.0 * PI : 12.0 * PI;
        c.Ab = (float)(1.0e-6 * Mb / (fa * Rb * Rb * ML));
        c.Cb = (float)(1.0e-6 * G_KPC * Mb * Mb / (fc * Rb * Rb * Rb * ML));
        c.GMb = (float)(G_KPC * Mb);
        c.Rb = (float)Rb;
        c.MLb = (float)ML;
        k += 3;
    }
    for (int j = 0; j < 2; ++j) {
        c.nl2Rd[j] = c.Ad[j] = c.inv2Rd[j] = c.Kd[j] = c.kf[j] = c.sf[j] = c.MLd[j] = 0.f;
        if (j < g.ndisc) {
            const double Md = exp10(th[k]), Rd = th[k + 1], ML = th[k + 2], kk = th[k + 3];
            ok = ok && Rd > 0.0 && ML > 0.0 && fabs(kk) <= 1.0;
            c.nl2Rd[j] = (float)(-1.4426950408889634 / Rd);
            c.Ad[j] = (float)(1.0e-6 * Md / (2.0 * PI * Rd * Rd * ci * ML));
            c.inv2Rd[j] = (float)(0.5 / Rd);
            c.Kd[j] = (float)(2.0 * G_KPC * Md / Rd);
            c.kf[j] = (float)(-kk * si);
            c.sf[j] = (float)((1.0 - kk * kk) / 3.0);
            c.MLd[j] = (float)ML;
            k += 4;
        }
    }
    c.H0 = c.H1 = 0.f;
    if (g.halo == 2) {            // NFW (M200, c)
        const double M200 = exp10(th[k]), conc = th[k + 1];
        ok = ok && conc > 0.0;
        const double r200 = cbrt(3.0 * M200 / (4.0 * PI * 200.0 * g.rho_crit));
        const double rs = r200 / conc;
        const double muc = log1p(conc) - conc / (1.0 + conc);
        c.H0 = (float)(1.0 / rs);
        c.H1 = (float)(G_KPC * M200 / (rs * muc));
    } else if (g.halo == 1) {     // Hernquist (Mh, Rh)
        const double Mh = exp10(th[k]), Rh = th[k + 1];
        ok = ok && Rh > 0.0;
        c.H0 = (float)Rh;
        c.H1 = (float)(G_KPC * Mh);
    }
    c.valid = ok ? 1 : 0;
    return c;
}

__device__ __forceinline__ float uni(float x) {
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x)));
}
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Make every field wave-uniform (the compiler keeps them in SGPRs).
__device__ __forceinline__ TC uniform_tc(const TC& a) {
    TC c;
    c.valid = uni(a.valid);
    c.Ui = uni(a.Ui); c.Vi = uni(a.Vi); c.Uf = uni(a.Uf); c.Vf = uni(a.Vf);
    c.ca = uni(a.ca); c.sa = uni(a.sa); c.sec2i = uni(a.sec2i);
    c.invRb = uni(a.invRb); c.Ab = uni(a.Ab); c.Cb = uni(a.Cb); c.GMb = uni(a.GMb);
    c.Rb = uni(a.Rb); c.MLb = uni(a.MLb);
    for (int j = 0; j < 2; ++j) {
        c.nl2Rd[j] = uni(a.nl2Rd[j]); c.Ad[j] = uni(a.Ad[j]); c.inv2Rd[j] = uni(a.inv2Rd[j]);
        c.Kd[j] = uni(a.Kd[j]); c.kf[j] = uni(a.kf[j]); c.sf[j] = uni(a.sf[j]);
        c.MLd[j] = uni(a.MLd[j]);
    }
    c.H0 = uni(a.H0); c.H1 = uni(a.H1);
    return c;
}

// ---------------------------------------------------------------------------
// FP32 special functions (piecewise-polynomial tables)
// ---------------------------------------------------------------------------
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ float fexp2(float x) { return __builtin_amdgcn_exp2f(x); }
__device__ __forceinline__ float flog2(float x) { return __builtin_amdgcn_logf(x); }

// Piece index and local coordinate u in [-1, 1) of x in [2^elo, 2^ehi):
// quarter-octave pieces selected by the exponent and the top two mantissa bits.
// Callers only pass x >= 2^elo; the bias is removed before the shift so the
// index is formed without a negative constant (the four table reads then
// share one address and use immediate offsets).
__device__ __forceinline__ int piece(float x, int elo, float& u) {
    const uint32_t b = __float_as_uint(x);
    u = __uint_as_float(0x3f800000u | ((b & 0x1FFFFFu) << 2)) * 2.0f - 3.0f;
    return (int)((b - ((uint32_t)(127 + elo) << 23)) >> 21);
}
// du/dx for the piece containing x: the piece has half-width 2^(e-3).
__device__ __forceinline__ float piece_dudx(float x) {
    const uint32_t E = (__float_as_uint(x) >> 23) & 0xFFu;
    return __uint_as_float((257u - E) << 23);
}

__device__ __forceinline__ float horner8(const float4 a, const float4 b, float u) {
    float p = fmaf(b.w, u, b.z);
    p = fmaf(p, u, b.y);
    p = fmaf(p, u, b.x);
    p = fmaf(p, u, a.w);
    p = fmaf(p, u, a.z);
    p = fmaf(p, u, a.y);
    return fmaf(p, u, a.x);
}
// value and derivative d/du
__device__ __forceinline__ float horner8d(const float4 a, const float4 b, float u, float& d) {
    float p = b.w, q = 0.f;
    q = fmaf(q, u, p); p = fmaf(p, u, b.z);
    q = fmaf(q, u, p); p = fmaf(p, u, b.y);
    q = fmaf(q, u, p); p = fmaf(p, u, b.x);
    q = fmaf(q, u, p); p = fmaf(p, u, a.w);
    q = fmaf(q, u, p); p = fmaf(p, u, a.z);
    q = fmaf(q, u, p); p = fmaf(p, u, a.y);
    q = fmaf(q, u, p); p = fmaf(p, u, a.x);
    d = q;
    return p;
}

// Value and derivative of a polynomial written as a Horner expression: the
// tail macros below evaluated on Dual arguments give P(w) and P'(w) exactly
// (forward-mode differentiation of the expression).
struct Dual {
    float v, d;
};
__device__ __forceinline__ Dual operator+(float a, Dual b) { return Dual{a + b.v, b.d}; }
__device__ __forceinline__ Dual operator*(Dual a, float b) { return Dual{a.v * b, a.d * b}; }
__device__ __forceinline__ Dual operator*(Dual a, Dual b) { return Dual{a.v * b.v, fmaf(a.d, b.v, a.v * b.d)}; }

// bulge g(s), h(s) for s >= 1e-6 from the staged table (Hernquist, or Jaffe
// when JF); beyond the table s^3 g and s^4 h are cubics in w = 1/s
template <bool JF, typename T>
__device__ __forceinline__ T tail_g(T w) { return JF ? GK_TAIL_JG(w) : GK_TAIL_G(w); }
template <bool JF, typename T>
__device__ __forceinline__ T tail_h(T w) { return JF ? GK_TAIL_JH(w) : GK_TAIL_H(w); }

template <bool JF>
__device__ __forceinline__ void eval_gh(const float4* __restrict__ T, float s, float& g, float& h) {
    if (s < 4096.0f) {
        float u;
        const int k = piece(s, GK_S_ELO, u);
        g = horner8(T[4 * k], T[4 * k + 1], u);
        h = horner8(T[4 * k + 2], T[4 * k + 3], u);
    } else {
        const float w = frcp(s), w3 = w * w * w;
        g = w3 * tail_g<JF>(w);
        h = w3 * w * tail_h<JF>(w);
    }
}
template <bool JF>
__device__ __forceinline__ void eval_gh_d(const float4* __restrict__ T, float s, float& g, float& h,
                                          float& dg, float& dh) {
    if (s < 4096.0f) {
        float u;
        const int k = piece(s, GK_S_ELO, u);
        const float dudx = piece_dudx(s);
        g = horner8d(T[4 * k], T[4 * k + 1], u, dg);
        h = horner8d(T[4 * k + 2], T[4 * k + 3], u, dh);
        dg *= dudx;
        dh *= dudx;
    } else {
        // s^3 g = Pg(w), s^4 h = Ph(w), w = 1/s: dg/ds = -w^4 (3 Pg + w Pg'), dh/ds = -w^5 (4 Ph + w Ph')
        const float w = frcp(s), w2 = w * w, w3 = w2 * w;
        const Dual W{w, 1.0f};
        const Dual pg = tail_g<JF>(W), ph = tail_h<JF>(W);     // cubics and their exact slopes
        g = w3 * pg.v;
        h = w3 * w * ph.v;
        dg = -w3 * w * (3.0f * pg.v + w * pg.d);
        dh = -w3 * w2 * (4.0f * ph.v + w * ph.d);
    }
}

// disc phi(y) = y^2 [I0 K0 - I1 K1](y)
__device__ __forceinline__ float eval_phi(const float4* __restrict__ T, float y) {
    if (y < 1024.0f) {
        if (y < 5.9604645e-8f) return 0.0f;                // 2^-24: phi < 1e-13
        float u;
        const int k = piece(y, GK_Y_ELO, u);
        return horner8(T[2 * k], T[2 * k + 1], u);
    }
    const float w = frcp(y);
    return 0.25f * w * GK_TAIL_PHI(w);
}
__device__ __forceinline__ float eval_phi_d(const float4* __restrict__ T, float y, float& d) {
    if (y < 1024.0f) {
        if (y < 5.9604645e-8f) { d = 0.0f; return 0.0f; }
        float u;
        const int k = piece(y, GK_Y_ELO, u);
        const float v = horner8d(T[2 * k], T[2 * k + 1], u, d);
        d *= piece_dudx(y);
        return v;
    }
    const float w = frcp(y);
    const Dual W{w, 1.0f};
    const Dual p = GK_TAIL_PHI(W);                     // 4 y phi = P(w): value and exact slope
    d = -0.25f * w * w * (p.v + w * p.d);
    return 0.25f * w * p.v;
}

// NFW m(x) = [ln(1+x) - x/(1+x)] / x
__device__ __forceinline__ float eval_m(const float4* __restrict__ T, float x) {
    if (x < 256.0f) {
        if (x < 5.9604645e-8f) return 0.5f * x;
        float u;
        const int k = piece(x, GK_X_ELO, u);
        return horner8(T[2 * k], T[2 * k + 1], u);
    }
    const float ix = frcp(x);
    return (0.69314718f * flog2(1.0f + x) - x * frcp(1.0f + x)) * ix;
}
__device__ __forceinline__ float eval_m_d(const float4* __restrict__ T, float x, float& d) {
    if (x < 256.0f) {
        if (x < 5.9604645e-8f) { d = 0.5f; return 0.5f * x; }
        float u;
        const int k = piece(x, GK_X_ELO, u);
        const float v = horner8d(T[2 * k], T[2 * k + 1], u, d);
        d *= piece_dudx(x);
        return v;
    }
    // m' = [x^2/(1+x)^2 - m x]... m = mu/x, mu' = x/(1+x)^2 -> m' = (mu' - m)/x
    const float ix = frcp(x), i1 = frcp(1.0f + x);
    const float m = (0.69314718f * flog2(1.0f + x) - x * i1) * ix;
    d = (x * i1 * i1 - m) * ix;
    return m;
}

// ---------------------------------------------------------------------------
// the model at one lattice point (paper Sec. 2.1-2.4)
// ---------------------------------------------------------------------------
struct Tabs {
    const float4* gh;
    const float4* phi;
    const float4* m;
};

// the constant-memory tables (read through the vector L1 cache: a lookup's
// piece index varies across the lanes); one bulge kind per grid
template <int BULGE>
__device__ __forceinline__ Tabs const_tabs() {
    return Tabs{(const float4*)(BULGE == 2 ? gk_tab_jgh : gk_tab_gh), (const float4*)gk_tab_phi,
                (const float4*)gk_tab_m};
}

// out: B_tot [Lsun/pc^2], v_los [km/s], sigma_los [km/s], <L/M> [Lsun/Msun]
template <int BULGE, int NDISC, int HALO>
__device__ __forceinline__ void point_model(const TC& c, const Tabs& T, float du, float dv,
                                            float& oB, float& oV, float& oS, float& oLM) {
    // frame: rotate by PA, deproject by i
    const float xp = fmaf(du, c.ca, dv * c.sa);
    const float yp = fmaf(dv, c.ca, -du * c.sa);
    const float x2 = xp * xp, y2 = yp * yp;
    const float r2 = fmaf(y2, c.sec2i, x2);
    const float rinv = r2 > 0.0f ? frsq(r2) : 0.0f;
    const float r = r2 * rinv;
    const float cphi = xp * rinv;
    float vc2 = 0.0f, Bt = 0.0f, BS = 0.0f, kB = 0.0f, sB = 0.0f, mass = 0.0f;
    float scale = 1.0f;
    if (BULGE) {
        const float R = fsqrt(fmaf(xp, xp, y2));
        const float sb = fmaxf(R * c.invRb, S_MIN);
        float g, h;
        eval_gh<BULGE == 2>(T.gh, sb, g, h);
        const float Bb = c.Ab * g;
        Bt = Bb;
        BS = c.Cb * h;
        mass = Bb * c.MLb;
        const float q = r + c.Rb;
        // Hernquist G M r / (r + Rb)^2; Jaffe G M / (r + Rb) (Appendix B)
        vc2 = BULGE == 2 ? c.GMb * frcp(q) : c.GMb * r * frcp(q * q);
    }
    // discs: without a bulge, weights are taken relative to the largest disc
    // exponential so that the ratios survive FP32 underflow far out
    float ex[2];
    float eref = 0.0f;
    if (!BULGE && NDISC > 0) {
        eref = r * c.nl2Rd[0];
        if (NDISC > 1) eref = fmaxf(eref, r * c.nl2Rd[1]);
        scale = fexp2(eref);
    }
#pragma unroll
    for (int j = 0; j < NDISC; ++j) {
        ex[j] = fexp2(fmaf(r, c.nl2Rd[j], -eref));
        const float Bd = c.Ad[j] * ex[j];
        Bt = fmaf(c.Ad[j], ex[j], Bt);              // as in point_model_b
        kB = fmaf(Bd, c.kf[j], kB);
        sB = fmaf(Bd, c.sf[j], sB);
        mass = fmaf(Bd, c.MLd[j], mass);
        vc2 = fmaf(c.Kd[j], eval_phi(T.phi, r * c.inv2Rd[j]), vc2);
    }
    if (HALO == 2) {
        vc2 = fmaf(c.H1, eval_m(T.m, r * c.H0), vc2);
    } else if (HALO == 1) {
        const float q = r + c.H0;
        vc2 = fmaf(c.H1 * r, frcp(q * q), vc2);
    }
    const float vint = fsqrt(vc2);
    const float ib = frcp(Bt);
    oB = Bt * scale;
    oV = cphi * vint * kB * ib;
    oS = fsqrt(fmaf(vc2, sB, BS) * ib);
    oLM = Bt * frcp(mass);
}

// The surface brightness alone (B of point_model, bit for bit: the same
// operations, every multiply-add written as one fmaf so that contraction
// cannot differ), for grids whose only valid map is B: the halo and the
// kinematics do not enter it.
template <bool JF>
__device__ __forceinline__ float eval_g(const float4* __restrict__ T, float s) {
    if (s < 4096.0f) {
        float u;
        const int k = piece(s, GK_S_ELO, u);
        return horner8(T[4 * k], T[4 * k + 1], u);
    }
    const float w = frcp(s), w3 = w * w * w;
    return w3 * tail_g<JF>(w);
}

template <int BULGE, int NDISC>
__device__ __forceinline__ float point_model_b(const TC& c, const Tabs& T, float du, float dv) {
    const float xp = fmaf(du, c.ca, dv * c.sa);
    const float yp = fmaf(dv, c.ca, -du * c.sa);
    const float y2 = yp * yp;
    float Bt = 0.0f, scale = 1.0f, r = 0.0f;
    if (NDISC > 0) {
        const float x2 = xp * xp;
        const float r2 = fmaf(y2, c.sec2i, x2);
        const float rinv = r2 > 0.0f ? frsq(r2) : 0.0f;
        r = r2 * rinv;
    }
    if (BULGE) {
        const float R = fsqrt(fmaf(xp, xp, y2));
        const float sb = fmaxf(R * c.invRb, S_MIN);
        Bt = c.Ab * eval_g<BULGE == 2>(T.gh, sb);
    }
    float eref = 0.0f;
    if (!BULGE && NDISC > 0) {
        eref = r * c.nl2Rd[0];
        if (NDISC > 1) eref = fmaxf(eref, r * c.nl2Rd[1]);
        scale = fexp2(eref);
    }
#pragma unroll
    for (int j = 0; j < NDISC; ++j) Bt = fmaf(c.Ad[j], fexp2(fmaf(r, c.nl2Rd[j], -eref)), Bt);
    return Bt * scale;
}

// ---------------------------------------------------------------------------
// reverse mode of point_model: given the adjoints fb = d logL / d(B, v, sigma,
// <L/M>) at one lattice point, accumulate d logL / d(constant) into ad[] for
// the FP32 per-theta constants below (the chain rule to theta is applied
// once per theta, in FP64).
// ---------------------------------------------------------------------------
enum {
    C_UF = 0, C_VF, C_CA, C_SA, C_SEC2I,
    C_INVRB, C_AB, C_CB, C_GMB, C_RB, C_MLB,
    C_D0 = 11,          // per disc j: C_D0 + 7 j + {0 nl2Rd, 1 Ad, 2 inv2Rd, 3 Kd, 4 kf, 5 sf, 6 MLd}
    C_H0 = 25, C_H1 = 26,
    NCONST = 27
};

template <int BULGE, int NDISC, int HALO>
__device__ __forceinline__ void point_model_adj(const TC& c, const Tabs& T, float du, float dv,
                                                float fB, float fV, float fS, float fL,
                                                float (&ad)[NCONST]) {
    // ---- forward recomputation (as point_model), keeping what the reverse needs
    const float xp = fmaf(du, c.ca, dv * c.sa);
    const float yp = fmaf(dv, c.ca, -du * c.sa);
    const float x2 = xp * xp, y2 = yp * yp;
    const float r2 = fmaf(y2, c.sec2i, x2);
    const float rinv = r2 > 0.0f ? frsq(r2) : 0.0f;
    const float r = r2 * rinv;
    const float cphi = xp * rinv;
    float vc2 = 0.0f, Bt = 0.0f, BS = 0.0f, kB = 0.0f, sB = 0.0f, mass = 0.0f;
    float scale = 1.0f;
    float R = 0.0f, g = 0.0f, h = 0.0f, dg = 0.0f, dh = 0.0f, Bb = 0.0f, iqb = 0.0f;
    bool clamped = true;
    if (BULGE) {
        R = fsqrt(x2 + y2);
        const float sbr = R * c.invRb;
        clamped = !(sbr > S_MIN);
        const float sb = clamped ? S_MIN : sbr;
        eval_gh_d<BULGE == 2>(T.gh, sb, g, h, dg, dh);
        Bb = c.Ab * g;
        Bt = Bb;
        BS = c.Cb * h;
        mass = Bb * c.MLb;
        iqb = frcp(r + c.Rb);
        vc2 = BULGE == 2 ? c.GMb * iqb : c.GMb * r * iqb * iqb;
    }
    float eref = 0.0f;
    if (!BULGE && NDISC > 0) {
        eref = r * c.nl2Rd[0];
        if (NDISC > 1) eref = fmaxf(eref, r * c.nl2Rd[1]);
        scale = fexp2(eref);
    }
    float ex[2] = {0.0f, 0.0f}, Bd[2] = {0.0f, 0.0f}, ph[2] = {0.0f, 0.0f}, dph[2] = {0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j < NDISC; ++j) {
        ex[j] = fexp2(fmaf(r, c.nl2Rd[j], -eref));
        Bd[j] = c.Ad[j] * ex[j];
        Bt += Bd[j];
        kB = fmaf(Bd[j], c.kf[j], kB);
        sB = fmaf(Bd[j], c.sf[j], sB);
        mass = fmaf(Bd[j], c.MLd[j], mass);
        ph[j] = eval_phi_d(T.phi, r * c.inv2Rd[j], dph[j]);
        vc2 = fmaf(c.Kd[j], ph[j], vc2);
    }
    float mv = 0.0f, dmv = 0.0f, iqh = 0.0f;
    if (HALO == 2) {
        mv = eval_m_d(T.m, r * c.H0, dmv);
        vc2 = fmaf(c.H1, mv, vc2);
    } else if (HALO == 1) {
        iqh = frcp(r + c.H0);
        vc2 = fmaf(c.H1 * r, iqh * iqh, vc2);
    }
    const float vint = fsqrt(vc2);
    const float ib = frcp(Bt);
    const float S2 = fmaf(vc2, sB, BS) * ib;
    const float oS = fsqrt(S2);
    const float imass = frcp(mass);

    // ---- reverse
    float Btb = fB * scale;
    // v = cphi vint kB ib
    const float vkb = vint * kB * ib;
    float cphib = fV * vkb;
    float vintb = fV * cphi * kB * ib;
    float kBb = fV * cphi * vint * ib;
    float ibb = fV * cphi * vint * kB;
    // sigma = sqrt(S2), S2 = (vc2 sB + BS) ib
    const float S2b = oS > 0.0f ? fS * 0.5f * frcp(oS) : 0.0f;
    float vc2b = S2b * sB * ib;
    const float sBb = S2b * vc2 * ib;
    const float BSb = S2b * ib;
    ibb = fmaf(S2b, fmaf(vc2, sB, BS), ibb);
    // <L/M> = Bt / mass
    Btb = fmaf(fL, imass, Btb);
    const float massb = -fL * Bt * imass * imass;
    // ib = 1 / Bt
    Btb = fmaf(-ibb, ib * ib, Btb);
    // vint = sqrt(vc2)
    if (vint > 0.0f) vc2b = fmaf(vintb, 0.5f * frcp(vint), vc2b);
    float rb = 0.0f;
    if (HALO == 2) {
        ad[C_H1] = fmaf(vc2b, mv, ad[C_H1]);
        const float xb = vc2b * c.H1 * dmv;
        rb = fmaf(xb, c.H0, rb);
        ad[C_H0] = fmaf(xb, r, ad[C_H0]);
    } else if (HALO == 1) {
        const float iq2 = iqh * iqh;
        ad[C_H1] = fmaf(vc2b, r * iq2, ad[C_H1]);
        // d/dr [r / q^2] = 1/q^2 - 2 r / q^3 ; d/dRh [r / q^2] = -2 r / q^3
        const float t = vc2b * c.H1;
        rb = fmaf(t, iq2 - 2.0f * r * iq2 * iqh, rb);
        ad[C_H0] = fmaf(t, -2.0f * r * iq2 * iqh, ad[C_H0]);
    }
#pragma unroll
    for (int j = 0; j < NDISC; ++j) {
        const int o = C_D0 + 7 * j;
        ad[o + 3] = fmaf(vc2b, ph[j], ad[o + 3]);
        const float yb = vc2b * c.Kd[j] * dph[j];
        rb = fmaf(yb, c.inv2Rd[j], rb);
        ad[o + 2] = fmaf(yb, r, ad[o + 2]);
        const float Bdb = fmaf(massb, c.MLd[j], fmaf(sBb, c.sf[j], fmaf(kBb, c.kf[j], Btb)));
        ad[o + 6] = fmaf(massb, Bd[j], ad[o + 6]);
        ad[o + 5] = fmaf(sBb, Bd[j], ad[o + 5]);
        ad[o + 4] = fmaf(kBb, Bd[j], ad[o + 4]);
        ad[o + 1] = fmaf(Bdb, ex[j], ad[o + 1]);
        const float argb = Bdb * c.Ad[j] * ex[j] * 0.69314718f;
        rb = fmaf(argb, c.nl2Rd[j], rb);
        ad[o + 0] = fmaf(argb, r, ad[o + 0]);
    }
    float x2b = 0.0f, y2b = 0.0f;
    if (BULGE) {
        const float iq2 = iqb * iqb;
        const float t = vc2b * c.GMb;
        if (BULGE == 2) {
            // v^2 = GM / q: d/dGM = 1/q; d/dr = d/dRb = -GM / q^2
            ad[C_GMB] = fmaf(vc2b, iqb, ad[C_GMB]);
            rb = fmaf(t, -iq2, rb);
            ad[C_RB] = fmaf(t, -iq2, ad[C_RB]);
        } else {
            ad[C_GMB] = fmaf(vc2b, r * iq2, ad[C_GMB]);
            rb = fmaf(t, iq2 - 2.0f * r * iq2 * iqb, rb);
            ad[C_RB] = fmaf(t, -2.0f * r * iq2 * iqb, ad[C_RB]);
        }
        const float Bbb = fmaf(massb, c.MLb, Btb);
        ad[C_MLB] = fmaf(massb, Bb, ad[C_MLB]);
        ad[C_CB] = fmaf(BSb, h, ad[C_CB]);
        ad[C_AB] = fmaf(Bbb, g, ad[C_AB]);
        if (!clamped) {
            const float sbb = fmaf(Bbb * c.Ab, dg, BSb * c.Cb * dh);
            const float Rb_ = sbb * c.invRb;
            ad[C_INVRB] = fmaf(sbb, R, ad[C_INVRB]);
            if (R > 0.0f) {
                const float t2 = Rb_ * 0.5f * frcp(R);
                x2b += t2;
                y2b += t2;
            }
        }
    }
    // frame: cphi = xp rinv, r = r2 rinv, rinv = r2^-1/2, r2 = y2 sec2i + x2
    float xpb = cphib * rinv;
    float r2b = 0.0f;
    if (r2 > 0.0f) {
        const float rinvb = fmaf(cphib, xp, rb * r2);
        r2b = fmaf(rb, rinv, -0.5f * rinvb * rinv * rinv * rinv);
    }
    y2b = fmaf(r2b, c.sec2i, y2b);
    ad[C_SEC2I] = fmaf(r2b, y2, ad[C_SEC2I]);
    x2b += r2b;
    xpb = fmaf(2.0f * xp, x2b, xpb);
    const float ypb = 2.0f * yp * y2b;
    // xp = du ca + dv sa, yp = dv ca - du sa, du = (u - Ui) - Uf
    ad[C_CA] = fmaf(xpb, du, fmaf(ypb, dv, ad[C_CA]));
    ad[C_SA] = fmaf(xpb, dv, fmaf(-ypb, du, ad[C_SA]));
    const float dub = fmaf(xpb, c.ca, -ypb * c.sa);
    const float dvb = fmaf(xpb, c.sa, ypb * c.ca);
    ad[C_UF] -= dub;
    ad[C_VF] -= dvb;
}

// Reverse mode of point_model_b: the adjoint fB = d logL / dB at one lattice
// point of a grid whose only valid map is B, accumulated into the adjoints
// of the constants B depends on (frame, bulge Ab and 1/Rb, discs Ad and
// -log2(e)/Rd); the other constants' adjoints are untouched.
template <bool JF>
__device__ __forceinline__ float eval_g_d(const float4* __restrict__ T, float s, float& dg) {
    if (s < 4096.0f) {
        float u;
        const int k = piece(s, GK_S_ELO, u);
        const float v = horner8d(T[4 * k], T[4 * k + 1], u, dg);
        dg *= piece_dudx(s);
        return v;
    }
    const float w = frcp(s), w2 = w * w, w3 = w2 * w;
    const Dual pg = tail_g<JF>(Dual{w, 1.0f});              // s^3 g = Pg(w), w = 1/s
    dg = -w3 * w * (3.0f * pg.v + w * pg.d);
    return w3 * pg.v;
}

template <int BULGE, int NDISC>
__device__ __forceinline__ void point_model_adj_b(const TC& c, const Tabs& T, float du, float dv, float fB,
                                                  float (&ad)[NCONST]) {
    const float xp = fmaf(du, c.ca, dv * c.sa);
    const float yp = fmaf(dv, c.ca, -du * c.sa);
    const float x2 = xp * xp, y2 = yp * yp;
    float r = 0.0f, r2 = 0.0f, rinv = 0.0f;
    if (NDISC > 0) {
        r2 = fmaf(y2, c.sec2i, x2);
        rinv = r2 > 0.0f ? frsq(r2) : 0.0f;
        r = r2 * rinv;
    }
    float scale = 1.0f, eref = 0.0f;
    if (!BULGE && NDISC > 0) {
        eref = r * c.nl2Rd[0];
        if (NDISC > 1) eref = fmaxf(eref, r * c.nl2Rd[1]);
        scale = fexp2(eref);
    }
    // B = scale (Ab g(R / Rb) + sum_j Ad_j 2^(r nl2Rd_j - eref)); eref cancels
    const float Btb = fB * scale;
    float rb = 0.0f, x2b = 0.0f, y2b = 0.0f;
#pragma unroll
    for (int j = 0; j < NDISC; ++j) {
        const int o = C_D0 + 7 * j;
        const float ex = fexp2(fmaf(r, c.nl2Rd[j], -eref));
        ad[o + 1] = fmaf(Btb, ex, ad[o + 1]);
        const float argb = Btb * c.Ad[j] * ex * 0.69314718f;
        rb = fmaf(argb, c.nl2Rd[j], rb);
        ad[o + 0] = fmaf(argb, r, ad[o + 0]);
    }
    if (BULGE) {
        const float R = fsqrt(fmaf(xp, xp, y2));
        const float sbr = R * c.invRb;
        const bool clamped = !(sbr > S_MIN);
        float dg;
        const float g = eval_g_d<BULGE == 2>(T.gh, clamped ? S_MIN : sbr, dg);
        ad[C_AB] = fmaf(Btb, g, ad[C_AB]);
        if (!clamped) {
            const float sbb = Btb * c.Ab * dg;
            ad[C_INVRB] = fmaf(sbb, R, ad[C_INVRB]);
            if (R > 0.0f) {
                const float t2 = sbb * c.invRb * 0.5f * frcp(R);
                x2b += t2;
                y2b += t2;
            }
        }
    }
    if (NDISC > 0 && r2 > 0.0f) {
        // r = r2 rinv, rinv = r2^-1/2, r2 = y2 sec2i + x2
        const float rinvb = rb * r2;
        const float r2b = fmaf(rb, rinv, -0.5f * rinvb * rinv * rinv * rinv);
        y2b = fmaf(r2b, c.sec2i, y2b);
        ad[C_SEC2I] = fmaf(r2b, y2, ad[C_SEC2I]);
        x2b += r2b;
    }
    const float xpb = 2.0f * xp * x2b;
    const float ypb = 2.0f * yp * y2b;
    ad[C_CA] = fmaf(xpb, du, fmaf(ypb, dv, ad[C_CA]));
    ad[C_SA] = fmaf(xpb, dv, fmaf(-ypb, du, ad[C_SA]));
    const float dub = fmaf(xpb, c.ca, -ypb * c.sa);
    const float dvb = fmaf(xpb, c.sa, ypb * c.ca);
    ad[C_UF] -= dub;
    ad[C_VF] -= dvb;
}

}  // namespace gk
