// Adjoint of the likelihood: d logL / d theta from the forward pass's
// per-pixel adjoints rbar = d logL / d F (written by the forward kernel in its
// adjoint-seed mode), compiled once per PSF mode and horizontal tap-pair
// count (-DGK_LW=0|1 -DGK_KH=4|6); the map-averaging units also carry the
// light-only variant for grids whose only valid map is B.
//
// One workgroup = one parameter vector x one block of the padded lattice.
// The gradient is the sum, over pixels p and maps m, of rbar_m(p)
// dF_m(p)/dtheta; F_m(p) averages the model over the lattice points of p's
// 3-sigma stencil (Sec. 3.1, PSF equation), so it equals the sum over lattice
// points x of fbar(x) dF(x)/dtheta with the transposed stencil
//   fbar(x, r) = (1/W) sum_p rbar(p) g(|x - x_p|) g(|r - r_p|) [inside the stencil].
// The blocks tile the lattice (a band of pixels owns the lattice points
// between its pixels' centres shifted by pad - s/2, the outer bands the
// margins), so every lattice point's reverse model runs once; a block reads
// the pixel adjoints of every pixel that reaches it (its frame: the band and
// a halo of about D pixels), which needs no exchange between workgroups.
// The block is streamed top to bottom in phases of R lattice rows (any R,
// independent of s):
//
//   ring       the pixel rows of rbar the phase reaches (a ring of
//              D + 1 + ceil((R - 1) / s) rows; a phase's new rows are loaded
//              while the previous phase's points are evaluated);
//   vertical   per (lattice row, pixel column): running sums S_l of
//              g(|b|) rbar over the pixel rows in reach, grouped by the
//              stencil half-width A(|b|) (largest first);
//   horizontal per lattice point: fbar = (1/W) sum over the D + 1 pixel
//              columns in reach of g(|t|) S_l(t), l(t) = groups with A >= |t|
//              (both tables are uniform per row phase and column phase and are
//              built on the host), then the reverse point model into 27 FP32
//              adjoints of the per-theta constants.
//
// The special-function tables are read from constant memory through the
// vector L1 cache (the luminosity-weighted body, which evaluates the model
// twice per point, copies them to LDS instead).  The constant adjoints are
// summed in FP64 (waves, then bands in order, by the last workgroup of the
// vector), and the chain rule to theta runs once.
#include "gk_fwd.h"

#ifndef GK_LW
#error "compile with -DGK_LW=<0|1>"
#endif
#ifndef GK_KH
#error "compile with -DGK_KH=<4|6>"
#endif

namespace gk {

// The pixel adjoints travel as one float4 per pixel (the four maps) or, for a
// grid whose only valid map is B, as one float.
template <int BO> struct AdjVec { using T = float4; };
template <> struct AdjVec<1> { using T = float; };
__device__ __forceinline__ void vzero(float4& v) { v = make_float4(0.f, 0.f, 0.f, 0.f); }
__device__ __forceinline__ void vzero(float& v) { v = 0.0f; }
__device__ __forceinline__ void vfma(float w, const float4& v, float4& acc) {
    acc.x = fmaf(w, v.x, acc.x);
    acc.y = fmaf(w, v.y, acc.y);
    acc.z = fmaf(w, v.z, acc.z);
    acc.w = fmaf(w, v.w, acc.w);
}
__device__ __forceinline__ void vfma(float w, float v, float& acc) { acc = fmaf(w, v, acc); }

// Chain rule from the adjoints of the FP32 constants of make_tc to the
// parameters (FP64), then writes the gradient row (zeros past P), or adds it
// to the row (accum; the padding columns are left alone).
__device__ inline void chain_rule(const double* th, const GridGeom& g, const double* cb, double* out,
                                  int stride, int accum) {
    const double d2r = PI / 180.0, LN10 = 2.302585092994046;
    double gr[32];
    for (int k = 0; k < 32; ++k) gr[k] = 0.0;
    const double pa = th[2] * d2r, inc = th[3] * d2r;
    double spa, cpa, si, ci;
    sincos(pa, &spa, &cpa);
    sincos(inc, &si, &ci);
    const double pks = g.pk / g.s;
    gr[0] = cb[C_UF] * g.s * g.fscale;
    gr[1] = cb[C_VF] * g.s * g.fscale;
    gr[2] = (cb[C_CA] * (-pks * spa) + cb[C_SA] * (pks * cpa)) * d2r;
    gr[3] = cb[C_SEC2I] * 2.0 * si / (ci * ci * ci) * d2r;
    int k = 4;
    if (g.bulge) {
        const double Mb = exp10(th[k]), Rb = th[k + 1], ML = th[k + 2];
        const double fa = g.bulge == 2 ? 1.0 : 2.0 * PI, fc = g.bulge == 2 ? 4.0 * PI : 12.0 * PI;
        const double Ab = 1.0e-6 * Mb / (fa * Rb * Rb * ML);
        const double Cb = 1.0e-6 * G_KPC * Mb * Mb / (fc * Rb * Rb * Rb * ML);
        const double GMb = G_KPC * Mb;
        gr[k] = (cb[C_AB] * Ab + 2.0 * cb[C_CB] * Cb + cb[C_GMB] * GMb) * LN10;
        gr[k + 1] = -cb[C_INVRB] / (Rb * Rb) - 2.0 * cb[C_AB] * Ab / Rb - 3.0 * cb[C_CB] * Cb / Rb + cb[C_RB];
        gr[k + 2] = -cb[C_AB] * Ab / ML - cb[C_CB] * Cb / ML + cb[C_MLB];
        k += 3;
    }
    for (int j = 0; j < g.ndisc; ++j) {
        const int o = C_D0 + 7 * j;
        const double Md = exp10(th[k]), Rd = th[k + 1], ML = th[k + 2], kk = th[k + 3];
        const double nl2Rd = -1.4426950408889634 / Rd;
        const double Ad = 1.0e-6 * Md / (2.0 * PI * Rd * Rd * ci * ML);
        const double inv2Rd = 0.5 / Rd;
        const double Kd = 2.0 * G_KPC * Md / Rd;
        gr[k] = (cb[o + 1] * Ad + cb[o + 3] * Kd) * LN10;
        gr[k + 1] = -(cb[o + 0] * nl2Rd + 2.0 * cb[o + 1] * Ad + cb[o + 2] * inv2Rd + cb[o + 3] * Kd) / Rd;
        gr[k + 2] = -cb[o + 1] * Ad / ML + cb[o + 6];
        gr[k + 3] = -cb[o + 4] * si - cb[o + 5] * 2.0 * kk / 3.0;
        gr[3] += (cb[o + 1] * Ad * si / ci - cb[o + 4] * kk * ci) * d2r;
        k += 4;
    }
    if (g.halo == 2) {
        const double M200 = exp10(th[k]), conc = th[k + 1];
        const double r200 = cbrt(3.0 * M200 / (4.0 * PI * 200.0 * g.rho_crit));
        const double rs = r200 / conc;
        const double muc = log1p(conc) - conc / (1.0 + conc);
        const double H0 = 1.0 / rs, H1 = G_KPC * M200 / (rs * muc);
        const double dmu = conc / ((1.0 + conc) * (1.0 + conc));
        gr[k] = (-cb[C_H0] * H0 / 3.0 + cb[C_H1] * H1 * 2.0 / 3.0) * LN10;
        gr[k + 1] = cb[C_H0] / r200 + cb[C_H1] * H1 * (1.0 / conc - dmu / muc);
        k += 2;
    } else if (g.halo == 1) {
        const double H1 = G_KPC * exp10(th[k]);
        gr[k] = cb[C_H1] * H1 * LN10;
        gr[k + 1] = cb[C_H0];
        k += 2;
    }
    if (accum)
        for (int q = 0; q < k; ++q) out[q] += gr[q];
    else
        for (int q = 0; q < stride; ++q) out[q] = q < k ? gr[q] : 0.0;
}

// KH: horizontal tap pairs per (row phase, column phase), the table's stride
// (pairs past (D + 1) / 2 are zero), so that the gather's loads issue together
// BO = 1: the grid's only valid map is B (never with LW): the light-only
// reverse model (point_model_adj_b), the other maps' adjoints being zero.
template <int BULGE, int NDISC, int HALO, int LW, int KH, int BO = 0>
__global__ void __launch_bounds__(ADJ_BS) adj_kernel(AdjArgs a) {
    static_assert(!BO || !LW, "the light-only reverse model carries B alone");
    extern __shared__ __align__(16) float smem[];
    const int tid = threadIdx.x, BS = blockDim.x;
    const int band = blockIdx.x % a.nbands;
    const int b = blockIdx.x / a.nbands;
    const GridGeom& G = a.geo;
    const int s = G.s, pad = G.pad, hs = G.hs, D = a.D;
    const int by = band / a.nbx, bx = band - by * a.nbx;
    const int j0 = by * a.band_h, j1 = min(G.ny, j0 + a.band_h);
    const int c0 = bx * a.band_w, c1 = min(G.nx, c0 + a.band_w);
    // the band owns a block of the lattice: rows [Lr0, Lr1) and columns
    // [Lc0, Lc1) of the whole padded lattice (lattice row g lies in the
    // stencils of pixel rows ceil((g - 2 pad) / s) .. floor(g / s)); the
    // blocks of all bands tile it, the outer bands taking the margins
    const int NLR = (G.ny - 1) * s + 2 * pad + 1, NLC = (G.nx - 1) * s + 2 * pad + 1;
    const int own = pad - s / 2;
    const int Lr0 = by == 0 ? 0 : j0 * s + own, Lr1 = j1 == G.ny ? NLR : j1 * s + own;
    const int Lc0 = bx == 0 ? 0 : c0 * s + own, Lc1 = c1 == G.nx ? NLC : c1 * s + own;
    // frame: the pixels whose stencils reach the block (their adjoints are
    // read, the halo included); frame lattice row r is lattice row jf0 s + r
    const int jf0 = max(0, ceil_div(Lr0 - 2 * pad, s)), jf1 = min(G.ny, (Lr1 - 1) / s + 1);
    const int cf0 = max(0, ceil_div(Lc0 - 2 * pad, s)), cf1 = min(G.nx, (Lc1 - 1) / s + 1);
    const int NR = jf1 - jf0, NC = cf1 - cf0;
    // block rows and columns before the frame's first lattice row / column
    // (possible when pad < s / 2) are reached by no pixel: they start at 0,
    // so every index below is non-negative
    const int rbeg = max(0, Lr0 - jf0 * s), rend = Lr1 - jf0 * s;
    const int xbeg = max(0, Lc0 - cf0 * s), xend = Lc1 - cf0 * s;
    const int vlo = jf0 * s + hs, ubase = cf0 * s + hs;
    const int RS = a.rows, NLEV = a.nlev, NCP = NC + 2 * D, RB = a.rb;
    const AdjLayout L = adj_layout(a.band_h, a.band_w, s, pad, D, RS, NLEV, RB, 2 * KH, LW);
    float* s_tab = smem + L.tab;                    // the LW body's copy of the tables
    using V = typename AdjVec<BO>::T;               // four maps, or B alone
    V* s_ring = (V*)(smem + L.ring);                // [RB][NC]
    V* s_S = (V*)(smem + L.S);                      // [RS][NCP][NLEV]
    const int4* s_ht = (const int4*)(smem + L.ht);  // [s][s][KH]
    const int2* s_vt = (const int2*)(smem + L.vt);  // [s][DSTRIDE]
    double* s_red = (double*)(smem + L.red);
    int2* s_span = (int2*)(smem + L.span);
    int* s_aof = (int*)(smem + L.aof);
    int* s_prange = (int*)(smem + L.prange);

    const double* th = a.theta + (size_t)b * a.stride;
    const TC tc = uniform_tc(make_tc(th, G));
    if (!tc.valid) {
        if (band == 0 && !a.accum)
            for (int q = tid; q < a.stride; q += BS) a.grad[(size_t)b * a.stride + q] = 0.0;
        return;
    }
    // ---- prologue: tables (LW), zeroed ring and S buffer, row spans
    {
        if constexpr (LW != 0) {
            const Tabs C = const_tabs<BULGE>();
            const float* tgh = (const float*)C.gh;
            for (int i = tid; i < TAB_GH; i += BS) s_tab[i] = tgh[i];
            for (int i = tid; i < TAB_PHI; i += BS) s_tab[TAB_GH + i] = gk_tab_phi[i];
            for (int i = tid; i < TAB_M; i += BS) s_tab[TAB_GH + TAB_PHI + i] = gk_tab_m[i];
        }
        int* ht = (int*)(smem + L.ht);
        const int* ght = (const int*)a.ht;
        for (int i = tid; i < s * s * KH * 4; i += BS) ht[i] = ght[i];
        int* vt = (int*)(smem + L.vt);
        const int* gvt = (const int*)a.vt;
        for (int i = tid; i < s * DSTRIDE * 2; i += BS) vt[i] = gvt[i];
        V z;
        vzero(z);
        for (int i = tid; i < RB * NC; i += BS) s_ring[i] = z;
        for (int i = tid; i < RS * NCP * NLEV; i += BS) s_S[i] = z;
        for (int i = tid; i < NR; i += BS) s_span[i] = a.span[jf0 + i];
        for (int i = tid; i <= pad; i += BS) s_aof[i] = a.aof[i];
    }
    __syncthreads();
    // needed lattice columns of each phase: the owned columns within the
    // union, over the phase's lattice rows, of the stencils of the frame's
    // valid pixels (elsewhere every pixel adjoint in reach is zero)
    const int nph = (rend - rbeg + RS - 1) / RS;
    for (int k = tid; k < nph; k += BS) {
        int lo = 1 << 30, hi = -(1 << 30);
        for (int r = rbeg + k * RS; r < min(rend, rbeg + (k + 1) * RS); ++r) {
            const int jlo = r >= 2 * pad ? (r - 2 * pad + s - 1) / s : 0;
            const int jhi = min(NR - 1, r / s);
            for (int jj = jlo; jj <= jhi; ++jj) {
                int bb = r - jj * s - pad;
                bb = bb < 0 ? -bb : bb;
                const int2 sp = s_span[jj];
                const int cl = max(cf0, sp.x), ch = min(cf1 - 1, sp.y);
                if (cl <= ch) {
                    const int A = s_aof[bb];
                    lo = min(lo, (cl - cf0) * s + pad - A);
                    hi = max(hi, (ch - cf0) * s + pad + A);
                }
            }
        }
        lo = max(lo, xbeg);
        hi = min(hi, xend - 1);
        // frame columns < 2^15 (band_w <= 128, D <= 10, s <= 15): both fields fit
        s_prange[k] = hi >= lo ? lo | ((hi - lo + 1) << 16) : 0;
    }
    const Tabs T = LW ? Tabs{(const float4*)s_tab, (const float4*)(s_tab + TAB_GH),
                             (const float4*)(s_tab + TAB_GH + TAB_PHI)}
                      : const_tabs<BULGE>();
    float ad[NCONST];
#pragma unroll
    for (int k = 0; k < NCONST; ++k) ad[k] = 0.0f;
    const float invW = a.invW;
    const float inv_s = 1.0f / (float)s;
    const float inv_nc = 1.0f / (float)NC;
    const size_t mstr = (size_t)G.ny * G.nx;
    const float* fb = a.fbar + (size_t)b * 4 * mstr;
    // Pixel rows of rbar enter a ring of RB rows, slot = row mod RB.  The rows
    // a phase reaches are loaded during the previous phase's gather (the ring
    // is not read then), so a phase needs two barriers: when they fit one per
    // thread, their global loads are issued before that gather and stored to
    // the ring after it, so that the gather hides their latency.
    // the first phase reaches pixel rows from rbeg / s - D on
    int loaded = max(-1, rbeg / s - D - 1);         // last pixel row put in the ring
    auto load_rows = [&](int rA_next) {
        const int nrow_n = min(RS, rend - rA_next);
        const int qlo_n = rA_next / s, qhi_n = (rA_next + nrow_n - 1) / s;
        const int base_n = ((qlo_n - D) % RB + RB) % RB;
        const int nnew = qhi_n - loaded;
        for (int p = tid; p < nnew * NC; p += BS) {
            const int k = (int)(((float)p + 0.5f) * inv_nc), cc = p - k * NC;
            const int jj = loaded + 1 + k;
            V v;
            vzero(v);
            if (jj < NR) {
                const size_t pix = (size_t)(jf0 + jj) * G.nx + cf0 + cc;
                if constexpr (BO)
                    v = fb[pix];
                else
                    v = make_float4(fb[pix], fb[mstr + pix], fb[2 * mstr + pix], fb[3 * mstr + pix]);
            }
            int slot = base_n + jj - (qlo_n - D);
            slot = slot >= RB ? slot - RB : slot;
            s_ring[slot * NC + cc] = v;
        }
        loaded = max(loaded, qhi_n);
    };
    load_rows(rbeg);
    __syncthreads();
    for (int rA = rbeg, ph_i = 0; rA < rend; rA += RS, ++ph_i) {
        const int nrow = min(RS, rend - rA);
        // pixel rows [qlo - D, qhi] are in reach of lattice rows [rA, rA + nrow); ring
        // slot of pixel row jj: base + jj - (qlo - D), wrapped, base = (qlo - D) mod RB
        const int qlo = rA / s;
        const int base = ((qlo - D) % RB + RB) % RB;
        // ---- vertical pass: group sums per (lattice row, pixel column)
        for (int p = tid; p < nrow * NC; p += BS) {
            const int rl = (int)(((float)p + 0.5f) * inv_nc), cc = p - rl * NC;
            const int r = rA + rl;
            const int qr = (int)(((float)r + 0.5f) * inv_s), ph = r - qr * s;
            const int2* vt = s_vt + ph * DSTRIDE;
            V* Sp = s_S + ((size_t)rl * NCP + cc + D) * NLEV;
            const int off0 = base + qr - qlo + D;       // ring position of pixel row qr, unwrapped
            // all DSTRIDE entries (zero past the phase's lags: weight 0, no
            // store), so that the table and ring loads issue together
            int2 e[DSTRIDE];
#pragma unroll
            for (int n = 0; n < DSTRIDE; ++n) e[n] = vt[n];
            V v[DSTRIDE];
#pragma unroll
            for (int n = 0; n < DSTRIDE; ++n) {
                int slot = off0 - (e[n].x & 255);
                slot = slot >= RB ? slot - RB : slot;
                v[n] = s_ring[slot * NC + cc];
            }
            V acc;
            vzero(acc);
#pragma unroll
            for (int n = 0; n < DSTRIDE; ++n) {
                vfma(__int_as_float(e[n].y), v[n], acc);
                if (e[n].x >> 16) Sp[(e[n].x >> 8) & 255] = acc;
            }
        }
        __syncthreads();
        // ---- the next phase's new pixel rows: global loads issued now
        const bool more = rA + RS < rend;
        bool pf_sync = false;
        int pf_at = -1;
        V pf_v;
        vzero(pf_v);
        if (more) {
            const int rA_next = rA + RS;
            const int nrow_n = min(RS, rend - rA_next);
            const int qlo_n = rA_next / s, qhi_n = (rA_next + nrow_n - 1) / s;
            const int base_n = ((qlo_n - D) % RB + RB) % RB;
            const int nnew = qhi_n - loaded;
            if (nnew * NC <= BS) {
                if (tid < nnew * NC) {
                    const int k = (int)(((float)tid + 0.5f) * inv_nc), cc = tid - k * NC;
                    const int jj = loaded + 1 + k;
                    if (jj < NR) {
                        const size_t pix = (size_t)(jf0 + jj) * G.nx + cf0 + cc;
                        if constexpr (BO)
                            pf_v = fb[pix];
                        else
                            pf_v = make_float4(fb[pix], fb[mstr + pix], fb[2 * mstr + pix], fb[3 * mstr + pix]);
                    }
                    int slot = base_n + jj - (qlo_n - D);
                    slot = slot >= RB ? slot - RB : slot;
                    pf_at = slot * NC + cc;
                }
                loaded = max(loaded, qhi_n);
            } else {
                pf_sync = true;
            }
        }
        // ---- horizontal gather and reverse point model, flat over the phase's points
        const int prange = s_prange[ph_i];
        const int plo = prange & 0xffff, pw = prange >> 16;
        const int npts = nrow * pw;
        const float inv_pw = 1.0f / (float)max(pw, 1);
        for (int qq = tid; qq < npts; qq += BS) {
            const int rl = (int)(((float)qq + 0.5f) * inv_pw);
            const int x = plo + (qq - rl * pw);
            const int qr = (int)(((float)(rA + rl) + 0.5f) * inv_s), ph = rA + rl - qr * s;
            const int qx = (int)(((float)x + 0.5f) * inv_s), ix = x - qx * s;
            const V* Sb = s_S + ((size_t)rl * NCP + qx + D) * NLEV;
            const int4* h = s_ht + (ph * s + ix) * KH;
            int4 e[KH];
#pragma unroll
            for (int k2 = 0; k2 < KH; ++k2) e[k2] = h[k2];
            V f;
            vzero(f);
#pragma unroll
            for (int k2 = 0; k2 < KH; ++k2) {
                const V v0 = Sb[e[k2].x], v1 = Sb[e[k2].z];
                vfma(__int_as_float(e[k2].y), v0, f);
                vfma(__int_as_float(e[k2].w), v1, f);
            }
            const int r = rA + rl;
            const float du = (float)(ubase + x - tc.Ui) - tc.Uf;
            const float dv = (float)(vlo + r - tc.Vi) - tc.Vf;
            if constexpr (BO) {
                point_model_adj_b<BULGE, NDISC>(tc, T, du, dv, f * invW, ad);
            } else {
                float4 fo = make_float4(f.x * invW, f.y * invW, f.z * invW, f.w * invW);
                if (LW) {
                    // the lattice carries (B, B v, B (sigma^2 + v^2), B / <L/M>): map their
                    // adjoints to those of (B, v, sigma, <L/M>) at this point
                    float pB, pV, pS, pL;
                    point_model<BULGE, NDISC, HALO>(tc, T, du, dv, pB, pV, pS, pL);
                    const float il = frcp(pL);
                    fo = make_float4(fo.x + fo.y * pV + fo.z * fmaf(pS, pS, pV * pV) + fo.w * il,
                                     fmaf(fo.y, pB, 2.0f * fo.z * pB * pV), 2.0f * fo.z * pB * pS,
                                     -fo.w * pB * il * il);
                }
                point_model_adj<BULGE, NDISC, HALO>(tc, T, du, dv, fo.x, fo.y, fo.z, fo.w, ad);
            }
        }
        if (pf_sync) load_rows(rA + RS);            // too many rows to prefetch in registers
        if (pf_at >= 0) s_ring[pf_at] = pf_v;
        __syncthreads();
    }

    // ---- FP64 reduction of the constant adjoints: waves (all constants
    // stepped together, so the shuffles overlap), then bands in order
    const int lane = tid & 63, wave = tid >> 6, nw = (BS + 63) >> 6;
    {
        double v[NCONST];
#pragma unroll
        for (int k = 0; k < NCONST; ++k) v[k] = (double)ad[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
            for (int k = 0; k < NCONST; ++k) v[k] += __shfl_down(v[k], o, 64);
        }
        if (lane == 0)
#pragma unroll
            for (int k = 0; k < NCONST; ++k) s_red[wave * NCONST + k] = v[k];
    }
    __syncthreads();
    double* gp = a.gpart + ((size_t)b * a.nbands + band) * NCONST;
    if (tid < NCONST) {
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += s_red[w * NCONST + tid];
        gp[tid] = t;
    }
    __syncthreads();
    if (tid == 0) {
        bool last = true;
        if (a.nbands > 1) {
            const unsigned ticket = __hip_atomic_fetch_add(a.counters + b, 1u, __ATOMIC_ACQ_REL,
                                                           __HIP_MEMORY_SCOPE_AGENT);
            last = ticket == (unsigned)a.nbands - 1;
        }
        if (last) {
            double cb[NCONST];
            for (int k = 0; k < NCONST; ++k) cb[k] = 0.0;
            for (int bnd = 0; bnd < a.nbands; ++bnd)
                for (int k = 0; k < NCONST; ++k)
                    cb[k] += __hip_atomic_load(a.gpart + ((size_t)b * a.nbands + bnd) * NCONST + k,
                                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            chain_rule(th, G, cb, a.grad + (size_t)b * a.stride, a.stride, a.accum);
            if (a.nbands > 1) __hip_atomic_store(a.counters + b, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

template <int LW, int KH>
hipError_t launch_adj_lw(int bulge, int nd, int halo, int bonly, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                         const AdjArgs& a) {
#if GK_LW == 0
    if (bonly) {                // light-only reverse model: the halo does not enter B
#define GK_BALAUNCH(BU, ND)                                                                     \
        if (bulge == BU && nd == ND) {                                                          \
            hipLaunchKernelGGL((adj_kernel<BU, ND, 0, LW, KH, 1>), grid, block, lds, st, a);   \
            return hipGetLastError();                                                           \
        }
        GK_BALAUNCH(1, 0) GK_BALAUNCH(1, 1) GK_BALAUNCH(1, 2)
        GK_BALAUNCH(2, 0) GK_BALAUNCH(2, 1) GK_BALAUNCH(2, 2)
        GK_BALAUNCH(0, 1) GK_BALAUNCH(0, 2)
#undef GK_BALAUNCH
        return hipErrorInvalidValue;
    }
#else
    if (bonly) return hipErrorInvalidValue;
#endif
#define GK_ALAUNCH(BU, ND, HA)                                                          \
    if (bulge == BU && nd == ND && halo == HA) {                                         \
        hipLaunchKernelGGL((adj_kernel<BU, ND, HA, LW, KH>), grid, block, lds, st, a);  \
        return hipGetLastError();                                                        \
    }
    GK_ALAUNCH(1, 0, 0) GK_ALAUNCH(1, 0, 1) GK_ALAUNCH(1, 0, 2)
    GK_ALAUNCH(1, 1, 0) GK_ALAUNCH(1, 1, 1) GK_ALAUNCH(1, 1, 2)
    GK_ALAUNCH(1, 2, 0) GK_ALAUNCH(1, 2, 1) GK_ALAUNCH(1, 2, 2)
    GK_ALAUNCH(2, 0, 0) GK_ALAUNCH(2, 0, 1) GK_ALAUNCH(2, 0, 2)
    GK_ALAUNCH(2, 1, 0) GK_ALAUNCH(2, 1, 1) GK_ALAUNCH(2, 1, 2)
    GK_ALAUNCH(2, 2, 0) GK_ALAUNCH(2, 2, 1) GK_ALAUNCH(2, 2, 2)
    GK_ALAUNCH(0, 1, 0) GK_ALAUNCH(0, 1, 1) GK_ALAUNCH(0, 1, 2)
    GK_ALAUNCH(0, 2, 0) GK_ALAUNCH(0, 2, 1) GK_ALAUNCH(0, 2, 2)
#undef GK_ALAUNCH
    return hipErrorInvalidValue;
}

template hipError_t launch_adj_lw<GK_LW, GK_KH>(int, int, int, int, dim3, dim3, size_t, hipStream_t, const AdjArgs&);

}  // namespace gk
