// The forward body: one parameter vector on one band of pixels (the model
// on the band's fine lattice, the separable PSF stencil and the chi^2), shared
// by the single-grid kernel and the many-grid kernel.
#pragma once

#include "gk_kern.h"

namespace gk {

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

typedef const __attribute__((address_space(4))) int* const_int_ptr;

// One pixel-row step of the separable stencil for one (map, pixel column).
// The step's s lattice rows (phases) each give horizontal partial sums
// H_0..H_PAD at the pixel centre from one batch of LDS loads; the pixel row
// at lag d (d steps back) takes weight g(|b|) times H_A(|b|), b = d s + ph - pad.
// acc[d] holds the running PSF sum of the pixel row d steps back; it is
// shifted by one each step, so acc[D] is complete after this call.  DL is the
// largest lag the tap count PAD admits (lag_cap): the loop over lags stops
// there instead of at DMAX.
template <int PAD, int DL>
__device__ __forceinline__ void stencil_sub(const float* __restrict__ L0, int rstride, int s,
                                            const float* __restrict__ gw, const int2* __restrict__ tab,
                                            float (&acc)[DMAX + 1]) {
    float g[PAD + 1];
#pragma unroll
    for (int k = 0; k <= PAD; ++k) g[k] = gw[k];
    float con[DL + 1];
#pragma unroll
    for (int d = 0; d <= DL; ++d) con[d] = 0.0f;
    for (int ph = 0; ph < s; ++ph) {
        const float* L = L0 + ph * rstride;
        float H[PAD + 1];
        H[0] = g[0] * L[0];
#pragma unroll
        for (int k = 1; k <= PAD; ++k) H[k] = fmaf(g[k], L[-k] + L[k], H[k - 1]);
        // table entries through the constant address space: scalar loads; lags
        // beyond D have weight 0, so the loop has a fixed trip count
        const_int_ptr t = (const_int_ptr)tab + 2 * ph * DSTRIDE;
#pragma unroll
        for (int d = 0; d <= DL; ++d) {
            const int A = t[2 * d];
            const float w = __int_as_float(t[2 * d + 1]);
            con[d] = fmaf(w, H[A], con[d]);
        }
    }
#pragma unroll
    for (int d = DL; d >= 1; --d) acc[d] = acc[d - 1] + con[d];
    acc[0] = con[0];
}

// One parameter vector (row b) on one band of one grid.  LW = 1:
// the PSF averages luminosity-weighted moments (a compile-time switch, so the
// map-averaging instantiations do not carry its registers).
// BO = 1: the grid's only valid map is B (a photometric grid; never with
// MODE_MAPS or LW): the model phase evaluates the surface brightness alone
// (point_model_b, equal bit for bit to point_model's B) and leaves the other
// three rows of the buffer at zero, which the stencil skips anyway.
// TL = 1: the special-function tables are copied to LDS (after the rest of
// the layout) and read there; else they are read from constant memory
// through the vector L1 cache.  The copy pays where the registers already
// cap the occupancy that the LDS it takes would lower: the many-grid kernel
// and the luminosity-weighted seed pass.
template <int BULGE, int NDISC, int HALO, int MODE, int LW, int BO = 0, int TL = 0>
__device__ __forceinline__ void fwd_band(const FwdArgs& a, const int b, const int band, float* smem) {
    static_assert(!BO || (MODE != MODE_MAPS && !LW), "the light-only body computes B alone");
    const int tid = threadIdx.x, BS = blockDim.x;
    const GridGeom& G = a.geo;
    const int s = G.s, pad = G.pad, hs = G.hs;
    const int by = band / a.nbx, bx = band - by * a.nbx;
    const int j0 = by * a.band_h, j1 = min(G.ny, j0 + a.band_h);
    const int c0 = bx * a.band_w, c1 = min(G.nx, c0 + a.band_w);
    const int NR = j1 - j0, NC = c1 - c0;
    const int NFR = (NR - 1) * s + 2 * pad + 1;
    const int vlo = j0 * s + hs;                    // lattice row of local row 0
    const int ubase = c0 * s + hs;                  // lattice column of local column 0
    const int nfrm = nfr_max(a.band_h, s, pad);
    const int RS = a.gsub * s;
    constexpr bool TAB_LDS = TL != 0;
    const Layout L = make_layout(RS, a.xw, nfrm, a.band_h, LW ? 8 * a.gsub * a.band_w : 0, TAB_LDS);
    float* s_tab = smem + L.tab;
    float* s_rows = smem + L.rows;
    double* s_red = (double*)(smem + L.red);
    int* s_prange = (int*)(smem + L.prange);
    float* s_fin = smem + L.fin;                    // [2][gsub][4][band_w] (luminosity-weighted mode)
    const int XW = a.xw;
    const int D = a.D;

    // --- parameters of this theta (FP64 -> FP32 constants, wave-uniform)
    const TC tc = uniform_tc(make_tc(a.theta + (size_t)b * a.stride, G));
    if (!tc.valid) {
        if (MODE == MODE_MAPS) {
            const float qnan = __int_as_float(0x7fc00000);
            for (int p = tid; p < 4 * NR * NC; p += BS) {
                const int m = p / (NR * NC), rem = p - m * NR * NC, jj = rem / NC, c = rem - jj * NC;
                a.maps[(size_t)b * 4 * G.ny * G.nx + ((size_t)m * G.ny + j0 + jj) * G.nx + c0 + c] = qnan;
            }
        } else if (band == 0 && tid == 0) {
            a.logL[b] = -INFINITY;
        }
        return;
    }

    // --- prologue: tables (TAB_LDS), zeroed row buffer, row spans
    if constexpr (TAB_LDS) {
        const Tabs C = const_tabs<BULGE>();
        const float* tgh = (const float*)C.gh;
        for (int i = tid; i < TAB_GH; i += BS) s_tab[i] = tgh[i];
        for (int i = tid; i < TAB_PHI; i += BS) s_tab[TAB_GH + i] = gk_tab_phi[i];
        for (int i = tid; i < TAB_M; i += BS) s_tab[TAB_GH + TAB_PHI + i] = gk_tab_m[i];
    }
    for (int i = tid; i < RS * 4 * XW; i += BS) s_rows[i] = 0.0f;
    // row spans of the band and stencil half-widths, staged for the span pass
    int2* s_span = (int2*)(smem + L.stage);
    int* s_aof = (int*)(s_span + a.band_h);
    for (int i = tid; i < NR; i += BS) s_span[i] = MODE != MODE_MAPS ? a.span[j0 + i] : make_int2(c0, c1 - 1);
    for (int i = tid; i <= pad; i += BS) s_aof[i] = a.aof[i];
    __syncthreads();
    // one column range per model phase: the union, over its lattice rows, of
    // the stencils of the band's valid pixels (about 3 % more points than row
    // by row, and no per-point row search); local columns < 2^15 (band_w <=
    // 128, s <= 15, pad <= 25), so first column and width pack in one int
    const int RSs = a.gsub * s;
    const int nph = (NFR + RSs - 1) / RSs;
    for (int k = tid; k < nph; k += BS) {
        int lo = 1 << 30, hi = -(1 << 30);
        for (int r = k * RSs; r < min(NFR, (k + 1) * RSs); ++r) {
            const int jlo = r >= 2 * pad ? (r - 2 * pad + s - 1) / s : 0;   // ceil((r - 2 pad) / s)
            const int jhi = min(NR - 1, r / s);
            for (int jj = jlo; jj <= jhi; ++jj) {
                int bb = r - jj * s - pad;
                bb = bb < 0 ? -bb : bb;
                const int2 sp = s_span[jj];
                const int cl = max(c0, sp.x), ch = min(c1 - 1, sp.y);
                if (cl <= ch) {
                    const int A = s_aof[bb];
                    lo = min(lo, (cl - c0) * s + pad - A);
                    hi = max(hi, (ch - c0) * s + pad + A);
                }
            }
        }
        s_prange[k] = hi >= lo ? lo | ((hi - lo + 1) << 16) : 0;
    }
    __syncthreads();

    const Tabs T = TAB_LDS ? Tabs{(const float4*)s_tab, (const float4*)(s_tab + TAB_GH),
                                  (const float4*)(s_tab + TAB_GH + TAB_PHI)}
                           : const_tabs<BULGE>();
    const float invW = a.invW;
    double chi2 = 0.0;
    const size_t mapoff = (size_t)b * 4 * G.ny * G.nx;
    // one (map, pixel column) pair per thread: blockDim >= 4 * band_w; the
    // threads beyond 4 NC run the same code on a clamped pair and store nothing,
    // which keeps the stencil phase free of divergent control flow
    const bool pact = tid < 4 * NC;
    const int tcl = pact ? tid : 4 * NC - 1;
    const int pm = tcl / NC, pc = tcl - (tcl / NC) * NC;
    float acc[DMAX + 1];
#pragma unroll
    for (int d = 0; d <= DMAX; ++d) acc[d] = 0.0f;
    const int Q = NR + D;                           // pixel-row steps

    for (int q0 = 0; q0 < Q; q0 += a.gsub) {
        // ---- lattice rows [rA, rA + nrow) of this phase, columns [plo, plo + pw)
        const int rA = q0 * s;
        const int nrow = max(0, min(RS, NFR - rA));
        const int ph = q0 / a.gsub;
        const int prange = uni(s_prange[ph]);
        const int plo = prange & 0xffff, pw = prange >> 16;
        const int npts = nrow * pw;
        const float inv_pw = 1.0f / (float)max(pw, 1);
        // ---- data of the pixel rows completed in this phase (prefetched)
        float pv[GSUB_CAP], pi[GSUB_CAP];
        if (MODE != MODE_MAPS) {
#pragma unroll
            for (int k = 0; k < GSUB_CAP; ++k) {
                if (k >= a.gsub) break;
                const int jj = q0 + k - D;
                const bool ok = jj >= 0 && jj < NR;
                const size_t pix = ((size_t)pm * G.ny + j0 + (ok ? jj : 0)) * G.nx + c0 + pc;
                const float vv = a.val[pix], ii = a.ivar[pix];
                pv[k] = vv;
                pi[k] = (ok && pact) ? ii : 0.0f;
            }
        }
        // ---- model phase: the phase's lattice points, flat over its rows
        for (int q = tid; q < npts; q += BS) {
            const int lr = (int)(((float)q + 0.5f) * inv_pw);
            const int r = rA + lr;
            const int x = plo + (q - lr * pw);                   // local column
            const int u = ubase + x;
            const int v = vlo + r;
            const float du = (float)(u - tc.Ui) - tc.Uf;
            const float dv = (float)(v - tc.Vi) - tc.Vf;
            float* row = s_rows + lr * 4 * XW + x;
            if (BO) {
                row[0] = point_model_b<BULGE, NDISC>(tc, T, du, dv);
                continue;
            }
            float fB, fV, fS, fL;
            point_model<BULGE, NDISC, HALO>(tc, T, du, dv, fB, fV, fS, fL);
            if (LW) {         // light, first and second velocity moments, mass
                row[0] = fB;
                row[XW] = fB * fV;
                row[2 * XW] = fB * fmaf(fS, fS, fV * fV);
                row[3 * XW] = fB * frcp(fL);
            } else {
                row[0] = fB;
                row[XW] = fV;
                row[2 * XW] = fS;
                row[3 * XW] = fL;
            }
        }
        __syncthreads();
        // ---- stencil phase: per (map, column) pair, in registers
        {
#pragma unroll
            for (int k = 0; k < GSUB_CAP; ++k) {
                if (k >= a.gsub) break;
                const int q = q0 + k;
                if (q >= Q) break;
                const float* L0 = s_rows + (k * s) * 4 * XW + pm * XW + pc * s + pad;
#define GK_SUB(PADV) stencil_sub<PADV, lag_cap(PADV)>(L0, 4 * XW, s, a.gw, a.tab, acc)
                if ((a.map_mask >> pm) & 1) {       // maps without valid pixels stay zero
                    switch (a.tpad) {
                        case 4: GK_SUB(4); break;
                        case 6: GK_SUB(6); break;
                        case 9: GK_SUB(9); break;
                        case 12: GK_SUB(12); break;
                        case 16: GK_SUB(16); break;
                        case 20: GK_SUB(20); break;
                        default: GK_SUB(25); break;
                    }
                }
#undef GK_SUB
                const int jj = q - D;                   // pixel row completed by this step
                if (jj >= 0 && LW) {
                    if (pact) s_fin[(k * 4 + pm) * a.band_w + pc] = acc[D] * invW;
                } else if (jj >= 0) {
                    const float F = acc[D] * invW;
                    const size_t pix = ((size_t)pm * G.ny + j0 + jj) * G.nx + c0 + pc;
                    if (MODE == MODE_MAPS) {
                        if (pact) a.maps[mapoff + pix] = (pm == 3) ? 1.0f / F : F;
                    } else {
                        const float iv = pi[k];
                        float gbar = 0.0f;
                        if (iv > 0.0f) {
                            const float Fm = (pm == 3) ? 1.0f / F : F;
                            const float res = Fm - pv[k];
                            chi2 += (double)res * (double)res * (double)iv;
                            // d logL / dF: -iv res, and for M/L = 1/F: +iv res / F^2
                            gbar = (pm == 3) ? iv * res * Fm * Fm : -iv * res;
                        }
                        if (MODE == MODE_FBAR && pact) a.fbar[mapoff + pix] = gbar;
                    }
                }
            }
        }
        if (LW) {
            // luminosity-weighted moments: every pixel's four PSF moments are in
            // s_fin; each (map, column) thread forms its own observable from them
            __syncthreads();
#pragma unroll
            for (int k = 0; k < GSUB_CAP; ++k) {
                if (k >= a.gsub) break;
                const int jj = q0 + k - D;
                if (jj < 0 || q0 + k >= Q) continue;
                const float* fk = s_fin + k * 4 * a.band_w + pc;
                const float F0 = fk[0], F1 = fk[a.band_w], F2 = fk[2 * a.band_w], F3 = fk[3 * a.band_w];
                const float i0 = frcp(F0);
                const float v = F1 * i0;
                const float s2 = fmaf(F2, i0, -v * v);
                const float sg = s2 > 0.0f ? fsqrt(s2) : 0.0f;
                const float obs = pm == 0 ? F0 : pm == 1 ? v : pm == 2 ? sg : F3 * i0;   // B, v, sigma, M/L
                const size_t pix = ((size_t)pm * G.ny + j0 + jj) * G.nx + c0 + pc;
                if (MODE == MODE_MAPS) {
                    if (pact) a.maps[mapoff + pix] = obs;
                } else {
                    const float iv = pi[k];
                    float ob = 0.0f;                    // d logL / d observable
                    if (iv > 0.0f) {
                        const float res = obs - pv[k];
                        chi2 += (double)res * (double)res * (double)iv;
                        ob = -iv * res;
                    }
                    // the clamped threads share an active thread's slot: only the owner writes
                    if (MODE == MODE_FBAR && pact) s_fin[(4 * a.gsub + k * 4 + pm) * a.band_w + pc] = ob;
                }
            }
            if (MODE == MODE_FBAR) {
                // d logL / d F_m through v = F1/F0, sigma = sqrt(F2/F0 - v^2), M/L = F3/F0
                __syncthreads();
#pragma unroll
                for (int k = 0; k < GSUB_CAP; ++k) {
                    if (k >= a.gsub) break;
                    const int jj = q0 + k - D;
                    if (jj < 0 || q0 + k >= Q) continue;
                    const float* fk = s_fin + k * 4 * a.band_w + pc;
                    const float* ok_ = s_fin + (4 * a.gsub + k * 4) * a.band_w + pc;
                    const float F0 = fk[0], F1 = fk[a.band_w], F2 = fk[2 * a.band_w], F3 = fk[3 * a.band_w];
                    const float o0 = ok_[0], o1 = ok_[a.band_w], o2 = ok_[2 * a.band_w], o3 = ok_[3 * a.band_w];
                    const float i0 = frcp(F0);
                    const float v = F1 * i0;
                    const float s2 = fmaf(F2, i0, -v * v);
                    const float sg = s2 > 0.0f ? fsqrt(s2) : 0.0f;
                    const float hs2 = sg > 0.0f ? 0.5f * frcp(sg) : 0.0f;          // d sigma / d s2
                    // s2 = F2/F0 - F1^2/F0^2
                    const float ds2_0 = (-F2 + 2.0f * F1 * v) * i0 * i0;
                    const float ds2_1 = -2.0f * v * i0;
                    const float ds2_2 = i0;
                    float gbar;
                    if (pm == 0)
                        gbar = o0 - o1 * v * i0 + o2 * hs2 * ds2_0 - o3 * F3 * i0 * i0;
                    else if (pm == 1)
                        gbar = o1 * i0 + o2 * hs2 * ds2_1;
                    else if (pm == 2)
                        gbar = o2 * hs2 * ds2_2;
                    else
                        gbar = o3 * i0;
                    // a pixel with no valid map (outside every map's column span the
                    // lattice is not evaluated, F0 may be 0) has a zero adjoint
                    const bool used = (o0 != 0.0f) | (o1 != 0.0f) | (o2 != 0.0f) | (o3 != 0.0f);
                    gbar = used ? gbar : 0.0f;
                    const size_t pix = ((size_t)pm * G.ny + j0 + jj) * G.nx + c0 + pc;
                    if (pact) a.fbar[mapoff + pix] = gbar;
                }
            }
        }
        __syncthreads();
    }

    if (MODE == MODE_MAPS) return;
    // ---- FP64 chi^2: wave sums, then waves in order, then bands in order
    chi2 = wave_sum(chi2);
    const int lane = tid & 63, wave = tid >> 6;
    if (lane == 0) s_red[wave] = chi2;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < (BS + 63) / 64; ++w) t += s_red[w];
        if (a.nbands == 1) {
            const double v = -0.5 * (t + *a.logdet);
            a.logL[b] = a.accum ? a.logL[b] + v : v;
        } else {
            a.partials[(size_t)b * a.pstride + band] = t;
            const unsigned ticket = __hip_atomic_fetch_add(a.counters + b, 1u, __ATOMIC_ACQ_REL,
                                                           __HIP_MEMORY_SCOPE_AGENT);
            if (ticket == (unsigned)a.nbands - 1) {
                double sum = 0.0;
                for (int k = 0; k < a.nbands; ++k)
                    sum += __hip_atomic_load(a.partials + (size_t)b * a.pstride + k, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
                const double v = -0.5 * (sum + *a.logdet);
                a.logL[b] = a.accum ? a.logL[b] + v : v;
                __hip_atomic_store(a.counters + b, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

// The map-averaging seed pass is held to 128 VGPRs (four waves per SIMD, as
// the other map-averaging bodies; it needs 129 unconstrained, and spills
// nothing at 128).
template <int BULGE, int NDISC, int HALO, int MODE, int LW, int BO = 0>
__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(MODE == MODE_FBAR && !LW ? 4 : 1)))
fwd_kernel(FwdArgs a) {
    extern __shared__ __align__(16) float smem[];
    fwd_band<BULGE, NDISC, HALO, MODE, LW, BO, MODE == MODE_FBAR && LW>(a, blockIdx.x / a.nbands,
                                                                         blockIdx.x % a.nbands, smem);
}

}  // namespace gk
