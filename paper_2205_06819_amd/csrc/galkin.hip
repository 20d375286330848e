// galkin: HIP implementation (gfx950) of the batched disc-galaxy likelihood.
//
// One workgroup evaluates one parameter vector (theta) on one rectangular
// band of pixels.  It streams the band's padded fine lattice row by row:
//
//   model phase   every thread evaluates lattice points of the next chunk
//                 (paper Sec. 2.1-2.4) into an LDS ring buffer;
//   stencil phase each (pixel column, map) pair forms the horizontal partial
//                 sums of the circular Gaussian stencil (Sec. 3.1, PSF
//                 equation) along each completed lattice row and pushes them,
//                 weighted by the vertical Gaussian factor, into LDS
//                 accumulators of the pixel rows that row reaches;
//   finalize      when the last lattice row of a pixel row is in, that row's
//                 PSF averages are complete: residuals against the data and
//                 the FP64 chi^2 (Sec. 2.5.1, likelihood equation).
//
// Only lattice points inside the union of the stencils of valid pixels are
// evaluated.  Per-band FP64 partial chi^2 are combined in band order by the
// last workgroup of each theta (deterministic, graph-capturable).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "galkin.h"
#include "gk_device.h"

namespace gk {

enum { MODE_LOGL = 0, MODE_FBAR = 1, MODE_MAPS = 2 };
constexpr int MAX_BANDS = 1024;       // per theta
constexpr int RED_SLOTS = 16;         // waves per workgroup (<= 1024 threads)

struct FwdArgs {
    GridGeom geo;
    const float* gw;        // [64] 1-D Gaussian factors exp(-a^2 / 2 (sigma s)^2), zero beyond pad
    const int* aof;         // [pad + 1] half-width A(|b|) of the stencil at row offset b
    const int2* tab;        // [s][DSTRIDE] (A(|b|), weight bits g(|b|)) for lattice-row phase ph and
                            // pixel-row lag d, b = d s + ph - pad; (0, 0) where |b| > pad
    float invW;             // 1 / sum of the 2-D stencil weights
    int D;                  // floor(2 pad / s): lag at which a pixel row is complete
    const float* val;       // data [4][ny][nx]
    const float* ivar;      // inverse variances [4][ny][nx], 0 = masked
    const int2* span;       // [ny] first / last column valid in any map
    const double* logdet;   // sum of ln(2 pi e^2) over valid pixels (device scalar)
    int band_h, band_w, nbx, nbands;
    int pstride;            // row stride of partials (>= nbands)
    int gsub;               // pixel-row steps per model phase (gsub * s <= RS_CAP lattice rows)
    int xw;                 // row stride of the row buffer (floats)
    int tpad;               // compile-time tap count used by the stencil (>= pad)
    const double* theta;
    int stride;
    double* logL;
    float* maps;            // MODE_MAPS output [B][4][ny][nx]
    float* fbar;            // MODE_FBAR output [B][4][ny][nx]: d logL / d F
    double* partials;       // [B][pstride]
    unsigned* counters;     // [B]
    int accum;              // 1: add the log-likelihood to logL[b] instead of storing it
    int map_mask;           // bit m set: map m is convolved (maps with no valid pixel are skipped)
};

constexpr int DMAX = 10;        // largest lag D = floor(2 pad / s) supported
constexpr int DSTRIDE = DMAX + 1;
constexpr int RS_CAP = 16;      // lattice rows per model phase
constexpr int GSUB_CAP = 4;     // pixel-row steps per model phase

struct Layout {                 // LDS carve-up, identical on host and device
    int tab, rows, red, rows_lo, rows_start, stage, fin, total_bytes;
};

__host__ __device__ inline int nfr_max(int band_h, int s, int pad) { return (band_h - 1) * s + 2 * pad + 1; }

// nfin: floats of the per-step exchange buffer of the luminosity-weighted
// mode (0 otherwise)
__host__ __device__ inline Layout make_layout(int rows, int xw, int nfrm, int band_h, int nfin) {
    Layout L;
    int off = 0;                                   // in 4-byte words
    L.rows = off;       off += rows * 4 * xw;
    off = (off + 3) & ~3;
    L.red = off;        off += 2 * RED_SLOTS;      // doubles
    L.rows_lo = off;    off += nfrm;
    L.rows_start = off; off += nfrm + 1 + RS_CAP;  // padded: phase lookups read ahead
    off = (off + 1) & ~1;
    L.stage = off;      off += 2 * band_h + 32;    // row spans and stencil half-widths
    L.fin = off;        off += nfin;
    // the tables last, at a launch-dependent offset: a table lookup is then one
    // base add and four reads with immediate offsets
    off = (off + 3) & ~3;
    L.tab = off;        off += TAB_ALL;
    L.total_bytes = 4 * off;
    return L;
}

// Block-wide exclusive scan of n ints in place (n small); returns the total.
__device__ inline int block_exclusive_scan(int* a, int n, int* scratch /*RED_SLOTS ints*/) {
    const int tid = threadIdx.x, BS = blockDim.x;
    const int per = (n + BS - 1) / BS;
    const int lo = min(n, tid * per), hi = min(n, lo + per);
    int sum = 0;
    for (int i = lo; i < hi; ++i) sum += a[i];
    const int lane = tid & 63, wave = tid >> 6;
    int x = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) scratch[wave] = x;
    __syncthreads();
    int wbase = 0;
    const int nw = (BS + 63) >> 6;
    for (int w = 0; w < wave; ++w) wbase += scratch[w];
    int total = 0;
    for (int w = 0; w < nw; ++w) total += scratch[w];
    int run = wbase + x - sum;                      // exclusive prefix of this thread
    for (int i = lo; i < hi; ++i) {
        const int v = a[i];
        a[i] = run;
        run += v;
    }
    __syncthreads();
    return total;
}

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
// shifted by one each step, so acc[D] is complete after this call.
template <int PAD>
__device__ __forceinline__ void stencil_sub(const float* __restrict__ L0, int rstride, int s,
                                            const float* __restrict__ gw, const int2* __restrict__ tab,
                                            float (&acc)[DMAX + 1]) {
    float g[PAD + 1];
#pragma unroll
    for (int k = 0; k <= PAD; ++k) g[k] = gw[k];
    float con[DMAX + 1];
#pragma unroll
    for (int d = 0; d <= DMAX; ++d) con[d] = 0.0f;
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
        for (int d = 0; d <= DMAX; ++d) {
            const int A = t[2 * d];
            const float w = __int_as_float(t[2 * d + 1]);
            con[d] = fmaf(w, H[A], con[d]);
        }
    }
#pragma unroll
    for (int d = DMAX; d >= 1; --d) acc[d] = acc[d - 1] + con[d];
    acc[0] = con[0];
}

// One parameter vector (row b) on one band of one grid.  load_tables = false
// when the caller already staged the special-function tables in LDS.  LW = 1:
// the PSF averages luminosity-weighted moments (a compile-time switch, so the
// map-averaging instantiations do not carry its registers).
template <int BULGE, int NDISC, int HALO, int MODE, int LW>
__device__ __forceinline__ void fwd_band(const FwdArgs& a, const int b, const int band, float* smem,
                                         const bool load_tables) {
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
    const Layout L = make_layout(RS, a.xw, nfrm, a.band_h, LW ? 8 * a.gsub * a.band_w : 0);
    float* s_tab = smem + L.tab;
    float* s_rows = smem + L.rows;
    double* s_red = (double*)(smem + L.red);
    int* s_lo = (int*)(smem + L.rows_lo);
    int* s_start = (int*)(smem + L.rows_start);
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

    // --- prologue: tables, zeroed row buffer, row spans
    if (load_tables) {
        const float* tgh = BULGE == 2 ? gk_tab_jgh : gk_tab_gh;     // one bulge kind per grid
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
    for (int r = tid; r < NFR; r += BS) {
        const int jlo = r >= 2 * pad ? (r - 2 * pad + s - 1) / s : 0;   // ceil((r - 2 pad) / s)
        const int jhi = min(NR - 1, r / s);
        int lo = 1 << 30, hi = -(1 << 30);
        for (int jj = jlo; jj <= jhi; ++jj) {
            int bb = r - jj * s - pad;
            bb = bb < 0 ? -bb : bb;
            const int2 sp = s_span[jj];
            const int cl = max(c0, sp.x), ch = min(c1 - 1, sp.y);
            if (cl <= ch) {
                const int A = s_aof[bb];
                lo = min(lo, cl * s + hs + pad - A);
                hi = max(hi, ch * s + hs + pad + A);
            }
        }
        s_lo[r] = hi >= lo ? lo - ubase : (1 << 30);  // local needed columns of lattice row r
        s_start[r] = hi >= lo ? hi - ubase : -(1 << 30);
    }
    __syncthreads();
    // one column range per model phase: the union of its lattice rows' ranges
    // (about 3 % more points than row by row, and no per-point row search)
    const int RSs = a.gsub * s;
    const int nph = (NFR + RSs - 1) / RSs;
    int* s_plo = (int*)(smem + L.stage);                // reuses the staging area
    int* s_pw = s_plo + nph;
    __syncthreads();
    for (int k = tid; k < nph; k += BS) {
        int lo = 1 << 30, hi = -(1 << 30);
        for (int r = k * RSs; r < min(NFR, (k + 1) * RSs); ++r) {
            lo = min(lo, s_lo[r]);
            hi = max(hi, s_start[r]);
        }
        s_plo[k] = hi >= lo ? lo : 0;
        s_pw[k] = hi >= lo ? hi - lo + 1 : 0;
    }
    __syncthreads();

    const Tabs T{(const float4*)s_tab, (const float4*)(s_tab + TAB_GH),
                 (const float4*)(s_tab + TAB_GH + TAB_PHI)};
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
        const int plo = uni(s_plo[ph]), pw = uni(s_pw[ph]);
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
            float fB, fV, fS, fL;
            point_model<BULGE, NDISC, HALO>(tc, T, du, dv, fB, fV, fS, fL);
            float* row = s_rows + lr * 4 * XW + x;
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
#define GK_SUB(PADV) stencil_sub<PADV>(L0, 4 * XW, s, a.gw, a.tab, acc)
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

template <int BULGE, int NDISC, int HALO, int MODE, int LW>
__global__ void __launch_bounds__(512) fwd_kernel(FwdArgs a) {
    extern __shared__ __align__(16) float smem[];
    fwd_band<BULGE, NDISC, HALO, MODE, LW>(a, blockIdx.x / a.nbands, blockIdx.x % a.nbands, smem, true);
}

// ============================================================================
// many grids in one launch: workgroup i takes work item i (grid, parameter row
// within the grid, band, first row of the grid in the batch); the host orders
// the items by decreasing cost, so the dispatcher hands out the longest items
// first and the short ones fill the tail.  (A persistent loop over an atomic
// queue kept loop-invariant state live across items: 206 instead of 125 VGPRs,
// half the occupancy, and slower overall.)
// ============================================================================
typedef const __attribute__((address_space(4))) int* const_word_ptr;

constexpr int MULTI_BS = 256;   // threads per workgroup of the many-grid launch

template <int LW>
__global__ void __launch_bounds__(MULTI_BS) multi_kernel(const FwdArgs* __restrict__ grids,
                                                         const int4* __restrict__ items,
                                                         const double* theta, int stride, double* logL) {
    extern __shared__ __align__(16) float smem[];
    const_word_ptr iw = (const_word_ptr)(items) + 4 * blockIdx.x;
    const int g = iw[0], row = iw[1], band = iw[2], off = iw[3];
    FwdArgs a = grids[g];
    a.theta = theta + (size_t)off * stride;   // this grid's rows start at row off
    a.stride = stride;
    a.logL = logL + off;
    const int comp = a.geo.bulge * 100 + a.geo.ndisc * 10 + a.geo.halo;
    switch (comp) {
#define GK_MCASE(BU, ND, HA)                                                                   \
    case BU * 100 + ND * 10 + HA:                                                              \
        fwd_band<BU, ND, HA, MODE_LOGL, LW>(a, row, band, smem, true);                          \
        break;
        GK_MCASE(1, 0, 0) GK_MCASE(1, 0, 1) GK_MCASE(1, 0, 2)
        GK_MCASE(1, 1, 0) GK_MCASE(1, 1, 1) GK_MCASE(1, 1, 2)
        GK_MCASE(1, 2, 0) GK_MCASE(1, 2, 1) GK_MCASE(1, 2, 2)
        GK_MCASE(2, 0, 0) GK_MCASE(2, 0, 1) GK_MCASE(2, 0, 2)
        GK_MCASE(2, 1, 0) GK_MCASE(2, 1, 1) GK_MCASE(2, 1, 2)
        GK_MCASE(2, 2, 0) GK_MCASE(2, 2, 1) GK_MCASE(2, 2, 2)
        GK_MCASE(0, 1, 0) GK_MCASE(0, 1, 1) GK_MCASE(0, 1, 2)
        GK_MCASE(0, 2, 0) GK_MCASE(0, 2, 1) GK_MCASE(0, 2, 2)
#undef GK_MCASE
        default: break;
    }
}

// ============================================================================
// adjoint: d logL / d theta
// ============================================================================
constexpr int MAX_BANDS_ADJ = 64;

struct AdjArgs {
    GridGeom geo;
    const float* gw;        // [64] 1-D Gaussian factors
    const int* aof;         // [pad + 1] stencil half-widths
    float invW;
    int D;                  // pixel-row lags of the stencil, floor(2 pad / s)
    const int2* span;       // [ny] valid column spans
    int band_h, band_w, nbx, nbands;
    const double* theta;
    int stride;
    const float* fbar;      // [B][4][ny][nx] d logL / d F from the forward pass
    double* gpart;          // [B][nbands][NCONST] per-band constant adjoints
    unsigned* counters;     // [B], zero on entry, reset by the last band
    double* grad;           // [B][stride]
    int accum;              // 1: add the gradient to grad[b] instead of storing it
};

__host__ __device__ inline int adj_lds_bytes(int band_h, int band_w, int s, int pad) {
    const int nfrm = nfr_max(band_h, s, pad);
    return 4 * (TAB_ALL + 4 * band_h * band_w + 64 + 2 * nfrm + 1 + RED_SLOTS * 2 * NCONST + 64 + 2 * band_h +
                32);
}

__device__ inline int floor_div(int n, int d) { return n >= 0 ? n / d : -((-n + d - 1) / d); }

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

template <int BULGE, int NDISC, int HALO>
__global__ void __launch_bounds__(256) adj_kernel(AdjArgs a) {
    extern __shared__ __align__(16) float smem[];
    const int tid = threadIdx.x, BS = blockDim.x;
    const int band = blockIdx.x % a.nbands;
    const int b = blockIdx.x / a.nbands;
    const GridGeom& G = a.geo;
    const int s = G.s, pad = G.pad, hs = G.hs;
    const int by = band / a.nbx, bx = band - by * a.nbx;
    const int j0 = by * a.band_h, j1 = min(G.ny, j0 + a.band_h);
    const int c0 = bx * a.band_w, c1 = min(G.nx, c0 + a.band_w);
    const int NR = j1 - j0, NC = c1 - c0;
    const int NFR = (NR - 1) * s + 2 * pad + 1;
    const int vlo = j0 * s + hs, ubase = c0 * s + hs;
    const int nfrm = nfr_max(a.band_h, s, pad);
    float* s_tab = smem;
    float4* s_fb = (float4*)(smem + TAB_ALL);                    // [NR][NC]
    float* s_gw = smem + TAB_ALL + 4 * a.band_h * a.band_w;       // [64]
    int* s_lo = (int*)(s_gw + 64);
    int* s_start = s_lo + nfrm;                                    // [nfrm + 1]
    double* s_red = (double*)(((uintptr_t)(s_start + nfrm + 1) + 15) & ~(uintptr_t)15);
    int2* s_span = (int2*)(s_red + RED_SLOTS * NCONST);           // [band_h] row spans
    int* s_aof = (int*)(s_span + a.band_h);                        // [pad + 1] half-widths

    const double* th = a.theta + (size_t)b * a.stride;
    const TC tc = uniform_tc(make_tc(th, G));
    if (!tc.valid) {
        if (band == 0 && !a.accum)
            for (int q = tid; q < a.stride; q += BS) a.grad[(size_t)b * a.stride + q] = 0.0;
        return;
    }
    const float* tgh = BULGE == 2 ? gk_tab_jgh : gk_tab_gh;
    for (int i = tid; i < TAB_GH; i += BS) s_tab[i] = tgh[i];
    for (int i = tid; i < TAB_PHI; i += BS) s_tab[TAB_GH + i] = gk_tab_phi[i];
    for (int i = tid; i < TAB_M; i += BS) s_tab[TAB_GH + TAB_PHI + i] = gk_tab_m[i];
    for (int i = tid; i < 64; i += BS) s_gw[i] = a.gw[i];
    for (int i = tid; i < NR; i += BS) s_span[i] = a.span[j0 + i];
    for (int i = tid; i <= pad; i += BS) s_aof[i] = a.aof[i];
    const size_t boff = (size_t)b * 4 * G.ny * G.nx, mstr = (size_t)G.ny * G.nx;
    for (int p = tid; p < NR * NC; p += BS) {
        const int jj = p / NC, cc = p - jj * NC;
        const size_t pix = boff + (size_t)(j0 + jj) * G.nx + c0 + cc;
        s_fb[p] = make_float4(a.fbar[pix], a.fbar[pix + mstr], a.fbar[pix + 2 * mstr], a.fbar[pix + 3 * mstr]);
    }
    __syncthreads();
    for (int r = tid; r < NFR; r += BS) {
        const int jlo = r >= 2 * pad ? (r - 2 * pad + s - 1) / s : 0;
        const int jhi = min(NR - 1, r / s);
        int lo = 1 << 30, hi = -(1 << 30);
        for (int jj = jlo; jj <= jhi; ++jj) {
            int bb = r - jj * s - pad;
            bb = bb < 0 ? -bb : bb;
            const int2 sp = s_span[jj];
            const int cl = max(c0, sp.x), ch = min(c1 - 1, sp.y);
            if (cl <= ch) {
                const int A = s_aof[bb];
                lo = min(lo, cl * s + hs + pad - A);
                hi = max(hi, ch * s + hs + pad + A);
            }
        }
        const int w = hi >= lo ? hi - lo + 1 : 0;
        s_lo[r] = w ? lo - ubase : 0;
        s_start[r] = w;
    }
    __syncthreads();
    const int total = block_exclusive_scan(s_start, NFR, (int*)s_red);
    if (tid == 0) s_start[NFR] = total;
    __syncthreads();

    const Tabs T{(const float4*)s_tab, (const float4*)(s_tab + TAB_GH),
                 (const float4*)(s_tab + TAB_GH + TAB_PHI)};
    float ad[NCONST];
#pragma unroll
    for (int k = 0; k < NCONST; ++k) ad[k] = 0.0f;
    const float invW = a.invW;
    const float inv_s = 1.0f / (float)s;
    const int D = a.D;
    int rcur = 0;
    for (int q = tid; q < total; q += BS) {
        while (s_start[rcur + 1] <= q) ++rcur;
        const int r = rcur;
        const int x = s_lo[r] + (q - s_start[r]);
        // transposed stencil: this lattice point's share of every band pixel
        // whose 3 sigma disc contains it, weighted by that pixel's adjoint
        float4 f = make_float4(0.f, 0.f, 0.f, 0.f);
        // pixel rows jj = jq - d and columns cc = cq - k around the point; the
        // divisions by s go through a float reciprocal (exact for these sizes)
        const int jq = (int)(((float)r + 0.5f) * inv_s), rr = r - jq * s - pad;
        const int cq = (int)(((float)x + 0.5f) * inv_s), rx = x - cq * s - pad;
        const int jlo = max(0, jq - D), jhi = min(NR - 1, jq);
        for (int jj = jlo; jj <= jhi; ++jj) {
            int bb = rr + (jq - jj) * s;
            bb = bb < 0 ? -bb : bb;
            if (bb > pad) continue;
            const int A = s_aof[bb];
            const float gb = s_gw[bb];
            // columns with |x - cc s - pad| <= A: k = cq - cc in [(pad - A - rx') / s, (pad + A - rx') / s]
            const int klo = max(0, (int)floorf((float)(-A - rx + s - 1) * inv_s + 1e-4f));
            const int khi = min(D, (int)floorf((float)(A - rx) * inv_s + 1e-4f));
            const int ccl = max(0, cq - khi), cch = min(NC - 1, cq - klo);
            const float4* fbr = s_fb + jj * NC;
            int cc = ccl;
            int t0 = x - cc * s - pad;
            for (; cc < cch; cc += 2, t0 -= 2 * s) {
                // two taps per trip: both pairs of LDS reads are in flight together
                const int a0 = t0 < 0 ? -t0 : t0;
                const int t1 = t0 - s, a1 = t1 < 0 ? -t1 : t1;
                const float g0 = s_gw[a0], g1 = s_gw[a1];
                const float4 b0 = fbr[cc], b1 = fbr[cc + 1];
                const float w0 = gb * g0, w1 = gb * g1;
                f.x = fmaf(w1, b1.x, fmaf(w0, b0.x, f.x));
                f.y = fmaf(w1, b1.y, fmaf(w0, b0.y, f.y));
                f.z = fmaf(w1, b1.z, fmaf(w0, b0.z, f.z));
                f.w = fmaf(w1, b1.w, fmaf(w0, b0.w, f.w));
            }
            if (cc == cch) {
                const int a0 = t0 < 0 ? -t0 : t0;
                const float w = gb * s_gw[a0];
                const float4 fb = fbr[cc];
                f.x = fmaf(w, fb.x, f.x);
                f.y = fmaf(w, fb.y, f.y);
                f.z = fmaf(w, fb.z, f.z);
                f.w = fmaf(w, fb.w, f.w);
            }
        }
        const float du = (float)(ubase + x - tc.Ui) - tc.Uf;
        const float dv = (float)(vlo + r - tc.Vi) - tc.Vf;
        float4 fo = make_float4(f.x * invW, f.y * invW, f.z * invW, f.w * invW);
        if (G.lw) {
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

// ============================================================================
// HMC leapfrog update (elementwise over the batch)
// ============================================================================
// stage 0: p += h g (half kick), then theta += eps M^-1 p (drift)
// stage 1: p += eps g, then drift
// stage 2: p += h g (closing half kick), no drift
// Rows whose log-likelihood is not finite are frozen (no update).
__global__ void __launch_bounds__(256) leapfrog_kernel(double* theta, double* mom, const double* grad,
                                                       const double* logL, const double* inv_mass,
                                                       double eps, int stage, int B, int P, int stride) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * P) return;
    const int b = i / P, k = i - b * P;
    const double L = logL[b];
    if (!(L > -INFINITY && L < INFINITY)) return;
    const size_t o = (size_t)b * stride + k;
    const double kick = (stage == 1) ? eps : 0.5 * eps;
    double p = mom[o] + kick * grad[o];
    mom[o] = p;
    if (stage != 2) theta[o] += eps * inv_mass[k] * p;
}

}  // namespace gk

// ============================================================================
// host side
// ============================================================================
using namespace gk;

static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHECK(call)                                                                  \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) return fail(GK_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

struct LaunchRule {
    int batch_min, band_h, band_w, steps;   // steps: pixel rows per model phase, 0 = automatic
};

struct gk_grid {
    gk_grid_desc d;
    GridGeom geo;
    int P = 0, K = 0, D = 0, max_batch = 0, device = 0, tpad = 0;
    float invW = 1.f;
    double logdet = 0.0;
    bool has_data = false;
    int map_mask = 15;      // maps with at least one valid pixel (all four in the moment mode)
    // device buffers
    float* d_gw = nullptr;
    int* d_aof = nullptr;
    int2* d_tab = nullptr;
    float* d_val = nullptr;
    float* d_ivar = nullptr;
    int2* d_span = nullptr;
    double* d_partials = nullptr;
    unsigned* d_counters = nullptr;
    float* d_fbar = nullptr;
    double* d_gpart = nullptr;
    double* d_logdet = nullptr;
    std::vector<LaunchRule> rules;
    int adj_band_h = 0, adj_band_w = 0;
};

static int valid_desc(const gk_grid_desc* d) {
    if (!d) return fail(GK_EINVAL, "desc is NULL");
    if (d->nx < 1 || d->ny < 1 || d->nx > 4096 || d->ny > 4096)
        return fail(GK_EINVAL, "nx, ny must be in [1, 4096] (got %d, %d)", d->nx, d->ny);
    if (!(d->pixel_kpc > 0.0) || !std::isfinite(d->pixel_kpc))
        return fail(GK_EINVAL, "pixel_kpc must be finite and > 0");
    if (d->supersample < 1 || d->supersample > 15 || d->supersample % 2 == 0)
        return fail(GK_EINVAL, "supersample must be odd and in [1, 15] (got %d)", d->supersample);
    if (!(d->psf_sigma_px >= 0.0) || d->psf_sigma_px > 64.0)
        return fail(GK_EINVAL, "psf_sigma_px must be in [0, 64]");
    if (d->bulge != GK_BULGE_NONE && d->bulge != GK_BULGE_HERNQUIST && d->bulge != GK_BULGE_JAFFE)
        return fail(GK_EINVAL, "unknown bulge kind %d", d->bulge);
    if (d->n_discs < 0 || d->n_discs > 2) return fail(GK_EINVAL, "n_discs must be 0, 1 or 2");
    if (d->halo < GK_HALO_NONE || d->halo > GK_HALO_NFW) return fail(GK_EINVAL, "unknown halo kind %d", d->halo);
    if (d->halo == GK_HALO_NFW && !(d->hubble_h > 0.0)) return fail(GK_EINVAL, "hubble_h must be > 0");
    if (d->psf_mode != GK_PSF_MAPS && d->psf_mode != GK_PSF_LUMINOSITY)
        return fail(GK_EINVAL, "unknown psf_mode %d", d->psf_mode);
    if (!(d->frame_px_kpc >= 0.0) || !std::isfinite(d->frame_px_kpc) || !std::isfinite(d->frame_dx) ||
        !std::isfinite(d->frame_dy))
        return fail(GK_EINVAL, "frame_px_kpc must be finite and >= 0, frame_dx and frame_dy finite");
    if (d->bulge == GK_BULGE_NONE && d->n_discs == 0)
        return fail(GK_EINVAL, "the model needs at least one luminous component");
    return GK_OK;
}

static void free_grid(gk_grid* g) {
    void* bufs[] = {g->d_gw, g->d_aof, g->d_tab, g->d_val, g->d_ivar,
                    g->d_span, g->d_partials, g->d_counters, g->d_fbar, g->d_gpart, g->d_logdet};
    for (void* p : bufs)
        if (p) (void)hipFree(p);
    delete g;
}

static int choose_rule(const gk_grid* g, int B, int& bh, int& bw, int& steps) {
    bh = g->d.ny;
    bw = g->d.nx;
    steps = 0;
    int best = -1;
    for (const auto& r : g->rules)
        if (r.batch_min <= B && r.batch_min > best) {
            best = r.batch_min;
            bh = r.band_h;
            bw = r.band_w;
            steps = r.steps;
        }
    bh = std::min(bh, g->d.ny);
    bw = std::min(bw, g->d.nx);
    return GK_OK;
}

struct LaunchCfg;
static int make_cfg(const gk_grid* g, int band_h, int band_w, LaunchCfg& c, int bs_fixed = 0, int steps = 0);

// Narrow (then shorten) a band until its launch fits the LDS and band limits.
static void fit_shape(const gk_grid* g, int& bh, int& bw, int bs_fixed);

static int default_rules(gk_grid* g) {
    // Large batches: bands of up to 40 x 40 pixels (measured best on the 3x3
    // lattice: enough workgroups per CU to overlap one band's model phase with
    // another's stencil phase).  Small batches: small square bands so that one
    // theta spreads over many CUs.
    const int nx = g->d.nx, ny = g->d.ny;
    g->rules.clear();
    // the grid split into near-equal bands of at most 40 pixels each way; a
    // wide PSF on a coarse lattice (lag D >= 9 pixel rows, e.g. no
    // supersampling) spends D of every band_h + D steps filling the lag, so
    // there bands grow to 16 D rows and 64 columns (measured 1.4x faster on a
    // 160 x 160 grid with D = 10)
    // (the luminosity-weighted mode, whose phases end in a moment exchange,
    // prefers 80-row bands: measured 6 % faster on the realistic cube)
    const int hmax = g->D >= 9 ? 16 * g->D : (g->geo.lw ? 80 : 40), wmax = g->D >= 9 ? 64 : 40;
    int bh = (ny + (ny + hmax - 1) / hmax - 1) / ((ny + hmax - 1) / hmax);
    int bw = (nx + (nx + wmax - 1) / wmax - 1) / ((nx + wmax - 1) / wmax);
    fit_shape(g, bh, bw, 0);
    // on the 3x3 lattice two pixel rows (six lattice rows) per model phase: the
    // smaller row buffer leaves LDS for a fifth workgroup per CU (measured 6 %
    // faster than three rows on the 80 x 80 realistic cube)
    const int steps_big = g->geo.s == 3 ? 2 : 0;
    g->rules.push_back({512, bh, bw, steps_big});
    // >= 4096 vectors fill the chip without splitting a grid finely: bands of
    // up to 128 rows and 64 columns recompute less of the stencil halo
    // (measured 1.45x faster than 34 x 34 bands on a 100 x 100 grid, B = 4096)
    if (g->D < 9) {
        const int hb = 128, wb = 64;
        int bh2 = (ny + (ny + hb - 1) / hb - 1) / ((ny + hb - 1) / hb);
        int bw2 = (nx + (nx + wb - 1) / wb - 1) / ((nx + wb - 1) / wb);
        fit_shape(g, bh2, bw2, 0);
        g->rules.push_back({4096, bh2, bw2, steps_big});
    }
    int side = std::max(4, (int)std::ceil(std::sqrt((double)nx * ny / 64.0)));
    bh = std::min(ny, side), bw = std::min(nx, side);
    fit_shape(g, bh, bw, 0);
    g->rules.push_back({1, bh, bw, 0});
    int mid = std::max(8, (int)std::ceil(std::sqrt((double)nx * ny / 8.0)));
    bh = std::min(ny, mid), bw = std::min(nx, std::max(mid, 16));
    fit_shape(g, bh, bw, 0);
    g->rules.push_back({32, bh, bw, 0});
    return GK_OK;
}

struct LaunchCfg {
    int band_h, band_w, nbx, nbands, BS, gsub, xw, lds;
};

static int make_cfg(const gk_grid* g, int band_h, int band_w, LaunchCfg& c, int bs_fixed, int steps) {
    const int s = g->geo.s, pad = g->geo.pad;
    c.band_h = band_h;
    c.band_w = band_w;
    c.nbx = (g->d.nx + band_w - 1) / band_w;
    const int nby = (g->d.ny + band_h - 1) / band_h;
    c.nbands = c.nbx * nby;
    if (c.nbands > MAX_BANDS) return fail(GK_EINVAL, "launch shape gives %d bands (> %d)", c.nbands, MAX_BANDS);
    if (band_w > 128) return fail(GK_EINVAL, "band_w %d > 128", band_w);
    c.BS = std::min(512, std::max(64, (4 * band_w + 63) / 64 * 64));
    if (bs_fixed) {
        if (4 * band_w > bs_fixed) return fail(GK_EINVAL, "band_w %d > %d", band_w, bs_fixed / 4);
        c.BS = bs_fixed;
    }
    c.xw = band_w * s + 2 * pad + 1;
    // pixel-row steps per model phase: about ten lattice rows (measured best on
    // the 3x3 lattice with 40x40 bands), at most RS_CAP lattice rows, and the
    // row buffer within ~40 KiB of LDS; an explicit count is honoured up to
    // those limits
    const int nfrm = nfr_max(band_h, s, pad);
    int gs = steps > 0 ? steps : std::max(1, (10 + s / 2) / s);
    gs = std::min({gs, GSUB_CAP, std::max(1, RS_CAP / s)});
    const int lw = g->geo.lw;
    while (gs > 1 && make_layout(gs * s, c.xw, nfrm, band_h, lw ? 8 * gs * band_w : 0).total_bytes >
                         (steps > 0 ? 64 : 40) * 1024)
        --gs;
    c.gsub = gs;
    c.lds = make_layout(gs * s, c.xw, nfrm, band_h, lw ? 8 * gs * band_w : 0).total_bytes;
    if (c.lds > 64 * 1024) return fail(GK_EINVAL, "launch shape needs %d bytes of LDS (> 64 KiB)", c.lds);
    return GK_OK;
}

static void fit_shape(const gk_grid* g, int& bh, int& bw, int bs_fixed) {
    const std::string saved = g_err;
    LaunchCfg c;
    bw = std::max(1, std::min(bw, bs_fixed ? bs_fixed / 4 : 128));
    while (make_cfg(g, bh, bw, c, bs_fixed) != GK_OK) {
        if (bw > 8) bw = (bw + 1) / 2;
        else if (bh > 1) bh = (bh + 1) / 2;
        else break;
    }
    g_err = saved;
}

template <int MODE>
static hipError_t launch_fwd(const gk_grid* g, const LaunchCfg& c, FwdArgs& a, int B, hipStream_t st) {
    const int bulge = g->d.bulge, nd = g->d.n_discs, halo = g->d.halo;
    if ((size_t)B * c.nbands * c.BS >= ((size_t)1 << 31)) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)(B * c.nbands)), block((unsigned)c.BS);
#define GK_LAUNCH(BU, ND, HA)                                                                    \
    if (bulge == BU && nd == ND && halo == HA) {                                                  \
        if (a.geo.lw)                                                                             \
            hipLaunchKernelGGL((fwd_kernel<BU, ND, HA, MODE, 1>), grid, block, c.lds, st, a);    \
        else                                                                                      \
            hipLaunchKernelGGL((fwd_kernel<BU, ND, HA, MODE, 0>), grid, block, c.lds, st, a);    \
        return hipGetLastError();                                                                 \
    }
    GK_LAUNCH(1, 0, 0) GK_LAUNCH(1, 0, 1) GK_LAUNCH(1, 0, 2)
    GK_LAUNCH(1, 1, 0) GK_LAUNCH(1, 1, 1) GK_LAUNCH(1, 1, 2)
    GK_LAUNCH(1, 2, 0) GK_LAUNCH(1, 2, 1) GK_LAUNCH(1, 2, 2)
    GK_LAUNCH(2, 0, 0) GK_LAUNCH(2, 0, 1) GK_LAUNCH(2, 0, 2)
    GK_LAUNCH(2, 1, 0) GK_LAUNCH(2, 1, 1) GK_LAUNCH(2, 1, 2)
    GK_LAUNCH(2, 2, 0) GK_LAUNCH(2, 2, 1) GK_LAUNCH(2, 2, 2)
    GK_LAUNCH(0, 1, 0) GK_LAUNCH(0, 1, 1) GK_LAUNCH(0, 1, 2)
    GK_LAUNCH(0, 2, 0) GK_LAUNCH(0, 2, 1) GK_LAUNCH(0, 2, 2)
#undef GK_LAUNCH
    return hipErrorInvalidValue;
}

static int check_call(const gk_grid* g, const double* theta, int B, int stride, const void* out) {
    if (!g) return fail(GK_EINVAL, "grid is NULL");
    if (B < 0 || B > g->max_batch) return fail(GK_EINVAL, "B = %d outside [0, max_batch = %d]", B, g->max_batch);
    if (stride < g->P) return fail(GK_EINVAL, "stride %d < number of parameters %d", stride, g->P);
    if (B > 0 && (!theta || !out)) return fail(GK_EINVAL, "NULL theta or output pointer");
    return GK_OK;
}

static void fill_args(const gk_grid* g, const LaunchCfg& c, FwdArgs& a, const double* theta, int stride) {
    a.geo = g->geo;
    a.gw = g->d_gw;
    a.aof = g->d_aof;
    a.tab = g->d_tab;
    a.invW = g->invW;
    a.D = g->D;
    a.val = g->d_val;
    a.ivar = g->d_ivar;
    a.span = g->d_span;
    a.logdet = g->d_logdet;
    a.pstride = MAX_BANDS;
    a.band_h = c.band_h;
    a.band_w = c.band_w;
    a.nbx = c.nbx;
    a.nbands = c.nbands;
    a.gsub = c.gsub;
    a.xw = c.xw;
    a.tpad = g->tpad;
    a.theta = theta;
    a.stride = stride;
    a.logL = nullptr;
    a.maps = nullptr;
    a.fbar = nullptr;
    a.partials = g->d_partials;
    a.counters = g->d_counters;
    a.accum = 0;
    a.map_mask = g->map_mask;
}

// ---------------------------------------------------------------------------
// many-grid plans: the per-grid argument blocks and the cost-ordered work
// items of one (grids, row offsets) combination, kept on the device so that a
// repeated call only enqueues the launch
// ---------------------------------------------------------------------------
struct MultiPlan {
    int device = 0;
    std::vector<const gk_grid*> grids;
    std::vector<int> offs;
    std::vector<int> shapes;        // band_h, band_w per grid at build time
    FwdArgs* d_args = nullptr;
    int4* d_items = nullptr;
    int n_items = 0, lds = 0;
    int n_items_lw = 0;             // the last n_items_lw items belong to luminosity-weighted grids
};

static std::mutex g_plan_mu;
static std::vector<MultiPlan*> g_plans;   // most recently used last
constexpr size_t MAX_PLANS = 8;

static void free_plan(MultiPlan* p) {
    if (p->d_args) (void)hipFree(p->d_args);
    if (p->d_items) (void)hipFree(p->d_items);
    delete p;
}

// Drop every cached plan that uses grid g (called when g is destroyed).
static void evict_plans(const gk_grid* g) {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (size_t i = 0; i < g_plans.size();) {
        MultiPlan* p = g_plans[i];
        if (std::find(p->grids.begin(), p->grids.end(), g) != p->grids.end()) {
            free_plan(p);
            g_plans.erase(g_plans.begin() + i);
        } else {
            ++i;
        }
    }
}

static void multi_band_shape(const gk_grid* g, int rows, int& bh, int& bw, int& steps) {
    choose_rule(g, rows, bh, bw, steps);
    fit_shape(g, bh, bw, MULTI_BS);
}

static bool plan_matches(const MultiPlan* p, int device, const gk_grid* const* grids, int n, const int* offs) {
    if (p->device != device || (int)p->grids.size() != n) return false;
    for (int i = 0; i < n; ++i) {
        if (p->grids[i] != grids[i] || p->offs[i] != offs[i]) return false;
        int bh, bw, st;
        multi_band_shape(grids[i], offs[i + 1] - offs[i], bh, bw, st);
        if (p->shapes[3 * i] != bh || p->shapes[3 * i + 1] != bw || p->shapes[3 * i + 2] != st) return false;
    }
    return p->offs[n] == offs[n];
}

// Relative cost of one band of one row: model points plus stencil taps.
static double band_cost(const gk_grid* g, const LaunchCfg& c, int band) {
    const int s = g->geo.s, pad = g->geo.pad;
    const int by = band / c.nbx, bx = band % c.nbx;
    const int nr = std::min(g->d.ny, (by + 1) * c.band_h) - by * c.band_h;
    const int nc = std::min(g->d.nx, (bx + 1) * c.band_w) - bx * c.band_w;
    const double pts = (double)((nr - 1) * s + 2 * pad + 1) * ((nc - 1) * s + 2 * pad + 1);
    const double ncomp = (g->d.bulge ? 1 : 0) + g->d.n_discs + (g->d.halo ? 1 : 0);
    return pts * (60.0 + 35.0 * ncomp) + 4.0 * nr * nc * (4.0 * (s * (1 + 3 * pad) + 2 * (2 * pad + 1)));
}

static int build_plan(int device, const gk_grid* const* grids, int n, const int* offs, MultiPlan*& out) {
    MultiPlan* p = new MultiPlan;
    p->device = device;
    p->grids.assign(grids, grids + n);
    p->offs.assign(offs, offs + n + 1);
    std::vector<FwdArgs> args(n);
    struct Item { double cost; int4 it; };
    std::vector<Item> items;
    int lds = 0;
    for (int i = 0; i < n; ++i) {
        const gk_grid* g = grids[i];
        const int rows = offs[i + 1] - offs[i];
        int bh, bw, st;
        multi_band_shape(g, rows, bh, bw, st);
        p->shapes.push_back(bh);
        p->shapes.push_back(bw);
        p->shapes.push_back(st);
        LaunchCfg c;
        int rc = make_cfg(g, bh, bw, c, MULTI_BS, st);
        if (rc) { free_plan(p); return rc; }
        lds = std::max(lds, c.lds);
        fill_args(g, c, args[i], nullptr, 0);
        for (int band = 0; band < c.nbands; ++band) {
            const double cost = band_cost(g, c, band);
            for (int r = 0; r < rows; ++r) items.push_back({cost, make_int4(i, r, band, offs[i])});
        }
    }
    // map-averaging items first, then the luminosity-weighted ones (a launch
    // each), each part in decreasing cost order
    std::stable_sort(items.begin(), items.end(), [&](const Item& x, const Item& y) {
        const int lx = grids[x.it.x]->geo.lw, ly = grids[y.it.x]->geo.lw;
        return lx != ly ? lx < ly : x.cost > y.cost;
    });
    std::vector<int4> it(items.size());
    int n_lw = 0;
    for (size_t k = 0; k < items.size(); ++k) {
        it[k] = items[k].it;
        n_lw += grids[items[k].it.x]->geo.lw;
    }
    p->n_items = (int)it.size();
    p->n_items_lw = n_lw;
    p->lds = lds;
    if (hipMalloc((void**)&p->d_args, sizeof(FwdArgs) * n) != hipSuccess ||
        hipMalloc((void**)&p->d_items, sizeof(int4) * std::max<size_t>(1, it.size())) != hipSuccess) {
        free_plan(p);
        return fail(GK_ENOMEM, "allocation of a many-grid plan failed");
    }
    if (hipMemcpy(p->d_args, args.data(), sizeof(FwdArgs) * n, hipMemcpyHostToDevice) != hipSuccess ||
        (!it.empty() && hipMemcpy(p->d_items, it.data(), sizeof(int4) * it.size(), hipMemcpyHostToDevice) != hipSuccess) ||
        hipDeviceSynchronize() != hipSuccess) {
        free_plan(p);
        return fail(GK_EHIP, "upload of a many-grid plan failed");
    }
    out = p;
    return GK_OK;
}

extern "C" {

const char* last_error(void) { return g_err.c_str(); }

int n_params(gk_grid_t g) {
    if (!g) return fail(GK_EINVAL, "grid is NULL");
    return g->P;
}

int create_grid(const gk_grid_desc* desc, int max_batch, gk_grid_t* out) {
    int rc = valid_desc(desc);
    if (rc) return rc;
    if (!out) return fail(GK_EINVAL, "out is NULL");
    if (max_batch < 1 || max_batch > (1 << 20)) return fail(GK_EINVAL, "max_batch must be in [1, 2^20]");
    *out = nullptr;
    gk_grid* g = new gk_grid();
    g->d = *desc;
    g->max_batch = max_batch;
    HIPCHECK(hipGetDevice(&g->device));
    const int s = desc->supersample;
    const double sig = desc->psf_sigma_px * s;             // stencil sigma in lattice units
    const double rad2 = 9.0 * sig * sig;
    const int pad = (int)std::floor(3.0 * sig);
    g->geo.nx = desc->nx;
    g->geo.ny = desc->ny;
    g->geo.s = s;
    g->geo.hs = (s - 1) / 2;
    g->geo.pad = pad;
    g->geo.pk = desc->pixel_kpc;
    g->geo.pk_over_s = (float)(desc->pixel_kpc / s);
    const double H = 0.1 * desc->hubble_h;                 // km/s/kpc
    g->geo.rho_crit = 3.0 * H * H / (8.0 * PI * G_KPC);
    g->geo.bulge = desc->bulge;
    g->geo.ndisc = desc->n_discs;
    g->geo.halo = desc->halo;
    g->geo.lw = desc->psf_mode == GK_PSF_LUMINOSITY ? 1 : 0;
    g->geo.fscale = desc->frame_px_kpc > 0.0 ? desc->frame_px_kpc / desc->pixel_kpc : 1.0;
    g->geo.fdx = desc->frame_dx;
    g->geo.fdy = desc->frame_dy;
    g->P = 4 + 3 * (desc->bulge != 0) + 4 * desc->n_discs + 2 * (desc->halo != 0);
    // 1-D Gaussian factors (FP32) and the stencil half-widths
    std::vector<float> gw(pad + 1);
    std::vector<int> aof(pad + 1);
    for (int a = 0; a <= pad; ++a) gw[a] = (float)std::exp(-(double)a * a / (2.0 * sig * sig + 1e-300));
    if (sig == 0.0) gw[0] = 1.0f;
    double W = 0.0;
    int K = 0;
    for (int bb = 0; bb <= pad; ++bb) {
        int A = -1;
        for (int a = 0; a <= pad; ++a)
            if ((double)a * a + (double)bb * bb <= rad2) A = a;
        aof[bb] = A;
    }
    for (int bb = -pad; bb <= pad; ++bb)
        for (int a = -pad; a <= pad; ++a)
            if ((double)a * a + (double)bb * bb <= rad2) {
                W += (double)gw[std::abs(a)] * (double)gw[std::abs(bb)];
                ++K;
            }
    if (K == 0) { gw[0] = 1.0f; W = 1.0; K = 1; aof[0] = 0; }
    g->K = K;
    g->invW = (float)(1.0 / W);
    // lag table: lattice row of phase ph (= row mod s) reaches the pixel row
    // d steps back with b = d s + ph - pad; weight g(|b|), half-width A(|b|)
    const int D = 2 * pad / s;
    if (pad > 25 || D > DMAX) {
        delete g;
        return fail(GK_EINVAL, "PSF too wide for this build: 3 sigma s = %d lattice points (max 25) and "
                               "2 pad / s = %d (max %d)", pad, D, DMAX);
    }
    g->D = D;
    std::vector<int2> tab((size_t)s * DSTRIDE, make_int2(0, 0));
    for (int ph = 0; ph < s; ++ph)
        for (int d = 0; d <= D; ++d) {
            const int bb = d * s + ph - pad;
            if (std::abs(bb) <= pad) {
                const float w = gw[std::abs(bb)];
                int wb;
                std::memcpy(&wb, &w, 4);
                tab[(size_t)ph * DSTRIDE + d] = make_int2(aof[std::abs(bb)], wb);
            }
        }
    const size_t npix = (size_t)desc->nx * desc->ny;
#define ALLOC(ptr, bytes)                                                                \
    if (hipMalloc((void**)&(ptr), (bytes)) != hipSuccess) {                              \
        free_grid(g);                                                                    \
        return fail(GK_ENOMEM, "hipMalloc of %zu bytes failed", (size_t)(bytes));       \
    }
    ALLOC(g->d_gw, sizeof(float) * std::max(pad + 1, 64));
    ALLOC(g->d_aof, sizeof(int) * (pad + 1));
    ALLOC(g->d_tab, sizeof(int2) * tab.size());
    ALLOC(g->d_val, sizeof(float) * 4 * npix);
    ALLOC(g->d_ivar, sizeof(float) * 4 * npix);
    ALLOC(g->d_span, sizeof(int2) * desc->ny);
    ALLOC(g->d_partials, sizeof(double) * (size_t)max_batch * MAX_BANDS);
    ALLOC(g->d_counters, sizeof(unsigned) * (size_t)max_batch);
    ALLOC(g->d_fbar, sizeof(float) * 4 * npix * (size_t)max_batch);
    ALLOC(g->d_gpart, sizeof(double) * NCONST * MAX_BANDS_ADJ * (size_t)max_batch);
    ALLOC(g->d_logdet, sizeof(double));
#undef ALLOC
    {
        // compile-time tap counts of the stencil (register arrays up to 26 entries
        // stay in VGPRs with uniform indexing; wider stencils are rejected above)
        static const int tpads[] = {4, 6, 9, 12, 16, 20, 25};
        g->tpad = 0;
        for (int t : tpads)
            if (t >= pad) { g->tpad = t; break; }
    }
    std::vector<float> gw64(std::max(pad + 1, 64), 0.0f);
    std::copy(gw.begin(), gw.end(), gw64.begin());
    if (hipMemcpy(g->d_gw, gw64.data(), sizeof(float) * gw64.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g->d_aof, aof.data(), sizeof(int) * (pad + 1), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g->d_tab, tab.data(), sizeof(int2) * tab.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(g->d_counters, 0, sizeof(unsigned) * (size_t)max_batch) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        free_grid(g);
        return fail(GK_EHIP, "upload of the stencil tables failed");
    }
    default_rules(g);
    // adjoint bands: at most 40 x 40 pixels (pixel adjoints are staged in LDS)
    g->adj_band_w = std::min(desc->nx, 40);
    g->adj_band_h = std::min(desc->ny, 40);
    while ((desc->nx + g->adj_band_w - 1) / g->adj_band_w * ((desc->ny + g->adj_band_h - 1) / g->adj_band_h) >
           MAX_BANDS_ADJ) {
        g->adj_band_w = std::min(desc->nx, g->adj_band_w + 8);
        g->adj_band_h = std::min(desc->ny, g->adj_band_h + 8);
    }
    if (adj_lds_bytes(g->adj_band_h, g->adj_band_w, s, pad) > 64 * 1024) {
        free_grid(g);
        return fail(GK_EINVAL, "grid too large for the adjoint's LDS tiles in this build");
    }
    *out = g;
    return GK_OK;
}

int destroy_grid(gk_grid_t g) {
    if (!g) return fail(GK_EINVAL, "grid is NULL");
    (void)hipDeviceSynchronize();
    evict_plans(g);
    free_grid(g);
    return GK_OK;
}

int set_launch_shape(gk_grid_t g, int batch_min, int band_h, int band_w, int steps) {
    if (!g) return fail(GK_EINVAL, "grid is NULL");
    if (batch_min < 1 || band_h < 1 || band_w < 1) return fail(GK_EINVAL, "batch_min, band_h, band_w must be >= 1");
    if (steps < 0 || steps > GSUB_CAP) return fail(GK_EINVAL, "steps must be in [0, %d]", GSUB_CAP);
    LaunchCfg c;
    int rc = make_cfg(g, std::min(band_h, g->d.ny), std::min(band_w, g->d.nx), c, 0, steps);
    if (rc) return rc;
    for (auto& r : g->rules)
        if (r.batch_min == batch_min) {
            r.band_h = band_h;
            r.band_w = band_w;
            r.steps = steps;
            return GK_OK;
        }
    g->rules.push_back({batch_min, band_h, band_w, steps});
    return GK_OK;
}

int get_launch_shape(gk_grid_t g, int B, int* band_h, int* band_w, int* steps) {
    if (!g || !band_h || !band_w || !steps) return fail(GK_EINVAL, "NULL grid or output pointer");
    if (B < 1) return fail(GK_EINVAL, "B must be >= 1");
    return choose_rule(g, B, *band_h, *band_w, *steps);
}

int set_data(gk_grid_t g, const float* value, const float* err, int on_device, void* stream) {
    if (!g) return fail(GK_EINVAL, "grid is NULL");
    if (!value || !err) return fail(GK_EINVAL, "NULL value or err");
    const int nx = g->d.nx, ny = g->d.ny;
    const size_t n = (size_t)4 * nx * ny;
    hipStream_t st = (hipStream_t)stream;
    std::vector<float> v(n), e(n);
    if (on_device) {
        HIPCHECK(hipMemcpyAsync(v.data(), value, n * sizeof(float), hipMemcpyDeviceToHost, st));
        HIPCHECK(hipMemcpyAsync(e.data(), err, n * sizeof(float), hipMemcpyDeviceToHost, st));
        HIPCHECK(hipStreamSynchronize(st));
    } else {
        std::memcpy(v.data(), value, n * sizeof(float));
        std::memcpy(e.data(), err, n * sizeof(float));
    }
    std::vector<float> iv(n, 0.0f), dv(n, 0.0f);
    std::vector<int2> span(ny, make_int2(1, 0));
    double logdet = 0.0;
    size_t nvalid = 0;
    for (int m = 0; m < 4; ++m)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t k = ((size_t)m * ny + j) * nx + i;
                const double ee = e[k];
                if (std::isfinite(v[k]) && std::isfinite(ee) && ee > 0.0) {
                    iv[k] = (float)(1.0 / (ee * ee));
                    dv[k] = v[k];
                    logdet += std::log(2.0 * PI * ee * ee);
                    ++nvalid;
                    int2& sp = span[j];
                    if (sp.x > sp.y) sp = make_int2(i, i);
                    else { sp.x = std::min(sp.x, i); sp.y = std::max(sp.y, i); }
                }
            }
    HIPCHECK(hipMemcpyAsync(g->d_val, dv.data(), n * sizeof(float), hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(g->d_ivar, iv.data(), n * sizeof(float), hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(g->d_span, span.data(), ny * sizeof(int2), hipMemcpyHostToDevice, st));
    HIPCHECK(hipMemcpyAsync(g->d_logdet, &logdet, sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHECK(hipStreamSynchronize(st));
    int mask = 0;
    for (int m = 0; m < 4; ++m)
        for (size_t k = (size_t)m * ny * nx; k < (size_t)(m + 1) * ny * nx; ++k)
            if (iv[k] > 0.0f) {
                mask |= 1 << m;
                break;
            }
    // the moment mode forms every observable from the four moment maps
    mask = g->geo.lw ? (mask ? 15 : 0) : mask;
    if (mask != g->map_mask) evict_plans(g);    // cached many-grid plans hold the mask
    g->map_mask = mask;
    g->logdet = logdet;
    g->has_data = true;
    (void)nvalid;
    return GK_OK;
}

// log-likelihood launch of one grid (arguments checked by the caller)
static int run_loglike(gk_grid* g, const double* theta, int B, int stride, double* logL, int accum,
                       hipStream_t st) {
    int bh, bw, steps;
    choose_rule(g, B, bh, bw, steps);
    LaunchCfg c;
    int rc = make_cfg(g, bh, bw, c, 0, steps);
    if (rc) return rc;
    FwdArgs a;
    fill_args(g, c, a, theta, stride);
    a.logL = logL;
    a.accum = accum;
    hipError_t e = launch_fwd<MODE_LOGL>(g, c, a, B, st);
    if (e != hipSuccess) return fail(GK_EHIP, "forward launch failed: %s", hipGetErrorString(e));
    return GK_OK;
}

static int run_grad(gk_grid* g, const double* theta, int B, int stride, double* logL, double* grad, int accum,
                    hipStream_t st);

int loglike_batch(gk_grid_t g, const double* theta, int B, int stride, double* logL, void* stream) {
    int rc = check_call(g, theta, B, stride, logL);
    if (rc) return rc;
    if (!g->has_data) return fail(GK_ESTATE, "loglike_batch before set_data");
    if (B == 0) return GK_OK;
    return run_loglike(g, theta, B, stride, logL, 0, (hipStream_t)stream);
}

int eval_maps(gk_grid_t g, const double* theta, int B, int stride, float* maps, void* stream) {
    int rc = check_call(g, theta, B, stride, maps);
    if (rc) return rc;
    if (B == 0) return GK_OK;
    int bh, bw, steps;
    choose_rule(g, B, bh, bw, steps);
    LaunchCfg c;
    rc = make_cfg(g, bh, bw, c, 0, steps);
    if (rc) return rc;
    FwdArgs a;
    fill_args(g, c, a, theta, stride);
    a.maps = maps;
    a.map_mask = 15;
    hipError_t e = launch_fwd<MODE_MAPS>(g, c, a, B, (hipStream_t)stream);
    if (e != hipSuccess) return fail(GK_EHIP, "maps launch failed: %s", hipGetErrorString(e));
    return GK_OK;
}

int loglike_grad_batch(gk_grid_t g, const double* theta, int B, int stride, double* logL, double* grad,
                       void* stream) {
    int rc = check_call(g, theta, B, stride, logL);
    if (rc) return rc;
    if (B > 0 && !grad) return fail(GK_EINVAL, "NULL grad");
    if (!g->has_data) return fail(GK_ESTATE, "loglike_grad_batch before set_data");
    if (B == 0) return GK_OK;
    return run_grad(g, theta, B, stride, logL, grad, 0, (hipStream_t)stream);
}

static int run_grad(gk_grid* g, const double* theta, int B, int stride, double* logL, double* grad, int accum,
                    hipStream_t st) {
    // pass 1: log-likelihood and d logL / d F at every pixel
    int bh, bw, steps;
    choose_rule(g, B, bh, bw, steps);
    LaunchCfg c;
    int rc = make_cfg(g, bh, bw, c, 0, steps);
    if (rc) return rc;
    FwdArgs fa;
    fill_args(g, c, fa, theta, stride);
    fa.logL = logL;
    fa.fbar = g->d_fbar;
    fa.accum = accum;
    hipError_t e = launch_fwd<MODE_FBAR>(g, c, fa, B, st);
    if (e != hipSuccess) return fail(GK_EHIP, "forward (adjoint seed) launch failed: %s", hipGetErrorString(e));
    // pass 2: adjoint of the PSF and of the model, chain rule to theta
    AdjArgs aa;
    aa.geo = g->geo;
    aa.gw = g->d_gw;
    aa.aof = g->d_aof;
    aa.invW = g->invW;
    aa.D = g->D;
    aa.span = g->d_span;
    aa.band_h = g->adj_band_h;
    aa.band_w = g->adj_band_w;
    aa.nbx = (g->d.nx + aa.band_w - 1) / aa.band_w;
    aa.nbands = aa.nbx * ((g->d.ny + aa.band_h - 1) / aa.band_h);
    aa.theta = theta;
    aa.stride = stride;
    aa.fbar = g->d_fbar;
    aa.gpart = g->d_gpart;
    aa.counters = g->d_counters;
    aa.grad = grad;
    aa.accum = accum;
    const int lds = adj_lds_bytes(aa.band_h, aa.band_w, g->geo.s, g->geo.pad);
    const dim3 grid2((unsigned)(B * aa.nbands)), block2(256);
    const int bulge = g->d.bulge, nd = g->d.n_discs, halo = g->d.halo;
    bool launched = false;
#define GK_ALAUNCH(BU, ND, HA)                                                                  \
    if (!launched && bulge == BU && nd == ND && halo == HA) {                                    \
        hipLaunchKernelGGL((adj_kernel<BU, ND, HA>), grid2, block2, lds, st, aa);               \
        launched = true;                                                                         \
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
    e = hipGetLastError();
    if (!launched || e != hipSuccess)
        return fail(GK_EHIP, "adjoint launch failed: %s", hipGetErrorString(e));
    return GK_OK;
}

int loglike_joint(const gk_grid_t* grids, int n_grids, const double* theta, int B, int stride, double* logL,
                  double* grad, void* stream) {
    if (n_grids < 1 || !grids) return fail(GK_EINVAL, "loglike_joint needs n_grids >= 1 and a grid list");
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return fail(GK_EHIP, "hipGetDevice failed");
    for (int i = 0; i < n_grids; ++i) {
        const gk_grid* g = grids[i];
        int rc = check_call(g, theta, B, stride, logL);
        if (rc) return rc;
        if (!g->has_data) return fail(GK_ESTATE, "grid %d has no data (set_data)", i);
        if (g->device != device) return fail(GK_EINVAL, "grid %d lives on device %d, not %d", i, g->device, device);
        const gk_grid* g0 = grids[0];
        if (g->d.bulge != g0->d.bulge || g->d.n_discs != g0->d.n_discs || g->d.halo != g0->d.halo)
            return fail(GK_EINVAL, "grid %d has another component set than grid 0", i);
        for (int k = 0; k < i; ++k)
            if (grids[k] == g) return fail(GK_EINVAL, "grid %d appears twice", i);
    }
    if (B == 0) return GK_OK;
    hipStream_t st = (hipStream_t)stream;
    // grid 0 stores, the others add, in stream order: the sum is taken in the
    // same order on every call
    for (int i = 0; i < n_grids; ++i) {
        const int rc = grad ? run_grad(grids[i], theta, B, stride, logL, grad, i > 0, st)
                            : run_loglike(grids[i], theta, B, stride, logL, i > 0, st);
        if (rc) return rc;
    }
    return GK_OK;
}

int hmc_leapfrog(gk_grid_t g, double* theta, double* momentum, const double* inv_mass, double eps,
                 int n_steps, int B, int stride, double* logL, double* grad, void* stream) {
    int rc = check_call(g, theta, B, stride, logL);
    if (rc) return rc;
    if (B > 0 && (!momentum || !inv_mass || !grad)) return fail(GK_EINVAL, "NULL momentum, inv_mass or grad");
    if (n_steps < 1) return fail(GK_EINVAL, "n_steps must be >= 1");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(GK_EINVAL, "eps must be finite and > 0");
    if (!g->has_data) return fail(GK_ESTATE, "hmc_leapfrog before set_data");
    if (B == 0) return GK_OK;
    hipStream_t st = (hipStream_t)stream;
    const int n = B * g->P;
    const dim3 grid((unsigned)((n + 255) / 256)), block(256);
    for (int k = 0; k <= n_steps; ++k) {
        rc = loglike_grad_batch(g, theta, B, stride, logL, grad, stream);
        if (rc) return rc;
        const int stage = (k == 0) ? 0 : (k == n_steps ? 2 : 1);
        hipLaunchKernelGGL(leapfrog_kernel, grid, block, 0, st, theta, momentum, grad, logL, inv_mass, eps,
                           stage, B, g->P, stride);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(GK_EHIP, "leapfrog launch failed: %s", hipGetErrorString(e));
    }
    return GK_OK;
}

int loglike_multi(const gk_grid_t* grids, int n_gal, const double* theta, const int* theta_offset, int stride,
                  double* logL, double* grad, void* stream) {
    if (n_gal < 0) return fail(GK_EINVAL, "n_gal must be >= 0");
    if (n_gal == 0) return GK_OK;
    if (!grids || !theta_offset) return fail(GK_EINVAL, "NULL grids or theta_offset");
    if (theta_offset[0] != 0) return fail(GK_EINVAL, "theta_offset[0] must be 0");
    for (int i = 0; i < n_gal; ++i)
        if (!grids[i]) return fail(GK_EINVAL, "grids[%d] is NULL", i);
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return fail(GK_EHIP, "hipGetDevice failed");
    for (int i = 0; i < n_gal; ++i) {
        const gk_grid* g = grids[i];
        const int rows = theta_offset[i + 1] - theta_offset[i];
        if (rows < 0 || rows > g->max_batch)
            return fail(GK_EINVAL, "galaxy %d has %d rows (max_batch %d)", i, rows, g->max_batch);
        if (stride < g->P) return fail(GK_EINVAL, "stride %d < number of parameters %d of galaxy %d", stride, g->P, i);
        if (!g->has_data) return fail(GK_ESTATE, "galaxy %d has no data (set_data)", i);
        if (g->device != device) return fail(GK_EINVAL, "galaxy %d lives on device %d, not %d", i, g->device, device);
        for (int k = 0; k < i; ++k)
            if (grids[k] == g) return fail(GK_EINVAL, "grid of galaxy %d appears twice", i);
    }
    const int total = theta_offset[n_gal];
    if (total == 0) return GK_OK;
    if (!theta || !logL) return fail(GK_EINVAL, "NULL theta or logL");
    hipStream_t st = (hipStream_t)stream;
    if (grad) {
        // gradient: one forward + adjoint launch pair per galaxy on the stream
        for (int i = 0; i < n_gal; ++i) {
            const int r0 = theta_offset[i], rows = theta_offset[i + 1] - r0;
            if (rows == 0) continue;
            int rc = loglike_grad_batch(grids[i], theta + (size_t)r0 * stride, rows, stride, logL + r0,
                                        grad + (size_t)r0 * stride, stream);
            if (rc) return rc;
        }
        return GK_OK;
    }
    MultiPlan* p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_plan_mu);
        for (size_t k = 0; k < g_plans.size(); ++k)
            if (plan_matches(g_plans[k], device, grids, n_gal, theta_offset)) {
                p = g_plans[k];
                g_plans.erase(g_plans.begin() + k);
                g_plans.push_back(p);
                break;
            }
        if (!p) {
            int rc = build_plan(device, grids, n_gal, theta_offset, p);
            if (rc) return rc;
            if (g_plans.size() >= MAX_PLANS) {
                (void)hipDeviceSynchronize();
                free_plan(g_plans.front());
                g_plans.erase(g_plans.begin());
            }
            g_plans.push_back(p);
        }
    }
    const int n0 = p->n_items - p->n_items_lw;
    if (n0 > 0)
        hipLaunchKernelGGL(multi_kernel<0>, dim3((unsigned)n0), dim3(MULTI_BS), p->lds, st, p->d_args, p->d_items,
                           theta, stride, logL);
    if (p->n_items_lw > 0)
        hipLaunchKernelGGL(multi_kernel<1>, dim3((unsigned)p->n_items_lw), dim3(MULTI_BS), p->lds, st, p->d_args,
                           p->d_items + n0, theta, stride, logL);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(GK_EHIP, "many-grid launch failed: %s", hipGetErrorString(e));
    return GK_OK;
}

}  // extern "C"

// ============================================================================
// data preparation: colour-M/L maps and the surface-brightness error model
// ============================================================================
namespace gk {

__global__ void __launch_bounds__(256) ml_colour_kernel(const float* __restrict__ mb, const float* __restrict__ mg,
                                                        const float* __restrict__ dmb,
                                                        const float* __restrict__ dmg, int n, float a, float b,
                                                        float s2, float* __restrict__ ml, float* __restrict__ err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float x = mb[i], y = mg[i], ex = dmb[i], ey = dmg[i];
    const bool ok = isfinite(x) && isfinite(y) && isfinite(ex) && isfinite(ey);
    // log10 (M/L) = a + b (m_beta - m_gamma); its error adds the magnitude errors
    // and the relation's scatter in quadrature
    const float lg = fmaf(b, x - y, a);
    const float m = exp10f(lg);
    const float el = sqrtf(fmaf(b * b, fmaf(ex, ex, ey * ey), s2));
    ml[i] = ok ? m : __int_as_float(0x7fc00000);
    err[i] = ok ? m * 2.302585093f * el : 0.0f;
}

__device__ __forceinline__ void ml_colour_one(float x, float y, float ex, float ey, float a, float b, float s2,
                                              float& m_out, float& e_out) {
    const bool ok = isfinite(x) && isfinite(y) && isfinite(ex) && isfinite(ey);
    const float m = exp10f(fmaf(b, x - y, a));
    const float el = sqrtf(fmaf(b * b, fmaf(ex, ex, ey * ey), s2));
    m_out = ok ? m : __int_as_float(0x7fc00000);
    e_out = ok ? m * 2.302585093f * el : 0.0f;
}

// four pixels per thread through 16-byte loads and stores (all six arrays
// 16-byte aligned); the last n % 4 pixels by the first threads, one each
__global__ void __launch_bounds__(256) ml_colour_kernel4(const float4* __restrict__ mb, const float4* __restrict__ mg,
                                                         const float4* __restrict__ dmb,
                                                         const float4* __restrict__ dmg, int n, float a, float b,
                                                         float s2, float4* __restrict__ ml, float4* __restrict__ err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int n4 = n >> 2;
    if (i < n4) {
        const float4 x = mb[i], y = mg[i], ex = dmb[i], ey = dmg[i];
        float4 m, e;
        ml_colour_one(x.x, y.x, ex.x, ey.x, a, b, s2, m.x, e.x);
        ml_colour_one(x.y, y.y, ex.y, ey.y, a, b, s2, m.y, e.y);
        ml_colour_one(x.z, y.z, ex.z, ey.z, a, b, s2, m.z, e.z);
        ml_colour_one(x.w, y.w, ex.w, ey.w, a, b, s2, m.w, e.w);
        ml[i] = m;
        err[i] = e;
    }
    const int t = 4 * n4 + i;
    if (i < (n & 3)) {
        const float* fmb = (const float*)mb;
        const float* fmg = (const float*)mg;
        const float* fdb = (const float*)dmb;
        const float* fdg = (const float*)dmg;
        ml_colour_one(fmb[t], fmg[t], fdb[t], fdg[t], a, b, s2, ((float*)ml)[t], ((float*)err)[t]);
    }
}

// one workgroup: the smallest positive finite B, then every pixel's error
__global__ void __launch_bounds__(1024) b_err_kernel(const float* __restrict__ B, int n, float rel, float floor_frac,
                                                     float* __restrict__ err) {
    __shared__ float s_min[16];
    const int tid = threadIdx.x, BS = blockDim.x;
    float mn = INFINITY;
    for (int i = tid; i < n; i += BS) {
        const float v = B[i];
        if (isfinite(v) && v > 0.0f) mn = fminf(mn, v);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mn = fminf(mn, __shfl_down(mn, o, 64));
    if ((tid & 63) == 0) s_min[tid >> 6] = mn;
    __syncthreads();
    mn = INFINITY;
    for (int w = 0; w < (BS + 63) / 64; ++w) mn = fminf(mn, s_min[w]);
    const float sys = isfinite(mn) ? floor_frac * mn : 0.0f;
    for (int i = tid; i < n; i += BS) {
        const float v = B[i];
        const float r = rel * v;
        err[i] = (isfinite(v) && v > 0.0f) ? sqrtf(fmaf(r, r, sys * sys)) : 0.0f;
    }
}

}  // namespace gk

extern "C" {

int ml_from_colour(const float* m_beta, const float* m_gamma, const float* dm_beta, const float* dm_gamma, int n,
                   double a, double b, double sigma_a, float* ml, float* err, void* stream) {
    if (n < 0) return fail(GK_EINVAL, "n must be >= 0");
    if (n == 0) return GK_OK;
    if (!m_beta || !m_gamma || !dm_beta || !dm_gamma || !ml || !err) return fail(GK_EINVAL, "NULL pointer");
    if (!std::isfinite(a) || !std::isfinite(b) || !(sigma_a >= 0.0)) return fail(GK_EINVAL, "bad a, b or sigma_a");
    auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
    const float fa = (float)a, fb = (float)b, s2 = (float)(sigma_a * sigma_a);
    if (al16(m_beta) && al16(m_gamma) && al16(dm_beta) && al16(dm_gamma) && al16(ml) && al16(err)) {
        const int n4 = std::max(n >> 2, n & 3);
        hipLaunchKernelGGL(ml_colour_kernel4, dim3((unsigned)((n4 + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                           (const float4*)m_beta, (const float4*)m_gamma, (const float4*)dm_beta,
                           (const float4*)dm_gamma, n, fa, fb, s2, (float4*)ml, (float4*)err);
    } else {
        hipLaunchKernelGGL(ml_colour_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)stream,
                           m_beta, m_gamma, dm_beta, dm_gamma, n, fa, fb, s2, ml, err);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(GK_EHIP, "colour-M/L launch failed: %s", hipGetErrorString(e));
    return GK_OK;
}

int brightness_errors(const float* B, int n, double rel, double floor_frac, float* err, void* stream) {
    if (n < 0) return fail(GK_EINVAL, "n must be >= 0");
    if (n == 0) return GK_OK;
    if (!B || !err) return fail(GK_EINVAL, "NULL pointer");
    if (!(rel >= 0.0) || !(floor_frac >= 0.0)) return fail(GK_EINVAL, "rel and floor_frac must be >= 0");
    hipLaunchKernelGGL(b_err_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, B, n, (float)rel,
                       (float)floor_frac, err);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(GK_EHIP, "error-model launch failed: %s", hipGetErrorString(e));
    return GK_OK;
}

}  // extern "C"
