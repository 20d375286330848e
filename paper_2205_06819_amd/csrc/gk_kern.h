// Kernel arguments, LDS layouts and the launch entry points shared by the
// host code (galkin.hip) and the kernel translation units (fwd_inst.hip,
// multi_inst.hip, adj.hip), which are compiled in parallel.
#pragma once

#include <hip/hip_runtime.h>

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
    int pstride;            // row stride of partials (= nbands: one FP64 partial per band of a vector)
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

// The forward stencil is compiled for a few tap counts (the smallest one >=
// pad is used).  For each, the largest lag D = floor(2 pad / s) that a grid
// accepted by create_grid (D <= DMAX) can have with that tap count: s = 1 only
// fits pad <= 5 (tap counts 4 and 6), s = 3 fits pad <= 16 and s >= 5 the rest.
__host__ __device__ constexpr int lag_cap(int tpad) {
    return tpad == 4 ? 8 : tpad == 6 ? 10 : tpad == 9 ? 6 : tpad == 12 ? 8 : tpad == 16 ? 10 : tpad == 20 ? 8 : 10;
}
constexpr int RS_CAP = 16;      // lattice rows per model phase
constexpr int GSUB_CAP = 4;     // pixel-row steps per model phase

struct Layout {                 // LDS carve-up, identical on host and device
    int rows, red, stage, prange, fin, tab, total_bytes;
};

__host__ __device__ inline int nfr_max(int band_h, int s, int pad) { return (band_h - 1) * s + 2 * pad + 1; }
// ceil(a / b) for b > 0 and any sign of a
__host__ __device__ inline int ceil_div(int a, int b) { return a >= 0 ? (a + b - 1) / b : -((-a) / b); }

// nfin: floats of the per-step exchange buffer of the luminosity-weighted
// mode (0 otherwise); tab_lds: an LDS copy of the special-function tables,
// last (the forward bodies that read it, see fwd_band)
__host__ __device__ inline Layout make_layout(int rows, int xw, int nfrm, int band_h, int nfin, bool tab_lds) {
    Layout L;
    int off = 0;                                   // in 4-byte words
    L.rows = off;       off += rows * 4 * xw;
    off = (off + 3) & ~3;
    L.red = off;        off += 2 * RED_SLOTS;      // doubles
    L.stage = off;      off += 2 * band_h + 32;    // row spans and stencil half-widths
    L.prange = off;     off += (nfrm + rows - 1) / rows + 1;   // per phase: first column | width << 16
    L.fin = off;        off += nfin;
    if (tab_lds) off = (off + 3) & ~3;
    L.tab = off;        off += tab_lds ? TAB_ALL : 0;
    L.total_bytes = 4 * off;
    return L;
}


constexpr int MAX_BANDS_ADJ = 1024;   // per theta
constexpr int ADJ_BS = 256;           // threads per workgroup of the adjoint

// The adjoint applies the transposed PSF stencil in separable form.  For a
// lattice row of phase ph (row index mod s) the pixel rows within reach sit
// at lags d = 0..D (pixel row = current step - d) and vertical offsets
// b_d = d s + ph - pad; sorted by decreasing half-width A(|b_d|) they fall
// into groups of equal A.  Per (lattice row, pixel column) the vertical pass
// stores the running sums S_l of g(|b_d|) rbar over groups 1..l; a lattice
// point at horizontal offset t from a pixel column then takes g(|t|) S_l with
// l = number of groups whose A >= |t|.
struct AdjArgs {
    GridGeom geo;
    const int* aof;         // [pad + 1] stencil half-widths A(|b|)
    const int2* vt;         // [s][DSTRIDE] vertical pass: (d | group << 8 | last-of-group << 16, weight bits)
    const int4* ht;         // [s][s][KP / 2] horizontal taps in pairs: (S offset, weight bits) x 2
    int KP;                 // table stride: horizontal taps per (phase, column phase), 2 adj_kh(D)
    int nlev;               // groups (S slots) per (lattice row, pixel column)
    int rb;                 // rows of the pixel-adjoint ring buffer, D + 1 + ceil((rows - 1) / s)
    float invW;
    int D;                  // pixel-row lags of the stencil, floor(2 pad / s)
    const int2* span;       // [ny] valid column spans
    int band_h, band_w, nbx, nbands;
    int rows;               // lattice rows per phase (1..RS_CAP)
    const double* theta;
    int stride;
    const float* fbar;      // [rows][4][ny][nx] d logL / d F from the forward pass
    double* gpart;          // [rows][nbands][NCONST] per-band constant adjoints
    unsigned* counters;     // [rows], zero on entry, reset by the last band
    double* grad;           // [rows][stride]
    int accum;              // 1: add the gradient to grad[b] instead of storing it
};

struct AdjLayout {              // LDS carve-up of the adjoint (4-byte words), host and device
    int tab, ring, S, vt, ht, red, span, aof, prange, total_bytes;
};

// tab_lds: the special-function tables get an LDS copy (the luminosity-
// weighted body, which evaluates the model twice per lattice point and runs
// faster so); the other bodies read the constant-memory tables through the
// vector L1 cache, which leaves the LDS for more lattice rows per phase
__host__ __device__ inline AdjLayout adj_layout(int band_h, int band_w, int s, int pad, int D, int rows, int nlev,
                                                int rb, int KP, bool tab_lds) {
    // a band of band_h x band_w pixels owns at most band_h s + 2 pad + 1
    // lattice rows, reached by at most band_h + D + 1 pixel rows (and columns)
    const int nrf = band_h + D + 1, ncf = band_w + D + 1;
    AdjLayout L;
    int off = 0;
    L.tab = off;  off += tab_lds ? TAB_ALL : 0;
    off = (off + 3) & ~3;
    L.ring = off; off += rb * ncf * 4;                             // float4 [rb][frame columns]
    L.S = off;    off += rows * (ncf + 2 * D) * nlev * 4;          // float4 [rows][frame columns + 2D][nlev]
    L.ht = off;   off += s * s * KP * 2;                           // int4 [s][s][KP / 2]
    L.vt = off;   off += s * DSTRIDE * 2;                          // int2 [s][DSTRIDE]
    off = (off + 1) & ~1;
    L.red = off;  off += (ADJ_BS / 64) * NCONST * 2;               // doubles, one row per wave
    L.span = off; off += 2 * nrf;
    L.aof = off;  off += pad + 1;
    const int nch = (band_h * s + 2 * pad + 1 + rows - 1) / rows + 1;
    L.prange = off; off += nch;                                    // per phase: first column | width << 16
    L.total_bytes = 4 * off;
    return L;
}

// tap pairs of the adjoint's horizontal table for lag depth D (a compile-time
// stride of the adjoint kernel; the D + 1 taps fill the first ceil((D + 1) / 2))
__host__ __device__ constexpr int adj_kh(int D) { return D <= 6 ? 4 : 6; }

constexpr int MULTI_BS = 256;   // threads per workgroup of the many-grid launch

// launch entry points (each defined in one kernel translation unit); they
// enqueue one launch on the stream and return hipGetLastError()
// bonly: the light-only body (a grid whose only valid map is B; log-likelihood
// modes of map averaging only, else hipErrorInvalidValue)
template <int MODE, int LW>
hipError_t launch_fwd(int bulge, int ndisc, int halo, int bonly, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                      const FwdArgs& a);
template <int LW>
hipError_t launch_multi(dim3 grid, dim3 block, size_t lds, hipStream_t st, const FwdArgs* grids, const int4* items,
                        const double* theta, int stride, double* logL);
// bonly: the light-only reverse model (a grid whose only valid map is B; map
// averaging only, else hipErrorInvalidValue)
template <int LW, int KH>
hipError_t launch_adj_lw(int bulge, int ndisc, int halo, int bonly, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                         const AdjArgs& a);

}  // namespace gk
