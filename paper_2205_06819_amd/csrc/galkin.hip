// galkin: host side of the C ABI (include/galkin.h) for gfx950: grid
// descriptors, stencil tables, data upload, launch shapes, the many-grid work
// plans, the HMC trajectory and the data-preparation kernels.  The likelihood
// kernels live in their own translation units (fwd_inst.hip, multi_inst.hip,
// adj.hip) behind the launch entry points of gk_kern.h.
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
#include "gk_kern.h"

namespace gk {

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

// Zero n counters (a kernel rather than a memset, so that callers may capture
// the enqueueing call in a HIP graph).
__global__ void __launch_bounds__(256) zero_u32_kernel(unsigned* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// Scratch of the allocation-free entry point (loglike_batch_noalloc): the
// band partials and tickets of its launch live here instead of in the grid's
// workspace.  Each device that loads the library holds its own copy until the
// process ends.  Host code never passes this name to a kernel or a copy: it
// uses the device address that hipGetSymbolAddress returns (per device, at
// grid creation; see scratch_ptr).
constexpr size_t SCRATCH_BYTES = (size_t)16 << 20;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

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
    float* d_fbar = nullptr;        // [grad_rows][4][ny][nx] pixel adjoints of one batch chunk
    double* d_gpart = nullptr;      // [grad_rows][adj nbands][NCONST]
    int2* d_adj_vt = nullptr;       // adjoint tables (AdjArgs::vt, AdjArgs::ht)
    int2* d_adj_ht = nullptr;
    double* d_logdet = nullptr;
    std::vector<LaunchRule> rules;
    // adjoint launch: bands of adj_band_h x adj_band_w pixels, adj_rows lattice
    // rows per phase; gradients of larger batches run in chunks of grad_rows
    int adj_band_h = 0, adj_band_w = 0, adj_rows = 1, adj_nbands = 0, adj_lds = 0;
    int adj_KP = 2, adj_nlev = 1, grad_rows = 1, gpart_bands = 0;   // gpart_bands: d_gpart capacity per row
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
                    g->d_span, g->d_partials, g->d_counters, g->d_fbar, g->d_gpart, g->d_logdet,
                    g->d_adj_vt, g->d_adj_ht};
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
    // Large batches: bands of up to 80 x 40 pixels (measured best on the 3x3
    // lattice: enough workgroups per CU to overlap one band's model phase with
    // another's stencil phase).  Small batches: small square bands so that one
    // theta spreads over many CUs.
    const int nx = g->d.nx, ny = g->d.ny;
    g->rules.clear();
    // the grid split into near-equal bands of at most 80 rows and 40 columns
    // (on the 80 x 80 realistic cube 0.556 ms per 1024 vectors against 0.582
    // for 40 x 40 bands; the luminosity-weighted mode, whose phases end in a
    // moment exchange, 0.583 against 0.606); a wide PSF on a coarse lattice
    // (lag D >= 9 pixel rows, e.g. no supersampling, or 5x5 supersampling of a
    // 4 px FWHM) spends D of every band_h + D steps filling the lag and
    // recomputes a 2 pad halo, so there bands grow to 32 D rows and 64 columns
    // (measured 1.4x faster on a 160 x 160 grid with D = 10; on the 300 x 300,
    // s = 5 grid 300 x 64 bands take 139.7 ms per 8192 vectors against 143.6
    // for 150 x 64 and 154.8 for 300 x 50); a grid with at least four full
    // 64-pixel bands uses exactly 64 columns, so that the stencil phase's
    // 4 x 64 threads are whole waves (the narrower last band costs less; with
    // fewer bands an even split measured faster)
    const int hmax = g->D >= 9 ? 32 * g->D : 80, wmax = g->D >= 9 ? 64 : 40;
    int bh = (ny + (ny + hmax - 1) / hmax - 1) / ((ny + hmax - 1) / hmax);
    int bw = (nx + (nx + wmax - 1) / wmax - 1) / ((nx + wmax - 1) / wmax);
    if (g->D >= 9 && nx >= 4 * 64) bw = 64;
    fit_shape(g, bh, bw, 0);
    // pixel-row steps per model phase: make_cfg's default (three on the 3x3
    // lattice: 0.556 ms against 0.570 for two on the realistic cube)
    g->rules.push_back({512, bh, bw, 0});
    // >= 4096 vectors fill the chip without splitting a grid finely: bands of
    // up to 128 rows and 64 columns recompute less of the stencil halo
    // (measured 1.45x faster than 34 x 34 bands on a 100 x 100 grid, B = 4096)
    if (g->D < 9) {
        const int hb = 128, wb = 64;
        int bh2 = (ny + (ny + hb - 1) / hb - 1) / ((ny + hb - 1) / hb);
        int bw2 = (nx + (nx + wb - 1) / wb - 1) / ((nx + wb - 1) / wb);
        fit_shape(g, bh2, bw2, 0);
        g->rules.push_back({4096, bh2, bw2, 0});
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

// ---------------------------------------------------------------------------
// adjoint launch shape
// ---------------------------------------------------------------------------
// LDS of one adjoint workgroup: at most 80 KiB (two per CU); shapes within
// 53 KiB (three per CU) are preferred by the default rule
constexpr int ADJ_LDS_MAX = 80 * 1024;
constexpr int ADJ_LDS_3 = 53 * 1024;

static int adj_ring_rows(const gk_grid* g, int rows) { return g->D + 1 + (rows - 1 + g->geo.s - 1) / g->geo.s; }

static int adj_lds_of(const gk_grid* g, int bh, int bw, int rows) {
    return adj_layout(bh, bw, g->geo.s, g->geo.pad, g->D, rows, g->adj_nlev, adj_ring_rows(g, rows), g->adj_KP,
                      g->geo.lw != 0)
        .total_bytes;
}

// Fraction of the workgroup's thread slots busy in a phase of `rows` lattice
// rows, over the column bands of width bw (a phase covers rows x the band's
// owned lattice columns, spread flat over the threads)
static double adj_fill(const gk_grid* g, int bw, int rows) {
    const int nx = g->d.nx, s = g->geo.s, pad = g->geo.pad;
    const int NLC = (nx - 1) * s + 2 * pad + 1, own = pad - s / 2;
    double pts = 0.0, slots = 0.0;
    for (int c0 = 0; c0 < nx; c0 += bw) {
        const int c1 = std::min(nx, c0 + bw);
        const int lo = c0 == 0 ? 0 : c0 * s + own, hi = c1 == nx ? NLC : c1 * s + own;
        const int p = rows * (hi - lo);
        pts += p;
        slots += (double)((p + ADJ_BS - 1) / ADJ_BS) * ADJ_BS;
    }
    return pts / slots;
}

// Install an adjoint shape (band_h x band_w pixels, `rows` lattice rows per
// phase, 0 = chosen here) if it fits the kernel's limits.
static int set_adj_shape(gk_grid* g, int bh, int bw, int rows) {
    bh = std::min(bh, g->d.ny);
    bw = std::min(bw, g->d.nx);
    if (bh < 1 || bw < 1) return fail(GK_EINVAL, "adjoint band must be at least 1 x 1");
    if (bw > 128) return fail(GK_EINVAL, "adjoint band_w %d > 128", bw);
    const int nb = ((g->d.nx + bw - 1) / bw) * ((g->d.ny + bh - 1) / bh);
    if (nb > MAX_BANDS_ADJ) return fail(GK_EINVAL, "adjoint shape gives %d bands (> %d)", nb, MAX_BANDS_ADJ);
    if (rows < 0 || rows > RS_CAP) return fail(GK_EINVAL, "adjoint rows must be in [0, %d]", RS_CAP);
    int best = 0;
    if (rows > 0) {
        best = adj_lds_of(g, bh, bw, rows) <= ADJ_LDS_MAX ? rows : 0;
    } else {
        // the most rows, up to 3, that keep >= 85 % of the threads busy, else
        // the best thread fill, among the shapes that leave room for three
        // workgroups per CU, else among those that fit at all
        for (int cap : {ADJ_LDS_3, ADJ_LDS_MAX}) {
            double fill = -1.0;
            int r85 = 0, rfill = 0;
            for (int r = 1; r <= RS_CAP; ++r) {
                if (adj_lds_of(g, bh, bw, r) > cap) break;
                const double f = adj_fill(g, bw, r);
                if (r <= 3 && f >= 0.85) r85 = r;
                if (f > fill + 1e-9) {
                    fill = f;
                    rfill = r;
                }
            }
            best = r85 ? r85 : rfill;
            if (best) break;
        }
    }
    if (!best) return fail(GK_EINVAL, "adjoint band %d x %d needs more than %d KiB of LDS", bh, bw, ADJ_LDS_MAX / 1024);
    g->adj_band_h = bh;
    g->adj_band_w = bw;
    g->adj_rows = best;
    g->adj_nbands = nb;
    g->adj_lds = adj_lds_of(g, bh, bw, best);
    return GK_OK;
}

// Default adjoint shape (measured on the 80 x 80, 160 x 160 and 300 x 300
// benchmark grids).  Rows per phase matter most: each phase costs two
// barriers and a vertical pass over the frame's columns, so the rule takes
// the most rows, up to 3, that keep >= 85 % of the threads busy within the
// LDS that leaves room for three workgroups per CU (on the 300 x 300 grid 3
// rows per phase take about 30 % less time than 1).  For that row count, a band's
// block reads a halo of D + 1 pixel columns and rows and restarts its ring,
// so wide and tall bands are cheapest: widths from even splits of the
// columns (at most 128, the kernel's limit, and at least 4 (D + 1) so that
// the halo stays within a quarter of the band) and from 256 / (s r) (a phase
// of r lattice rows then fills the threads once), widest first, then the
// tallest bands for which a vector still spans at least two bands (more
// workgroups) and the grid at most MAX_BANDS_ADJ bands (on a 100 x 100 grid,
// B = 4096, a gradient with bands of 50 x 100 pixels takes 0.94 of the time
// with 100 x 50).  A grid whose adjoint fits no shape keeps
// adj_nbands = 0: its forward calls work and its gradient calls return
// GK_EINVAL.
static int default_adj_shape(gk_grid* g) {
    const int nx = g->d.nx, ny = g->d.ny, s = g->geo.s;
    const std::string saved = g_err;
    auto split = [](int n, int m) { const int k = (n + m - 1) / m; return (n + k - 1) / k; };
    std::vector<int> widths;
    for (int m : {128, 80, 64, 40, 32, 20, 16, 8}) widths.push_back(split(nx, m));
    for (int r = 1; r <= 4; ++r)
        if (256 / (s * r) >= 8) widths.push_back(std::min(nx, 256 / (s * r)));
    std::sort(widths.begin(), widths.end(), [](int x, int y) { return x > y; });
    widths.erase(std::unique(widths.begin(), widths.end()), widths.end());
    const bool big = nx >= 40 || ny >= 40;          // room for two bands
    auto try_set = [&](int bh, int bw, int rows) {
        if (set_adj_shape(g, bh, bw, rows) != GK_OK) return false;
        g_err = saved;
        return true;
    };
    for (int cap : {ADJ_LDS_3, ADJ_LDS_MAX})
        for (int pass = 0; pass < 2; ++pass)        // pass 1: single-band shapes allowed
            for (int rows = 3; rows >= 1; --rows)
                for (int bw : widths) {
                    if (bw > 128 || (bw < 4 * (g->D + 1) && bw < nx) || adj_fill(g, bw, rows) < 0.85) continue;
                    for (int hmax : {4096, 2048, 1024, 512, 256, 128, 64}) {
                        const int bh = split(ny, hmax);
                        const int nb = ((nx + bw - 1) / bw) * ((ny + bh - 1) / bh);
                        if (nb > MAX_BANDS_ADJ || (pass == 0 && big && nb < 2)) continue;
                        if (adj_lds_of(g, bh, bw, rows) <= cap && try_set(bh, bw, rows)) return GK_OK;
                    }
                }
    // nothing reached the fill target: the best fill of the default heights
    for (int cap : {ADJ_LDS_3, ADJ_LDS_MAX})
        for (int hmax = 64; hmax <= 4096; hmax *= 2) {
            const int bh = split(ny, hmax);
            int bbw = 0, brows = 0;
            double bfill = -1.0;
            for (int bw : widths) {
                if (((nx + bw - 1) / bw) * ((ny + bh - 1) / bh) > MAX_BANDS_ADJ) continue;
                for (int r = 1; r <= RS_CAP; ++r) {
                    if (adj_lds_of(g, bh, bw, r) > cap) break;
                    const double f = adj_fill(g, bw, r);
                    if (f > bfill + 1e-9) {
                        bfill = f;
                        bbw = bw;
                        brows = r;
                    }
                }
            }
            if (bbw && try_set(bh, bbw, brows)) return GK_OK;
        }
    g_err = saved;
    g->adj_nbands = 0;
    return GK_OK;
}

struct LaunchCfg {
    int band_h, band_w, nbx, nbands, BS, gsub, xw, lds;
    int lds_tab;    // with the LDS copy of the tables (many-grid kernel, luminosity-weighted seed pass)
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
    // the 3x3 lattice with 80x40 bands), at most RS_CAP lattice rows, the row
    // buffer within ~40 KiB of LDS (64 KiB for an explicit count) and, with
    // the LDS copy of the tables, within 80 KiB; an explicit count is honoured
    // up to those limits
    const int nfrm = nfr_max(band_h, s, pad);
    int gs = steps > 0 ? steps : std::max(1, (10 + s / 2) / s);
    gs = std::min({gs, GSUB_CAP, std::max(1, RS_CAP / s)});
    const int lw = g->geo.lw;
    auto lds_of = [&](int gsub, bool tab) {
        return make_layout(gsub * s, c.xw, nfrm, band_h, lw ? 8 * gsub * band_w : 0, tab).total_bytes;
    };
    while (gs > 1 && (lds_of(gs, false) > (steps > 0 ? 64 : 40) * 1024 || lds_of(gs, true) > 80 * 1024)) --gs;
    c.gsub = gs;
    c.lds = lds_of(gs, false);
    c.lds_tab = lds_of(gs, true);
    if (c.lds > 64 * 1024) return fail(GK_EINVAL, "launch shape needs %d bytes of LDS (> 64 KiB)", c.lds);
    if (c.lds_tab > 80 * 1024)
        return fail(GK_EINVAL, "launch shape needs %d bytes of LDS with the tables (> 80 KiB)", c.lds_tab);
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
static hipError_t enqueue_fwd(const gk_grid* g, const LaunchCfg& c, FwdArgs& a, int B, hipStream_t st) {
    if ((size_t)B * c.nbands * c.BS >= ((size_t)1 << 31)) return hipErrorInvalidConfiguration;
    const dim3 grid((unsigned)(B * c.nbands)), block((unsigned)c.BS);
    // a grid whose only valid map is B runs the light-only model
    const int bonly = MODE != MODE_MAPS && !a.geo.lw && a.map_mask == 1;
    const size_t lds = MODE == MODE_FBAR && a.geo.lw ? c.lds_tab : c.lds;
    return a.geo.lw ? launch_fwd<MODE, 1>(g->d.bulge, g->d.n_discs, g->d.halo, 0, grid, block, lds, st, a)
                    : launch_fwd<MODE, 0>(g->d.bulge, g->d.n_discs, g->d.halo, bonly, grid, block, lds, st, a);
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
    a.pstride = c.nbands;          // partials packed per vector: [B][nbands]
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
        lds = std::max(lds, c.lds_tab);
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

// Device address of `scratch` on the given device (which must be current),
// looked up once per device and kept.
constexpr int SCRATCH_MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_dev[SCRATCH_MAX_DEVICES];

static int scratch_ptr(int device, void** out) {
    if (device < 0 || device >= SCRATCH_MAX_DEVICES)
        return fail(GK_EINVAL, "device %d beyond the %d devices the scratch table covers", device,
                    SCRATCH_MAX_DEVICES);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(gk::scratch));
        if (e != hipSuccess || !p)
            return fail(GK_EHIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch_dev[device] = p;
    }
    *out = g_scratch_dev[device];
    return GK_OK;
}

int create_grid(const gk_grid_desc* desc, int max_batch, gk_grid_t* out) {
    int rc = valid_desc(desc);
    if (rc) return rc;
    if (!out) return fail(GK_EINVAL, "out is NULL");
    if (max_batch < 1 || max_batch > (1 << 20)) return fail(GK_EINVAL, "max_batch must be in [1, 2^20]");
    *out = nullptr;
    int device = 0;
    HIPCHECK(hipGetDevice(&device));
    {
        // set-up of the allocation-free entry point's scratch on this device
        void* sp = nullptr;
        rc = scratch_ptr(device, &sp);
        if (rc) return rc;
    }
    gk_grid* g = new gk_grid();
    g->d = *desc;
    g->max_batch = max_batch;
    g->device = device;
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
    // adjoint tables (transposed stencil in separable form): for each lattice
    // row phase, the lags in reach sorted by decreasing half-width and grouped
    // by equal half-width; for each (row phase, column phase) the D + 1 pixel
    // columns in reach with their weight and group count
    std::vector<int2> avt((size_t)s * DSTRIDE, make_int2(0, 0));
    std::vector<std::vector<int>> groupA(s);
    int nlev = 1;
    for (int ph = 0; ph < s; ++ph) {
        std::vector<std::pair<int, int>> lags;         // (A, d)
        for (int d = 0; d <= D; ++d) {
            const int bb = std::abs(d * s + ph - pad);
            if (bb <= pad) lags.push_back({aof[bb], d});
        }
        std::sort(lags.begin(), lags.end(), [](const std::pair<int, int>& x, const std::pair<int, int>& y) {
            return x.first != y.first ? x.first > y.first : x.second < y.second;
        });
        int grp = -1;
        for (size_t n = 0; n < lags.size(); ++n) {
            const int A = lags[n].first, d = lags[n].second;
            if (n == 0 || A != lags[n - 1].first) {
                ++grp;
                groupA[ph].push_back(A);
            }
            const int last = (n + 1 == lags.size() || lags[n + 1].first != A) ? 1 : 0;
            const float w = gw[std::abs(d * s + ph - pad)];
            int wb;
            std::memcpy(&wb, &w, 4);
            avt[(size_t)ph * DSTRIDE + n] = make_int2(d | (grp << 8) | (last << 16), wb);
        }
        nlev = std::max(nlev, (int)groupA[ph].size());
    }
    const int KP = 2 * adj_kh(D);                      // table stride, even, >= D + 1
    std::vector<int2> aht((size_t)s * s * KP, make_int2(0, 0));
    for (int ph = 0; ph < s; ++ph)
        for (int i = 0; i < s; ++i)
            for (int k = 0; k <= D; ++k) {
                const int at = std::abs(k * s + i - pad);
                int l = 0;
                for (int A : groupA[ph]) l += A >= at ? 1 : 0;
                if (l == 0) continue;
                int wb;
                std::memcpy(&wb, &gw[at], 4);
                aht[((size_t)ph * s + i) * KP + k] = make_int2(-k * nlev + (l - 1), wb);
            }
    g->adj_KP = KP;
    g->adj_nlev = nlev;
    const size_t npix = (size_t)desc->nx * desc->ny;
    // the gradient's pixel-adjoint buffer holds at most ~2 GiB: larger batches
    // run in chunks of grad_rows vectors (one forward + adjoint pair each)
    g->grad_rows = (int)std::max<size_t>(1, std::min<size_t>((size_t)max_batch,
                                                              ((size_t)2 << 30) / (16 * npix)));
    int arc = default_adj_shape(g);
    if (arc) {
        delete g;
        return arc;
    }
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
    ALLOC(g->d_fbar, sizeof(float) * 4 * npix * (size_t)g->grad_rows);
    g->gpart_bands = std::max(1, g->adj_nbands);
    ALLOC(g->d_gpart, sizeof(double) * NCONST * g->gpart_bands * (size_t)g->grad_rows);
    ALLOC(g->d_adj_vt, sizeof(int2) * avt.size());
    ALLOC(g->d_adj_ht, sizeof(int2) * aht.size());
    ALLOC(g->d_logdet, sizeof(double));
#undef ALLOC
    {
        // compile-time tap counts of the stencil (register arrays up to 26 entries
        // stay in VGPRs with uniform indexing; wider stencils are rejected above)
        static const int tpads[] = {4, 6, 9, 12, 16, 20, 25};
        g->tpad = 0;
        for (int t : tpads)
            if (t >= pad && lag_cap(t) >= D) { g->tpad = t; break; }
        if (!g->tpad) {
            free_grid(g);
            return fail(GK_EINVAL, "no compiled stencil for pad = %d and lag %d", pad, D);
        }
    }
    std::vector<float> gw64(std::max(pad + 1, 64), 0.0f);
    std::copy(gw.begin(), gw.end(), gw64.begin());
    if (hipMemcpy(g->d_gw, gw64.data(), sizeof(float) * gw64.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g->d_aof, aof.data(), sizeof(int) * (pad + 1), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g->d_tab, tab.data(), sizeof(int2) * tab.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g->d_adj_vt, avt.data(), sizeof(int2) * avt.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(g->d_adj_ht, aht.data(), sizeof(int2) * aht.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemset(g->d_counters, 0, sizeof(unsigned) * (size_t)max_batch) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        free_grid(g);
        return fail(GK_EHIP, "upload of the stencil tables failed");
    }
    default_rules(g);
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

int set_adjoint_shape(gk_grid_t g, int band_h, int band_w, int rows) {
    if (!g) return fail(GK_EINVAL, "grid is NULL");
    if (band_h < 1 || band_w < 1) return fail(GK_EINVAL, "band_h, band_w must be >= 1");
    const int old[5] = {g->adj_band_h, g->adj_band_w, g->adj_rows, g->adj_nbands, g->adj_lds};
    int rc = set_adj_shape(g, band_h, band_w, rows);   // changes g only on success
    if (rc) return rc;
    if (g->adj_nbands > g->gpart_bands) {
        // more bands than the per-band gradient partials were sized for: grow them
        double* p = nullptr;
        if (hipDeviceSynchronize() != hipSuccess ||
            hipMalloc((void**)&p, sizeof(double) * NCONST * g->adj_nbands * (size_t)g->grad_rows) != hipSuccess) {
            g->adj_band_h = old[0];
            g->adj_band_w = old[1];
            g->adj_rows = old[2];
            g->adj_nbands = old[3];
            g->adj_lds = old[4];
            return fail(GK_ENOMEM, "allocation of the adjoint's band partials failed");
        }
        (void)hipFree(g->d_gpart);
        g->d_gpart = p;
        g->gpart_bands = g->adj_nbands;
    }
    return GK_OK;
}

int get_adjoint_shape(gk_grid_t g, int* band_h, int* band_w, int* rows) {
    if (!g || !band_h || !band_w || !rows) return fail(GK_EINVAL, "NULL grid or output pointer");
    if (g->adj_nbands <= 0) return fail(GK_EINVAL, "this grid fits no adjoint band shape of this build");
    *band_h = g->adj_band_h;
    *band_w = g->adj_band_w;
    *rows = g->adj_rows;
    return GK_OK;
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
    hipError_t e = enqueue_fwd<MODE_LOGL>(g, c, a, B, st);
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

int loglike_batch_noalloc(gk_grid_t g, const double* theta, int B, int stride, double* logL, void* stream) {
    int rc = check_call(g, theta, B, stride, logL);
    if (rc) return rc;
    if (!g->has_data) return fail(GK_ESTATE, "loglike_batch_noalloc before set_data");
    if (B == 0) return GK_OK;
    int device = -1;
    if (hipGetDevice(&device) != hipSuccess) return fail(GK_EHIP, "hipGetDevice failed");
    if (device != g->device) return fail(GK_EINVAL, "grid lives on device %d, current device is %d", g->device, device);
    void* base = nullptr;
    rc = scratch_ptr(device, &base);
    if (rc) return rc;
    int bh, bw, steps;
    choose_rule(g, B, bh, bw, steps);
    LaunchCfg c;
    rc = make_cfg(g, bh, bw, c, 0, steps);
    if (rc) return rc;
    // [B] tickets, then [B][nbands] FP64 band partials
    const size_t cnt_bytes = ((size_t)B * sizeof(unsigned) + 255) & ~(size_t)255;
    const size_t need = c.nbands > 1 ? cnt_bytes + (size_t)B * c.nbands * sizeof(double) : 0;
    if (need > SCRATCH_BYTES)
        return fail(GK_EINVAL,
                    "loglike_batch_noalloc: %d vectors x %d bands need %zu bytes of scratch (limit %zu: "
                    "B x (8 bands + 4) bytes); use a smaller batch or wider bands (set_launch_shape)",
                    B, c.nbands, need, SCRATCH_BYTES);
    hipStream_t st = (hipStream_t)stream;
    FwdArgs a;
    fill_args(g, c, a, theta, stride);
    a.logL = logL;
    a.counters = (unsigned*)base;
    a.partials = (double*)((char*)base + cnt_bytes);
    a.pstride = c.nbands;
    if (c.nbands > 1) {
        // the tickets must start at zero; the previous call on this device left
        // them zero unless it was interrupted, so clear them anyway
        hipLaunchKernelGGL(zero_u32_kernel, dim3((unsigned)((B + 255) / 256)), dim3(256), 0, st, a.counters, B);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(GK_EHIP, "scratch clear failed: %s", hipGetErrorString(e));
    }
    hipError_t e = enqueue_fwd<MODE_LOGL>(g, c, a, B, st);
    if (e != hipSuccess) return fail(GK_EHIP, "forward launch failed: %s", hipGetErrorString(e));
    return GK_OK;
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
    hipError_t e = enqueue_fwd<MODE_MAPS>(g, c, a, B, (hipStream_t)stream);
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
    if (g->adj_nbands <= 0)
        return fail(GK_EINVAL, "this grid (%d x %d, s = %d) fits no adjoint band shape of this build", g->d.nx,
                    g->d.ny, g->geo.s);
    // the whole batch's forward launch shape (band partials and tickets per row)
    int bh, bw, steps;
    choose_rule(g, B, bh, bw, steps);
    LaunchCfg c;
    int rc = make_cfg(g, bh, bw, c, 0, steps);
    if (rc) return rc;
    // chunks of at most grad_rows vectors share the pixel-adjoint buffer
    for (int r0 = 0; r0 < B; r0 += g->grad_rows) {
        const int n = std::min(g->grad_rows, B - r0);
        const double* th = theta + (size_t)r0 * stride;
        // pass 1: log-likelihood and d logL / d F at every pixel
        FwdArgs fa;
        fill_args(g, c, fa, th, stride);
        fa.logL = logL + r0;
        fa.fbar = g->d_fbar;
        fa.accum = accum;
        hipError_t e = enqueue_fwd<MODE_FBAR>(g, c, fa, n, st);
        if (e != hipSuccess)
            return fail(GK_EHIP, "forward (adjoint seed) launch failed: %s", hipGetErrorString(e));
        // pass 2: transposed stencil and reverse point model per band, chain rule to theta
        AdjArgs aa;
        aa.geo = g->geo;
        aa.aof = g->d_aof;
        aa.vt = g->d_adj_vt;
        aa.ht = (const int4*)g->d_adj_ht;
        aa.KP = g->adj_KP;
        aa.nlev = g->adj_nlev;
        aa.rb = adj_ring_rows(g, g->adj_rows);
        aa.invW = g->invW;
        aa.D = g->D;
        aa.span = g->d_span;
        aa.band_h = g->adj_band_h;
        aa.band_w = g->adj_band_w;
        aa.nbx = (g->d.nx + aa.band_w - 1) / aa.band_w;
        aa.nbands = g->adj_nbands;
        aa.rows = g->adj_rows;
        aa.theta = th;
        aa.stride = stride;
        aa.fbar = g->d_fbar;
        aa.gpart = g->d_gpart;
        aa.counters = g->d_counters;
        aa.grad = grad + (size_t)r0 * stride;
        aa.accum = accum;
        if ((size_t)n * aa.nbands >= ((size_t)1 << 31)) return fail(GK_EINVAL, "adjoint grid too large");
        const dim3 grid2((unsigned)(n * aa.nbands)), block2(ADJ_BS);
        const bool kh4 = g->adj_KP == 8;
        const int bu = g->d.bulge, nd = g->d.n_discs, ha = g->d.halo;
        const int bonly = !g->geo.lw && g->map_mask == 1;     // only B has valid pixels
        if (g->geo.lw)
            e = kh4 ? launch_adj_lw<1, 4>(bu, nd, ha, 0, grid2, block2, g->adj_lds, st, aa)
                    : launch_adj_lw<1, 6>(bu, nd, ha, 0, grid2, block2, g->adj_lds, st, aa);
        else
            e = kh4 ? launch_adj_lw<0, 4>(bu, nd, ha, bonly, grid2, block2, g->adj_lds, st, aa)
                    : launch_adj_lw<0, 6>(bu, nd, ha, bonly, grid2, block2, g->adj_lds, st, aa);
        if (e != hipSuccess) return fail(GK_EHIP, "adjoint launch failed: %s", hipGetErrorString(e));
    }
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
    hipError_t e = hipSuccess;
    if (n0 > 0)
        e = launch_multi<0>(dim3((unsigned)n0), dim3(MULTI_BS), p->lds, st, p->d_args, p->d_items, theta, stride, logL);
    if (e == hipSuccess && p->n_items_lw > 0)
        e = launch_multi<1>(dim3((unsigned)p->n_items_lw), dim3(MULTI_BS), p->lds, st, p->d_args, p->d_items + n0,
                            theta, stride, logL);
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
