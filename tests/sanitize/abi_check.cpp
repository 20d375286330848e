// Host paths of the C ABI (include/galkin.h) under AddressSanitizer and
// UndefinedBehaviorSanitizer, which instrument host code only (the kernels are
// built as usual).  Always: argument validation of every entry point.  With a
// GPU present, also: grid creation across descriptor edge cases, the set_data
// host path (masks, non-finite entries, a map without valid pixels), launch
// and adjoint shape rules, the batched calls on device buffers, the many-grid
// plan cache (build, reuse, eviction on a mask change and on destroy), the
// allocation-free entry point's size check, and the data-preparation calls.
// Exit status 0 when every check passed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "galkin.h"

static int g_fail = 0, g_checks = 0;
#define CHECK(cond)                                                                              \
    do {                                                                                         \
        ++g_checks;                                                                              \
        if (!(cond)) {                                                                           \
            std::fprintf(stderr, "CHECK failed at line %d: %s [last_error: %s]\n", __LINE__,    \
                         #cond, last_error());                                                   \
            ++g_fail;                                                                            \
        }                                                                                        \
    } while (0)

static gk_grid_desc make(int nx, int ny, int s, double sig, int bulge, int nd, int halo) {
    gk_grid_desc d;
    std::memset(&d, 0, sizeof d);
    d.nx = nx;
    d.ny = ny;
    d.pixel_kpc = 0.2;
    d.supersample = s;
    d.psf_sigma_px = sig;
    d.bulge = bulge;
    d.n_discs = nd;
    d.halo = halo;
    d.hubble_h = 0.7;
    d.psf_mode = GK_PSF_MAPS;
    return d;
}

static void validation() {
    gk_grid_t g = nullptr;
    CHECK(create_grid(nullptr, 4, &g) == GK_EINVAL);
    CHECK(last_error() != nullptr && std::strlen(last_error()) > 0);
    const gk_grid_desc good = make(10, 10, 3, 1.0, GK_BULGE_HERNQUIST, 1, GK_HALO_NFW);
    CHECK(create_grid(&good, 4, nullptr) == GK_EINVAL);
    CHECK(create_grid(&good, 0, &g) == GK_EINVAL);
    CHECK(create_grid(&good, (1 << 20) + 1, &g) == GK_EINVAL);
    std::vector<gk_grid_desc> bad;
    for (int k = 0; k < 16; ++k) bad.push_back(good);
    bad[0].nx = 0;
    bad[1].ny = 5000;
    bad[2].supersample = 2;
    bad[3].supersample = 17;
    bad[4].psf_sigma_px = -1.0;
    bad[5].psf_sigma_px = NAN;
    bad[6].n_discs = 3;
    bad[7].halo = 7;
    bad[8].bulge = 3;
    bad[9].bulge = GK_BULGE_NONE;
    bad[9].n_discs = 0;
    bad[10].pixel_kpc = 0.0;
    bad[11].pixel_kpc = INFINITY;
    bad[12].psf_mode = 2;
    bad[13].frame_px_kpc = -1.0;
    bad[14].frame_dx = NAN;
    bad[15].hubble_h = 0.0;
    for (const auto& d : bad) CHECK(create_grid(&d, 4, &g) == GK_EINVAL);
    CHECK(destroy_grid(nullptr) == GK_EINVAL);
    CHECK(n_params(nullptr) == GK_EINVAL);
    CHECK(set_data(nullptr, nullptr, nullptr, 0, nullptr) == GK_EINVAL);
    CHECK(loglike_batch(nullptr, nullptr, 1, 13, nullptr, nullptr) == GK_EINVAL);
    CHECK(loglike_batch_noalloc(nullptr, nullptr, 1, 13, nullptr, nullptr) == GK_EINVAL);
    CHECK(loglike_grad_batch(nullptr, nullptr, 1, 13, nullptr, nullptr, nullptr) == GK_EINVAL);
    CHECK(eval_maps(nullptr, nullptr, 1, 13, nullptr, nullptr) == GK_EINVAL);
    CHECK(hmc_leapfrog(nullptr, nullptr, nullptr, nullptr, 0.1, 2, 1, 13, nullptr, nullptr, nullptr) == GK_EINVAL);
    CHECK(loglike_joint(nullptr, 1, nullptr, 1, 13, nullptr, nullptr, nullptr) == GK_EINVAL);
    CHECK(loglike_joint(nullptr, 0, nullptr, 1, 13, nullptr, nullptr, nullptr) == GK_EINVAL);
    CHECK(loglike_multi(nullptr, -1, nullptr, nullptr, 13, nullptr, nullptr, nullptr) == GK_EINVAL);
    CHECK(loglike_multi(nullptr, 0, nullptr, nullptr, 13, nullptr, nullptr, nullptr) == GK_OK);
    gk_grid_t nulls[2] = {nullptr, nullptr};
    int offs[3] = {0, 1, 2};
    CHECK(loglike_multi(nulls, 2, nullptr, offs, 13, nullptr, nullptr, nullptr) == GK_EINVAL);
    int offs_bad[3] = {1, 1, 2};
    CHECK(loglike_multi(nulls, 2, nullptr, offs_bad, 13, nullptr, nullptr, nullptr) == GK_EINVAL);
    CHECK(set_launch_shape(nullptr, 1, 1, 1, 0) == GK_EINVAL);
    int h, w, st;
    CHECK(get_launch_shape(nullptr, 1, &h, &w, &st) == GK_EINVAL);
    CHECK(set_adjoint_shape(nullptr, 8, 8, 0) == GK_EINVAL);
    CHECK(get_adjoint_shape(nullptr, &h, &w, &st) == GK_EINVAL);
    CHECK(ml_from_colour(nullptr, nullptr, nullptr, nullptr, 4, 0.0, 1.0, 0.1, nullptr, nullptr, nullptr) == GK_EINVAL);
    CHECK(ml_from_colour(nullptr, nullptr, nullptr, nullptr, 0, 0.0, 1.0, 0.1, nullptr, nullptr, nullptr) == GK_OK);
    CHECK(ml_from_colour(nullptr, nullptr, nullptr, nullptr, -1, 0.0, 1.0, 0.1, nullptr, nullptr, nullptr) == GK_EINVAL);
    CHECK(brightness_errors(nullptr, 4, 0.05, 0.1, nullptr, nullptr) == GK_EINVAL);
    CHECK(brightness_errors(nullptr, -1, 0.05, 0.1, nullptr, nullptr) == GK_EINVAL);
}

// data maps [4][ny][nx] with a smooth pattern, some masked entries
static void maps(int nx, int ny, std::vector<float>& v, std::vector<float>& e, bool holes) {
    const size_t n = (size_t)nx * ny;
    v.assign(4 * n, 0.f);
    e.assign(4 * n, 0.f);
    for (int m = 0; m < 4; ++m)
        for (size_t i = 0; i < n; ++i) {
            const float x = (float)(i % nx) - 0.5f * nx, y = (float)(i / nx) - 0.5f * ny;
            const float r = std::sqrt(x * x + y * y);
            v[m * n + i] = m == 0 ? 100.f * std::exp(-0.2f * r) : m == 1 ? 3.f * x : m == 2 ? 80.f : 2.f;
            e[m * n + i] = m == 0 ? 5.f : m == 3 ? 0.2f : 10.f;
        }
    if (holes && n > 8) {
        v[0] = NAN;
        v[n + 3] = INFINITY;
        e[2 * n + 5] = -1.f;
        e[3 * n + 7] = NAN;
        for (size_t i = 0; i < n; ++i) e[3 * n + i] = 0.f;      // M/L map fully masked
    }
}

template <class T>
static T* dev(const std::vector<T>& h) {
    T* p = nullptr;
    if (hipMalloc((void**)&p, sizeof(T) * std::max<size_t>(1, h.size())) != hipSuccess) return nullptr;
    if (!h.empty()) (void)hipMemcpy(p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice);
    return p;
}

static void with_device() {
    const int P = 17;
    std::vector<double> th(8 * P);
    const double row[P] = {0.3, -0.2, 40.0, 55.0, 10.0, 0.8, 3.0, 10.2, 1.5, 2.0, 0.8, 10.8, 4.0, 3.0, 0.3, 12.0, 10.0};
    for (int b = 0; b < 8; ++b)
        for (int k = 0; k < P; ++k) th[b * P + k] = row[k] + 0.01 * b;
    th[3 * P + 3] = 95.0;                                   // outside the domain
    double* d_th = dev(th);
    double* d_l = dev(std::vector<double>(64));
    double* d_g = dev(std::vector<double>(64 * P));
    CHECK(d_th && d_l && d_g);

    // grids across descriptor edge cases
    const gk_grid_desc descs[] = {
        make(30, 24, 3, 1.06, GK_BULGE_HERNQUIST, 2, GK_HALO_NFW),
        make(1, 1, 3, 1.0, GK_BULGE_HERNQUIST, 2, GK_HALO_NFW),
        make(17, 1, 1, 1.5, GK_BULGE_JAFFE, 2, GK_HALO_NFW),
        make(12, 9, 5, 1.6986, GK_BULGE_HERNQUIST, 2, GK_HALO_NFW),      // widest stencil
        make(9, 7, 15, 0.3, GK_BULGE_HERNQUIST, 2, GK_HALO_NFW),
        make(385, 385, 1, 0.0, GK_BULGE_HERNQUIST, 2, GK_HALO_NFW),      // beyond the old 384 px limit
    };
    std::vector<gk_grid_t> grids;
    for (const auto& d : descs) {
        gk_grid_t g = nullptr;
        CHECK(create_grid(&d, 64, &g) == GK_OK);
        CHECK(n_params(g) == P);
        std::vector<float> v, e;
        maps(d.nx, d.ny, v, e, true);
        CHECK(loglike_batch(g, d_th, 8, P, d_l, nullptr) == GK_ESTATE);
        CHECK(set_data(g, v.data(), e.data(), 0, nullptr) == GK_OK);
        CHECK(set_data(g, nullptr, e.data(), 0, nullptr) == GK_EINVAL);
        CHECK(loglike_batch(g, d_th, 8, P, d_l, nullptr) == GK_OK);
        CHECK(loglike_batch(g, d_th, 0, P, d_l, nullptr) == GK_OK);
        CHECK(loglike_batch(g, d_th, 65, P, d_l, nullptr) == GK_EINVAL);
        CHECK(loglike_batch(g, d_th, 8, P - 1, d_l, nullptr) == GK_EINVAL);
        CHECK(loglike_batch(g, nullptr, 8, P, d_l, nullptr) == GK_EINVAL);
        CHECK(loglike_grad_batch(g, d_th, 8, P, d_l, d_g, nullptr) == GK_OK);
        CHECK(loglike_grad_batch(g, d_th, 8, P, d_l, nullptr, nullptr) == GK_EINVAL);
        CHECK(loglike_batch_noalloc(g, d_th, 8, P, d_l, nullptr) == GK_OK);
        CHECK(hipDeviceSynchronize() == hipSuccess);
        std::vector<double> l(8);
        (void)hipMemcpy(l.data(), d_l, sizeof(double) * 8, hipMemcpyDeviceToHost);
        CHECK(std::isinf(l[3]) && l[3] < 0);
        CHECK(std::isfinite(l[0]));
        grids.push_back(g);
    }
    gk_grid_t g0 = grids[0];
    int h, w, st;
    CHECK(set_launch_shape(g0, 1, 5, 7, 9) == GK_EINVAL);
    CHECK(set_launch_shape(g0, 1, 5, 7, 2) == GK_OK);
    CHECK(get_launch_shape(g0, 3, &h, &w, &st) == GK_OK && h == 5 && w == 7 && st == 2);
    CHECK(get_launch_shape(g0, 0, &h, &w, &st) == GK_EINVAL);
    CHECK(set_adjoint_shape(g0, 8, 200, 0) == GK_OK);        // clipped to the grid's 30 columns
    CHECK(get_adjoint_shape(g0, &h, &w, &st) == GK_OK && w == 30);
    CHECK(set_adjoint_shape(grids[5], 8, 200, 0) == GK_EINVAL);   // 200 columns of a 385-wide grid > 128
    CHECK(set_adjoint_shape(g0, 8, 8, 17) == GK_EINVAL);
    CHECK(set_adjoint_shape(g0, 3, 3, 2) == GK_OK);         // more bands: partials grow
    CHECK(get_adjoint_shape(g0, &h, &w, &st) == GK_OK && h == 3 && w == 3 && st == 2);
    CHECK(loglike_grad_batch(g0, d_th, 8, P, d_l, d_g, nullptr) == GK_OK);
    CHECK(hmc_leapfrog(g0, d_th, d_g, d_l, -1.0, 2, 8, P, d_l, d_g, nullptr) == GK_EINVAL);
    CHECK(hmc_leapfrog(g0, d_th, d_g, d_l, 0.1, 0, 8, P, d_l, d_g, nullptr) == GK_EINVAL);
    // the allocation-free call rejects requests beyond its scratch
    gk_grid_t gbig = nullptr;
    gk_grid_desc dbig = make(80, 80, 3, 1.06, GK_BULGE_HERNQUIST, 2, GK_HALO_NFW);
    CHECK(create_grid(&dbig, 8192, &gbig) == GK_OK);
    std::vector<float> v, e;
    maps(80, 80, v, e, false);
    CHECK(set_data(gbig, v.data(), e.data(), 0, nullptr) == GK_OK);
    for (int bm : {1, 32, 512, 4096}) CHECK(set_launch_shape(gbig, bm, 4, 4, 0) == GK_OK);
    CHECK(loglike_batch_noalloc(gbig, d_th, 8192, P, d_l, nullptr) == GK_EINVAL);
    CHECK(destroy_grid(gbig) == GK_OK);
    // many-grid plans: build, reuse, drop on a mask change, drop on destroy
    gk_grid_t mg[3] = {grids[0], grids[3], grids[4]};
    int moff[4] = {0, 3, 5, 8};
    CHECK(loglike_multi(mg, 3, d_th, moff, P, d_l, nullptr, nullptr) == GK_OK);
    CHECK(loglike_multi(mg, 3, d_th, moff, P, d_l, nullptr, nullptr) == GK_OK);
    int moff_bad[4] = {0, 3, 2, 8};
    CHECK(loglike_multi(mg, 3, d_th, moff_bad, P, d_l, nullptr, nullptr) == GK_EINVAL);
    gk_grid_t dup[2] = {grids[0], grids[0]};
    int doff[3] = {0, 1, 2};
    CHECK(loglike_multi(dup, 2, d_th, doff, P, d_l, nullptr, nullptr) == GK_EINVAL);
    maps(descs[3].nx, descs[3].ny, v, e, false);            // M/L map valid again: mask changes
    CHECK(set_data(grids[3], v.data(), e.data(), 0, nullptr) == GK_OK);
    CHECK(loglike_multi(mg, 3, d_th, moff, P, d_l, d_g, nullptr) == GK_OK);
    CHECK(loglike_joint(mg, 2, d_th, 8, P, d_l, d_g, nullptr) == GK_OK);
    CHECK(hipDeviceSynchronize() == hipSuccess);
    // data preparation on small arrays
    std::vector<float> mb(13, 16.f), mgm(13, 15.f), em(13, 0.05f);
    mb[4] = NAN;
    float *a = dev(mb), *b = dev(mgm), *c = dev(em), *o1 = dev(em), *o2 = dev(em);
    CHECK(ml_from_colour(a + 1, b, c, c, 12, -0.7, 0.9, 0.07, o1, o2, nullptr) == GK_OK);   // unaligned path
    CHECK(ml_from_colour(a, b, c, c, 13, -0.7, 0.9, 0.07, o1, o2, nullptr) == GK_OK);
    CHECK(brightness_errors(a, 13, 0.05, 0.1, o2, nullptr) == GK_OK);
    CHECK(hipDeviceSynchronize() == hipSuccess);
    for (float* p : {a, b, c, o1, o2}) (void)hipFree(p);
    for (gk_grid_t g : grids) CHECK(destroy_grid(g) == GK_OK);
    (void)hipFree(d_th);
    (void)hipFree(d_l);
    (void)hipFree(d_g);
}

int main() {
    validation();
    int ndev = 0;
    const bool device = hipGetDeviceCount(&ndev) == hipSuccess && ndev > 0;
    if (device) with_device();
    std::printf("%s: %d checks, %d failed\n", device ? "device checks" : "validation only (no device)", g_checks,
                g_fail);
    return g_fail ? 1 : 0;
}
