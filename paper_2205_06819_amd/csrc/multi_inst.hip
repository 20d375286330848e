// The many-grid forward kernel (one launch per catalogue), compiled once per
// PSF mode (-DGK_LW=0|1).
#include "gk_fwd.h"

#ifndef GK_LW
#error "compile with -DGK_LW=<0|1>"
#endif

namespace gk {

// ============================================================================
// many grids in one launch: workgroup i takes work item i (grid, parameter row
// within the grid, band, first row of the grid in the batch); the host orders
// the items by decreasing cost, so the dispatcher hands out the longest items
// first and the short ones fill the tail.  (A persistent loop over an atomic
// queue kept loop-invariant state live across items: 206 instead of 125 VGPRs,
// half the occupancy, and slower overall.)  The special-function tables are
// copied to LDS: the registers cap the occupancy at four waves per SIMD, which
// the small bands' LDS with the copy still allows.
// ============================================================================
typedef const __attribute__((address_space(4))) int* const_word_ptr;

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
        fwd_band<BU, ND, HA, MODE_LOGL, LW, 0, 1>(a, row, band, smem);                         \
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

template <int LW>
hipError_t launch_multi(dim3 grid, dim3 block, size_t lds, hipStream_t st, const FwdArgs* grids, const int4* items,
                        const double* theta, int stride, double* logL) {
    hipLaunchKernelGGL(multi_kernel<LW>, grid, block, lds, st, grids, items, theta, stride, logL);
    return hipGetLastError();
}

template hipError_t launch_multi<GK_LW>(dim3, dim3, size_t, hipStream_t, const FwdArgs*, const int4*, const double*,
                                        int, double*);

}  // namespace gk
