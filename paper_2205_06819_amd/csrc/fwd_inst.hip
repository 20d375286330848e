// Instantiations of the single-grid forward kernel for one (MODE, LW) pair:
// this file is compiled once per pair (-DGK_MODE=0|1|2 -DGK_LW=0|1), so the
// 24 component sets x 6 pairs build in parallel; the log-likelihood modes of
// map averaging also carry the light-only body for the 8 (bulge, discs) sets.
#include "gk_fwd.h"

#ifndef GK_MODE
#error "compile with -DGK_MODE=<0|1|2> -DGK_LW=<0|1>"
#endif

namespace gk {

template <int MODE, int LW>
hipError_t launch_fwd(int bulge, int nd, int halo, int bonly, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                      const FwdArgs& a) {
#if GK_MODE != 2 && GK_LW == 0
    // light-only body: the halo does not enter B
    if (bonly) {
#define GK_BLAUNCH(BU, ND)                                                                       \
        if (bulge == BU && nd == ND) {                                                           \
            hipLaunchKernelGGL((fwd_kernel<BU, ND, 0, MODE, LW, 1>), grid, block, lds, st, a);  \
            return hipGetLastError();                                                            \
        }
        GK_BLAUNCH(1, 0) GK_BLAUNCH(1, 1) GK_BLAUNCH(1, 2)
        GK_BLAUNCH(2, 0) GK_BLAUNCH(2, 1) GK_BLAUNCH(2, 2)
        GK_BLAUNCH(0, 1) GK_BLAUNCH(0, 2)
#undef GK_BLAUNCH
        return hipErrorInvalidValue;
    }
#else
    if (bonly) return hipErrorInvalidValue;
#endif
#define GK_LAUNCH(BU, ND, HA)                                                               \
    if (bulge == BU && nd == ND && halo == HA) {                                             \
        hipLaunchKernelGGL((fwd_kernel<BU, ND, HA, MODE, LW>), grid, block, lds, st, a);    \
        return hipGetLastError();                                                            \
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

template hipError_t launch_fwd<GK_MODE, GK_LW>(int, int, int, int, dim3, dim3, size_t, hipStream_t, const FwdArgs&);

}  // namespace gk
