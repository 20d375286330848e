// Instantiations of the single-grid forward kernel for one (MODE, LW) pair:
// this file is compiled once per pair (-DGK_MODE=0|1|2 -DGK_LW=0|1), so the
// 24 component sets x 6 pairs build in parallel.
#include "gk_fwd.h"

#ifndef GK_MODE
#error "compile with -DGK_MODE=<0|1|2> -DGK_LW=<0|1>"
#endif

namespace gk {

template <int MODE, int LW>
hipError_t launch_fwd(int bulge, int nd, int halo, dim3 grid, dim3 block, size_t lds, hipStream_t st,
                      const FwdArgs& a) {
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

template hipError_t launch_fwd<GK_MODE, GK_LW>(int, int, int, dim3, dim3, size_t, hipStream_t, const FwdArgs&);

}  // namespace gk
