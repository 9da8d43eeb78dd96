// One instantiation unit of the two pass kernels, for the mask radii
// LOGFX_RA <= LOGFX_RB given on the command line.  The build compiles this
// file once per supported pair of radii, so the units compile in parallel;
// logfx_dispatch.hip selects among them at run time.
#include "logfx_kernels.h"

#if !defined(LOGFX_RA) || !defined(LOGFX_RB)
#error "compile with -DLOGFX_RA=<radius of mask 1> -DLOGFX_RB=<radius of mask 2>"
#endif

#define LOGFX_FN3(n, a, b) n##_r##a##_##b
#define LOGFX_FN2(n, a, b) LOGFX_FN3(n, a, b)
#define LOGFX_FN(n) LOGFX_FN2(n, LOGFX_RA, LOGFX_RB)

namespace logfx {

hipError_t LOGFX_FN(pass1_i)(const Pass1Args<OrbitTapsI> &a, int mode, int grid, hipStream_t s,
                             int *max_grid) {
    if (mode == 1) return kern::p1<int, LOGFX_RA, LOGFX_RB, 1>(a, grid, s, max_grid);
    if (mode == 2) return kern::p1<int, LOGFX_RA, LOGFX_RB, 2>(a, grid, s, max_grid);
    return kern::p1<int, LOGFX_RA, LOGFX_RB, 0>(a, grid, s, max_grid);
}
hipError_t LOGFX_FN(pass1_d)(const Pass1Args<OrbitTapsD> &a, int mode, int grid, hipStream_t s,
                             int *max_grid) {
    if (mode == 1) return kern::p1<double, LOGFX_RA, LOGFX_RB, 1>(a, grid, s, max_grid);
    if (mode == 2) return kern::p1<double, LOGFX_RA, LOGFX_RB, 2>(a, grid, s, max_grid);
    return kern::p1<double, LOGFX_RA, LOGFX_RB, 0>(a, grid, s, max_grid);
}
hipError_t LOGFX_FN(pass2_i)(const Pass2Args<OrbitTapsI> &a, int grid, hipStream_t s, int *max_grid) {
    return kern::p2<int, LOGFX_RA, LOGFX_RB>(a, grid, s, max_grid);
}
hipError_t LOGFX_FN(pass2_d)(const Pass2Args<OrbitTapsD> &a, int grid, hipStream_t s, int *max_grid) {
    return kern::p2<double, LOGFX_RA, LOGFX_RB>(a, grid, s, max_grid);
}

}  // namespace logfx
