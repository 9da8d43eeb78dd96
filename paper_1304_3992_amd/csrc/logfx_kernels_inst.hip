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

namespace {   // one copy per radius pair: internal linkage keeps the units' copies apart

// Pass-1 variants built: statistics only, maps, cells, stored strengths,
// stored strengths with cells; on the integer path each also in the packed
// form.
template <class Acc>
hipError_t pass1_any(const Pass1Args<typename kern::AccOps<Acc>::Taps> &a, int mode, int grid, hipStream_t s,
                     int *max_grid) {
    switch (mode) {
    case 0: return kern::p1<Acc, LOGFX_RA, LOGFX_RB, 0>(a, grid, s, max_grid);
    case kP1Maps: return kern::p1<Acc, LOGFX_RA, LOGFX_RB, kP1Maps>(a, grid, s, max_grid);
    case kP1Cells: return kern::p1<Acc, LOGFX_RA, LOGFX_RB, kP1Cells>(a, grid, s, max_grid);
    case kP1StoreZ: return kern::p1<Acc, LOGFX_RA, LOGFX_RB, kP1StoreZ>(a, grid, s, max_grid);
    case kP1StoreZ | kP1Cells: return kern::p1<Acc, LOGFX_RA, LOGFX_RB, kP1StoreZ | kP1Cells>(a, grid, s, max_grid);
    }
    if constexpr (std::is_same<Acc, int>::value) {   // the same on packed 16-bit sums
        constexpr int K = kP1Packed;
        switch (mode) {
        case K: return kern::p1<int, LOGFX_RA, LOGFX_RB, K>(a, grid, s, max_grid);
        case K | kP1Maps: return kern::p1<int, LOGFX_RA, LOGFX_RB, K | kP1Maps>(a, grid, s, max_grid);
        case K | kP1Cells: return kern::p1<int, LOGFX_RA, LOGFX_RB, K | kP1Cells>(a, grid, s, max_grid);
        case K | kP1StoreZ: return kern::p1<int, LOGFX_RA, LOGFX_RB, K | kP1StoreZ>(a, grid, s, max_grid);
        case K | kP1StoreZ | kP1Cells:
            return kern::p1<int, LOGFX_RA, LOGFX_RB, K | kP1StoreZ | kP1Cells>(a, grid, s, max_grid);
        }
    }
    return hipErrorInvalidValue;
}
}  // namespace

hipError_t LOGFX_FN(pass1_i)(const Pass1Args<OrbitTapsI> &a, int mode, int grid, hipStream_t s,
                             int *max_grid) {
    return pass1_any<int>(a, mode, grid, s, max_grid);
}
hipError_t LOGFX_FN(pass1_d)(const Pass1Args<OrbitTapsD> &a, int mode, int grid, hipStream_t s,
                             int *max_grid) {
    return pass1_any<double>(a, mode, grid, s, max_grid);
}
hipError_t LOGFX_FN(pass2_i)(const Pass2Args<OrbitTapsI> &a, int grid, hipStream_t s, int *max_grid) {
    return kern::p2<int, LOGFX_RA, LOGFX_RB>(a, grid, s, max_grid);
}
hipError_t LOGFX_FN(pass2_d)(const Pass2Args<OrbitTapsD> &a, int grid, hipStream_t s, int *max_grid) {
    return kern::p2<double, LOGFX_RA, LOGFX_RB>(a, grid, s, max_grid);
}

}  // namespace logfx
