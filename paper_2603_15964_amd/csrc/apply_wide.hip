// One-step launches of the banded apply kernel (apply.hpp) for non-uniform
// grids: stationary weights stored per node ([kind][k][node], built once by
// the wide build), stencils up to 25 points, pointwise nonlinearity only
// (none or Allen-Cahn; Sec. 4.3.3).
#include "apply.hpp"

namespace lmep {
namespace {

// Tiles of 64 nodes as well: non-uniform instances are often small (the
// paper's Chebyshev grid has 64 nodes).
template <int NN, int SCH, int NL>
hipError_t go_nu(int tile, const DevProb* p, const int* ti, int64_t tiles, const double* fd, const double* w,
                 const double* ui, double* uo, hipStream_t s) {
    if (tile == 64) {
        hipLaunchKernelGGL((apply_kernel<NN, SCH, NL, true, 64>), dim3((unsigned)tiles), dim3(NT), 0, s, p, ti, fd, w,
                           ui, uo);
        return hipGetLastError();
    }
    return go<NN, SCH, NL, true>(tile, p, ti, tiles, fd, w, ui, uo, s);
}

template <int NN>
hipError_t dispatch_nonuniform(int tile, int scheme, int nonlin, const DevProb* p, const int* ti, int64_t tiles,
                               const double* fd, const double* w, const double* ui, double* uo, hipStream_t s) {
    if (nonlin == NL_NONE) {
        switch (scheme) {
            case SCH_LINEAR: return go_nu<NN, SCH_LINEAR, NL_NONE>(tile, p, ti, tiles, fd, w, ui, uo, s);
            case SCH_ETD1: return go_nu<NN, SCH_ETD1, NL_NONE>(tile, p, ti, tiles, fd, w, ui, uo, s);
            case SCH_ETD2RK: return go_nu<NN, SCH_ETD2RK, NL_NONE>(tile, p, ti, tiles, fd, w, ui, uo, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (nonlin == NL_AC) {
        switch (scheme) {
            case SCH_ETD1: return go_nu<NN, SCH_ETD1, NL_AC>(tile, p, ti, tiles, fd, w, ui, uo, s);
            case SCH_ETD2RK: return go_nu<NN, SCH_ETD2RK, NL_AC>(tile, p, ti, tiles, fd, w, ui, uo, s);
            default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_apply_nonuniform(int n, int tile, int scheme, int nonlin, const DevProb* d_probs,
                                   const int* d_tile_inst, int64_t tiles, const double* fd, const double* d_w,
                                   const double* d_u_in, double* d_u_out, hipStream_t stream) {
    if (tiles <= 0) return hipSuccess;
#define LMEP_NU_CASE(NN) \
    case NN: return dispatch_nonuniform<NN>(tile, scheme, nonlin, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
    switch (n) {
        LMEP_NU_CASE(3) LMEP_NU_CASE(5) LMEP_NU_CASE(7) LMEP_NU_CASE(9) LMEP_NU_CASE(11) LMEP_NU_CASE(13)
        LMEP_NU_CASE(15) LMEP_NU_CASE(17) LMEP_NU_CASE(19) LMEP_NU_CASE(21) LMEP_NU_CASE(23) LMEP_NU_CASE(25)
        default: return hipErrorInvalidValue;
    }
#undef LMEP_NU_CASE
}

}  // namespace lmep
