// Launch of the multi-step stationary apply (stepk.hpp) at a given depth.
#include "lmep_internal.hpp"

namespace lmep {

hipError_t launch_stepk(int n, int scheme, int nonlin, int kb, int ksteps, const DevProb* d_probs,
                        const int* d_tile_inst, int64_t tiles, const double* fd, const double* d_w,
                        const double* d_u_in, double* d_u_out, hipStream_t stream, int side) {
    if (tiles <= 0) return hipSuccess;
    if (ksteps < 1 || ksteps > kb || side < 0 || side > 2) return hipErrorInvalidValue;
    if (side != 0) {
        if (scheme == SCH_ETDRK4) return hipErrorInvalidValue;
        switch (kb) {
            case 1: return launch_stepk_upwind_depth<1>(side, n, scheme, nonlin, ksteps, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
            case 2: return launch_stepk_upwind_depth<2>(side, n, scheme, nonlin, ksteps, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
            case 4: return launch_stepk_upwind_depth<4>(side, n, scheme, nonlin, ksteps, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
            case 8: return launch_stepk_upwind_depth<8>(side, n, scheme, nonlin, ksteps, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
            case 16: return launch_stepk_upwind_depth<16>(side, n, scheme, nonlin, ksteps, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
            default: return hipErrorInvalidValue;
        }
    }
    switch (kb) {
        case 1: return launch_stepk_depth<1>(n, scheme, nonlin, ksteps, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
        case 2: return launch_stepk_depth<2>(n, scheme, nonlin, ksteps, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
        case 4: return launch_stepk_depth<4>(n, scheme, nonlin, ksteps, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
        case 8: return launch_stepk_depth<8>(n, scheme, nonlin, ksteps, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
        case 16: return launch_stepk_depth<16>(n, scheme, nonlin, ksteps, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stepk_mixed(int nmax, int scheme, int nonlin, int kb, int ksteps, const DevProb* d_probs,
                              const int* d_tile_inst, int64_t tiles, const double* fd, const double* d_w,
                              const double* d_u_in, double* d_u_out, hipStream_t stream) {
    if (tiles <= 0) return hipSuccess;
    if (ksteps < 1 || ksteps > kb) return hipErrorInvalidValue;
    switch (kb) {
        case 8: return launch_stepk_mixed_depth<8>(nmax, scheme, nonlin, ksteps, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
        case 16: return launch_stepk_mixed_depth<16>(nmax, scheme, nonlin, ksteps, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lmep
