// Multi-step stationary apply kernels on one-sided (upwind) windows advancing up to 16 step(s) per launch.
#include "stepk.hpp"

namespace lmep {

template <>
hipError_t launch_stepk_upwind_depth<16>(int side, int n, int scheme, int nonlin, int ksteps, const DevProb* d_probs,
                                         const int* d_tile_inst, int64_t tiles, const double* fd, const double* d_w,
                                         const double* d_u_in, double* d_u_out, hipStream_t stream) {
    if (side == 1)
        return dispatch_n<16, 1>(n, scheme, nonlin, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, ksteps,
                                 stream);
    if (side == 2)
        return dispatch_n<16, 2>(n, scheme, nonlin, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, ksteps,
                                 stream);
    return hipErrorInvalidValue;
}

}  // namespace lmep
