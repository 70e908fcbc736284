// Multi-step stationary apply kernels (ETD schemes) advancing up to 16 steps per launch; ETDRK4 stops at 8.
#include "stepk.hpp"

namespace lmep {

template <>
hipError_t launch_stepk_depth<16>(int n, int scheme, int nonlin, int ksteps, const DevProb* d_probs,
                                   const int* d_tile_inst, int64_t tiles, const double* fd, const double* d_w,
                                   const double* d_u_in, double* d_u_out, hipStream_t stream) {
    if (scheme == SCH_ETDRK4) return hipErrorInvalidValue;
    return dispatch_n<16, 0>(n, scheme, nonlin, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, ksteps, stream);
}

}  // namespace lmep
