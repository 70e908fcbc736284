// Multi-step stationary apply kernels (ETD schemes and ETDRK4) advancing up to 4 step(s) per launch.
#include "stepk_rk4.hpp"

namespace lmep {

template <>
hipError_t launch_stepk_depth<4>(int n, int scheme, int nonlin, int ksteps, const DevProb* d_probs,
                                  const int* d_tile_inst, int64_t tiles, const double* fd, const double* d_w,
                                  const double* d_u_in, double* d_u_out, hipStream_t stream) {
    if (scheme == SCH_ETDRK4)
        return dispatch_n_rk4<4>(n, nonlin, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, ksteps, stream);
    return dispatch_n<4, 0>(n, scheme, nonlin, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, ksteps, stream);
}

}  // namespace lmep
