// Multi-step stationary apply over several stencil sizes in one launch, up to 8 steps per launch.
#include "stepk.hpp"

namespace lmep {

template <>
hipError_t launch_stepk_mixed_depth<8>(int nmax, int scheme, int nonlin, int ksteps, const DevProb* d_probs,
                                        const int* d_tile_inst, int64_t tiles, const double* fd, const double* d_w,
                                        const double* d_u_in, double* d_u_out, hipStream_t stream) {
    return dispatch_mixed<8>(nmax, scheme, nonlin, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, ksteps,
                              stream);
}

}  // namespace lmep
