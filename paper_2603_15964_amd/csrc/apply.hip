// One-step launches of the banded apply kernel (apply.hpp): uniform grids with
// stationary weight tables, and frozen-velocity Burgers with per-node weights.
#include "apply.hpp"

namespace lmep {
namespace {

// Supported (scheme, nonlinearity, weights) combinations.
template <int NN>
hipError_t dispatch(int tile, int scheme, int nonlin, bool pernode, const DevProb* p, const int* ti, int64_t tiles,
                    const double* fd, const double* w, const double* ui, double* uo, hipStream_t s) {
    if (pernode) {
        if (scheme == SCH_ETD1 && nonlin == NL_BURGERS)
            return go<NN, SCH_ETD1, NL_BURGERS, true>(tile, p, ti, tiles, fd, w, ui, uo, s);
        return hipErrorInvalidValue;
    }
    if (scheme == SCH_LINEAR) return go<NN, SCH_LINEAR, NL_NONE, false>(tile, p, ti, tiles, fd, w, ui, uo, s);
    switch (nonlin) {
        case NL_NONE:
            return scheme == SCH_ETD1 ? go<NN, SCH_ETD1, NL_NONE, false>(tile, p, ti, tiles, fd, w, ui, uo, s)
                                      : go<NN, SCH_ETD2RK, NL_NONE, false>(tile, p, ti, tiles, fd, w, ui, uo, s);
        case NL_AC:
            return scheme == SCH_ETD1 ? go<NN, SCH_ETD1, NL_AC, false>(tile, p, ti, tiles, fd, w, ui, uo, s)
                                      : go<NN, SCH_ETD2RK, NL_AC, false>(tile, p, ti, tiles, fd, w, ui, uo, s);
        case NL_KDV:
            return scheme == SCH_ETD1 ? go<NN, SCH_ETD1, NL_KDV, false>(tile, p, ti, tiles, fd, w, ui, uo, s)
                                      : go<NN, SCH_ETD2RK, NL_KDV, false>(tile, p, ti, tiles, fd, w, ui, uo, s);
        default: return hipErrorInvalidValue;
    }
}

__global__ void check_finite_kernel(const double* __restrict__ x, int64_t count, int* __restrict__ flag) {
    int bad = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(x[q]);
    if (bad) atomicOr(flag, 1);
}

}  // namespace

hipError_t launch_apply(int n, int tile, int scheme, int nonlin, bool pernode, const DevProb* d_probs,
                        const int* d_tile_inst, int64_t tiles, const double* fd, const double* d_w,
                        const double* d_u_in, double* d_u_out, hipStream_t stream) {
    if (tiles <= 0) return hipSuccess;
    switch (n) {
        case 3: return dispatch<3>(tile, scheme, nonlin, pernode, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
        case 5: return dispatch<5>(tile, scheme, nonlin, pernode, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
        case 7: return dispatch<7>(tile, scheme, nonlin, pernode, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
        case 9: return dispatch<9>(tile, scheme, nonlin, pernode, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
        case 11: return dispatch<11>(tile, scheme, nonlin, pernode, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
        case 13: return dispatch<13>(tile, scheme, nonlin, pernode, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
        case 15: return dispatch<15>(tile, scheme, nonlin, pernode, d_probs, d_tile_inst, tiles, fd, d_w, d_u_in, d_u_out, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_check_finite(const double* d_x, int64_t count, int* d_flag, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(check_finite_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, d_x, count, d_flag);
    return hipGetLastError();
}

}  // namespace lmep
