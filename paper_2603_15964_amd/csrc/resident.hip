// Many steps per launch for small instances (Sec. 4.3.3's Chebyshev grid has
// 64 nodes; the advection-diffusion workload 256): one block holds a whole
// instance, one thread per node, the node's weights in registers (its own
// per-node row on a non-uniform grid, the row its window harvests from the
// stationary table on a uniform one) and the state (and the stage arrays) in
// LDS, and advances it ksteps steps before writing it back.
// HBM then sees the weights and the state once per launch instead of once per
// step.  u_in may equal u_out: each thread reads its node before any thread
// writes.  Each node's value is formed by the same expressions in the same order
// as in the one-step kernel, so the two paths agree bit for bit.
//
// Per step (Dirichlet ends held):
//   ETD1 / LINEAR : u+_i = sum_k W0_i[k] u_S(k) (+ W1_i[k] N_S(k))
//   ETD2RK        : a_i = the same; u+_i = a_i + sum_k W2_i[k] (N(a) - N(u))_S(k)
// with the pointwise N = g (u - u^3) (or none).  On a uniform grid the window
// S(k) of node i wraps (periodic) or reflects (Neumann) as in the one-step
// kernel; each thread keeps the LDS slots of its window.
#include "lmep_device.hpp"

namespace lmep {
namespace {

template <int NN, int SCH, int NL, bool UNI>
__global__ __launch_bounds__(kResidentMaxN) void resident_kernel(const DevProb* __restrict__ probs,
                                                                const double* __restrict__ w,
                                                                const double* u_in, double* u_out, int ksteps) {
    constexpr int PP = (SCH == SCH_ETD2RK) ? 2 : (SCH == SCH_ETD1 ? 1 : 0);
    constexpr bool HAS_N = (PP > 0) && (NL != NL_NONE);
    constexpr bool RK2 = (SCH == SCH_ETD2RK);
    extern __shared__ double lds[];
    const DevProb& P = probs[blockIdx.x];
    const int N = (int)P.N;
    const int i = threadIdx.x;
    const bool node = i < N;
    const double g = P.nl_coef;
    double* su = lds;             // state
    double* sN = su + N;          // N(u)
    double* sa = sN + N;          // first ETD2RK stage
    double* sNa = sa + N;         // N(a)

    const int bc = UNI ? P.bc : BC_DIRICHLET;
    // a uniform grid's window may be one-sided (stationary: the side of c)
    const int o = node ? (int)window_offset(i, N, NN, bc, UNI ? P.window : WIN_CENTRED, P.c) : 0;
    const bool fixed = bc == BC_DIRICHLET && ((i == 0) || (i == N - 1));
    double W0[NN], W1[NN], W2[NN];
    int slot[NN];  // LDS slot of window position k
    const double* __restrict__ wn = w + P.weight_off;
    const int r = -o;
#pragma unroll
    for (int k = 0; k < NN; ++k) {
        if constexpr (UNI) {  // stationary table [kind][r][k]
            W0[k] = node ? wn[r * NN + k] : 0.0;
            W1[k] = (node && PP >= 1) ? wn[(NN + r) * NN + k] : 0.0;
            W2[k] = (node && PP >= 2) ? wn[(2 * NN + r) * NN + k] : 0.0;
            slot[k] = node ? (int)map_index(i + o + k, N, bc) : 0;
        } else {  // per node [kind][k][i]
            W0[k] = node ? wn[(int64_t)k * N + i] : 0.0;
            W1[k] = (node && PP >= 1) ? wn[(int64_t)(NN + k) * N + i] : 0.0;
            W2[k] = (node && PP >= 2) ? wn[(int64_t)(2 * NN + k) * N + i] : 0.0;
            slot[k] = i + o + k;
        }
    }
    if (node) su[i] = u_in[P.state_off + i];
    __syncthreads();

    for (int st = 0; st < ksteps; ++st) {
        if constexpr (HAS_N && RK2) {  // N(u) is needed again by the second stage
            if (node) {
                const double x = su[i];
                sN[i] = g * (x - x * x * x);
            }
        }
        double acc = 0.0;
        if (node) {
            if (fixed) {
                acc = (i == 0) ? P.bc_left : P.bc_right;
            } else {
                // N of each window value is formed here rather than read from
                // an array (half the LDS traffic); it is the expression the
                // one-step kernel stores, so the values are the same
#pragma unroll
                for (int k = 0; k < NN; ++k) {
                    const double x = su[slot[k]];
                    acc += W0[k] * x;
                    if constexpr (HAS_N) acc += W1[k] * (g * (x - x * x * x));
                }
            }
        }
        if constexpr (RK2) {
            if (node) sa[i] = acc;
            __syncthreads();
            if constexpr (HAS_N) {
                if (node) {
                    const double x = sa[i];
                    sNa[i] = g * (x - x * x * x);
                }
                __syncthreads();
                if (node && !fixed) {
#pragma unroll
                    for (int k = 0; k < NN; ++k) acc += W2[k] * (sNa[slot[k]] - sN[slot[k]]);
                }
            }
        }
        __syncthreads();  // every read of su / sN of this step is done
        if (node) su[i] = acc;
        __syncthreads();
    }
    if (node) u_out[P.state_off + i] = su[i];
}

template <int NN, int SCH, int NL, bool UNI>
hipError_t go_res(const DevProb* p, int count, int block, const double* w, const double* ui, double* uo,
                  int ksteps, hipStream_t s) {
    const size_t lds = sizeof(double) * 4 * (size_t)block;
    hipLaunchKernelGGL((resident_kernel<NN, SCH, NL, UNI>), dim3((unsigned)count), dim3(block), lds, s, p, w, ui, uo,
                       ksteps);
    return hipGetLastError();
}

template <int NN, bool UNI>
hipError_t dispatch_res(int scheme, int nonlin, const DevProb* p, int count, int block, const double* w,
                        const double* ui, double* uo, int ksteps, hipStream_t s) {
    if (nonlin == NL_NONE) {
        switch (scheme) {
            case SCH_LINEAR: return go_res<NN, SCH_LINEAR, NL_NONE, UNI>(p, count, block, w, ui, uo, ksteps, s);
            case SCH_ETD1: return go_res<NN, SCH_ETD1, NL_NONE, UNI>(p, count, block, w, ui, uo, ksteps, s);
            case SCH_ETD2RK: return go_res<NN, SCH_ETD2RK, NL_NONE, UNI>(p, count, block, w, ui, uo, ksteps, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (nonlin == NL_AC) {
        switch (scheme) {
            case SCH_ETD1: return go_res<NN, SCH_ETD1, NL_AC, UNI>(p, count, block, w, ui, uo, ksteps, s);
            case SCH_ETD2RK: return go_res<NN, SCH_ETD2RK, NL_AC, UNI>(p, count, block, w, ui, uo, ksteps, s);
            default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

template <int NN>
hipError_t dispatch_res_grid(bool uniform, int scheme, int nonlin, const DevProb* p, int count, int block,
                             const double* w, const double* ui, double* uo, int ksteps, hipStream_t s) {
    if constexpr (NN <= kMaxN) {
        if (uniform) return dispatch_res<NN, true>(scheme, nonlin, p, count, block, w, ui, uo, ksteps, s);
    } else {
        if (uniform) return hipErrorInvalidValue;
    }
    return dispatch_res<NN, false>(scheme, nonlin, p, count, block, w, ui, uo, ksteps, s);
}

}  // namespace

hipError_t launch_resident(int n, int scheme, int nonlin, bool uniform, const DevProb* d_probs, int count,
                           int64_t max_nodes, const double* d_w, const double* d_u_in, double* d_u_out, int ksteps,
                           hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    if (max_nodes < 1 || max_nodes > kResidentMaxN || ksteps < 1) return hipErrorInvalidValue;
    const int block = (int)((max_nodes + 63) / 64 * 64);
#define LMEP_RES_CASE(NN)                                                                                          \
    case NN:                                                                                                       \
        return dispatch_res_grid<NN>(uniform, scheme, nonlin, d_probs, count, block, d_w, d_u_in, d_u_out, ksteps, \
                                     stream);
    switch (n) {
        LMEP_RES_CASE(3) LMEP_RES_CASE(5) LMEP_RES_CASE(7) LMEP_RES_CASE(9) LMEP_RES_CASE(11) LMEP_RES_CASE(13)
        LMEP_RES_CASE(15) LMEP_RES_CASE(17) LMEP_RES_CASE(19) LMEP_RES_CASE(21) LMEP_RES_CASE(23) LMEP_RES_CASE(25)
        default: return hipErrorInvalidValue;
    }
#undef LMEP_RES_CASE
}

}  // namespace lmep
