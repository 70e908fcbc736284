// Banded apply (steps a7-a8): one time step of the assembled banded
// integrator, node by node, with the harvested weights (Sec. 3.1 step 3):
//   LINEAR : u+_i = W0_i . u_S
//   ETD1   : u+_i = W0_i . u_S + W1_i . N_S
//   ETD2RK : a_i  = W0_i . u_S + W1_i . N(u)_S                    (stage 0)
//            u+_i = a_i + W2_i . (N(a) - N(u))_S                  (stage 1)
// with the nonlinear terms
//   frozen-velocity Burgers : N^(i)_j = -g (u_j - u_i) (du/dx)_j
//   KdV                     : N_j = -(g/2) (d/dx u^2)_j
//   Allen-Cahn              : N_j = g (u_j - u_j^3)
// where d/dx at node j uses row r_j of D1 on j's own stencil.
//
// One block covers a tile of kApplyTile consecutive nodes of one instance.
// A node's stencil lies within 2R of it (R = (n-1)/2; one-sided stencils next
// to Dirichlet ends reach 2R to one side), so N is needed over the tile plus a
// halo of 2R, and the state (and the stage value a) is staged in LDS over a
// halo of 4R when N needs a derivative, 2R otherwise.  Every global read of
// the state is coalesced and happens once per block.  N is
// evaluated once per position into LDS.  Per-node weights (structure of
// arrays, [kind][k][node]) are read coalesced straight from HBM; stationary
// weights ([kind][r][k], a few KB) are staged in LDS.  Dirichlet end nodes
// hold their boundary values.
#include "lmep_device.hpp"

namespace lmep {
namespace {

constexpr int T = kApplyTile;

template <int NN, int SCH, int NL, bool PERNODE, int STAGE>
__global__ __launch_bounds__(T) void apply_kernel(const DevProb* __restrict__ probs, int nprob,
                                                  const double* __restrict__ fd, const double* __restrict__ w,
                                                  const double* __restrict__ u_in,
                                                  const double* __restrict__ u_stage, double* __restrict__ u_out) {
    constexpr int R = (NN - 1) / 2;
    constexpr bool DERIV = (NL == NL_BURGERS) || (NL == NL_KDV);
    constexpr int HN = 2 * R;               // halo of the N (or du/dx) positions
    constexpr int H = DERIV ? 4 * R : 2 * R; // halo of the staged state
    constexpr int LU = T + 2 * H;          // staged state positions
    constexpr int LN = T + 2 * HN;         // positions where N (or du/dx) is needed
    constexpr int PP = (SCH == SCH_ETD2RK) ? 2 : (SCH == SCH_ETD1 ? 1 : 0);
    constexpr bool TWO = (STAGE == 1);     // ETD2RK second stage: needs u and a

    __shared__ double su[LU];
    __shared__ double sa[TWO ? LU : 1];
    __shared__ double sN[(PP > 0) ? LN : 1];
    __shared__ double sNa[TWO ? LN : 1];
    __shared__ double sD1[DERIV ? NN * NN : 1];
    __shared__ double sw[PERNODE ? 1 : (PP + 1) * NN * NN];

    const int tid = threadIdx.x;
    const int64_t tile = blockIdx.x;
    const DevProb& P = probs[find_instance(probs, nprob, tile)];
    const int64_t N = P.N;
    const int bc = P.bc;
    const int64_t t0 = (tile - P.item_begin) * T;
    const double* __restrict__ u = u_in + P.state_off;
    const double* __restrict__ a = u_stage + P.state_off;
    const double g = P.nl_coef;

    // stage the state over [t0 - H, t0 + T + H); positions no valid node needs
    // are clamped into the grid so that no read leaves the instance.
    for (int q = tid; q < LU; q += T) {
        int64_t j = map_index(t0 - H + q, N, bc);
        j = j < 0 ? 0 : (j > N - 1 ? N - 1 : j);
        su[q] = u[j];
        if constexpr (TWO) sa[q] = a[j];
    }
    if constexpr (DERIV) {
        const double ih = 1.0 / P.h;
        for (int q = tid; q < NN * NN; q += T) sD1[q] = fd[fd_index(NN, 0, q / NN, q % NN)] * ih;
    }
    if constexpr (!PERNODE) {
        for (int q = tid; q < (PP + 1) * NN * NN; q += T) sw[q] = w[P.weight_off + q];
    }
    __syncthreads();

    // nonlinear term (or du/dx for the frozen-velocity case) over [t0 - HN, t0 + T + HN)
    if constexpr (PP > 0 && NL != NL_NONE) {
        for (int q = tid; q < LN; q += T) {
            const int64_t j = t0 - HN + q;  // unwrapped position
            double vN = 0.0, vNa = 0.0;
            if constexpr (NL == NL_AC) {
                const double x = su[q + H - HN];
                vN = g * (x - x * x * x);
                if constexpr (TWO) {
                    const double y = sa[q + H - HN];
                    vNa = g * (y - y * y * y);
                }
            } else {
                // derivative at position j from j's own stencil (row r_j of D1)
                int64_t jj = j;
                if (bc == BC_DIRICHLET) jj = jj < 0 ? 0 : (jj > N - 1 ? N - 1 : jj);
                const int64_t o = (bc == BC_DIRICHLET) ? window_offset(jj, N, NN, bc) : -(int64_t)R;
                const int rr = (int)(-o);
                int base = (int)(jj + o - (t0 - H));
                base = base < 0 ? 0 : (base > LU - NN ? LU - NN : base);
                double acc = 0.0, acca = 0.0;
#pragma unroll
                for (int k = 0; k < NN; ++k) {
                    const double d = sD1[rr * NN + k];
                    const double x = su[base + k];
                    if constexpr (NL == NL_KDV) {
                        acc += d * x * x;
                        if constexpr (TWO) acca += d * sa[base + k] * sa[base + k];
                    } else {
                        acc += d * x;
                    }
                }
                if constexpr (NL == NL_KDV) {
                    vN = -0.5 * g * acc;
                    vNa = -0.5 * g * acca;
                } else {
                    vN = acc;  // du/dx for the frozen-velocity remainder
                }
            }
            sN[q] = vN;
            if constexpr (TWO) sNa[q] = vNa;
        }
        __syncthreads();
    }

    const int64_t i = t0 + tid;
    if (i >= N) return;
    double* __restrict__ out = u_out + P.state_off;
    if (bc == BC_DIRICHLET && (i == 0 || i == N - 1)) {
        out[i] = (i == 0) ? P.bc_left : P.bc_right;
        return;
    }
    const int64_t o = window_offset(i, N, NN, bc);
    const int r = (int)(-o);
    int bu = (int)(i + o - (t0 - H));   // first stencil position in su
    int bn = (int)(i + o - (t0 - HN));  // first stencil position in sN
    bu = bu < 0 ? 0 : (bu > LU - NN ? LU - NN : bu);
    bn = bn < 0 ? 0 : (bn > LN - NN ? LN - NN : bn);
    const double* __restrict__ wn = w + P.weight_off;

    auto weight = [&](int kind, int k) -> double {
        if constexpr (PERNODE) return wn[(int64_t)(kind * NN + k) * N + i];
        else return sw[(kind * NN + r) * NN + k];
    };

    double acc;
    if constexpr (!TWO) {
        acc = 0.0;
        const double ui = su[tid + H];
#pragma unroll
        for (int k = 0; k < NN; ++k) {
            acc += weight(0, k) * su[bu + k];
            if constexpr (PP > 0 && NL != NL_NONE) {
                if constexpr (NL == NL_BURGERS) acc += weight(1, k) * (-g * (su[bu + k] - ui) * sN[bn + k]);
                else acc += weight(1, k) * sN[bn + k];
            }
        }
    } else {
        acc = sa[tid + H];
        if constexpr (NL != NL_NONE) {
#pragma unroll
            for (int k = 0; k < NN; ++k) acc += weight(2, k) * (sNa[bn + k] - sN[bn + k]);
        }
    }
    out[i] = acc;
}

template <int NN, int SCH, int NL, bool PN, int ST>
hipError_t go(const DevProb* p, int np, int64_t tiles, const double* fd, const double* w, const double* ui,
              const double* us, double* uo, hipStream_t s) {
    hipLaunchKernelGGL((apply_kernel<NN, SCH, NL, PN, ST>), dim3((unsigned)tiles), dim3(T), 0, s, p, np, fd, w, ui, us,
                       uo);
    return hipGetLastError();
}

// Supported (scheme, nonlinearity, weights) combinations.
template <int NN>
hipError_t dispatch(int scheme, int nonlin, bool pernode, int stage, const DevProb* p, int np, int64_t tiles,
                    const double* fd, const double* w, const double* ui, const double* us, double* uo,
                    hipStream_t s) {
    if (scheme == SCH_LINEAR && !pernode) return go<NN, SCH_LINEAR, NL_NONE, false, 0>(p, np, tiles, fd, w, ui, us, uo, s);
    if (scheme == SCH_ETD1 && !pernode) {
        switch (nonlin) {
            case NL_NONE: return go<NN, SCH_ETD1, NL_NONE, false, 0>(p, np, tiles, fd, w, ui, us, uo, s);
            case NL_AC: return go<NN, SCH_ETD1, NL_AC, false, 0>(p, np, tiles, fd, w, ui, us, uo, s);
            case NL_KDV: return go<NN, SCH_ETD1, NL_KDV, false, 0>(p, np, tiles, fd, w, ui, us, uo, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (scheme == SCH_ETD1 && pernode && nonlin == NL_BURGERS)
        return go<NN, SCH_ETD1, NL_BURGERS, true, 0>(p, np, tiles, fd, w, ui, us, uo, s);
    if (scheme == SCH_ETD2RK && !pernode) {
        switch (nonlin) {
            case NL_NONE:
                return stage == 0 ? go<NN, SCH_ETD2RK, NL_NONE, false, 0>(p, np, tiles, fd, w, ui, us, uo, s)
                                  : go<NN, SCH_ETD2RK, NL_NONE, false, 1>(p, np, tiles, fd, w, ui, us, uo, s);
            case NL_AC:
                return stage == 0 ? go<NN, SCH_ETD2RK, NL_AC, false, 0>(p, np, tiles, fd, w, ui, us, uo, s)
                                  : go<NN, SCH_ETD2RK, NL_AC, false, 1>(p, np, tiles, fd, w, ui, us, uo, s);
            case NL_KDV:
                return stage == 0 ? go<NN, SCH_ETD2RK, NL_KDV, false, 0>(p, np, tiles, fd, w, ui, us, uo, s)
                                  : go<NN, SCH_ETD2RK, NL_KDV, false, 1>(p, np, tiles, fd, w, ui, us, uo, s);
            default: return hipErrorInvalidValue;
        }
    }
    return hipErrorInvalidValue;
}

__global__ void check_finite_kernel(const double* __restrict__ x, int64_t count, int* __restrict__ flag) {
    int bad = 0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < count; q += (int64_t)gridDim.x * blockDim.x)
        bad |= !isfinite(x[q]);
    if (bad) atomicOr(flag, 1);
}

}  // namespace

hipError_t launch_apply(int n, int scheme, int nonlin, bool pernode, int stage, const DevProb* d_probs, int nprob,
                        int64_t tiles, const double* fd, const double* d_w, const double* d_u_in,
                        const double* d_u_stage, double* d_u_out, hipStream_t stream) {
    if (tiles <= 0) return hipSuccess;
    switch (n) {
        case 3: return dispatch<3>(scheme, nonlin, pernode, stage, d_probs, nprob, tiles, fd, d_w, d_u_in, d_u_stage, d_u_out, stream);
        case 5: return dispatch<5>(scheme, nonlin, pernode, stage, d_probs, nprob, tiles, fd, d_w, d_u_in, d_u_stage, d_u_out, stream);
        case 7: return dispatch<7>(scheme, nonlin, pernode, stage, d_probs, nprob, tiles, fd, d_w, d_u_in, d_u_stage, d_u_out, stream);
        case 9: return dispatch<9>(scheme, nonlin, pernode, stage, d_probs, nprob, tiles, fd, d_w, d_u_in, d_u_stage, d_u_out, stream);
        case 11: return dispatch<11>(scheme, nonlin, pernode, stage, d_probs, nprob, tiles, fd, d_w, d_u_in, d_u_stage, d_u_out, stream);
        case 13: return dispatch<13>(scheme, nonlin, pernode, stage, d_probs, nprob, tiles, fd, d_w, d_u_in, d_u_stage, d_u_out, stream);
        case 15: return dispatch<15>(scheme, nonlin, pernode, stage, d_probs, nprob, tiles, fd, d_w, d_u_in, d_u_stage, d_u_out, stream);
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
