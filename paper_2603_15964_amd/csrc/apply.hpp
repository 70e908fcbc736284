// Banded apply (steps a7-a8): one time step of the assembled banded
// integrator, node by node, with the harvested weights (Sec. 3.1 step 3):
//   LINEAR : u+_i = W0_i . u_S
//   ETD1   : u+_i = W0_i . u_S + W1_i . N_S
//   ETD2RK : a_i  = W0_i . u_S + W1_i . N(u)_S
//            u+_i = a_i + W2_i . (N(a) - N(u))_S          (both stages fused)
// with the nonlinear terms
//   frozen-velocity Burgers : N^(i)_j = -g (u_j - u_i) (du/dx)_j
//   KdV                     : N_j = -(g/2) (d/dx u^2)_j
//   Allen-Cahn              : N_j = g (u_j - u_j^3)
// where d/dx at node j uses row r_j of D1 on j's own stencil.
//
// One block covers a tile of kApplyTile consecutive nodes of one instance
// (block -> instance through a host-built table).  A node's stencil lies
// within 2R of it (R = (n-1)/2; one-sided stencils next to Dirichlet ends
// reach 2R to one side) and a derivative adds another 2R, so the state is
// staged in LDS over the tile plus a halo covering every value the tile's
// outputs depend on: 2R (LINEAR, pointwise N), 4R (derivative N), and for the
// fused ETD2RK 4R (pointwise) or 8R (derivative) since a and N(a) are formed
// in LDS around the tile.  Each global value of the state is read once per
// block, coalesced; per-node weights (structure of arrays [kind][k][node]) are
// read coalesced from HBM; stationary weights ([kind][r][k]) sit in LDS.
// Dirichlet end nodes hold their boundary values.
#pragma once

#include "lmep_device.hpp"

namespace lmep {
namespace {

constexpr int NT = 256;  // threads per block

template <int NN, int NL>
struct Halo {
    static constexpr int R = (NN - 1) / 2;
    static constexpr bool DERIV = (NL == NL_BURGERS) || (NL == NL_KDV);
    static constexpr int STEN = 2 * R;            // reach of a stencil (edge rows included)
    static constexpr int NR = DERIV ? 2 * R : 0;  // extra reach of N
};

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Position whose neighbourhood in the staged arrays stands for unwrapped
// position j: j itself on periodic grids (translation invariance) and inside a
// Dirichlet grid; the reflected node on Neumann grids, since every nodal
// quantity at a reflected position is the reflected node's own value.
__device__ __forceinline__ int64_t source_position(int64_t j, int64_t N, int bc) {
    return bc == BC_NEUMANN ? map_index(j, N, bc) : j;
}

// N at unwrapped position j, from the LDS array v that starts at unwrapped
// position base.  KdV and the frozen-velocity du/dx use j's own stencil, whose
// side for upwind windows follows j's advection speed (c, or c + g u_j).
template <int NN, int NL>
__device__ __forceinline__ double nonlinear_at(const double* __restrict__ v, int len, int64_t base, int64_t j,
                                               int64_t N, int bc, int window, double c,
                                               const double* __restrict__ sD1, double g) {
    if constexpr (NL == NL_AC) {
        const double x = v[clampi((int)(j - base), 0, len - 1)];
        return g * (x - x * x * x);
    } else {
        int64_t jj = source_position(j, N, bc);
        if (bc == BC_DIRICHLET) jj = jj < 0 ? 0 : (jj > N - 1 ? N - 1 : jj);
        double a = c;
        if constexpr (NL == NL_BURGERS) a += g * v[clampi((int)(jj - base), 0, len - 1)];
        const int64_t o = window_offset(jj, N, NN, bc, window, a);
        const int rr = (int)(-o);
        const int b = clampi((int)(jj + o - base), 0, len - NN);
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < NN; ++k) {
            const double x = v[b + k];
            if constexpr (NL == NL_KDV) acc += sD1[rr * NN + k] * x * x;
            else acc += sD1[rr * NN + k] * x;
        }
        if constexpr (NL == NL_KDV) return -0.5 * g * acc;
        else return acc;  // du/dx (frozen-velocity remainder)
    }
}

template <int NN, int SCH, int NL, bool PERNODE, int TILE>
__global__ __launch_bounds__(NT) void apply_kernel(const DevProb* __restrict__ probs, const int* __restrict__ tile_inst,
                                                   const double* __restrict__ fd, const double* __restrict__ w,
                                                   const double* __restrict__ u_in, double* __restrict__ u_out) {
    using Hh = Halo<NN, NL>;
    constexpr int PP = (SCH == SCH_ETD2RK) ? 2 : (SCH == SCH_ETD1 ? 1 : 0);
    constexpr bool HAS_N = (PP > 0) && (NL != NL_NONE);
    constexpr bool RK2 = (SCH == SCH_ETD2RK);
    // reach of each stage around the tile (in nodes)
    constexpr int A_REACH = RK2 ? Hh::STEN + (HAS_N ? Hh::NR : 0) : 0;  // a and N(a) region halo
    constexpr int AR = A_REACH;                                          // a region halo
    constexpr int NU_REACH = AR + Hh::STEN;                              // N(u) region halo
    constexpr int U_REACH = NU_REACH + (HAS_N ? Hh::NR : 0);             // staged state halo
    constexpr int LU = TILE + 2 * U_REACH;
    constexpr int LNU = TILE + 2 * NU_REACH;
    constexpr int LA = TILE + 2 * AR;

    __shared__ double su[LU];
    __shared__ double sNu[HAS_N ? LNU : 1];
    __shared__ double sa[RK2 ? LA : 1];
    __shared__ double sNa[(RK2 && HAS_N) ? LA : 1];
    __shared__ double sD1[Hh::DERIV ? NN * NN : 1];
    __shared__ double sw[PERNODE ? 1 : (PP + 1) * NN * NN];

    const int tid = threadIdx.x;
    const DevProb& P = probs[tile_inst[blockIdx.x]];
    const int64_t N = P.N;
    const int bc = P.bc;
    const int64_t t0 = ((int64_t)blockIdx.x - P.item_begin) * TILE;
    const double* __restrict__ u = u_in + P.state_off;
    const double g = P.nl_coef;
    const int64_t ubase = t0 - U_REACH;

    {  // all loads of the staged state in flight before the LDS stores
        constexpr int ITER = (LU + NT - 1) / NT;
        double v[ITER];
#pragma unroll
        for (int t = 0; t < ITER; ++t) {
            const int q = tid + t * NT;
            int64_t j = map_index(ubase + q, N, bc);
            j = j < 0 ? 0 : (j > N - 1 ? N - 1 : j);
            v[t] = (q < LU) ? u[j] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < ITER; ++t)
            if (tid + t * NT < LU) su[tid + t * NT] = v[t];
    }
    if constexpr (Hh::DERIV) {
        const double ih = 1.0 / P.h;
        for (int q = tid; q < NN * NN; q += NT) sD1[q] = fd[fd_index(NN, 0, q / NN, q % NN)] * ih;
    }
    if constexpr (!PERNODE) {
        for (int q = tid; q < (PP + 1) * NN * NN; q += NT) sw[q] = w[P.weight_off + q];
    }
    __syncthreads();

    const int64_t nubase = t0 - NU_REACH;
    if constexpr (HAS_N) {
        for (int q = tid; q < LNU; q += NT)
            sNu[q] = nonlinear_at<NN, NL>(su, LU, ubase, nubase + q, N, bc, P.window, P.c, sD1, g);
        __syncthreads();
    }

    const double* __restrict__ wn = w + P.weight_off;
    auto weight = [&](int kind, int r, int k, int64_t i) -> double {
        if constexpr (PERNODE) return wn[(int64_t)(kind * NN + k) * N + i];
        else return sw[(kind * NN + r) * NN + k];
    };
    // first stage (or the whole LINEAR / ETD1 step) at unwrapped position i
    auto stage_a = [&](int64_t i) -> double {
        int64_t ii = i;
        if (bc == BC_DIRICHLET) {
            if (ii <= 0) return P.bc_left;
            if (ii >= N - 1) return P.bc_right;
        } else {
            ii = map_index(i, N, bc);
        }
        const int64_t c = source_position(i, N, bc);  // where the stencil of node ii is read
        const double ui = su[clampi((int)(c - ubase), 0, LU - 1)];
        const int64_t o = window_offset(ii, N, NN, bc, P.window, NL == NL_BURGERS ? P.c + g * ui : P.c);
        const int r = (int)(-o);
        const int bu = clampi((int)(c + o - ubase), 0, LU - NN);
        const int bn = clampi((int)(c + o - nubase), 0, (HAS_N ? LNU : NN) - NN);
        double acc = 0.0;
#pragma unroll
        for (int k = 0; k < NN; ++k) {
            acc += weight(0, r, k, ii) * su[bu + k];
            if constexpr (HAS_N) {
                if constexpr (NL == NL_BURGERS) acc += weight(1, r, k, ii) * (-g * (su[bu + k] - ui) * sNu[bn + k]);
                else acc += weight(1, r, k, ii) * sNu[bn + k];
            }
        }
        return acc;
    };

    double* __restrict__ out = u_out + P.state_off;
    if constexpr (!RK2) {
        for (int q = tid; q < TILE; q += NT) {
            const int64_t i = t0 + q;
            if (i < N) out[i] = stage_a(i);
        }
    } else {
        const int64_t abase = t0 - AR;
        for (int q = tid; q < LA; q += NT) sa[q] = stage_a(abase + q);
        __syncthreads();
        if constexpr (HAS_N) {
            for (int q = tid; q < LA; q += NT)
                sNa[q] = nonlinear_at<NN, NL>(sa, LA, abase, abase + q, N, bc, P.window, P.c, sD1, g);
            __syncthreads();
        }
        for (int q = tid; q < TILE; q += NT) {
            const int64_t i = t0 + q;
            if (i >= N) continue;
            double acc = sa[q + AR];
            if (bc == BC_DIRICHLET && (i == 0 || i == N - 1)) {
                out[i] = acc;
                continue;
            }
            if constexpr (HAS_N) {
                const int64_t o = window_offset(i, N, NN, bc, P.window, P.c);
                const int r = (int)(-o);
                const int ba = clampi((int)(i + o - abase), 0, LA - NN);
                const int bn = clampi((int)(i + o - nubase), 0, LNU - NN);
#pragma unroll
                for (int k = 0; k < NN; ++k) acc += weight(2, r, k, i) * (sNa[ba + k] - sNu[bn + k]);
            }
            out[i] = acc;
        }
    }
}

template <int NN, int SCH, int NL, bool PN>
hipError_t go(int tile, const DevProb* p, const int* ti, int64_t tiles, const double* fd, const double* w,
              const double* ui, double* uo, hipStream_t s) {
    if (tile == 256)
        hipLaunchKernelGGL((apply_kernel<NN, SCH, NL, PN, 256>), dim3((unsigned)tiles), dim3(NT), 0, s, p, ti, fd, w,
                           ui, uo);
    else if (tile == 1024)
        hipLaunchKernelGGL((apply_kernel<NN, SCH, NL, PN, 1024>), dim3((unsigned)tiles), dim3(NT), 0, s, p, ti, fd, w,
                           ui, uo);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace
}  // namespace lmep
