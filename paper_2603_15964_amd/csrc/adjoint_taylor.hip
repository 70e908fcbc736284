// Reverse step, per-node part, by the finite Taylor series (step a10 for
// instances without a reaction term on uniform grids): the weights W0, W1 of
// each node and the derivatives of lam_i u+_i with respect to nu, c and delta
// through those weights -- what adj_frechet_kernel reads off the
// block-triangular Pade exponential, here in O(n^2) per node.
//
// As in the forward finite-Taylor build, with q(x) = a x + b x^2 + e x^3
// (a = -c dt/h, b = nu dt/h^2, e = -delta dt/h^3) and the moments
// e^{theta q} = sum_k M_k(theta) x^k / k!, the rows are
//     W0 = sum_k M_k(1) T_k[r'],   W1 = dt sum_k (int_0^1 M_k) T_k[r']
// (expanded about node r' = r + s, s the integer nearest a/2, per node).  Differentiating
// e^{theta q} by a, b or e multiplies it by theta x, theta x^2 or theta x^3,
// which shifts the moments:
//     dM_k/da = theta k M_{k-1},  dM_k/db = theta k (k-1) M_{k-2},
//     dM_k/de = theta k (k-1) (k-2) M_{k-3},
// so the derivatives need no recursion of their own: with
// I_1(j) = int_0^1 theta M_j(theta) dtheta,
//     dW0/da = sum_k k M_{k-1}(1) T_k[r'],  dW1/da = dt sum_k k I_1(k-1) T_k[r'],
// and likewise for b and e.  The forward update of node i is
// u+_i = W0 . U + W1 . V over its window (U the window's u, V its N), so
//     d(lam_i u+_i)/da = lam_i sum_k k (M_{k-1}(1) tau_k + dt I_1(k-1) nu_k)
// with tau_k = T_k[r'] . U and nu_k = T_k[r'] . V, and the chain rule gives
// nu, c and delta.  The derivative in c also serves c_i = c + g u_i of the
// frozen velocity.  Blocks cover 256-node tiles of one instance (the tile
// table of the reverse step), so a node's result does not depend on how the
// instances are batched.
#include "lmep_device.hpp"

namespace lmep {
namespace {

constexpr int T = kAdjTile;

template <int NN, int PP, bool SHIFT>
__device__ __forceinline__ void adj_taylor_node(double a, double b, double e, double s, double dt,
                                                const double* __restrict__ Tr, const double (&U)[NN],
                                                const double (&V)[NN], double (&W0)[NN], double (&W1)[NN],
                                                double& Ga, double& Gb, double& Ge) {
    double m2[NN], m1[NN], m0[NN];  // mu[k-2][.], mu[k-1][.], mu[k][.] (M_k = sum_m mu[k][m] theta^m)
    double Eh[NN], Ih[NN];          // M_j(1) and I_1(j) of the orders done so far
#pragma unroll
    for (int m = 0; m < NN; ++m) {
        m2[m] = 0.0;
        m1[m] = 0.0;
        m0[m] = 0.0;
    }
    m0[0] = 1.0;
    Eh[0] = 1.0;
    Ih[0] = 0.5;
    Ga = 0.0;
    Gb = 0.0;
    Ge = 0.0;
#pragma unroll
    for (int j = 0; j < NN; ++j) {  // order 0
        const double t = Tr[j];
        W0[j] = t;
        W1[j] = t;
    }
#pragma unroll
    for (int k = 0; k + 1 < NN; ++k) {
        const int K = k + 1;  // order formed in this pass
        const double bk = (double)(2 * k) * b;
        const double ek = (double)(3 * k * (k - 1)) * e;
        double nx[NN];
#pragma unroll
        for (int m = 0; m < NN; ++m) {
            double v = 0.0;
            if (m <= K) {
                if (SHIFT && m <= k) v = -s * m0[m];
                if (m >= 1) {
                    v = fma(a, m0[m - 1], v);
                    if (k >= 1) v = fma(bk, m1[m - 1], v);
                    if (k >= 2) v = fma(ek, m2[m - 1], v);
                }
            }
            nx[m] = v;
        }
        double E = -0.0, F = -0.0, I1 = -0.0;
#pragma unroll
        for (int m = 0; m < NN; ++m) {
            m2[m] = m1[m];
            m1[m] = m0[m];
            m0[m] = nx[m];
            if (m <= K && (SHIFT || m >= 1)) {
                E += nx[m];
                F = fma(nx[m], 1.0 / (double)(m + 1), F);
                I1 = fma(nx[m], 1.0 / (double)(m + 2), I1);
            }
        }
        Eh[K] = E;
        Ih[K] = I1;
        const double* __restrict__ Tk = Tr + K * kMaxN;
        double tau = -0.0, nuk = -0.0;
#pragma unroll
        for (int j = 0; j < NN; ++j) {
            const double t = Tk[j];
            W0[j] = fma(E, t, W0[j]);
            tau = fma(t, U[j], tau);
            if constexpr (PP >= 1) {
                W1[j] = fma(F, t, W1[j]);
                nuk = fma(t, V[j], nuk);
            }
        }
        // derivative terms of order K: K M_{K-1}, K (K-1) M_{K-2}, K (K-1) (K-2) M_{K-3}
        double da = (double)K * Eh[K - 1] * tau;
        if constexpr (PP >= 1) da = fma((double)K * dt * Ih[K - 1], nuk, da);
        Ga += da;
        if (K >= 2) {
            double db = (double)(K * (K - 1)) * Eh[K - 2] * tau;
            if constexpr (PP >= 1) db = fma((double)(K * (K - 1)) * dt * Ih[K - 2], nuk, db);
            Gb += db;
        }
        if (K >= 3) {
            double de = (double)(K * (K - 1) * (K - 2)) * Eh[K - 3] * tau;
            if constexpr (PP >= 1) de = fma((double)(K * (K - 1) * (K - 2)) * dt * Ih[K - 3], nuk, de);
            Ge += de;
        }
    }
}

template <int NN, int PP>
__global__ __launch_bounds__(T) void adj_taylor_kernel(const DevProb* __restrict__ probs, int nprob,
                                                       const double* __restrict__ taylor,
                                                       const double* __restrict__ u_all,
                                                       const double* __restrict__ lam_all,
                                                       const double* __restrict__ g_all, double* __restrict__ ws,
                                                       int ws_stride, double* __restrict__ dparam) {
    const int64_t tile = blockIdx.x;
    const DevProb& P = probs[find_instance(probs, nprob, tile)];
    const int64_t N = P.N;
    const int64_t node = (tile - P.item_begin) * T + threadIdx.x;
    // lane 0 holds the wavefront's first node: past the end, so is every lane
    if (__builtin_amdgcn_readfirstlane(node < N ? 1 : 0) == 0) return;
    const bool active = node < N;
    const int64_t i = active ? node : N - 1;  // idle lanes repeat the last node; their results are dropped
    const int bc = P.bc;
    const double* __restrict__ u = u_all + P.state_off;
    const bool fixed = (bc == BC_DIRICHLET) && (i == 0 || i == N - 1);
    const double lam = fixed ? 0.0 : lam_all[P.state_off + i];
    const int64_t o = window_offset(i, N, NN, bc);
    const int r = (int)(-o);
    const double dt = P.dt, g = P.nl_coef, ih = 1.0 / P.h;
    const double ui = u[i];
    const double ceff = P.c + (P.nonlin == NL_BURGERS ? g * ui : 0.0);
    const double a = -ceff * ih * dt, b = P.nu * ih * ih * dt, e = -P.delta * ih * ih * ih * dt;

    double U[NN], V[NN];
#pragma unroll
    for (int j = 0; j < NN; ++j) {
        const int64_t jj = map_index(i + o + j, N, bc);
        U[j] = u[jj];
        double v = 0.0;
        if constexpr (PP >= 1) {
            if (P.nonlin == NL_BURGERS) v = -g * (U[j] - ui) * g_all[P.state_off + jj];
            else if (P.nonlin == NL_AC) v = g * (U[j] - U[j] * U[j] * U[j]);
        }
        V[j] = v;
    }

    const double half = fmin(fmax(0.5 * a, -(double)NN), (double)NN);
    const int sh = (int)rint(half);
    const double* __restrict__ tb = taylor + taylor_index(NN, 0, 0, 0);
    double W0[NN], W1[NN], Ga, Gb, Ge;
    int rp = r + sh;
    rp = rp < 0 ? 0 : (rp > NN - 1 ? NN - 1 : rp);
    const int r0 = __builtin_amdgcn_readfirstlane(r), rp0 = __builtin_amdgcn_readfirstlane(rp);
    if (__ballot(active && (r != r0 || rp != rp0)) == 0) {  // one expansion row for the wavefront
        const double* __restrict__ Tr = tb + rp0 * (kMaxN * kMaxN);
        if (rp0 == r0)
            adj_taylor_node<NN, PP, false>(a, b, e, 0.0, dt, Tr, U, V, W0, W1, Ga, Gb, Ge);
        else
            adj_taylor_node<NN, PP, true>(a, b, e, (double)(rp0 - r0), dt, Tr, U, V, W0, W1, Ga, Gb, Ge);
    } else {
        adj_taylor_node<NN, PP, true>(a, b, e, (double)(rp - r), dt, tb + rp * (kMaxN * kMaxN), U, V, W0, W1, Ga,
                                      Gb, Ge);
    }
    if (!active) return;
    double* __restrict__ wsb = ws + P.state_off * (int64_t)ws_stride;  // [kind][k][N]
    double* __restrict__ dp = dparam + 3 * P.state_off;
#pragma unroll
    for (int j = 0; j < NN; ++j) {
        wsb[(int64_t)j * N + i] = W0[j];
        if constexpr (PP >= 1) wsb[(int64_t)(NN + j) * N + i] = dt * W1[j];
    }
    dp[i] = fixed ? 0.0 : lam * (dt * ih * ih) * Gb;                // d/dnu
    dp[N + i] = fixed ? 0.0 : lam * (-dt * ih) * Ga;                // d/dc (also d/dc_i)
    dp[2 * N + i] = fixed ? 0.0 : lam * (-dt * ih * ih * ih) * Ge;  // d/ddelta
}

template <int NN>
hipError_t go_adj_taylor(const AdjointLaunch& a, hipStream_t s) {
    if (a.p == 0)
        hipLaunchKernelGGL((adj_taylor_kernel<NN, 0>), dim3((unsigned)a.tiles), dim3(T), 0, s, a.tile_probs, a.nprob,
                           a.taylor, a.u, a.lam, a.g, a.ws, a.ws_stride, a.dparam);
    else
        hipLaunchKernelGGL((adj_taylor_kernel<NN, 1>), dim3((unsigned)a.tiles), dim3(T), 0, s, a.tile_probs, a.nprob,
                           a.taylor, a.u, a.lam, a.g, a.ws, a.ws_stride, a.dparam);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_adj_taylor(const AdjointLaunch& a, hipStream_t s) {
    if (a.tiles <= 0) return hipSuccess;
    if (a.p < 0 || a.p > 1 || !a.taylor) return hipErrorInvalidValue;
    switch (a.n) {
        case 3: return go_adj_taylor<3>(a, s);
        case 5: return go_adj_taylor<5>(a, s);
        case 7: return go_adj_taylor<7>(a, s);
        case 9: return go_adj_taylor<9>(a, s);
        case 11: return go_adj_taylor<11>(a, s);
        case 13: return go_adj_taylor<13>(a, s);
        case 15: return go_adj_taylor<15>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lmep
