// Reverse step by the finite Taylor series (step a10 for instances without a
// reaction term on uniform grids).  Per node: the weights W0, W1 and the
// derivatives of lam_i u+_i with respect to nu, c and delta through those
// weights -- what adj_frechet_kernel reads off the block-triangular Pade
// exponential, here in O(n^2) per node -- and, in the same kernel, the
// gathers of the reverse step over a tile.
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
// frozen velocity.  Blocks cover tiles of one instance, so a node's result
// does not depend on how the instances are batched.
#include "lmep_device.hpp"

namespace lmep {
namespace {

constexpr int T = kAdjTile;

// One side of a node's work.  ROLE 0 forms W0 and the terms of the
// derivatives that go through it (M_{K-1}(1) tau_K and its b, e analogues);
// ROLE 1 forms W1 and the terms through it (dt I_1(K-1) nu_K ...).  Each side
// runs the moment recursion itself and keeps only the per-order sums it
// uses, so a thread holds one window vector (X = U or V) and one weight row:
// the two sides of a node run in different wavefronts of the block, and the
// parameter terms are the sum of the two sides' parts.
template <int NN, int ROLE, bool SHIFT, bool DISP = true>
__device__ __forceinline__ void adj_taylor_side(double a, double b, double e, double s, double dt,
                                                const double* __restrict__ Tr, const double (&X)[NN],
                                                double (&W)[NN], double& Ga, double& Gb, double& Ge) {
    double m2[NN], m1[NN], m0[NN];  // mu[k-2][.], mu[k-1][.], mu[k][.] (M_k = sum_m mu[k][m] theta^m)
    double Hh[NN];                  // M_j(1) (ROLE 0) or I_1(j) (ROLE 1) of the orders done so far
#pragma unroll
    for (int m = 0; m < NN; ++m) {
        m2[m] = 0.0;
        m1[m] = 0.0;
        m0[m] = 0.0;
    }
    m0[0] = 1.0;
    Hh[0] = ROLE == 0 ? 1.0 : 0.5;
    Ga = 0.0;
    Gb = 0.0;
    Ge = 0.0;
#pragma unroll
    for (int j = 0; j < NN; ++j) W[j] = Tr[j];  // order 0
    // Without a shift mu[k][m] can be non-zero only for lo(k) <= m <= k (the
    // forward series states why); terms on the exact zeros outside that range,
    // and the cubic term when e = 0 (DISP false), are skipped: each remaining
    // term is the same fma as before, so the values do not change.
    constexpr auto lo = [](int k) constexpr { return SHIFT ? 0 : (DISP ? (k + 2) / 3 : (k + 1) / 2); };
#pragma unroll
    for (int k = 0; k + 1 < NN; ++k) {
        const int K = k + 1;  // order formed in this pass
        const double bk = (double)(2 * k) * b;
        const double ek = (double)(3 * k * (k - 1)) * e;
        double nx[NN];
#pragma unroll
        for (int m = 0; m < NN; ++m) {
            double v = 0.0;
            if (m <= K && m >= lo(K)) {
                if (SHIFT && m <= k) v = -s * m0[m];
                if (m >= 1 && m - 1 >= lo(k)) v = fma(a, m0[m - 1], v);
                if (k >= 1 && m >= 1 && m - 1 >= lo(k - 1) && m <= k) v = fma(bk, m1[m - 1], v);
                if (DISP && k >= 2 && m >= 1 && m - 1 >= lo(k - 2) && m <= k - 1) v = fma(ek, m2[m - 1], v);
            }
            nx[m] = v;
        }
        // ROLE 0: C = E = M_K(1); ROLE 1: C = F = int_0^1 M_K, I1 = I_1(K)
        double C = -0.0, I1 = -0.0;
#pragma unroll
        for (int m = 0; m < NN; ++m) {
            m2[m] = m1[m];
            m1[m] = m0[m];
            m0[m] = nx[m];
            if (m <= K && m >= lo(K) && (SHIFT || m >= 1)) {
                if constexpr (ROLE == 0) {
                    C += nx[m];
                } else {
                    C = fma(nx[m], 1.0 / (double)(m + 1), C);
                    I1 = fma(nx[m], 1.0 / (double)(m + 2), I1);
                }
            }
        }
        Hh[K] = ROLE == 0 ? C : I1;
        const double* __restrict__ Tk = Tr + K * kMaxN;
        double dot = -0.0;  // tau_K (ROLE 0) or nu_K (ROLE 1)
#pragma unroll
        for (int j = 0; j < NN; ++j) {
            const double t = Tk[j];
            W[j] = fma(C, t, W[j]);
            dot = fma(t, X[j], dot);
        }
        // derivative terms of order K: K M_{K-1}, K (K-1) M_{K-2}, K (K-1) (K-2) M_{K-3}
        // (through W1: the same with dt I_1 in place of M(1))
        const double f = ROLE == 0 ? 1.0 : dt;
        Ga = fma((double)K * f * Hh[K - 1], dot, Ga);
        if (K >= 2) Gb = fma((double)(K * (K - 1)) * f * Hh[K - 2], dot, Gb);
        if (K >= 3) Ge = fma((double)(K * (K - 1) * (K - 2)) * f * Hh[K - 3], dot, Ge);
    }
}

// Stencils S_i that contain position j, as in the reverse step's gathers, but
// with periodic candidates left unwrapped: calls f(x, k) with x the node's
// index (its unwrapped position on a periodic grid) and k its stencil
// position, in the same order as the one-kernel-per-gather path.
template <class F>
__device__ __forceinline__ void stencils_containing(int64_t j, int64_t N, int n, int bc, F&& f) {
    const int R = (n - 1) / 2;
    int64_t ps[3];
    int np = 0;
    ps[np++] = j;
    if (bc == BC_NEUMANN) {
        if (j > 0 && j <= 2 * R) ps[np++] = -j;
        if (j < N - 1 && j >= N - 1 - 2 * R) ps[np++] = 2 * (N - 1) - j;
    }
    for (int q = 0; q < np; ++q) {
        const int64_t p = ps[q];
        for (int d = -(n - 1); d <= n - 1; ++d) {
            const int64_t x = p + d;
            int64_t i = x;
            if (bc == BC_PERIODIC) {
                i = map_index(x, N, bc);
            } else if (i < 0 || i > N - 1) {
                continue;
            }
            if (bc == BC_DIRICHLET && (i == 0 || i == N - 1)) continue;
            const int64_t o = window_offset(i, N, n, bc);
            const int64_t k = -d - o;
            if (k < 0 || k >= n) continue;
            f(bc == BC_PERIODIC ? x : i, (int)k);
        }
    }
}

// The whole reverse step of a tile of T - 4 (n - 1) nodes in one block of
// 2 T threads:
//   1. stage u, du/dx and lambda over the block's T = 256 weight positions
//      (the tile and 2 (n - 1) on each side) plus the windows' reach;
//   2. each position's weights and parameter terms (adj_taylor_side): threads
//      [0, T) take the W0 side, threads [T, 2T) the W1 side; the weights go
//      to LDS times lambda of their node -- positions next to the tile are
//      recomputed by the neighbouring blocks instead of being exchanged;
//   3. ghat at the positions within n - 1 of the tile (gather over LDS, on
//      threads [T, 2T)), while threads [0, T) sum the part of lambda_k that
//      does not read ghat;
//   4. the ghat terms of lambda_k (gather over LDS), lambda_k written to HBM;
//   5. the tile's parameter terms summed in a fixed order into part[].
// The per-node weights never reach HBM.  Every sum runs in a fixed order, so
// the results do not depend on the launch or on how instances are batched.
// DISP false: no instance of the launch has a dispersion term, and the cubic
// term of the moment recursion (exact zeros then) is left out; the kernel
// then fits in 128 registers, four wavefronts per SIMD.
template <int NN, int PP, bool DISP>
__global__ __launch_bounds__(2 * T) void adj_fused_kernel(const DevProb* __restrict__ probs, int nprob,
                                                      const double* __restrict__ fd,
                                                      const double* __restrict__ taylor,
                                                      const double* __restrict__ u_all,
                                                      const double* __restrict__ lam_all,
                                                      const double* __restrict__ g_all,
                                                      double* __restrict__ lam_out_all, double* __restrict__ part) {
    constexpr int R = (NN - 1) / 2;
    constexpr int H = NN - 1;   // reach of a window
    constexpr int HW = 2 * H;   // weight positions on each side of the tile
    constexpr int TO = T - 2 * HW;  // nodes of the tile
    constexpr int SU = T + 2 * H;   // staged u and du/dx positions
    __shared__ double su[SU], sg[SU], sl[T], sgh[T], sdc[T], sW[2 * NN * T];
    __shared__ double red[3][T];

    const int64_t tile = blockIdx.x;
    const DevProb& P = probs[find_instance(probs, nprob, tile)];
    const int64_t N = P.N;
    const int64_t t0 = (tile - P.item_begin) * TO;  // first node of the tile
    const int64_t base = t0 - HW;                    // position of weight slot 0
    const int bc = P.bc;
    const bool dir = bc == BC_DIRICHLET, per = bc == BC_PERIODIC;
    const double* __restrict__ u = u_all + P.state_off;
    const double* __restrict__ gg = g_all + P.state_off;
    const double dt = P.dt, g = P.nl_coef, ih = 1.0 / P.h;
    const bool burgers = P.nonlin == NL_BURGERS;
    const int tid = threadIdx.x;
    // a position holds a node: inside the grid, or anywhere on a periodic grid
    auto holds = [&](int64_t x) { return per || (x >= 0 && x < N); };

    // 1. staging.  Positions outside a Dirichlet grid, or more than one
    // reflection away from a Neumann grid, are never read (a node's window
    // reaches at most (n-1)/2 beyond an end).
    for (int q = tid; q < SU; q += 2 * T) {
        const int64_t x = base - H + q;
        const bool ok = per || (dir ? (x >= 0 && x < N) : (x >= -(N - 1) && x <= 2 * (N - 1)));
        const int64_t xi = ok ? map_index(x, N, bc) : 0;
        su[q] = ok ? u[xi] : 0.0;
        sg[q] = ok ? gg[xi] : 0.0;
    }
    if (tid < T) {
        const int64_t x = base + tid;
        sl[tid] = holds(x) ? lam_all[P.state_off + map_index(x, N, bc)] : 0.0;
    }
    __syncthreads();

    // 2. weights and parameter terms of weight slot pos: threads [0, T) take
    // the W0 side of slot tid, threads [T, 2T) the W1 side of slot tid - T
    // (whole wavefronts per side)
    double d0 = 0.0, d1 = 0.0, d2 = 0.0;
    {
        const int role = tid >= T ? 1 : 0;
        const int pos = tid - role * T;
        const int64_t x = base + pos;
        const bool active = holds(x);
        // idle lanes take a node of the tile (results dropped)
        const int64_t i = active ? map_index(x, N, bc) : (t0 < N ? t0 : N - 1);
        const int64_t xs = active ? x : i;  // position whose staged window is read
        const int us0 = (int)(xs - (base - H));
        const double ui = su[us0];
        const double ceff = P.c + (burgers ? g * ui : 0.0);
        const int o = (int)window_offset(i, N, NN, bc);
        const int r = -o;
        const double a = -ceff * ih * dt, b = P.nu * ih * ih * dt, e = -P.delta * ih * ih * ih * dt;
        const double half = fmin(fmax(0.5 * a, -(double)NN), (double)NN);
        const int sh = (int)rint(half);
        const double* __restrict__ tb = taylor + taylor_index(NN, 0, 0, 0);
        int rp = r + sh;
        rp = rp < 0 ? 0 : (rp > NN - 1 ? NN - 1 : rp);
        const int r0 = __builtin_amdgcn_readfirstlane(r), rp0 = __builtin_amdgcn_readfirstlane(rp);
        const bool uniform = __ballot(active && (r != r0 || rp != rp0)) == 0;
        double Ga = 0.0, Gb = 0.0, Ge = 0.0;
        // one side of slot pos: the window's U or V, the weights to LDS, the
        // parameter terms to (Ga, Gb, Ge)
        const double lq = sl[pos];  // the weights are stored times lambda of their node
        auto side = [&](auto role_c) {
            constexpr int RL = decltype(role_c)::value;
            double X[NN], W[NN];
#pragma unroll
            for (int j = 0; j < NN; ++j) {
                const double uj = su[us0 + o + j];
                double v = uj;
                if constexpr (RL == 1) {
                    v = 0.0;
                    if (burgers) v = -g * (uj - ui) * sg[us0 + o + j];
                    else if (P.nonlin == NL_AC) v = g * (uj - uj * uj * uj);
                }
                X[j] = v;
            }
            if (uniform) {
                const double* __restrict__ Tr = tb + rp0 * (kMaxN * kMaxN);
                if (rp0 == r0)
                    adj_taylor_side<NN, RL, false, DISP>(a, b, e, 0.0, dt, Tr, X, W, Ga, Gb, Ge);
                else
                    adj_taylor_side<NN, RL, true, DISP>(a, b, e, (double)(rp0 - r0), dt, Tr, X, W, Ga, Gb, Ge);
#pragma unroll
                for (int j = 0; j < NN; ++j) sW[(RL * NN + j) * T + pos] = lq * (RL == 0 ? W[j] : dt * W[j]);
            } else {
                // lanes of several window or table rows (next to an end, or
                // shifts that differ): one pass per distinct (r, r'), each with
                // wave-uniform table rows
                for (;;) {
                    // the lowest lane still here picks the rows of this pass;
                    // it matches itself, so every pass retires at least one lane
                    const int rf = __builtin_amdgcn_readfirstlane(r);
                    const int rpf = __builtin_amdgcn_readfirstlane(rp);
                    if (r == rf && rp == rpf) {
                        adj_taylor_side<NN, RL, true, DISP>(a, b, e, (double)(rpf - rf), dt, tb + rpf * (kMaxN * kMaxN),
                                                            X, W, Ga, Gb, Ge);
#pragma unroll
                        for (int j = 0; j < NN; ++j) sW[(RL * NN + j) * T + pos] = lq * (RL == 0 ? W[j] : dt * W[j]);
                        break;
                    }
                }
            }
        };
        if (role == 0) {
            side(std::integral_constant<int, 0>{});
        } else if constexpr (PP >= 1) {
            side(std::integral_constant<int, 1>{});
            red[0][pos] = Ga;  // the W1 side's parts, added by the W0 side below
            red[1][pos] = Gb;
            red[2][pos] = Ge;
        }
        __syncthreads();
        if (role == 0) {
            if constexpr (PP >= 1) {
                Ga += red[0][pos];
                Gb += red[1][pos];
                Ge += red[2][pos];
            }
            const bool fixed = dir && (i == 0 || i == N - 1);
            const double lam = (active && !fixed) ? sl[pos] : 0.0;
            const bool mine = active && pos >= HW && pos < HW + TO && x < N;  // a node of the tile
            if (mine) {
                d0 = lam * (dt * ih * ih) * Gb;
                d1 = lam * (-dt * ih) * Ga;
                d2 = lam * (-dt * ih * ih * ih) * Ge;
            }
            sdc[pos] = d1;
        }
    }
    __syncthreads();

    // 3. ghat at the weight slots within n - 1 of the tile (threads [T, 2T)),
    // while threads [0, TO) form the part of lambda_k that does not read ghat
    const int64_t j = t0 + tid;
    const bool node_thread = tid < TO && j < N;
    double acc = 0.0;  // lambda_k of node j, summed in the order of the stencil terms
    if (tid >= T) {
        const int q3 = tid - T;
        if (burgers && q3 >= H && q3 < T - H) {
            const int64_t m = base + q3;
            double gacc = 0.0;
            if (holds(m)) {
                const int64_t mi = map_index(m, N, bc);
                const double um = su[q3 + H];
                auto term = [&](int64_t x, int k) {
                    const int q = (int)(x - base);
                    gacc += sW[(NN + k) * T + q] * (-g) * (um - su[q + H]);
                };
                if (gather_interior(mi, N, NN)) {
#pragma unroll
                    for (int d = -R; d <= R; ++d) term(m + d, R - d);
                } else {
                    stencils_containing(per ? m : mi, N, NN, bc, term);
                }
            }
            sgh[q3] = gacc;
        }
    } else if (node_thread) {
        // 4a. the gathers over the weights and the node's own window
        const int qj = HW + tid;  // weight slot of node j
        const double uj = su[qj + H];
        const bool etd = P.scheme == SCH_ETD1;
        double dNj = 0.0;
        if (etd && burgers) dNj = -g * sg[qj + H];
        if (etd && P.nonlin == NL_AC) dNj = g * (1.0 - 3.0 * uj * uj);
        auto term = [&](int64_t x, int k) {
            const int q = (int)(x - base);
            const double w0 = sW[k * T + q];
            acc += etd ? fma(dNj, sW[(NN + k) * T + q], w0) : w0;
        };
        if (gather_interior(j, N, NN)) {
#pragma unroll
            for (int d = -R; d <= R; ++d) term(j + d, R - d);
        } else {
            stencils_containing(j, N, NN, bc, term);
        }
        const bool fixed = dir && (j == 0 || j == N - 1);
        if (burgers && !fixed) {
            const int o = (int)window_offset(j, N, NN, bc);
            double sacc = 0.0;
#pragma unroll
            for (int k = 0; k < NN; ++k) sacc += sW[(NN + k) * T + qj] * sg[qj + H + o + k];
            acc += g * sacc + g * sdc[qj];
        }
    }
    __syncthreads();

    // 4b. the ghat terms of lambda_k, then lambda_k to HBM
    if (node_thread) {
        const int qj = HW + tid;
        if (burgers) {
            if (gather_interior(j, N, NN)) {
#pragma unroll
                for (int d = -R; d <= R; ++d) acc += sgh[qj + d] * fd[fd_index(NN, 0, R, R - d)] * ih;
            } else {
                int64_t ps[3];
                int np = 0;
                ps[np++] = j;
                if (bc == BC_NEUMANN) {
                    if (j > 0 && j <= 2 * R) ps[np++] = -j;
                    if (j < N - 1 && j >= N - 1 - 2 * R) ps[np++] = 2 * (N - 1) - j;
                }
                for (int q = 0; q < np; ++q) {
                    for (int d = -(NN - 1); d <= NN - 1; ++d) {
                        const int64_t x = ps[q] + d;
                        int64_t m = x;
                        if (bc == BC_PERIODIC) m = map_index(x, N, bc);
                        else if (m < 0 || m > N - 1) continue;
                        const int64_t o = window_offset(m, N, NN, bc);
                        const int64_t l = -d - o;
                        if (l < 0 || l >= NN) continue;
                        acc += sgh[(int)((per ? x : m) - base)] * fd[fd_index(NN, 0, (int)(-o), (int)l)] * ih;
                    }
                }
            }
        }
        lam_out_all[P.state_off + j] = acc;
    }

    // 5. the tile's parameter terms, in a fixed order: each wavefront of the
    // W0 side sums its lanes (shuffles), then thread 0 the four wavefront sums
    if (tid < T) {
        double v[3] = {d0, d1 * (tid >= HW && tid < HW + TO ? 1.0 : 0.0), d2};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_down(v[c], off, 64);
            if ((tid & 63) == 0) red[c][tid >> 6] = v[c];
        }
    }
    __syncthreads();
    if (tid == 0)
        for (int c = 0; c < 3; ++c) part[3 * tile + c] = (red[c][0] + red[c][1]) + (red[c][2] + red[c][3]);
}

template <int NN, int PP>
hipError_t go_adj_fused_p(const AdjointLaunch& a, hipStream_t s) {
    if (a.disp)
        hipLaunchKernelGGL((adj_fused_kernel<NN, PP, true>), dim3((unsigned)a.fused_tiles), dim3(2 * T), 0, s,
                           a.fused_probs, a.nprob, a.fd, a.taylor, a.u, a.lam, a.g, a.lam_out, a.part);
    else
        hipLaunchKernelGGL((adj_fused_kernel<NN, PP, false>), dim3((unsigned)a.fused_tiles), dim3(2 * T), 0, s,
                           a.fused_probs, a.nprob, a.fd, a.taylor, a.u, a.lam, a.g, a.lam_out, a.part);
    return hipGetLastError();
}

template <int NN>
hipError_t go_adj_fused(const AdjointLaunch& a, hipStream_t s) {
    return a.p == 0 ? go_adj_fused_p<NN, 0>(a, s) : go_adj_fused_p<NN, 1>(a, s);
}

}  // namespace

hipError_t launch_adj_fused(const AdjointLaunch& a, hipStream_t s) {
    if (a.fused_tiles <= 0) return hipSuccess;
    if (a.p < 0 || a.p > 1 || !a.taylor || !a.fused_probs) return hipErrorInvalidValue;
    switch (a.n) {
        case 3: return go_adj_fused<3>(a, s);
        case 5: return go_adj_fused<5>(a, s);
        case 7: return go_adj_fused<7>(a, s);
        case 9: return go_adj_fused<9>(a, s);
        case 11: return go_adj_fused<11>(a, s);
        case 13: return go_adj_fused<13>(a, s);
        case 15: return go_adj_fused<15>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lmep
