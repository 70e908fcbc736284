// Frozen-velocity weight build by a finite Taylor series (steps a3-a6 for the
// frozen-velocity Burgers operator under ETD1; with FUSE also a7-a8).
//
// Why a finite series is exact.  On a uniform grid the window's derivative
// matrices are those of its interpolating polynomial (Sec. 2.1): with D the
// first-derivative matrix on unit spacing, D^(2) = D^2, D^(3) = D^3, and
// D^n = 0 because n derivatives annihilate a polynomial of degree n - 1.  So
// dt L = q(D) with q(x) = a x + b x^2 + e x^3 (a = -c dt/h, b = nu dt/h^2,
// e = -delta dt/h^3; no reaction term), every function of dt L is a
// polynomial of degree n - 1 in D, and the augmented matrix of Sec. 3.1 is
// nilpotent as well: its exponential is a finite sum, no Pade approximant and
// no squarings are needed.  With
//     e^{theta q(x)} = sum_k M_k(theta) x^k / k!,
//     M_0 = 1,  M_{k+1} = theta a M_k + 2 theta b k M_{k-1} + 3 theta e k (k-1) M_{k-2}
// (from d/dx e^{theta q} = theta q' e^{theta q}), the harvested rows are
//     row r of e^{dt L}        = sum_k M_k(1) T_k[r],
//     row r of dt phi1(dt L)   = dt sum_k (int_0^1 M_k(theta) dtheta) T_k[r],
// where T_k[r][j] = (D^k)[r][j] / k! is the coefficient of y^k in l_j(x_r + y)
// for the window's Lagrange basis polynomial l_j (a per-device table).  M_k is
// a polynomial in theta, M_k = sum_m mu[k][m] theta^m, so the integral is
// sum_m mu[k][m] / (m + 1).  This is O(n^2) work per node against the
// O(n^3 log) of a Pade exponential of the (n+1) x (n+1) augmented matrix.
//
// Conditioning.  e^{theta a D} translates a polynomial by theta a, so the
// sums above add large terms of both signs when |a| spans several nodes.  As
// e^{s D} is an exact translation by s, the same weights follow from the
// expansion about node r' = r + s with theta a replaced by theta a - s in the
// moment recursion:
//     mu[k+1][m] = a mu[k][m-1] - s mu[k][m] + 2 b k mu[k-1][m-1] + 3 e k (k-1) mu[k-2][m-1],
// taking T_k[r'] in place of T_k[r].  s is the integer nearest a / 2 (the
// middle of the translation range [0, a] that theta sweeps), kept inside the
// window; each node picks its own, so its result does not depend on which
// wavefront it falls in.  When every lane of a wavefront expands about the
// same row (every interior wavefront while |a| < 1, and most of them beyond),
// the table row is read through the scalar unit; otherwise per lane.
//
// Layout: one thread per node, kTaylorTile consecutive nodes of one instance
// per block.  With FUSE the block first stages u and the frozen-velocity
// derivative (du/dx)_j (from each position's own window, as in the Pade
// kernel's fused step) for its nodes and a halo of n - 1 positions on each side
// in LDS; each node then forms u+_i = sum_j W0[j] u_j + W1[j] N_j with
// N_j = -g (u_j - u_i) (du/dx)_j over its window (the factor -g rides on W1
// with dt), and the weights never leave registers.  Without FUSE the weights
// are written in the per-node layout.
//
// One-sided windows of 9 or more points take the same build in double-double
// (build_taylor_dd_kernel, one step per launch; the weight routine is in
// taylor_dd.hpp), and so do stationary one-sided tables (build_table_dd_kernel).
#include "lmep_device.hpp"
#include "taylor_dd.hpp"

namespace lmep {
namespace {

// The recursion's per-order coefficients 2 k b and 3 k (k - 1) e.  They are
// fixed for an instance and step size: the multi-step kernel forms them once
// per launch (CoefTable); elsewhere each is formed where it is used
// (CoefAtUse), which keeps fewer registers live.  Same values either way.
struct CoefAtUse {
    double b, e;
    __device__ __forceinline__ double bk(int k) const { return (double)(2 * k) * b; }
    __device__ __forceinline__ double ek(int k) const { return (double)(3 * k * (k - 1)) * e; }
};
template <int NN>
struct CoefTable {
    double bk_[NN], ek_[NN];
    __device__ __forceinline__ double bk(int k) const { return bk_[k]; }
    __device__ __forceinline__ double ek(int k) const { return ek_[k]; }
};
template <int NN>
__device__ __forceinline__ CoefTable<NN> coef_table(double b, double e) {
    const CoefAtUse u{b, e};
    CoefTable<NN> c;
#pragma unroll
    for (int k = 0; k < NN; ++k) {
        c.bk_[k] = u.bk(k);
        c.ek_[k] = u.ek(k);
    }
    return c;
}

// Weights of one node from table row T (T[k * TS + j] = T_k[r'][j]).
// SHIFT: s != 0; DISP: e != 0.
template <int NN, bool SHIFT, bool DISP, int TS, class CF>
__device__ __forceinline__ void taylor_weights(double a, const CF& cf, double s,
                                               const double* __restrict__ T, double (&W0)[NN], double (&W1)[NN]) {
    double m2[NN], m1[NN], m0[NN];  // mu[k-2][.], mu[k-1][.], mu[k][.]
#pragma unroll
    for (int m = 0; m < NN; ++m) {
        m2[m] = 0.0;
        m1[m] = 0.0;
        m0[m] = 0.0;
    }
    m0[0] = 1.0;
#pragma unroll
    for (int j = 0; j < NN; ++j) {  // order 0: M_0 = 1, its integral 1
        const double t = T[j];
        W0[j] = t;
        W1[j] = t;
    }
    // Without a shift mu[k][m] can be non-zero only for lo(k) <= m <= k: the
    // coefficient of x^k in (theta q(x))^m / m! needs m <= k <= 2m (3m with
    // the cubic term).  Terms whose moment lies outside that range are exact
    // zeros and are skipped (multiplying by a zero is not folded away for us).
    constexpr auto lo = [](int k) constexpr { return SHIFT ? 0 : (DISP ? (k + 2) / 3 : (k + 1) / 2); };
#pragma unroll
    for (int k = 0; k + 1 < NN; ++k) {
        const double bk = cf.bk(k);
        const double ek = cf.ek(k);
        double nx[NN];
#pragma unroll
        for (int m = 0; m < NN; ++m) {
            // every term an explicit fma (a plain first product could be
            // contracted into the sums below differently in different kernels)
            double v = 0.0;
            if (m <= k + 1 && m >= lo(k + 1)) {
                if (SHIFT && m <= k) v = -s * m0[m];
                if (m >= 1 && m - 1 >= lo(k)) v = fma(a, m0[m - 1], v);
                if (k >= 1 && m >= 1 && m - 1 >= lo(k - 1) && m <= k) v = fma(bk, m1[m - 1], v);
                if (DISP && k >= 2 && m >= 1 && m - 1 >= lo(k - 2) && m <= k - 1) v = fma(ek, m2[m - 1], v);
            }
            nx[m] = v;
        }
        double E = -0.0, F = -0.0;  // -0.0: the first sum term needs no add
#pragma unroll
        for (int m = 0; m < NN; ++m) {
            m2[m] = m1[m];
            m1[m] = m0[m];
            m0[m] = nx[m];
            if (m <= k + 1 && m >= lo(k + 1) && (SHIFT || m >= 1)) {
                E += nx[m];
                F = fma(nx[m], 1.0 / (double)(m + 1), F);
            }
        }
        const double* __restrict__ Tk = T + (k + 1) * TS;
#pragma unroll
        for (int j = 0; j < NN; ++j) {
            const double t = Tk[j];
            W0[j] = fma(E, t, W0[j]);
            W1[j] = fma(F, t, W1[j]);
        }
    }
}

template <int NN, bool SHIFT, int TS = kMaxN, class CF>
__device__ __forceinline__ void taylor_weights_d(bool disp, double a, const CF& cf, double s,
                                                 const double* __restrict__ T, double (&W0)[NN], double (&W1)[NN]) {
    if (disp)
        taylor_weights<NN, SHIFT, true, TS, CF>(a, cf, s, T, W0, W1);
    else
        taylor_weights<NN, SHIFT, false, TS, CF>(a, cf, s, T, W0, W1);
}

// The n x n x n block of the table for this stencil size, copied to LDS as
// lt[(r' * NN + k) * NN + j]: mixed wavefronts read their rows from there.
template <int NN>
__device__ __forceinline__ void stage_taylor_block(const double* __restrict__ taylor, double* lt, int tid, int nt) {
    for (int i = tid; i < NN * NN * NN; i += nt) {
        const int rp = i / (NN * NN), k = (i / NN) % NN, j = i % NN;
        lt[i] = taylor[taylor_index(NN, rp, k, j)];
    }
}

// Weights of this lane's node (harvest row r, shift sh) with the expansion
// row r + sh read through the scalar unit when the wavefront's active lanes
// share it; otherwise each lane reads its own row, from the LDS copy of the
// table block when the kernel holds one (lt != nullptr), else from the table
// in global memory.  Lanes with the same (r, sh) get the same values either
// way.
template <int NN, class CF>
__device__ __forceinline__ void node_weights(bool active, int r, int sh, bool disp, double a, const CF& cf,
                                             const double* __restrict__ taylor, const double* lt, double (&W0)[NN],
                                             double (&W1)[NN]) {
    const double* __restrict__ tb = taylor + taylor_index(NN, 0, 0, 0);
    int rp = r + sh;
    rp = rp < 0 ? 0 : (rp > NN - 1 ? NN - 1 : rp);
    const int r0 = __builtin_amdgcn_readfirstlane(r), rp0 = __builtin_amdgcn_readfirstlane(rp);
    if (__ballot(active && (r != r0 || rp != rp0)) == 0) {
        const double* __restrict__ T = tb + rp0 * (kMaxN * kMaxN);
        if (rp0 == r0)
            taylor_weights_d<NN, false>(disp, a, cf, 0.0, T, W0, W1);
        else
            taylor_weights_d<NN, true>(disp, a, cf, (double)(rp0 - r0), T, W0, W1);
    } else if (lt) {
        const double* lr = lt + rp * (NN * NN);
        if constexpr (NN <= 7) {
            // the whole row in registers first: one round of LDS reads instead
            // of one per order (larger rows would spill)
            double Tl[NN * NN];
#pragma unroll
            for (int i = 0; i < NN * NN; ++i) Tl[i] = lr[i];
            taylor_weights_d<NN, true, NN>(disp, a, cf, (double)(rp - r), Tl, W0, W1);
        } else {
            taylor_weights_d<NN, true, NN>(disp, a, cf, (double)(rp - r), lr, W0, W1);
        }
    } else {
        taylor_weights_d<NN, true>(disp, a, cf, (double)(rp - r), tb + rp * (kMaxN * kMaxN), W0, W1);
    }
}

// The one-step kernel's body; DD: weights in double-double from the
// double-double table (`taylor` is then that table).
template <int NN, bool FUSE, bool DD>
__device__ __forceinline__ void build_taylor_body(const DevProb* __restrict__ probs, int nprob,
                                                  const double* __restrict__ fd, const double* __restrict__ taylor,
                                                  const double* __restrict__ u, double* __restrict__ w,
                                                  unsigned long long* __restrict__ stats, double* __restrict__ u_out) {
    constexpr int R = (NN - 1) / 2;
    constexpr int H = NN - 1;  // staged halo: a one-sided window reaches n - 1 positions
    constexpr int S = kTaylorTile + 2 * H;
    __shared__ double su[FUSE ? S : 1], sd[FUSE ? S : 1];

    const int64_t tile = xcd_block(blockIdx.x, gridDim.x);
    const DevProb& P = probs[find_instance(probs, nprob, tile)];
    const int64_t N = P.N;
    const int64_t node0 = (tile - P.item_begin) * kTaylorTile;
    const int bc = P.bc;
    const double* __restrict__ us = u + P.state_off;
    const double ih = 1.0 / P.h, g = P.nl_coef;
    const int tid = threadIdx.x;
    if (stats && tid == 0) atomicAdd(stats, (unsigned long long)(N - node0 < kTaylorTile ? N - node0 : kTaylorTile));

    if constexpr (FUSE) {
        // positions node0 - H .. min(node0 + tile, N) - 1 + H; on Dirichlet grids
        // only those inside the grid (windows never leave it)
        const int64_t vend = (node0 + kTaylorTile < N ? node0 + kTaylorTile : N) + H;
        for (int sl = tid; sl < S; sl += kTaylorTile) {
            const int64_t v = node0 - H + sl;
            double uv = 0.0, dv = 0.0;
            if (v < vend && (bc != BC_DIRICHLET || (v >= 0 && v < N))) {
                const int64_t j = map_index(v, N, bc);
                uv = us[j];
                const int64_t oj = window_offset(j, N, NN, bc, P.window, P.c + g * uv);
                if (oj == -R && j >= R && j + R <= N - 1) {
#pragma unroll
                    for (int l = 0; l < NN; ++l) dv += (fd[fd_index(NN, 0, R, l)] * ih) * us[j - R + l];
                } else if (j + oj >= 0 && j + oj + NN - 1 <= N - 1) {
                    const int rj = (int)(-oj);
#pragma unroll
                    for (int l = 0; l < NN; ++l) dv += (fd[fd_index(NN, 0, rj, l)] * ih) * us[j + oj + l];
                } else {
                    const int rj = (int)(-oj);
#pragma unroll
                    for (int l = 0; l < NN; ++l)
                        dv += (fd[fd_index(NN, 0, rj, l)] * ih) * us[map_index(j + oj + l, N, bc)];
                }
            }
            su[sl] = uv;
            sd[sl] = dv;
        }
        __syncthreads();
    }

    const int64_t node = node0 + tid;
    const bool active = node < N;
    // lane 0 holds the wavefront's first node: past the end, so is every lane
    if (__builtin_amdgcn_readfirstlane(active ? 1 : 0) == 0) return;
    const int64_t nd = active ? node : N - 1;  // idle lanes repeat the last node; their results are dropped
    const double ui = FUSE ? su[tid + H] : us[nd];
    const double ceff = P.c + g * ui;
    const int r = (int)(-window_offset(nd, N, NN, bc, P.window, ceff));
    const double dt = P.dt;
    const double a = -ceff * ih * dt, b = P.nu * ih * ih * dt, e = -P.delta * ih * ih * ih * dt;
    const bool disp = P.delta != 0.0;
    const double half = fmin(fmax(0.5 * a, -(double)NN), (double)NN);
    const int sh = (int)rint(half);

    double W0[NN], W1[NN];
    // fused: W1 carries -g dt, so the window term is (u_j - u_i) d_j
    const double w1s = FUSE ? -g * dt : dt;
    if constexpr (DD) {
        double W2[NN];
        node_weights_dd<NN, 1>(r, sh, a, b, e, w1s, taylor, W0, W1, W2);
    } else {
        node_weights<NN>(active, r, sh, disp, a, CoefAtUse{b, e}, taylor, nullptr, W0, W1);
#pragma unroll
        for (int j = 0; j < NN; ++j) W1[j] *= w1s;
    }

    if constexpr (FUSE) {
        const int base = tid + H - r;  // slot of window position 0
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < NN; ++j) {
            const double uj = su[base + j];
            const double Nj = (uj - ui) * sd[base + j];
            acc = fma(W0[j], uj, acc);
            acc = fma(W1[j], Nj, acc);
        }
        if (active) {
            const bool fixed = bc == BC_DIRICHLET && (node == 0 || node == N - 1);
            u_out[P.state_off + node] = fixed ? (node == 0 ? P.bc_left : P.bc_right) : acc;
        }
    } else if (active) {
        double* __restrict__ wb = w + P.weight_off;
#pragma unroll
        for (int j = 0; j < NN; ++j) {
            wb[(int64_t)j * N + node] = W0[j];
            wb[(int64_t)(NN + j) * N + node] = W1[j];
        }
    }
}

template <int NN, bool FUSE>
__global__ __launch_bounds__(kTaylorTile) void build_taylor_kernel(const DevProb* __restrict__ probs, int nprob,
                                                                   const double* __restrict__ fd,
                                                                   const double* __restrict__ taylor,
                                                                   const double* __restrict__ u,
                                                                   double* __restrict__ w,
                                                                   unsigned long long* __restrict__ stats,
                                                                   double* __restrict__ u_out) {
    build_taylor_body<NN, FUSE, false>(probs, nprob, fd, taylor, u, w, stats, u_out);
}
template <int NN, bool FUSE>
__global__ __launch_bounds__(kTaylorTile) void build_taylor_dd_kernel(const DevProb* __restrict__ probs, int nprob,
                                                                      const double* __restrict__ fd,
                                                                      const double* __restrict__ tdd,
                                                                      const double* __restrict__ u,
                                                                      double* __restrict__ w,
                                                                      unsigned long long* __restrict__ stats,
                                                                      double* __restrict__ u_out) {
    build_taylor_body<NN, FUSE, true>(probs, nprob, fd, tdd, u, w, stats, u_out);
}

// Several frozen-velocity steps per launch (LMEP_F_PERSISTENT; centred or
// one-sided windows on Dirichlet or periodic grids).  A block stages reg <=
// kTaylorRegion consecutive positions of its instance in LDS, advances them
// ksteps <= kb steps there and writes the middle reg - 2 kb (n - 1) of them.
// Each step spoils n - 1 positions at each open end of the valid range (a
// node's window reaches (n-1)/2 positions and the frozen-velocity derivative
// at a window position another (n-1)/2), 2 (n - 1) with one-sided windows; at
// a Dirichlet end inside the region the windows are clamped and nothing is
// spoilt.  Every node is formed by the
// same expressions in the same order as in the one-step kernel (derivative
// from the position's own window, weights of the node, stencil sum), so the
// two paths agree bit for bit.  The block copies the first-derivative rows of
// its stencil size to LDS, and on a Dirichlet grid the table block as well:
// the wavefronts next to an end, whose lanes harvest different window rows,
// read their rows from there at every step instead of from global memory.
// Elsewhere a wavefront's lanes part only where the shift or the window side
// changes; those few read the table in global memory, which measured faster.
template <int NN>
__device__ __forceinline__ void taylor_stepk_body(const DevProb* __restrict__ probs, int nprob, int kb, int ksteps,
                                                  int reg, const double* __restrict__ fd,
                                                  const double* __restrict__ taylor,
                                                  const double* __restrict__ u_in, double* __restrict__ u_out,
                                                  unsigned long long* __restrict__ stats) {
    constexpr int R = (NN - 1) / 2;
    constexpr int H = NN - 1;
    constexpr int MAXR = kTaylorRegion;
    __shared__ double lds[3 * MAXR];  // current u, next u, derivative: addressed by offsets
    __shared__ double lt[NN * NN * NN];  // this stencil size's table block
    __shared__ double lfd[NN * NN];      // first-derivative rows of the clamped and one-sided windows
    const int REG = reg;
    const int nt = blockDim.x;  // threads: one staged position each per pass (normally nt = reg)
    const int64_t tile = xcd_block(blockIdx.x, gridDim.x);
    const DevProb& P = probs[find_instance(probs, nprob, tile)];
    const int64_t N = P.N;
    const bool upw = P.window == WIN_UPWIND;
    const int rw = upw ? H : R;       // reach of a window and of a derivative's window
    const int halo = kb * taylor_stepk_reach(NN, upw);
    const int tw = REG - 2 * halo;  // nodes written per block
    const int bc = P.bc;
    const bool dir = bc == BC_DIRICHLET;
    const int64_t own = (tile - P.item_begin) * tw;  // first node this block is responsible for
    // On a Dirichlet grid the last block is moved back to end at node N - 1
    // (it rewrites part of its neighbour's tile with the same values): a node
    // next to an end has its window shifted inwards by up to (n-1)/2, and the
    // derivatives at that window reach (n-1)/2 further, so a short last region
    // would not hold what its nodes depend on.
    const int64_t first = (dir && N >= tw && own > N - tw) ? N - tw : own;
    const int64_t v0 = first - halo;  // grid position of slot 0
    const double* __restrict__ us = u_in + P.state_off;
    const double ih = 1.0 / P.h, g = P.nl_coef, dt = P.dt;
    const bool disp = P.delta != 0.0;
    const int tid = threadIdx.x;
    if (stats && tid == 0) {
        const int64_t wn = N - own < tw ? N - own : tw;
        atomicAdd(stats, (unsigned long long)(wn * ksteps));
    }
    // slots holding grid nodes: on Dirichlet grids the part of the region inside the grid
    const int g_lo = dir ? (int)(v0 < 0 ? -v0 : 0) : 0;
    const int g_hi = dir ? (int)(N - v0 < REG ? N - v0 : REG) : REG;
    int cu = 0, cn = MAXR;
    const int cd = 2 * MAXR;
    for (int t = tid; t < REG; t += nt)
        lds[cu + t] = (t >= g_lo && t < g_hi) ? us[map_index(v0 + t, N, bc)] : 0.0;
    if (dir) stage_taylor_block<NN>(taylor, lt, tid, nt);
    for (int i = tid; i < NN * NN; i += nt) lfd[i] = fd[fd_index(NN, 0, i / NN, i % NN)] * ih;
    __syncthreads();
    int lo = g_lo, hi = g_hi;  // slots whose current u is valid
    // loop invariants, formed by the same expressions as in the one-step
    // kernel; held in registers across the steps up to n = 9 (beyond, they
    // would spill and are formed at each use instead)
    constexpr bool HOIST = NN <= 9;
    const CoefTable<NN> cf0 =
        coef_table<NN>(HOIST ? P.nu * ih * ih * dt : 0.0, HOIST ? -P.delta * ih * ih * ih * dt : 0.0);
    double fdc[NN];  // centred first-derivative row
#pragma unroll
    for (int l = 0; l < NN; ++l) fdc[l] = HOIST ? fd[fd_index(NN, 0, R, l)] * ih : 0.0;
    for (int st = 0; st < ksteps; ++st) {
        const bool lend = dir && v0 + lo == 0, rend = dir && v0 + hi == N;  // grid ends: nothing spoilt
        const int nlo = lend ? lo : lo + 2 * rw, nhi = rend ? hi : hi - 2 * rw;  // slots updated this step
        const int dlo = lend ? lo : lo + rw, dhi = rend ? hi : hi - rw;          // slots whose derivative they read
        for (int t = dlo + tid; t < dhi; t += nt) {
            const int64_t j = map_index(v0 + t, N, bc);
            const int oj = (int)window_offset(j, N, NN, bc, P.window, P.c + g * lds[cu + t]);
            double dv = 0.0;
            if (oj == -R) {  // centred row
#pragma unroll
                for (int l = 0; l < NN; ++l)
                    dv += (HOIST ? fdc[l] : fd[fd_index(NN, 0, R, l)] * ih) * lds[cu + t - R + l];
            } else {
                const double* fr = lfd + (-oj) * NN;
#pragma unroll
                for (int l = 0; l < NN; ++l) dv += fr[l] * lds[cu + t + oj + l];
            }
            lds[cd + t] = dv;
        }
        __syncthreads();
        for (int base = 0; base < REG; base += nt) {
            const int t = base + tid;
            const bool active = t >= nlo && t < nhi;
            if (__ballot(active) == 0) continue;  // the whole wavefront idles (uniform)
            const int te = active ? t : nlo;     // idle lanes repeat a valid slot; their results are dropped
            const int64_t i = map_index(v0 + te, N, bc);
            const double ui = lds[cu + te];
            const double ceff = P.c + g * ui;
            const int o = (int)window_offset(i, N, NN, bc, P.window, ceff);
            const int r = -o;
            const double a = -ceff * ih * dt;
            const double half = fmin(fmax(0.5 * a, -(double)NN), (double)NN);
            const int sh = (int)rint(half);
            double W0[NN], W1[NN];
            if constexpr (HOIST)
                node_weights<NN>(active, r, sh, disp, a, cf0, taylor, dir ? lt : nullptr, W0, W1);
            else
                node_weights<NN>(active, r, sh, disp, a, CoefAtUse{P.nu * ih * ih * dt, -P.delta * ih * ih * ih * dt},
                                 taylor, dir ? lt : nullptr, W0, W1);
            const double w1s = -g * dt;  // as in the one-step kernel
#pragma unroll
            for (int j = 0; j < NN; ++j) W1[j] *= w1s;
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < NN; ++j) {
                const double uj = lds[cu + te + o + j];
                const double Nj = (uj - ui) * lds[cd + te + o + j];
                acc = fma(W0[j], uj, acc);
                acc = fma(W1[j], Nj, acc);
            }
            if (active) {
                const bool fixed = dir && (i == 0 || i == N - 1);
                lds[cn + t] = fixed ? (i == 0 ? P.bc_left : P.bc_right) : acc;
            }
        }
        __syncthreads();
        const int tmp = cu;
        cu = cn;
        cn = tmp;
        lo = nlo;
        hi = nhi;
    }
    double* __restrict__ uo = u_out + P.state_off;
    for (int t = halo + tid; t < halo + tw; t += nt) {
        const int64_t node = v0 + t;
        if (node < N) uo[node] = lds[cu + t];
    }
}

template <int NN>
__global__ __launch_bounds__(kTaylorRegion) void taylor_stepk_kernel(const DevProb* __restrict__ probs, int nprob,
                                                                   int kb, int ksteps, int reg,
                                                                   const double* __restrict__ fd,
                                                                   const double* __restrict__ taylor,
                                                                   const double* __restrict__ u_in,
                                                                   double* __restrict__ u_out,
                                                                   unsigned long long* __restrict__ stats) {
    taylor_stepk_body<NN>(probs, nprob, kb, ksteps, reg, fd, taylor, u_in, u_out, stats);
}
// Stationary one-sided tables in double-double: one thread per harvested row
// (items = n per instance, item_begin = the instance's first row), the plain
// layout [kind][r][k] with W1 = dt phi1 and W2 = dt phi2 rows.
template <int NN, int PP>
__global__ __launch_bounds__(64) void build_table_dd_kernel(const DevProb* __restrict__ probs, int nprob,
                                                            int64_t items, const double* __restrict__ tdd,
                                                            double* __restrict__ w) {
    const int64_t item = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (item >= items) return;
    const DevProb& P = probs[find_instance(probs, nprob, item)];
    const int r = (int)(item - P.item_begin);
    const double ih = 1.0 / P.h, dt = P.dt;
    const double a = -P.c * ih * dt, b = P.nu * ih * ih * dt, e = -P.delta * ih * ih * ih * dt;
    const double half = fmin(fmax(0.5 * a, -(double)NN), (double)NN);
    double W0[NN], W1[NN], W2[NN];
    node_weights_dd<NN, PP>(r, (int)rint(half), a, b, e, dt, tdd, W0, W1, W2);
    double* __restrict__ wb = w + P.weight_off;
#pragma unroll
    for (int k = 0; k < NN; ++k) {
        wb[r * NN + k] = W0[k];
        if constexpr (PP >= 1) wb[(NN + r) * NN + k] = W1[k];
        if constexpr (PP >= 2) wb[(2 * NN + r) * NN + k] = W2[k];
    }
}

template <int NN>
hipError_t go_taylor(bool dd, const DevProb* d_probs, int nprob, int64_t tiles, const double* fd, const double* taylor,
                     const double* d_u, double* d_w, unsigned long long* stats, double* d_u_out, hipStream_t stream) {
    if constexpr (NN < kTaylorDdMinN) {
        if (dd) return hipErrorInvalidValue;
    } else if (dd) {
        if (d_u_out)
            hipLaunchKernelGGL((build_taylor_dd_kernel<NN, true>), dim3((unsigned)tiles), dim3(kTaylorTile), 0,
                               stream, d_probs, nprob, fd, taylor, d_u, d_w, stats, d_u_out);
        else
            hipLaunchKernelGGL((build_taylor_dd_kernel<NN, false>), dim3((unsigned)tiles), dim3(kTaylorTile), 0,
                               stream, d_probs, nprob, fd, taylor, d_u, d_w, stats, d_u_out);
        return hipGetLastError();
    }
    if (d_u_out)
        hipLaunchKernelGGL((build_taylor_kernel<NN, true>), dim3((unsigned)tiles), dim3(kTaylorTile), 0, stream,
                           d_probs, nprob, fd, taylor, d_u, d_w, stats, d_u_out);
    else
        hipLaunchKernelGGL((build_taylor_kernel<NN, false>), dim3((unsigned)tiles), dim3(kTaylorTile), 0, stream,
                           d_probs, nprob, fd, taylor, d_u, d_w, stats, d_u_out);
    return hipGetLastError();
}

template <int NN, int PP>
hipError_t go_table_dd(const DevProb* d_probs, int nprob, int64_t items, const double* tdd, double* d_w,
                       hipStream_t stream) {
    hipLaunchKernelGGL((build_table_dd_kernel<NN, PP>), dim3((unsigned)((items + 63) / 64)), dim3(64), 0, stream,
                       d_probs, nprob, items, tdd, d_w);
    return hipGetLastError();
}
template <int NN>
hipError_t go_table_dd_p(int p, const DevProb* d_probs, int nprob, int64_t items, const double* tdd, double* d_w,
                         hipStream_t stream) {
    switch (p) {
        case 0: return go_table_dd<NN, 0>(d_probs, nprob, items, tdd, d_w, stream);
        case 1: return go_table_dd<NN, 1>(d_probs, nprob, items, tdd, d_w, stream);
        case 2: return go_table_dd<NN, 2>(d_probs, nprob, items, tdd, d_w, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_taylor_stepk(int n, int kb, int ksteps, int reg, const DevProb* d_probs, int nprob, int64_t tiles,
                               const double* fd, const double* taylor, const double* d_u_in, double* d_u_out,
                               unsigned long long* stats, hipStream_t stream) {
    if (tiles <= 0) return hipSuccess;
    if (tiles > 0x7fffffff || kb < 1 || kb > 8 || ksteps < 1 || ksteps > kb || reg < 64 || reg > kTaylorRegion ||
        reg % 64 != 0 || taylor_stepk_tile(n, kb, reg, false) < 1)
        return hipErrorInvalidValue;
#define LMEP_TSK_CASE(NN)                                                                                         \
    case NN:                                                                                                      \
        hipLaunchKernelGGL((taylor_stepk_kernel<NN>), dim3((unsigned)tiles), dim3(reg), 0, stream, d_probs, nprob,  \
                           kb, ksteps, reg, fd, taylor, d_u_in, d_u_out, stats);                                  \
        return hipGetLastError();
    switch (n) {
        LMEP_TSK_CASE(3) LMEP_TSK_CASE(5) LMEP_TSK_CASE(7) LMEP_TSK_CASE(9) LMEP_TSK_CASE(11) LMEP_TSK_CASE(13)
        LMEP_TSK_CASE(15)
        default: return hipErrorInvalidValue;
    }
#undef LMEP_TSK_CASE
}

hipError_t launch_build_table_dd(int n, int p, const DevProb* d_probs, int nprob, int64_t items, const double* tdd,
                                 double* d_w, hipStream_t stream) {
    if (items <= 0) return hipSuccess;
    if (items > 0x7fffffffLL * 64) return hipErrorInvalidValue;
    switch (n) {
        case 3: return go_table_dd_p<3>(p, d_probs, nprob, items, tdd, d_w, stream);
        case 5: return go_table_dd_p<5>(p, d_probs, nprob, items, tdd, d_w, stream);
        case 7: return go_table_dd_p<7>(p, d_probs, nprob, items, tdd, d_w, stream);
        case 9: return go_table_dd_p<9>(p, d_probs, nprob, items, tdd, d_w, stream);
        case 11: return go_table_dd_p<11>(p, d_probs, nprob, items, tdd, d_w, stream);
        case 13: return go_table_dd_p<13>(p, d_probs, nprob, items, tdd, d_w, stream);
        case 15: return go_table_dd_p<15>(p, d_probs, nprob, items, tdd, d_w, stream);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_build_taylor(int n, const DevProb* d_probs, int nprob, int64_t tiles, const double* fd,
                               const double* taylor, const double* d_u, double* d_w, unsigned long long* stats,
                               hipStream_t stream, double* d_u_out, bool dd) {
    if (tiles <= 0) return hipSuccess;
    if (tiles > 0x7fffffff) return hipErrorInvalidValue;
    switch (n) {
        case 3: return go_taylor<3>(dd, d_probs, nprob, tiles, fd, taylor, d_u, d_w, stats, d_u_out, stream);
        case 5: return go_taylor<5>(dd, d_probs, nprob, tiles, fd, taylor, d_u, d_w, stats, d_u_out, stream);
        case 7: return go_taylor<7>(dd, d_probs, nprob, tiles, fd, taylor, d_u, d_w, stats, d_u_out, stream);
        case 9: return go_taylor<9>(dd, d_probs, nprob, tiles, fd, taylor, d_u, d_w, stats, d_u_out, stream);
        case 11: return go_taylor<11>(dd, d_probs, nprob, tiles, fd, taylor, d_u, d_w, stats, d_u_out, stream);
        case 13: return go_taylor<13>(dd, d_probs, nprob, tiles, fd, taylor, d_u, d_w, stats, d_u_out, stream);
        case 15: return go_taylor<15>(dd, d_probs, nprob, tiles, fd, taylor, d_u, d_w, stats, d_u_out, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lmep
