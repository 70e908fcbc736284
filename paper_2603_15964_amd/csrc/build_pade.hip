// Weight build (steps a3-a6): per local matrix, form the augmented local
// operator, take its exponential by FP64 Pade scaling-and-squaring, and
// harvest the node's row of each block.
//
// Local matrix (compact, transposed form of the paper's augmented block matrix
// of Sec. 3.1, size M = n + p):
//     Mt = dt * [[L^T, e_r, 0], [0, 0, 1], [0, 0, 0]]
// exp(Mt) holds, in rows < n, column r of e^{dt L^T} (= row r of e^{dt L},
// the W0 harvest), column n = dt phi1(dt L^T) e_r (= row r of dt phi1(dt L),
// W1) and column n+1 = dt^2 phi2(dt L^T) e_r (row r of dt^2 phi2, W2 * dt).
// Transposing puts the harvested rows into columns, so lane k (= stencil
// position k) ends up holding weight k of every kind, ready for the
// structure-of-arrays weight layout that the apply kernel reads coalesced.
//
// Exponential: degree-13 diagonal Pade approximant with scaling and squaring
// (Higham 2005, "The scaling and squaring method for the matrix exponential
// revisited"): s = max(0, ceil(log2(||Mt|| / theta13))) chosen per matrix from
// its own norm (so no matrix is over-scaled), U and V from A^2, A^4, A^6, one
// linear solve, s squarings.  The norm is the infinity norm of Mt (the 1-norm
// of the untransposed augmented matrix).  One local matrix per 16-lane DPP
// row, lane i holding row i; four matrices per wavefront.
#include "lmep_device.hpp"

namespace lmep {
namespace {

constexpr double kTheta13 = 5.371920351148152;  // Higham 2005, Table 2.3

// [13/13] Pade coefficients of e^x normalised to c_0 = 1:
// c_j = (26 - j)! 13! / (26! j! (13 - j)!), via c_{j+1} = c_j (13 - j) / ((26 - j)(j + 1)).
constexpr double pade13c(int j) {
    double c = 1.0;
    for (int i = 0; i < j; ++i) c = c * (double)(13 - i) / ((double)(26 - i) * (double)(i + 1));
    return c;
}

template <int M>
__device__ __forceinline__ void add_identity(double (&X)[M], double a, int lane) {
#pragma unroll
    for (int j = 0; j < M; ++j) X[j] += (j == lane) ? a : 0.0;
}

// P = V + U, Q = V - U for the degree-13 approximant of A (row matrices):
//   U = A (A6 (c13 A6 + c11 A4 + c9 A2) + c7 A6 + c5 A4 + c3 A2 + c1 I)
//   V =    A6 (c12 A6 + c10 A4 + c8 A2) + c6 A6 + c4 A4 + c2 A2 + c0 I
// The inner products accumulate into the linear combination they are added to.
template <int M, int NB>
__device__ __forceinline__ void pade13(const double (&A)[M], double (&P)[M], double (&Q)[M], int lane) {
    constexpr double c[14] = {pade13c(0), pade13c(1), pade13c(2),  pade13c(3),  pade13c(4),
                              pade13c(5), pade13c(6), pade13c(7),  pade13c(8),  pade13c(9),
                              pade13c(10), pade13c(11), pade13c(12), pade13c(13)};
    double A2[M], A4[M], A6[M], T[M], W[M];
    mul<M, NB>(A, A, A2);
    mul<M, NB>(A2, A2, A4);
    mul<M, NB>(A4, A2, A6);
#pragma unroll
    for (int j = 0; j < M; ++j) {
        T[j] = c[13] * A6[j] + c[11] * A4[j] + c[9] * A2[j];
        W[j] = c[7] * A6[j] + c[5] * A4[j] + c[3] * A2[j];
    }
    add_identity(W, c[1], lane);
    mul_acc<M, NB>(A6, T, W);  // W = inner factor of U
#pragma unroll
    for (int j = 0; j < M; ++j) {
        T[j] = c[12] * A6[j] + c[10] * A4[j] + c[8] * A2[j];
        Q[j] = c[6] * A6[j] + c[4] * A4[j] + c[2] * A2[j];
    }
    add_identity(Q, c[0], lane);
    mul_acc<M, NB>(A6, T, Q);  // Q = V
    mul<M, NB>(A, W, T);  // T = U
#pragma unroll
    for (int j = 0; j < M; ++j) {  // V and U are formed separately: V - U may cancel
        const double v = Q[j], u = T[j];
        P[j] = v + u;
        Q[j] = v - u;
    }
}

// Column `col` of the row matrix X, one entry per lane (lane i gets X[i][col]).
template <int M>
__device__ __forceinline__ double column(const double (&X)[M], int col) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < M; ++k) v = (k == col) ? X[k] : v;
    return v;
}

// Power-of-two balancing of a row matrix (lane i holds row i): B = D^-1 A D
// with D = diag(d) chosen to equalise each row's and column's off-diagonal
// 1-norms (Parlett and Reinsch 1969; LAPACK's gebal without permutations).
// Scaling by powers of two is exact and exp(A) = D exp(B) D^-1.  Returns this
// lane's d.  Used for the stationary tables of one-sided windows, whose edge
// rows make the local matrix badly scaled: there it cuts the squarings and
// the FP64 error of the harvested row by one to three orders of magnitude.
template <int M>
__device__ __forceinline__ double balance_rows(double (&A)[M], int lane) {
    double d = 1.0;
    for (int sweep = 0; sweep < 32; ++sweep) {
        bool changed = false;
        sfor<M>([&](auto ic) {
            constexpr int I = decltype(ic)::value;
            const double c = row_sum16(lane != I ? fabs(A[I]) : 0.0);  // column I, off-diagonal
            double rs = 0.0;
#pragma unroll
            for (int j = 0; j < M; ++j) rs += (j != lane) ? fabs(A[j]) : 0.0;
            const double r = bcast<I>(rs);  // row I, off-diagonal
            if (c != 0.0 && r != 0.0) {
                double f = 1.0, cc = c;
                while (cc < 0.5 * r) { f *= 2.0; cc *= 4.0; }
                while (cc >= 2.0 * r) { f *= 0.5; cc *= 0.25; }
                if ((cc + r) / f < 0.95 * (c + r)) {
                    changed = true;
                    if (lane == I) {
#pragma unroll
                        for (int j = 0; j < M; ++j) A[j] /= f;
                        d *= f;
                    }
                    A[I] *= f;
                }
            }
        });
        if (!changed) break;
    }
    return d;
}

// (X * X)[:, col] given the column v = X[:, col] distributed over the lanes.
template <int M>
__device__ __forceinline__ double square_column(const double (&X)[M], double v) {
    double c = 0.0;
    exec_guard();
    sfor<M>([&](auto kc) {
        constexpr int K = decltype(kc)::value;
        fmac_b1<K>(c, v, X[K]);
    });
    return c;
}

// FUSE (frozen-velocity ETD1 only): instead of writing the weights, the row
// goes on to the node's update (step a8): lane k forms W0[k] u_j + W1[k] N_j at
// stencil position j = S_i(k), with N_j = -g (u_j - u_i) (du/dx)_j and
// (du/dx)_j from j's own stencil, and the sixteen lanes' terms are summed into
// u_out[i].  The weights never reach HBM.
template <int NN, int PP, bool FUSE>
__global__ __launch_bounds__(256) void build_pade_kernel(const DevProb* __restrict__ probs, int nprob, int64_t items,
                                                         const double* __restrict__ fd, const double* __restrict__ u,
                                                         double* __restrict__ w,
                                                         unsigned long long* __restrict__ stats,
                                                         double* __restrict__ u_out) {
    constexpr int M = NN + PP;
    static_assert(!FUSE || PP == 1, "the fused update is ETD1");
    static_assert(M <= kMaxM, "local matrix exceeds one DPP row");
    const int lane = threadIdx.x & 15;
    const int64_t item = xcd_block(blockIdx.x, gridDim.x) * 16 + (threadIdx.x >> 4);
    if (item >= items) return;  // the whole 16-lane row leaves together

    const DevProb& P = probs[find_instance(probs, nprob, item)];
    const int64_t local = item - P.item_begin;
    const bool frozen = P.frozen != 0;
    const int64_t node = frozen ? local : 0;
    const double dt = P.dt;
    double ceff = P.c;
    if (frozen) ceff += P.nl_coef * u[P.state_off + node];
    const int r = frozen ? (int)(-window_offset(node, P.N, NN, P.bc, P.window, ceff)) : (int)local;

    // Row `lane` of Mt: dt * L[k][lane] for k < n (column `lane` of the local
    // operator L = -c D1 + nu D2 - delta D3 + react I on the stencil).
    const double ih = 1.0 / P.h;
    const double a1 = -ceff * ih * dt, a2 = P.nu * ih * ih * dt, a3 = -P.delta * ih * ih * ih * dt;
    const double ar = P.react * dt;
    double A[M];
    const int lc = lane < NN ? lane : 0;
#pragma unroll
    for (int k = 0; k < NN; ++k) {
        const double d1 = fd[fd_index(NN, 0, k, lc)], d2 = fd[fd_index(NN, 1, k, lc)],
                     d3 = fd[fd_index(NN, 2, k, lc)];
        const double v = a1 * d1 + a2 * d2 + a3 * d3 + (k == lane ? ar : 0.0);
        A[k] = lane < NN ? v : 0.0;
    }
    if constexpr (PP >= 1) A[NN] = (lane == r) ? dt : 0.0;
    if constexpr (PP >= 2) A[NN + 1] = (lane == NN) ? dt : 0.0;
    if constexpr (PP >= 3) A[NN + 2] = (lane == NN + 1) ? dt : 0.0;
    // balancing costs about as much as the exponential here, so it is kept to
    // stationary tables (built once); frozen-velocity one-sided windows are
    // stable only for small n, where the unbalanced FP64 rows are accurate
    const bool balanced = P.window == WIN_UPWIND && !frozen;
    const double dbal = balanced ? balance_rows(A, lane) : 1.0;

    double rs = 0.0;
#pragma unroll
    for (int k = 0; k < M; ++k) rs += fabs(A[k]);
    const double nrm = row_max16(rs);
    int s = 0;
    if (nrm > kTheta13) {
        int e;
        const double f = frexp(nrm / kTheta13, &e);
        s = (f == 0.5) ? e - 1 : e;
    }
#pragma unroll
    for (int k = 0; k < M; ++k) A[k] = ldexp(A[k], -s);

    double X[M], Q[M];
    pade13<M, NN>(A, X, Q, lane);
    solve_inplace<M, NN>(Q, X, lane);
    // s squarings, alternating between X and A; only the harvested columns
    // (r and the augmented ones) of the last square are formed
    int q = s;
    while (q >= 3) {
        mul<M, NN>(X, X, A);
        mul<M, NN>(A, A, X);
        q -= 2;
    }
    if (q == 2) {
        mul<M, NN>(X, X, A);
#pragma unroll
        for (int j = 0; j < M; ++j) X[j] = A[j];
    }
    double w0 = column(X, r), w1 = 0.0, w2 = 0.0, w3 = 0.0;
    if constexpr (PP >= 1) w1 = X[NN];
    if constexpr (PP >= 2) w2 = X[NN + 1];
    if constexpr (PP >= 3) w3 = X[NN + 2];
    if (q >= 1) {
        w0 = square_column(X, w0);
        if constexpr (PP >= 1) w1 = square_column(X, w1);
        if constexpr (PP >= 2) w2 = square_column(X, w2);
        if constexpr (PP >= 3) w3 = square_column(X, w3);
    }
    if (balanced) {  // entry (k, j) of exp(Mt) is d_k exp(B)[k][j] / d_j
        w0 *= dbal / __shfl(dbal, r, 16);
        if constexpr (PP >= 1) w1 *= dbal / bcast<NN>(dbal);
        if constexpr (PP >= 2) w2 *= dbal / bcast<NN + 1>(dbal);
        if constexpr (PP >= 3) w3 *= dbal / bcast<NN + 2>(dbal);
    }

    if (stats && lane == 0) {  // profiling only: matrices built and squarings done
        atomicAdd(stats, 1ull);
        atomicAdd(stats + 1, (unsigned long long)s);
    }
    if constexpr (FUSE) {
        const int64_t N = P.N;
        const int bc = P.bc;
        const double* __restrict__ us = u + P.state_off;
        constexpr int R = (NN - 1) / 2;
        double term = 0.0;
        if (lane < NN) {
            const double ih = 1.0 / P.h;
            double uj, d = 0.0;
            if (P.window == WIN_CENTRED && node >= 2 * R && node + 2 * R <= N - 1) {
                // interior: the node's window and each window node's own window
                // are centred and in the grid
                const double* __restrict__ wj = us + (node - 2 * R + lane);
                uj = wj[R];
#pragma unroll
                for (int l = 0; l < NN; ++l) d += (fd[fd_index(NN, 0, R, l)] * ih) * wj[l];
            } else if (P.window == WIN_UPWIND && node >= 4 * R && node + 4 * R <= N - 1) {
                // interior, one-sided: every window involved lies in the grid
                // (no wrap, reflection or clamp); each lane picks its own side
                const int64_t j = node - r + lane;
                uj = us[j];
                const double aj = P.c + P.nl_coef * uj;
                const int oj = aj > 0.0 ? -(NN - 1) : (aj < 0.0 ? 0 : -R);
                const double* __restrict__ wj = us + (j + oj);
#pragma unroll
                for (int l = 0; l < NN; ++l) d += (fd[fd_index(NN, 0, -oj, l)] * ih) * wj[l];
            } else {
                const int64_t j = map_index(node - r + lane, N, bc);  // stencil position (mirror node for Neumann)
                uj = us[j];
                const int64_t oj = window_offset(j, N, NN, bc, P.window, P.c + P.nl_coef * uj);
                const int rj = (int)(-oj);
#pragma unroll
                for (int l = 0; l < NN; ++l)
                    d += (fd[fd_index(NN, 0, rj, l)] * ih) * us[map_index(j + oj + l, N, bc)];
            }
            const double Nj = -P.nl_coef * (uj - us[node]) * d;
            term = w0 * uj;
            term += w1 * Nj;
        }
        const double sum = row_sum16(term);
        if (lane == 0) {
            const bool fixed = bc == BC_DIRICHLET && (node == 0 || node == N - 1);
            u_out[P.state_off + node] = fixed ? (node == 0 ? P.bc_left : P.bc_right) : sum;
        }
        return;
    }
    if (lane >= NN) return;
    double* __restrict__ wb = w + P.weight_off;
    if (frozen) {
        const int64_t N = P.N;
        wb[(int64_t)lane * N + node] = w0;
        if constexpr (PP >= 1) wb[(int64_t)(NN + lane) * N + node] = w1;
        if constexpr (PP == 2) wb[(int64_t)(2 * NN + lane) * N + node] = w2 / dt;
    } else if constexpr (PP == 3) {
        // ETDRK4 full step: e^{L dt} and dt alpha, dt beta, dt gamma from the
        // rows dt phi1 = w1, dt phi2 = w2 / dt, dt phi3 = w3 / dt^2 (Sec. 3)
        const double f1 = w1, f2 = w2 / dt, f3 = w3 / (dt * dt);
        wb[(2 * NN + r) * NN + lane] = w0;
        wb[(3 * NN + r) * NN + lane] = f1 - 3.0 * f2 + 4.0 * f3;
        wb[(4 * NN + r) * NN + lane] = 2.0 * f2 - 4.0 * f3;
        wb[(5 * NN + r) * NN + lane] = 4.0 * f3 - f2;
    } else {
        // plain harvest, or the ETDRK4 half step (p = 1 at dt / 2: kinds 0, 1)
        wb[r * NN + lane] = w0;
        if constexpr (PP >= 1) wb[(NN + r) * NN + lane] = w1;
        if constexpr (PP == 2) wb[(2 * NN + r) * NN + lane] = w2 / dt;
    }
}

template <int NN, int PP>
hipError_t launch_np(const DevProb* d_probs, int nprob, int64_t items, const double* fd, const double* d_u,
                     double* d_w, unsigned long long* stats, double* d_u_out, hipStream_t stream) {
    if constexpr (NN + PP > kMaxM) {
        return hipErrorInvalidValue;
    } else {
        const int64_t blocks = (items + 15) / 16;
        if (d_u_out) {
            if constexpr (PP == 1)
                hipLaunchKernelGGL((build_pade_kernel<NN, PP, true>), dim3((unsigned)blocks), dim3(256), 0, stream,
                                   d_probs, nprob, items, fd, d_u, d_w, stats, d_u_out);
            else
                return hipErrorInvalidValue;
        } else {
            hipLaunchKernelGGL((build_pade_kernel<NN, PP, false>), dim3((unsigned)blocks), dim3(256), 0, stream,
                               d_probs, nprob, items, fd, d_u, d_w, stats, d_u_out);
        }
        return hipGetLastError();
    }
}

template <int NN>
hipError_t launch_n(int p, const DevProb* d_probs, int nprob, int64_t items, const double* fd, const double* d_u,
                    double* d_w, unsigned long long* stats, double* d_u_out, hipStream_t stream) {
    switch (p) {
        case 0: return launch_np<NN, 0>(d_probs, nprob, items, fd, d_u, d_w, stats, d_u_out, stream);
        case 1: return launch_np<NN, 1>(d_probs, nprob, items, fd, d_u, d_w, stats, d_u_out, stream);
        case 2: return launch_np<NN, 2>(d_probs, nprob, items, fd, d_u, d_w, stats, d_u_out, stream);
        case 3: return launch_np<NN, 3>(d_probs, nprob, items, fd, d_u, d_w, stats, d_u_out, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

hipError_t launch_build(int n, int p, const DevProb* d_probs, int nprob, int64_t items, const double* fd,
                        const double* d_u, double* d_w, unsigned long long* stats, hipStream_t stream,
                        double* d_u_out) {
    if (items <= 0) return hipSuccess;
    switch (n) {
        case 3: return launch_n<3>(p, d_probs, nprob, items, fd, d_u, d_w, stats, d_u_out, stream);
        case 5: return launch_n<5>(p, d_probs, nprob, items, fd, d_u, d_w, stats, d_u_out, stream);
        case 7: return launch_n<7>(p, d_probs, nprob, items, fd, d_u, d_w, stats, d_u_out, stream);
        case 9: return launch_n<9>(p, d_probs, nprob, items, fd, d_u, d_w, stats, d_u_out, stream);
        case 11: return launch_n<11>(p, d_probs, nprob, items, fd, d_u, d_w, stats, d_u_out, stream);
        case 13: return launch_n<13>(p, d_probs, nprob, items, fd, d_u, d_w, stats, d_u_out, stream);
        case 15: return launch_n<15>(p, d_probs, nprob, items, fd, d_u, d_w, stats, d_u_out, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace lmep
