// Weight build on non-uniform grids (steps a2-a6 with per-node stencils,
// Sec. 4.3.3): every node has its own local operator, built from the
// differentiation matrices of its own window's coordinates, and its own
// exponential, harvested once (the weights are stationary).  The same kernel
// builds the stationary table of a uniform instance whose augmented matrix
// is too large for a 16-lane DPP row (ETDRK4 with n + 3 > 16): one matrix per
// harvested row r, on the window x_a = (a - r) h, written as [kind][r][k].
//
// Per node:
//   * coordinates of the window relative to the node, xs_a = x_{i+o+a} - x_i;
//   * D1 from the derivative of the Lagrange basis on those nodes,
//       D1[a][b] = pi_a / (pi_b (xs_a - xs_b)) (a != b),
//       D1[a][a] = sum_{b != a} 1 / (xs_a - xs_b),   pi_b = prod_{l != b} (xs_b - xs_l),
//     and D2 = D1 D1, D3 = D2 D1 (D1 maps polynomials of degree < n to their
//     derivatives, so its powers are the higher-derivative matrices);
//   * L = -c D1 + nu D2 - delta D3 + react I and the compact transposed
//     augmented matrix Mt = dt [[L^T, e_r, 0], [0, 0, 1], [0, 0, 0]] of order
//     m = n + p, as in the uniform build;
//   * balancing: a diagonal similarity by powers of two, Mt = D B D^-1, that
//     equalises row and column norms (Parlett and Reinsch 1969, the scheme of
//     LAPACK's gebal without permutations); the windows next to clustered
//     Chebyshev ends have entries spread over ten orders of magnitude, which
//     scaling-and-squaring on Mt itself turns into errors up to 1e-3 (n = 21)
//     while on B it needs no squaring at all.  Scaling by powers of two is
//     exact, and exp(Mt) = D exp(B) D^-1;
//   * exp(B) by degree-13 Pade scaling-and-squaring (s from the infinity norm
//     of B, the uniform build's rule), with the linear solve done by
//     Gauss-Jordan elimination with partial pivoting;
//   * columns r, n, n+1 of exp(Mt) -> W0, W1, W2 of the node, stored per node
//     ([kind][k][node]); for an ETDRK4 table also column n+2 (dt^3 phi3), and
//     the rows e^{L dt}, dt alpha, dt beta, dt gamma of Sec. 3 from them.
//
// Orders up to 32 (stencils up to 25 points) do not fit the 16-lane DPP rows
// of the uniform build, and these weights are built once, so the layout here
// is plain: one wavefront per node, its matrices in LDS (row stride m + 1),
// each product spread over the 64 lanes one output entry at a time.
#include "lmep_device.hpp"

namespace lmep {
namespace {

constexpr int kWaveThreads = 64;
constexpr double kTheta13w = 5.371920351148152;  // Higham 2005, Table 2.3

constexpr double pade13w(int j) {
    double c = 1.0;
    for (int i = 0; i < j; ++i) c = c * (double)(13 - i) / ((double)(26 - i) * (double)(i + 1));
    return c;
}

// C = X Y for m x m matrices with row stride ld (C distinct from X and Y).
__device__ __forceinline__ void mm(const double* __restrict__ X, const double* __restrict__ Y,
                                   double* __restrict__ C, int m, int ld, int lane) {
    for (int e = lane; e < m * m; e += kWaveThreads) {
        const int i = e / m, j = e - i * m;
        double acc = 0.0;
        for (int k = 0; k < m; ++k) acc = fma(X[i * ld + k], Y[k * ld + j], acc);
        C[i * ld + j] = acc;
    }
    __syncthreads();
}

__global__ __launch_bounds__(kWaveThreads) void build_wide_kernel(const DevProb* __restrict__ probs, int nprob,
                                                                 double* __restrict__ w) {
    extern __shared__ double lds[];
    constexpr double c0 = pade13w(0), c1 = pade13w(1), c2 = pade13w(2), c3 = pade13w(3), c4 = pade13w(4),
                     c5 = pade13w(5), c6 = pade13w(6), c7 = pade13w(7), c8 = pade13w(8), c9 = pade13w(9),
                     c10 = pade13w(10), c11 = pade13w(11), c12 = pade13w(12), c13 = pade13w(13);
    const int lane = threadIdx.x;
    const int64_t item = blockIdx.x;  // one node per block
    const DevProb& P = probs[find_instance(probs, nprob, item)];
    const int64_t node = item - P.item_begin;  // node, or harvested row of a uniform table
    const int64_t N = P.N;
    const bool uni = P.x == nullptr;
    const int n = P.n, m = n + P.p, ld = m + 1, sz = m * ld;
    double* A = lds;
    double* A2 = A + sz;
    double* A4 = A2 + sz;
    double* A6 = A4 + sz;
    double* W1 = A6 + sz;
    double* W2 = W1 + sz;
    double* W3 = W2 + sz;
    double* xs = W3 + sz;   // n window coordinates
    double* pis = xs + n;   // n products pi_b
    double* red = pis + n;  // row sums
    double* dsc = red + m;  // balancing scale factors
    int* piv = (int*)(dsc + m);

    const int64_t o = uni ? -node : window_offset(node, N, n, P.bc);
    const int r = (int)(-o);
    const double* __restrict__ x = P.x;
    if (lane < n) xs[lane] = uni ? (double)(lane - r) * P.h : x[node + o + lane] - x[node];
    __syncthreads();
    if (lane < n) {
        double pr = 1.0;
        for (int l = 0; l < n; ++l)
            if (l != lane) pr *= xs[lane] - xs[l];
        pis[lane] = pr;
    }
    __syncthreads();
    // D1 in W1, D2 in W2, D3 in W3 (n x n, stride ld)
    for (int e = lane; e < n * n; e += kWaveThreads) {
        const int a = e / n, b = e - a * n;
        double v = 0.0;
        if (a != b) {
            v = (pis[a] / pis[b]) / (xs[a] - xs[b]);
        } else {
            for (int l = 0; l < n; ++l)
                if (l != a) v += 1.0 / (xs[a] - xs[l]);
        }
        W1[a * ld + b] = v;
    }
    __syncthreads();
    mm(W1, W1, W2, n, ld, lane);
    mm(W2, W1, W3, n, ld, lane);

    // Mt = dt [[L^T, e_r, 0], [0, 0, 1], [0, 0, 0]]
    const double dt = P.dt;
    for (int e = lane; e < m * m; e += kWaveThreads) {
        const int i = e / m, j = e - i * m;
        double v = 0.0;
        if (i < n && j < n) {
            // row i of L^T = column i of L: L[j][i]
            v = -P.c * W1[j * ld + i] + P.nu * W2[j * ld + i] - P.delta * W3[j * ld + i];
            if (i == j) v += P.react;
            v *= dt;
        } else if ((i == r && j == n) || (i >= n && j == i + 1)) {
            v = dt;
        }
        A[i * ld + j] = v;
    }
    __syncthreads();

    // balancing: B = D^-1 Mt D with D = diag(dsc), powers of two
    if (lane < m) dsc[lane] = 1.0;
    __syncthreads();
    for (int sweep = 0; sweep < 32; ++sweep) {
        bool changed = false;
        for (int i = 0; i < m; ++i) {
            double cv = (lane < m && lane != i) ? fabs(A[lane * ld + i]) : 0.0;  // column i, off-diagonal
            double rv = (lane < m && lane != i) ? fabs(A[i * ld + lane]) : 0.0;  // row i, off-diagonal
            for (int off = 32; off >= 1; off >>= 1) {  // butterfly: every lane ends with the same sums
                cv += __shfl_xor(cv, off);
                rv += __shfl_xor(rv, off);
            }
            if (cv == 0.0 || rv == 0.0) continue;
            double f = 1.0, c = cv;
            const double total = cv + rv;
            while (c < 0.5 * rv) { f *= 2.0; c *= 4.0; }
            while (c >= 2.0 * rv) { f *= 0.5; c *= 0.25; }
            if ((c + rv) / f < 0.95 * total) {
                changed = true;
                __syncthreads();
                if (lane < m) {
                    A[i * ld + lane] /= f;
                    A[lane * ld + i] *= f;
                }
                if (lane == 0) dsc[i] *= f;
                __syncthreads();
            }
        }
        if (!changed) break;
    }
    if (lane < m) {
        double rs = 0.0;
        for (int j = 0; j < m; ++j) rs += fabs(A[lane * ld + j]);
        red[lane] = rs;
    }
    __syncthreads();
    double nrm = 0.0;
    for (int i = 0; i < m; ++i) nrm = fmax(nrm, red[i]);
    int s = 0;
    if (nrm > kTheta13w) {
        int ex;
        const double f = frexp(nrm / kTheta13w, &ex);
        s = (f == 0.5) ? ex - 1 : ex;
    }
    for (int e = lane; e < m * m; e += kWaveThreads) {
        const int i = e / m, j = e - i * m;
        A[i * ld + j] = ldexp(A[i * ld + j], -s);
    }
    __syncthreads();

    // degree-13 Pade: U = A (A6 (c13 A6 + c11 A4 + c9 A2) + c7 A6 + c5 A4 + c3 A2 + c1 I)
    //                 V =    A6 (c12 A6 + c10 A4 + c8 A2) + c6 A6 + c4 A4 + c2 A2 + c0 I
    mm(A, A, A2, m, ld, lane);
    mm(A2, A2, A4, m, ld, lane);
    mm(A4, A2, A6, m, ld, lane);
    for (int e = lane; e < m * m; e += kWaveThreads) {
        const int i = e / m, j = e - i * m, q = i * ld + j;
        W1[q] = c13 * A6[q] + c11 * A4[q] + c9 * A2[q];
    }
    __syncthreads();
    mm(A6, W1, W2, m, ld, lane);
    for (int e = lane; e < m * m; e += kWaveThreads) {
        const int i = e / m, j = e - i * m, q = i * ld + j;
        W2[q] += c7 * A6[q] + c5 * A4[q] + c3 * A2[q] + (i == j ? c1 : 0.0);
    }
    __syncthreads();
    mm(A, W2, W1, m, ld, lane);  // U
    for (int e = lane; e < m * m; e += kWaveThreads) {
        const int i = e / m, j = e - i * m, q = i * ld + j;
        W2[q] = c12 * A6[q] + c10 * A4[q] + c8 * A2[q];
    }
    __syncthreads();
    mm(A6, W2, W3, m, ld, lane);
    for (int e = lane; e < m * m; e += kWaveThreads) {
        const int i = e / m, j = e - i * m, q = i * ld + j;
        const double v = W3[q] + c6 * A6[q] + c4 * A4[q] + c2 * A2[q] + (i == j ? c0 : 0.0);  // V
        W2[q] = v + W1[q];  // P = V + U
        W3[q] = v - W1[q];  // Q = V - U
    }
    __syncthreads();

    // Q X = P by Gauss-Jordan elimination with partial pivoting; X in W2
    for (int c = 0; c < m; ++c) {
        if (lane == 0) {
            int p = c;
            double best = fabs(W3[c * ld + c]);
            for (int i = c + 1; i < m; ++i) {
                const double v = fabs(W3[i * ld + c]);
                if (v > best) { best = v; p = i; }
            }
            piv[0] = p;
        }
        __syncthreads();
        const int p = piv[0];
        if (p != c) {
            for (int j = lane; j < m; j += kWaveThreads) {
                double t = W3[c * ld + j]; W3[c * ld + j] = W3[p * ld + j]; W3[p * ld + j] = t;
                t = W2[c * ld + j]; W2[c * ld + j] = W2[p * ld + j]; W2[p * ld + j] = t;
            }
            __syncthreads();
        }
        if (lane < m) red[lane] = (lane == c) ? 0.0 : W3[lane * ld + c] / W3[c * ld + c];
        __syncthreads();
        for (int e = lane; e < m * m; e += kWaveThreads) {
            const int i = e / m, j = e - i * m;
            if (i == c) continue;
            const double f = red[i];
            if (j > c) W3[i * ld + j] -= f * W3[c * ld + j];
            W2[i * ld + j] -= f * W2[c * ld + j];
        }
        __syncthreads();
    }
    for (int e = lane; e < m * m; e += kWaveThreads) {
        const int i = e / m, j = e - i * m;
        W2[i * ld + j] /= W3[i * ld + i];
    }
    __syncthreads();

    // s squarings, alternating between W2 and W1 (chosen by parity, so the
    // pointers stay plain offsets into lds and keep their address space)
    for (int q = 0; q < s; ++q) {
        if (q & 1) mm(W1, W1, W2, m, ld, lane);
        else mm(W2, W2, W1, m, ld, lane);
    }
    const double* X = lds + ((s & 1) ? 4 : 5) * sz;  // W1 or W2
    // exp(Mt) = D exp(B) D^-1: entry (k, j) is dsc[k] X[k][j] / dsc[j]
    if (lane < n) {
        double* __restrict__ wb = w + P.weight_off;
        const double dk = dsc[lane];
        const double w0 = dk * X[lane * ld + r] / dsc[r];
        const double w1 = P.p >= 1 ? dk * X[lane * ld + n] / dsc[n] : 0.0;          // row of dt phi1
        const double w2 = P.p >= 2 ? dk * X[lane * ld + n + 1] / dsc[n + 1] : 0.0;  // dt^2 phi2
        const double w3 = P.p >= 3 ? dk * X[lane * ld + n + 2] / dsc[n + 2] : 0.0;  // dt^3 phi3
        if (!uni) {
            wb[(int64_t)lane * N + node] = w0;
            if (P.p >= 1) wb[(int64_t)(n + lane) * N + node] = w1;
            if (P.p >= 2) wb[(int64_t)(2 * n + lane) * N + node] = w2 / dt;
        } else if (P.harvest == HARVEST_RK4_FULL) {
            const double f1 = w1, f2 = w2 / dt, f3 = w3 / (dt * dt);
            wb[(2 * n + r) * n + lane] = w0;
            wb[(3 * n + r) * n + lane] = f1 - 3.0 * f2 + 4.0 * f3;
            wb[(4 * n + r) * n + lane] = 2.0 * f2 - 4.0 * f3;
            wb[(5 * n + r) * n + lane] = 4.0 * f3 - f2;
        } else {  // plain rows, or the ETDRK4 half step (kinds 0, 1)
            wb[r * n + lane] = w0;
            if (P.p >= 1) wb[(n + r) * n + lane] = w1;
            if (P.p >= 2) wb[(2 * n + r) * n + lane] = w2 / dt;
        }
    }
}

}  // namespace

size_t build_wide_lds_bytes(int n, int p) {
    const int m = n + p;
    return sizeof(double) * (size_t)(7 * m * (m + 1) + 2 * n + 2 * m) + 16;
}

hipError_t launch_build_wide(int n, int p, const DevProb* d_probs, int nprob, int64_t items, double* d_w,
                             hipStream_t stream) {
    if (items <= 0) return hipSuccess;
    if (n < 3 || n > kMaxNWide || (n % 2) == 0 || p < 0 || p > 3 || n + p > kMaxMWide) return hipErrorInvalidValue;
    hipLaunchKernelGGL(build_wide_kernel, dim3((unsigned)items), dim3(kWaveThreads), build_wide_lds_bytes(n, p),
                       stream, d_probs, nprob, d_w);
    return hipGetLastError();
}

}  // namespace lmep
