// Step a2 -- finite-difference weights on the stencil (Sec. 2.1 step 1: the
// standard differentiation matrix of the stencil, computed with Fornberg's
// recursion for arbitrarily spaced nodes).  On a uniform grid the stencil
// matrix does not depend on where the stencil sits, so one table per stencil
// size serves every node: weights on the centred integer nodes
// x_k = k - (n-1)/2, scaled by h^-d where they are used.  The table is a
// static device array filled once per device by fd_table_kernel.
//
// A second table serves the finite-Taylor build (build_taylor.hip): the
// derivatives of every order 0..n-1 of the window's Lagrange basis
// polynomials at each window node, divided by the order's factorial, i.e. the
// rows of D1^k / k! (D1 the unit-spacing first-derivative matrix).
#include <mutex>

#include "dd.hpp"
#include "lmep_device.hpp"

namespace lmep {
namespace {

__device__ double g_fd_table[kFdTableDoubles];
__device__ double g_taylor_table[kTaylorTableDoubles];
__device__ double g_taylor_dd_table[2 * kTaylorTableDoubles];  // high parts, then low parts

// Fornberg (1988), "Generation of finite difference formulas on arbitrarily
// spaced grids": weights c[j][d] of node j for the d-th derivative at z,
// built up one node at a time; derivatives up to order MD.
template <int MD>
__device__ void fornberg_weights(int n, double z, const double* x, double (*c)[MD + 1]) {
    for (int j = 0; j < n; ++j)
        for (int d = 0; d <= MD; ++d) c[j][d] = 0.0;
    c[0][0] = 1.0;
    double c1 = 1.0, c4 = x[0] - z;
    for (int i = 1; i < n; ++i) {
        const int mn = i < MD ? i : MD;
        double c2 = 1.0;
        const double c5 = c4;
        c4 = x[i] - z;
        for (int j = 0; j < i; ++j) {
            const double c3 = x[i] - x[j];
            c2 *= c3;
            if (j == i - 1) {  // new node i, from node i-1's weights before they are updated
                for (int d = mn; d >= 1; --d) c[i][d] = c1 * (d * c[i - 1][d - 1] - c5 * c[i - 1][d]) / c2;
                c[i][0] = -c1 * c5 * c[i - 1][0] / c2;
            }
            for (int d = mn; d >= 1; --d) c[j][d] = (c4 * c[j][d] - d * c[j][d - 1]) / c3;
            c[j][0] = c4 * c[j][0] / c3;
        }
        c1 = c2;
    }
}

// One thread per (stencil size, evaluation node a).
__global__ void fd_table_kernel(double* __restrict__ tab) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kNumFd * kFdMaxN) return;
    const int n = 3 + 2 * (t / kFdMaxN);
    const int a = t % kFdMaxN;
    if (a >= n) return;
    double x[kFdMaxN];
    for (int k = 0; k < n; ++k) x[k] = (double)k - 0.5 * (double)(n - 1);
    double c[kFdMaxN][4];
    fornberg_weights<3>(n, x[a], x, c);
    for (int d = 0; d < kFdDerivs; ++d)
        for (int k = 0; k < n; ++k) tab[fd_index(n, d, a, k)] = c[k][d + 1];
}

// One thread per (stencil size, expansion node a): entry (a, k, j) is the
// k-th derivative of basis polynomial j at node a over k! -- the coefficient
// of y^k in l_j(x_a + y).
__global__ void taylor_table_kernel(double* __restrict__ tab) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kNumN * kMaxN) return;
    const int n = 3 + 2 * (t / kMaxN);
    const int a = t % kMaxN;
    if (a >= n) return;
    double x[kMaxN];
    for (int k = 0; k < n; ++k) x[k] = (double)k - 0.5 * (double)(n - 1);
    double c[kMaxN][kMaxN];
    fornberg_weights<kMaxN - 1>(n, x[a], x, c);
    double fact = 1.0;
    for (int d = 0; d < n; ++d) {
        if (d > 1) fact *= (double)d;
        for (int j = 0; j < n; ++j) tab[taylor_index(n, a, d, j)] = c[j][d] / fact;
    }
}

std::mutex g_mu;
const double* g_ptr[64] = {};
const double* g_taylor_ptr[64] = {};

// The same table in double-double, exactly rounded: on the integer stencil
// l_j(x_a + y) = prod_{m != j} (y + a - m) / prod_{m != j} (j - m), whose
// numerator coefficients and denominator are integers below 2^53 for n <= 15
// (products of at most 14 factors of size <= 14), so each entry is one
// double-double quotient of two exact doubles.  One thread per (stencil size,
// expansion node a, basis polynomial j).
__global__ void taylor_dd_table_kernel(double* __restrict__ hi, double* __restrict__ lo) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= kNumN * kMaxN * kMaxN) return;
    const int n = 3 + 2 * (t / (kMaxN * kMaxN));
    const int a = (t / kMaxN) % kMaxN, j = t % kMaxN;
    if (a >= n || j >= n) return;
    double c[kMaxN] = {};  // coefficients of the numerator, lowest first
    c[0] = 1.0;
    int deg = 0;
    double den = 1.0;
    for (int m = 0; m < n; ++m) {
        if (m == j) continue;
        const double d = (double)(a - m);
        for (int k = deg + 1; k >= 1; --k) c[k] = c[k - 1] + d * c[k];
        c[0] *= d;
        ++deg;
        den *= (double)(j - m);
    }
    for (int k = 0; k < n; ++k) {
        const dd q = dd_div_d(dd_of(c[k]), den);
        hi[taylor_index(n, a, k, j)] = q.hi;
        lo[taylor_index(n, a, k, j)] = q.lo;
    }
}

}  // namespace

hipError_t taylor_dd_table_init(const double** d_table_out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    static const double* ptr[64] = {};
    std::lock_guard<std::mutex> lock(g_mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_taylor_dd_table))) != hipSuccess) return e;
        double* hi = (double*)p;
        const int threads = kNumN * kMaxN * kMaxN;
        hipLaunchKernelGGL(taylor_dd_table_kernel, dim3((threads + 255) / 256), dim3(256), 0, nullptr, hi,
                           hi + kTaylorTableDoubles);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
        ptr[dev] = hi;
    }
    *d_table_out = ptr[dev];
    return hipSuccess;
}

hipError_t fd_table_init(const double** d_table_out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_fd_table))) != hipSuccess) return e;
        hipLaunchKernelGGL(fd_table_kernel, dim3(1), dim3(kNumFd * kFdMaxN), 0, nullptr, (double*)p);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
        g_ptr[dev] = (const double*)p;
    }
    *d_table_out = g_ptr[dev];
    return hipSuccess;
}

hipError_t taylor_table_init(const double** d_table_out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_taylor_ptr[dev]) {
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_taylor_table))) != hipSuccess) return e;
        hipLaunchKernelGGL(taylor_table_kernel, dim3(1), dim3(kNumN * kMaxN), 0, nullptr, (double*)p);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
        g_taylor_ptr[dev] = (const double*)p;
    }
    *d_table_out = g_taylor_ptr[dev];
    return hipSuccess;
}

}  // namespace lmep
