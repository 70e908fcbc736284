// Device helpers shared by the kernel files of liblmep.
//
//  * stencil window / index mapping (step a1),
//  * compile-time loops,
//  * "row matrices": an M x M FP64 matrix (M <= 16) held by one 16-lane DPP
//    row of a wavefront, lane i keeping row i in registers.  A product
//    C = X * Y needs, in lane i, X[i][k] (own register) times Y[k][j] (lane
//    k's register); gfx950's 64-bit DPP broadcast `row_newbcast:k` delivers
//    lane k's register to the whole row as the first source of v_fmac_f64, so
//    every multiply-add of the product is one VALU instruction and no LDS or
//    permute traffic is needed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "lmep_internal.hpp"

namespace lmep {

// ------------------------------------------------------------- step a1 ----
// Stencil of node i: grid indices i+o .. i+o+n-1.  Centred (o = -(n-1)/2),
// or for upwind windows fully one-sided against the node's advection speed a
// (Sec. 4.1): o = -(n-1) for a > 0, o = 0 for a < 0, centred for a = 0.  On
// Dirichlet grids the window is then moved to the n nearest in-domain nodes
// (edge rows next to the ends).  The harvested row is r = -o.
__device__ __forceinline__ int64_t window_offset(int64_t i, int64_t N, int n, int bc, int window = WIN_CENTRED,
                                                 double a = 0.0) {
    int64_t o = -(int64_t)((n - 1) / 2);
    if (window == WIN_UPWIND && a != 0.0) o = a > 0.0 ? -(int64_t)(n - 1) : 0;
    if (bc == BC_DIRICHLET) {
        o = o < -i ? -i : o;
        o = o > N - n - i ? N - n - i : o;
    }
    return o;
}

// Grid index of (unwrapped) position j: periodic wrap, even reflection about
// the end nodes (Neumann), identity (Dirichlet windows never leave the grid).
__device__ __forceinline__ int64_t map_index(int64_t j, int64_t N, int bc) {
    if (bc == BC_PERIODIC) {
        if (j >= 0 && j < N) return j;
        if (j < 0 && j >= -N) return j + N;
        if (j >= N && j < 2 * N) return j - N;
        j = j % N;  // halos wider than the grid (tiny instances)
        return j < 0 ? j + N : j;
    }
    if (bc == BC_NEUMANN) {
        j = j < 0 ? -j : j;
        return j > N - 1 ? 2 * (N - 1) - j : j;
    }
    return j;
}

// Reverse-step gathers: nodes j whose gathers see only interior nodes (every
// node within n - 1 of j has a centred window, none is a held Dirichlet end,
// no Neumann mirror or periodic wrap is involved).  The stencils containing j
// are then those of i = j + d, d = -(n-1)/2 .. (n-1)/2, at position
// k = (n-1)/2 - d -- the same terms, in the same order (d ascending), as the
// general loop over candidates, so the fast paths agree with it bit for bit.
__device__ __forceinline__ bool gather_interior(int64_t j, int64_t N, int n) {
    return j >= 2 * (n - 1) && j <= N - 1 - 2 * (n - 1);
}

// Instance owning work item `item`: a division when the group records a common
// item count per instance, else a binary search over item_begin.
__device__ __forceinline__ int find_instance(const DevProb* __restrict__ probs, int nprob, int64_t item) {
    const int each = probs[0].each;  // equal item counts: no search (the same answer)
    if (each > 0) {
        const uint64_t k = (uint64_t)item / (uint32_t)each;
        return k < (uint64_t)nprob ? (int)k : nprob - 1;
    }
    int lo = 0, hi = nprob - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (probs[mid].item_begin <= item) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Blocks of a launch are handed to the 8 XCDs round-robin (block b runs on
// XCD b % 8), and each XCD has its own L2.  Renumbering so that XCD x works
// through a contiguous range of logical blocks keeps neighbouring nodes, and
// the stencil windows they share, in one L2.  A bijection of [0, gridDim.x).
constexpr int kXcds = 8;
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t blocks) {
    const int64_t x = b % kXcds, idx = b / kXcds;
    const int64_t cnt = blocks / kXcds, rem = blocks % kXcds;
    return x * cnt + (x < rem ? x : rem) + idx;
}

// --------------------------------------------------------- compile-time for
template <class F, int... Is>
__device__ __forceinline__ void sfor_impl(F&& f, std::integer_sequence<int, Is...>) {
    (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void sfor(F&& f) {
    sfor_impl(f, std::make_integer_sequence<int, N>{});
}

// --------------------------------------------------------- DPP primitives -
// A VALU write of a VGPR needs two wait states before a DPP instruction reads
// it, and a VALU write of EXEC five; the compiler does not insert them for
// inline assembly, so every block starts with its own s_nop.

// c_j += bcast_K(y_j) * x for a group of 1..8 columns.  One s_nop covers the
// whole group: its DPP sources are only read, never written, inside the block.
#define LMEP_FMAC_DPP(c, y) "v_fmac_f64_dpp " c ", " y ", %[x] row_newbcast:%[k] row_mask:0xf bank_mask:0xf\n\t"
template <int K>
__device__ __forceinline__ void fmac_b8(double& c0, double& c1, double& c2, double& c3, double& c4, double& c5,
                                        double& c6, double& c7, double y0, double y1, double y2, double y3,
                                        double y4, double y5, double y6, double y7, double x) {
    asm("s_nop 1\n\t" LMEP_FMAC_DPP("%0", "%[y0]") LMEP_FMAC_DPP("%1", "%[y1]") LMEP_FMAC_DPP("%2", "%[y2]")
            LMEP_FMAC_DPP("%3", "%[y3]") LMEP_FMAC_DPP("%4", "%[y4]") LMEP_FMAC_DPP("%5", "%[y5]")
                LMEP_FMAC_DPP("%6", "%[y6]") LMEP_FMAC_DPP("%7", "%[y7]")
        : "+v"(c0), "+v"(c1), "+v"(c2), "+v"(c3), "+v"(c4), "+v"(c5), "+v"(c6), "+v"(c7)
        : [y0] "v"(y0), [y1] "v"(y1), [y2] "v"(y2), [y3] "v"(y3), [y4] "v"(y4), [y5] "v"(y5), [y6] "v"(y6),
          [y7] "v"(y7), [x] "v"(x), [k] "n"(K));
}
template <int K>
__device__ __forceinline__ void fmac_b4(double& c0, double& c1, double& c2, double& c3, double y0, double y1,
                                        double y2, double y3, double x) {
    asm("s_nop 1\n\t" LMEP_FMAC_DPP("%0", "%[y0]") LMEP_FMAC_DPP("%1", "%[y1]") LMEP_FMAC_DPP("%2", "%[y2]")
            LMEP_FMAC_DPP("%3", "%[y3]")
        : "+v"(c0), "+v"(c1), "+v"(c2), "+v"(c3)
        : [y0] "v"(y0), [y1] "v"(y1), [y2] "v"(y2), [y3] "v"(y3), [x] "v"(x), [k] "n"(K));
}
template <int K>
__device__ __forceinline__ void fmac_b2(double& c0, double& c1, double y0, double y1, double x) {
    asm("s_nop 1\n\t" LMEP_FMAC_DPP("%0", "%[y0]") LMEP_FMAC_DPP("%1", "%[y1]")
        : "+v"(c0), "+v"(c1)
        : [y0] "v"(y0), [y1] "v"(y1), [x] "v"(x), [k] "n"(K));
}
template <int K>
__device__ __forceinline__ void fmac_b1(double& c0, double y0, double x) {
    asm("s_nop 1\n\t" LMEP_FMAC_DPP("%0", "%[y0]")
        : "+v"(c0)
        : [y0] "v"(y0), [x] "v"(x), [k] "n"(K));
}
#undef LMEP_FMAC_DPP

__device__ __forceinline__ void exec_guard() { asm volatile("s_nop 4" ::: "memory"); }

// Lane K's value of v, broadcast to its whole 16-lane row.
template <int K>
__device__ __forceinline__ double bcast(double v) {
    return __builtin_amdgcn_update_dpp(0.0, v, 0x150 + K, 0xf, 0xf, false);  // row_newbcast:K
}

// C[j] += x * bcast_K(Y[j]) for columns [J0, J1).
template <int M, int K, int J0, int J1>
__device__ __forceinline__ void fmac_cols(double (&C)[M], const double (&Y)[M], double x) {
    if constexpr (J1 - J0 >= 8) {
        fmac_b8<K>(C[J0], C[J0 + 1], C[J0 + 2], C[J0 + 3], C[J0 + 4], C[J0 + 5], C[J0 + 6], C[J0 + 7], Y[J0],
                   Y[J0 + 1], Y[J0 + 2], Y[J0 + 3], Y[J0 + 4], Y[J0 + 5], Y[J0 + 6], Y[J0 + 7], x);
        fmac_cols<M, K, J0 + 8, J1>(C, Y, x);
    } else if constexpr (J1 - J0 >= 4) {
        fmac_b4<K>(C[J0], C[J0 + 1], C[J0 + 2], C[J0 + 3], Y[J0], Y[J0 + 1], Y[J0 + 2], Y[J0 + 3], x);
        fmac_cols<M, K, J0 + 4, J1>(C, Y, x);
    } else if constexpr (J1 - J0 >= 2) {
        fmac_b2<K>(C[J0], C[J0 + 1], Y[J0], Y[J0 + 1], x);
        fmac_cols<M, K, J0 + 2, J1>(C, Y, x);
    } else if constexpr (J1 - J0 == 1) {
        fmac_b1<K>(C[J0], Y[J0], x);
    }
}

// C += X * Y for row matrices of order M whose rows and columns >= NB form the
// augmented block: rows k >= NB of Y vanish in columns < NB, so those products
// are skipped (the local matrix is block upper triangular).
template <int M, int NB>
__device__ __forceinline__ void mul_acc(const double (&X)[M], const double (&Y)[M], double (&C)[M]) {
    exec_guard();
    sfor<M>([&](auto kc) {
        constexpr int K = decltype(kc)::value;
        constexpr int J0 = (K < NB) ? 0 : NB;
        fmac_cols<M, K, J0, M>(C, Y, X[K]);
    });
}

template <int M, int NB>
__device__ __forceinline__ void mul(const double (&X)[M], const double (&Y)[M], double (&C)[M]) {
#pragma unroll
    for (int j = 0; j < M; ++j) C[j] = 0.0;
    mul_acc<M, NB>(X, Y, C);
}

// 1/x to within rounding: hardware reciprocal estimate refined by two Newton
// steps (each squares the relative error of the estimate).
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// Solve Q X = P in place (P becomes X) by Gaussian elimination without
// pivoting, rows distributed over the DPP row (lane = row).  The Pade
// denominators are well conditioned and, for these block-triangular local
// matrices, elimination in natural order keeps growth near 1.  Rows are
// eliminated downwards, then upwards with the unnormalised pivot rows, and
// each lane divides its own row by its pivot once at the end.  Q and P are
// block upper triangular with the augmented block (rows and columns >= NB)
// upper triangular, so downward steps on augmented pivots and the left
// columns of augmented pivot rows are skipped.
template <int M, int NB>
__device__ __forceinline__ void solve_inplace(double (&Q)[M], double (&P)[M], int lane) {
    exec_guard();
    double own_pivot = 1.0;
    double rp[M];
    sfor<M>([&](auto kc) {
        constexpr int K = decltype(kc)::value;
        own_pivot = (lane == K) ? Q[K] : own_pivot;
        rp[K] = recip(bcast<K>(Q[K]));
        if constexpr (K < NB) {
            const double l = (lane > K) ? -Q[K] * rp[K] : 0.0;
            fmac_cols<M, K, K + 1, M>(Q, Q, l);
            fmac_cols<M, K, 0, M>(P, P, l);
        }
    });
    sfor<M>([&](auto kc) {
        constexpr int K = M - 1 - decltype(kc)::value;
        if constexpr (K > 0) {
            const double l = (lane < K) ? -Q[K] * rp[K] : 0.0;
            fmac_cols<M, K, (K < NB) ? 0 : NB, M>(P, P, l);
        }
    });
    const double inv = recip(own_pivot);
#pragma unroll
    for (int j = 0; j < M; ++j) P[j] *= inv;
}

// Max over the 16 lanes of a DPP row.
__device__ __forceinline__ double row_max16(double v) {
    v = fmax(v, __shfl_xor(v, 8, 16));
    v = fmax(v, __shfl_xor(v, 4, 16));
    v = fmax(v, __shfl_xor(v, 2, 16));
    v = fmax(v, __shfl_xor(v, 1, 16));
    return v;
}

// Sum over the 16 lanes of a DPP row, in a fixed order.
__device__ __forceinline__ double row_sum16(double v) {
    v += __shfl_xor(v, 8, 16);
    v += __shfl_xor(v, 4, 16);
    v += __shfl_xor(v, 2, 16);
    v += __shfl_xor(v, 1, 16);
    return v;
}

}  // namespace lmep
