// The finite-Taylor weights (the moment recursion and contraction of the
// finite-Taylor build) carried in double-double, for one-sided windows.
//
// Why one-sided rows need it.  A one-sided window harvests its last (or first)
// row, and the translation theta a that the exponential applies runs across
// the whole window (|a| up to (n + 1) / 2 in the stable band of Sec. 4.1).
// The rows are then sums of the window's Lagrange-basis Taylor coefficients
// T_k (alternating, growing like (n/2)!^2) against moments that grow like
// |a / 2|^k: even about the best expansion node the terms cancel by a factor
// of millions for n = 15 with pure advection, and by more with diffusion.  FP64
// sums lose that many digits; a double-double sum (106 bits) loses them from
// far below the FP64 rounding of the result, so the rounded weights are the
// exact rows to within half an ulp of their largest entry.
//
// Everything is the same computation as the FP64 build: with the shift s the
// moments of M'_k(theta) = sum_m mu[k][m] theta^m are
//     mu[k+1][m] = a mu[k][m-1] - s mu[k][m] + 2 b k mu[k-1][m-1] + 3 e k (k-1) mu[k-2][m-1],
// and the rows are
//     W0 = sum_k E_k T_k[r'],  E_k = sum_m mu[k][m]                 (row of e^{dt L})
//     W1 = sum_k F_k T_k[r'],  F_k = sum_m mu[k][m] / (m + 1)       (row of phi1(dt L))
//     W2 = sum_k G_k T_k[r'],  G_k = sum_m mu[k][m] / ((m+1)(m+2))  (row of phi2(dt L))
// since the integral of theta^m over [0, 1] is 1 / (m + 1) and that of
// (1 - theta) theta^m is 1 / ((m + 1)(m + 2)) (phi2(z) is the integral of
// (1 - theta) e^{theta z}).  The inputs a, b, e, s and the scale are doubles;
// the coefficients 2 k b and 3 k (k - 1) e are formed exactly (two_prod); the
// table row T (high and low parts) is the double-double table.
#pragma once

#include "dd.hpp"
#include "lmep_internal.hpp"

namespace lmep {

// PP = 0: W0; 1: W0, W1; 2: W0, W1, W2 (W1 and W2 multiplied by `scale` in
// double-double before rounding).  T_k[j] = (Th + k kMaxN)[j] + (Tl + k kMaxN)[j].
// The dispersion term is always carried (with e = 0 it adds exact zeros).
// The order loop is not unrolled: the moment rows stay in registers (their
// indices are fixed) and the code stays small.
template <int NN, int PP>
__device__ __forceinline__ void taylor_weights_dd(double a, double b, double e, double s, double scale,
                                                  const double* __restrict__ Th, const double* __restrict__ Tl,
                                                  double (&W0)[NN], double (&W1)[NN], double (&W2)[NN]) {
    dd m2[NN], m1[NN], m0[NN];  // mu[k-2][.], mu[k-1][.], mu[k][.]
    dd A0[NN], A1[NN], A2[NN];
#pragma unroll
    for (int m = 0; m < NN; ++m) {
        m2[m] = dd_of(0.0);
        m1[m] = dd_of(0.0);
        m0[m] = dd_of(0.0);
    }
    m0[0] = dd_of(1.0);
    // order 0: M'_0 = 1, so E_0 = F_0 = 1 and G_0 = 1/2
#pragma unroll
    for (int j = 0; j < NN; ++j) {
        const dd t = {Th[j], Tl[j]};
        A0[j] = t;
        A1[j] = t;
        A2[j] = {0.5 * t.hi, 0.5 * t.lo};
    }
    const dd ns = dd_of(-s);
#pragma unroll 1
    for (int k = 0; k + 1 < NN; ++k) {
        const dd bk = two_prod((double)(2 * k), b);
        const dd ek = two_prod((double)(3 * k * (k - 1)), e);
        dd E = dd_of(0.0), F = dd_of(0.0), G = dd_of(0.0);
        // the new row overwrites mu[k-2] from the top down: entry m of it is
        // the last use of mu[k-2][m] (entry m + 1 reads it)
#pragma unroll
        for (int m = NN - 1; m >= 0; --m) {
            dd v = dd_of(0.0);
            if (m <= k + 1) {  // mu[k+1][m] = 0 beyond
                v = dd_mul(ns, m0[m]);
                if (m >= 1) {
                    v = dd_add(v, dd_mul_d(m0[m - 1], a));
                    v = dd_add(v, dd_mul(bk, m1[m - 1]));
                    v = dd_add(v, dd_mul(ek, m2[m - 1]));
                }
                E = dd_add(E, v);
                if constexpr (PP >= 1) F = dd_add(F, dd_div_d(v, (double)(m + 1)));
                if constexpr (PP >= 2) G = dd_add(G, dd_div_d(v, (double)((m + 1) * (m + 2))));
            }
            m2[m] = v;
        }
#pragma unroll
        for (int m = 0; m < NN; ++m) {  // (m2, m1, m0) <- (m1, m0, new)
            const dd t = m2[m];
            m2[m] = m1[m];
            m1[m] = m0[m];
            m0[m] = t;
        }
        const double* __restrict__ Tkh = Th + (k + 1) * kMaxN;
        const double* __restrict__ Tkl = Tl + (k + 1) * kMaxN;
#pragma unroll
        for (int j = 0; j < NN; ++j) {
            const dd t = {Tkh[j], Tkl[j]};
            A0[j] = dd_fma(E, t, A0[j]);
            if constexpr (PP >= 1) A1[j] = dd_fma(F, t, A1[j]);
            if constexpr (PP >= 2) A2[j] = dd_fma(G, t, A2[j]);
        }
    }
#pragma unroll
    for (int j = 0; j < NN; ++j) {
        W0[j] = dd_round(A0[j]);
        W1[j] = PP >= 1 ? dd_round(dd_mul_d(A1[j], scale)) : 0.0;
        W2[j] = PP >= 2 ? dd_round(dd_mul_d(A2[j], scale)) : 0.0;
    }
}

// The weights of a node that harvests window row r, expanded about row
// r + sh (clamped to the window), from the double-double table `tdd`.
template <int NN, int PP>
__device__ __forceinline__ void node_weights_dd(int r, int sh, double a, double b, double e, double scale,
                                                const double* __restrict__ tdd, double (&W0)[NN], double (&W1)[NN],
                                                double (&W2)[NN]) {
    int rp = r + sh;
    rp = rp < 0 ? 0 : (rp > NN - 1 ? NN - 1 : rp);
    const double* __restrict__ Th = tdd + taylor_index(NN, rp, 0, 0);
    const double* __restrict__ Tl = Th + kTaylorTableDoubles;
    taylor_weights_dd<NN, PP>(a, b, e, (double)(rp - r), scale, Th, Tl, W0, W1, W2);
}

}  // namespace lmep
