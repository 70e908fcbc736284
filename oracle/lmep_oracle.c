/*
 * lmep_oracle.c -- plain CPU FP64 oracle for the Local Matrix Exponential
 * Propagator (LMEP) hot path.  TEST INFRASTRUCTURE ONLY: only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It shares
 * no code with the HIP library and takes every input (states, parameters) from
 * its caller.
 *
 * What it computes, following the paper's order:
 *   a1  stencil window of each node (centred, or fully one-sided against the
 *       flow, Sec. 4.1; one-sided "edge rows" next to Dirichlet ends,
 *       Sec. 2.1 step 3; reflected for Neumann ends),
 *   a2  differentiation matrices on the stencil (Sec. 2.1 step 1), on the
 *       node's own coordinates for non-uniform grids (Sec. 4.3.3),
 *   a3  local operator L = -c D1 + nu D2 - delta D3 + react I (Thm 2, Remark),
 *   a4  the paper's s n x s n augmented block matrix (Sec. 3.1 step 1),
 *   a5  its exponential by the terminating Taylor series (Remark on
 *       nilpotency; Thm 2 proof),
 *   a6  harvest of the node's row of each block (Sec. 3.1 step 2),
 *   a7  nonlinear terms, a8 the LINEAR / ETD1 / ETD2RK update (Sec. 3,
 *       Sec. 3.1 step 3), a9 the step loop, a10 the reverse (adjoint) step.
 *
 * Parity unpinned: none.  Every exported function is checked by the
 * "not gpu" tests against values printed in the paper, closed forms,
 * invariants, exact rational arithmetic or complex-step derivatives.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { BC_PERIODIC = 0, BC_DIRICHLET = 1, BC_NEUMANN = 2 };
enum { SCH_LINEAR = 0, SCH_ETD1 = 1, SCH_ETD2RK = 2, SCH_ETDRK4 = 3 };
enum { NL_NONE = 0, NL_BURGERS_FROZEN = 1, NL_KDV = 2, NL_ALLEN_CAHN = 3 };
enum { WIN_CENTRED = 0, WIN_UPWIND = 1 };

/* The oracle's own problem record (the GPU library has its own, unrelated one). */
typedef struct {
    int64_t N;       /* grid nodes */
    int32_t n;       /* stencil size (odd) */
    int32_t bc;      /* BC_* */
    double h;        /* uniform grid spacing */
    double dt;       /* time step */
    double c, nu, delta, react; /* u_t = -c u_x + nu u_xx - delta u_xxx + react u + N(u) */
    int32_t scheme;  /* SCH_* */
    int32_t nonlin;  /* NL_* */
    double nl_coef;  /* coefficient g of the nonlinear term */
    double bc_left, bc_right; /* Dirichlet end values */
    int32_t window;  /* WIN_*: centred stencils, or fully one-sided against the flow */
    const double *x; /* node coordinates of a non-uniform grid (increasing), or NULL: uniform, spacing h */
} ora_prob;

/* Highest phi-function a scheme needs (blocks of the augmented matrix minus one). */
static int scheme_p(int scheme)
{
    return scheme == SCH_ETDRK4 ? 3 : (scheme == SCH_ETD2RK ? 2 : (scheme == SCH_ETD1 ? 1 : 0));
}

/* Weight vectors stored per node: W0..Wp, or for ETDRK4 the six rows
 * E(dt/2), (dt/2) phi1(dt/2), E(dt), dt alpha, dt beta, dt gamma. */
static int scheme_kinds(int scheme) { return scheme == SCH_ETDRK4 ? 6 : scheme_p(scheme) + 1; }

/* Step a1 -- stencil of node i: grid indices i+o .. i+o+n-1 (before wrapping).
 * Centred windows: o = -(n-1)/2.  Upwind windows (the fully one-sided stencils
 * of Sec. 4.1, which the paper runs up to CFL (n+1)/2): the window ends at i
 * when the node's advection speed a is positive (o = -(n-1)), starts at i when
 * it is negative (o = 0), and is centred when a = 0.  Dirichlet: the window is
 * then moved to the n nearest in-domain nodes where it would leave the grid,
 * so nodes next to an end use an edge row (Sec. 2.1 step 3; Example 1's
 * Beam-Warming row).  Periodic windows wrap; Neumann windows reflect.  The
 * harvest row is r = -o. */
static int64_t window_offset_a(int64_t i, int64_t N, int n, int bc, int window, double a)
{
    int64_t o = -(int64_t)(n - 1) / 2;
    if (window == WIN_UPWIND) {
        if (a > 0) o = -(int64_t)(n - 1);
        else if (a < 0) o = 0;
    }
    if (bc == BC_DIRICHLET) {
        if (o < -i) o = -i;
        if (o > N - n - i) o = N - n - i;
    }
    return o;
}

/* Window of node i of problem P for a node whose advection speed is a. */
static int64_t window_offset_p(const ora_prob *P, int64_t i, double a)
{
    return window_offset_a(i, P->N, P->n, P->bc, P->window, a);
}

/* Grid index of stencil position j: wrapped (periodic), reflected about the end
 * nodes (Neumann, even extension), unchanged (Dirichlet, always in range). */
static int64_t grid_index(int64_t j, int64_t N, int bc)
{
    if (bc == BC_PERIODIC) {
        j %= N;
        if (j < 0) j += N;
    } else if (bc == BC_NEUMANN) {
        if (j < 0) j = -j;
        if (j > N - 1) j = 2 * (N - 1) - j;
    }
    return j;
}

static int is_fixed_node(const ora_prob *P, int64_t i)
{
    return P->bc == BC_DIRICHLET && (i == 0 || i == P->N - 1);
}

/* Step a2 -- differentiation matrices on the stencil.  Row a of D^(m) holds
 * the weights that return the m-th derivative, at node a, of the polynomial
 * interpolant of degree < n through the stencil values (the "standard finite
 * difference matrix", Sec. 2.1 step 1).  D1 is written from the derivative
 * of the Lagrange basis,
 *     D1[a][b] = l_b'(x_a) = pi_a / (pi_b (x_a - x_b))   (a != b),
 *     D1[a][a] = sum_{b != a} 1 / (x_a - x_b),
 * with pi_b = prod_{l != b} (x_b - x_l).  Because D1 maps the values of any
 * polynomial of degree < n to the values of its derivative (again of degree
 * < n), the m-th derivative matrix is the m-th power of D1 (proof of Thm 1).
 * The nodes are the centred integers (a - (n-1)/2), the result is scaled by
 * h^-m; a uniform stencil's matrix does not depend on where it sits.
 * Arithmetic in long double (binary128 for one-sided windows); the weights are
 * built from these wide matrices and rounded to double once, at the end. */
#define FDT long double
#define FDFN fd_matrices_ld
#define FDNODES fd_nodes_ld
#include "lmep_oracle_fd.inc"
#undef FDT
#undef FDFN
#undef FDNODES
#define FDT __float128
#define FDFN fd_matrices_q
#define FDNODES fd_nodes_q
#include "lmep_oracle_fd.inc"
#undef FDT
#undef FDFN
#undef FDNODES

/* The same matrices rounded to double (exported; also used for the
 * derivative terms of the nonlinearity, which are plain FP64 dot products). */
int ora_fd_matrices(int n, double h, double *D1, double *D2, double *D3)
{
    long double A1[64 * 64], A2[64 * 64], A3[64 * 64];
    if (fd_matrices_ld(n, h, A1, A2, A3)) return -1;
    for (int a = 0; a < n * n; ++a) {
        D1[a] = (double)A1[a];
        D2[a] = (double)A2[a];
        D3[a] = (double)A3[a];
    }
    return 0;
}

/* ---- the type-generic part: real, complex, and real carried in binary128 ---- */
static __float128 absq_(__float128 x) { return x < 0 ? -x : x; }

#define T double
#define TW long double
#define RW long double
#define DW long double
#define EPSW 0x1p-80L
#define FD_WIDE fd_matrices_ld
#define FD_NODES_WIDE fd_nodes_ld
#define ABSW(x) fabsl(x)
#define FN(name) name##_d
#define RE(x) (x)
#include "lmep_oracle_core.inc"
#undef T
#undef TW
#undef ABSW
#undef FN
#define T double complex
#define TW long double complex
#define ABSW(x) cabsl(x)
#define FN(name) name##_z
#undef RE
#define RE(x) creal(x)
#include "lmep_oracle_core.inc"
#undef T
#undef TW
#undef RW
#undef DW
#undef EPSW
#undef FD_WIDE
#undef FD_NODES_WIDE
#undef ABSW
#undef FN
#undef RE
#define T double
#define TW __float128
#define RW __float128
#define DW __float128
#define EPSW ((__float128)0x1p-120)
#define FD_WIDE fd_matrices_q
#define FD_NODES_WIDE fd_nodes_q
#define ABSW(x) absq_(x)
#define FN(name) name##_q
#define RE(x) (x)
#include "lmep_oracle_core.inc"
#undef T
#undef TW
#undef RW
#undef DW
#undef EPSW
#undef FD_WIDE
#undef FD_NODES_WIDE
#undef ABSW
#undef FN
#undef RE

static int check_prob(const ora_prob *P)
{
    if (!P || P->n < 1 || (P->n % 2) == 0 || P->N < P->n || !(P->h > 0) || !(P->dt > 0)) return -1;
    if (P->bc < 0 || P->bc > 2 || P->scheme < 0 || P->scheme > 3 || P->nonlin < 0 || P->nonlin > 3) return -1;
    if (P->bc == BC_NEUMANN && (P->n - 1) / 2 > P->N - 1) return -1;
    if (P->nonlin == NL_BURGERS_FROZEN && P->scheme != SCH_ETD1) return -1;
    if (P->window != WIN_CENTRED && P->window != WIN_UPWIND) return -1;
    if (P->x) { /* non-uniform grids: Dirichlet ends, centred windows, pointwise N */
        if (P->bc != BC_DIRICHLET || P->window != WIN_CENTRED) return -1;
        if (P->nonlin != NL_NONE && P->nonlin != NL_ALLEN_CAHN) return -1;
        for (int64_t j = 1; j < P->N; ++j)
            if (!(P->x[j] > P->x[j - 1])) return -1;
    }
    return 0;
}

/* ---------------------------- exported API ---------------------------- */

/* Stencil offset o of node i (integer step a1). */
int64_t ora_window_offset(const ora_prob *P, int64_t i, double a) { return window_offset_p(P, i, a); }

/* Differentiation matrices (rounded to double) on n given nodes. */
int ora_fd_nodes(int n, const double *x, double *D1, double *D2, double *D3)
{
    long double xs[64], A1[64 * 64], A2[64 * 64], A3[64 * 64];
    if (n < 1 || n > 63) return -1;
    for (int a = 0; a < n; ++a) xs[a] = x[a];
    if (fd_nodes_ld(n, xs, A1, A2, A3)) return -1;
    for (int a = 0; a < n * n; ++a) {
        D1[a] = (double)A1[a];
        D2[a] = (double)A2[a];
        D3[a] = (double)A3[a];
    }
    return 0;
}

/* Row r of the augmented exponential for a given local operator L (n x n,
 * row major): out = [W0 | W1 | W2 | W3] as in augmented_row (p + 1 parts). */
int ora_augmented_row(int n, int p, const double *L, double dt, int r, int nilpotent, double *out)
{
    if (n < 1 || n > 63 || p < 0 || p > 3 || r < 0 || r >= n) return -1;
    long double Lw[64 * 64];
    for (int a = 0; a < n * n; ++a) Lw[a] = L[a];
    augmented_row_d(n, p, Lw, dt, r, nilpotent, out);
    return 0;
}

/* Same for a complex local operator (complex-step checks of the exponential). */
int ora_augmented_row_z(int n, int p, const double complex *L, double dt, int r, double complex *out)
{
    if (n < 1 || n > 63 || p < 0 || p > 3 || r < 0 || r >= n) return -1;
    long double complex Lw[64 * 64];
    for (int a = 0; a < n * n; ++a) Lw[a] = L[a];
    augmented_row_z(n, p, Lw, dt, r, 1, out);
    return 0;
}

/* Weights of every node: w[i][kind][k], kind = W0, W1 (ETD), W2 (ETD2RK), or
 * the six ETDRK4 rows (scheme_kinds).
 * u is read only for the frozen-velocity case (may be NULL otherwise). */
int ora_build_weights(const ora_prob *P, const double *u, double *w)
{
    if (check_prob(P)) return -1;
    const int n = P->n;
    if (P->nonlin == NL_BURGERS_FROZEN && !u) return -1;
    if (P->window == WIN_UPWIND) {
        __float128 Q1[64 * 64], Q2[64 * 64], Q3[64 * 64];
        if (fd_matrices_q(n, P->h, Q1, Q2, Q3)) return -1;
        all_weights_q(P, Q1, Q2, Q3, P->c, P->nu, P->delta, u, w);
        return 0;
    }
    long double D1[64 * 64], D2[64 * 64], D3[64 * 64];
    if (fd_matrices_ld(n, P->h, D1, D2, D3)) return -1;
    all_weights_d(P, D1, D2, D3, P->c, P->nu, P->delta, u, w);
    return 0;
}

/* Advance `steps` steps from u0; result in uT. */
int ora_run(const ora_prob *P, const double *u0, int64_t steps, double *uT)
{
    if (check_prob(P) || steps < 0) return -1;
    if (P->window == WIN_UPWIND) return run_q(P, P->c, P->nu, P->delta, u0, steps, uT);
    return run_d(P, P->c, P->nu, P->delta, u0, steps, uT);
}

/* Complex-step forward: parameters c + i*c_im, nu + i*nu_im, delta + i*delta_im
 * and initial state u0_re + i*u0_im.  Used only to differentiate the forward
 * map (Im(f(x + i e)) / e is the derivative to rounding for analytic f). */
int ora_run_z(const ora_prob *P, double c_im, double nu_im, double delta_im,
              const double *u0_re, const double *u0_im, int64_t steps,
              double *uT_re, double *uT_im)
{
    if (check_prob(P) || steps < 0 || P->react != 0.0 || P->window != WIN_CENTRED) return -1;
    const int64_t N = P->N;
    double complex *u0 = (double complex *)calloc(N, sizeof(double complex));
    double complex *uT = (double complex *)malloc(sizeof(double complex) * N);
    for (int64_t j = 0; j < N; ++j) u0[j] = u0_re[j] + I * (u0_im ? u0_im[j] : 0.0);
    int rc = run_z(P, P->c + I * c_im, P->nu + I * nu_im, P->delta + I * delta_im, u0, steps, uT);
    for (int64_t j = 0; j < N; ++j) { uT_re[j] = creal(uT[j]); uT_im[j] = cimag(uT[j]); }
    free(u0); free(uT);
    return rc;
}

/* Step a10 -- reverse of one LINEAR or ETD1 step (not ETD2RK).  Given the
 * forward state u (= u^k) and lam = d loss / d u^{k+1}, writes
 * lam_out = d loss / d u^k and adds this step's parameter derivatives to
 * grad[0..2] = (d/d nu, d/d c, d/d delta).  Written as the plain chain rule
 * of the forward step, in scatter form:
 *   u+_i = sum_k W0_i[k] u_{S_i(k)} + sum_k W1_i[k] N^(i)_{S_i(k)}.
 * The weights' dependence on a parameter theta enters through the directional
 * derivative of the harvested row along dL/dtheta (dL/dc = -D1, dL/dnu = D2,
 * dL/ddelta = -D3), taken from the block exponential [[X, E], [0, X]].  For
 * the frozen-velocity case the node's own value u_i moves c_i = c + g u_i.
 * Dirichlet end nodes are not updated, so their entries of lam are unused. */
int ora_adjoint_step(const ora_prob *P, const double *u, const double *lam, double *lam_out, double *grad)
{
    if (check_prob(P) || P->scheme >= SCH_ETD2RK || P->nonlin == NL_KDV || P->react != 0.0 ||
        P->window != WIN_CENTRED || P->x)
        return -1;
    const int n = P->n, p = scheme_p(P->scheme), W = (p + 1) * n;
    const int64_t N = P->N;
    const double gam = P->nl_coef;
    const int frozen = (P->nonlin == NL_BURGERS_FROZEN);
    long double D1[64 * 64], D2[64 * 64], D3[64 * 64];
    double D1d[64 * 64], D2d[64 * 64], D3d[64 * 64];
    if (fd_matrices_ld(n, P->h, D1, D2, D3) || ora_fd_matrices(n, P->h, D1d, D2d, D3d)) return -1;
    double *w = (double *)malloc(sizeof(double) * (size_t)N * W);
    double *dw = (double *)malloc(sizeof(double) * (size_t)N * 3 * W); /* per node, per direction */
    double *g = (double *)calloc(N, sizeof(double));
    double *gbar = (double *)calloc(N, sizeof(double));
    all_weights_d(P, D1, D2, D3, P->c, P->nu, P->delta, u, w);
    if (frozen)
        for (int64_t j = 0; j < N; ++j) g[j] = own_derivative_d(P, D1d, u, j, 0.0); /* centred windows only */

    /* derivative of each node's harvested row along the three directions */
    const long double *dirs[3] = {D2, D1, D3};
    const double sgn[3] = {+1.0, -1.0, -1.0}; /* dL/dnu = D2, dL/dc = -D1, dL/ddelta = -D3 */
    int have_r[64] = {0};
    double *row_cache = (double *)malloc(sizeof(double) * 64 * 3 * W);
#pragma omp parallel for schedule(dynamic, 16) if (frozen)
    for (int64_t i = 0; i < N; ++i) {
        if (!frozen) continue;
        const int r = (int)(-window_offset_a(i, N, n, P->bc, WIN_CENTRED, 0.0));
        long double L[64 * 64], dL[64 * 64];
        local_operator_d(n, D1, D2, D3, P->c + gam * u[i], P->nu, P->delta, 0.0, L);
        for (int d = 0; d < 3; ++d) {
            for (int q = 0; q < n * n; ++q) dL[q] = sgn[d] * dirs[d][q];
            augmented_row_derivative_d(n, p, L, dL, P->dt, r, dw + (i * 3 + d) * W);
        }
    }
    if (!frozen) { /* stationary: one derivative per distinct harvest row */
        for (int64_t i = 0; i < N; ++i) {
            const int r = (int)(-window_offset_a(i, N, n, P->bc, WIN_CENTRED, 0.0));
            if (!have_r[r]) {
                long double L[64 * 64], dL[64 * 64];
                local_operator_d(n, D1, D2, D3, P->c, P->nu, P->delta, 0.0, L);
                for (int d = 0; d < 3; ++d) {
                    for (int q = 0; q < n * n; ++q) dL[q] = sgn[d] * dirs[d][q];
                    augmented_row_derivative_d(n, p, L, dL, P->dt, r, row_cache + (r * 3 + d) * W);
                }
                have_r[r] = 1;
            }
            memcpy(dw + i * 3 * W, row_cache + r * 3 * W, sizeof(double) * 3 * W);
        }
    }

    for (int64_t j = 0; j < N; ++j) lam_out[j] = 0.0;
    double gsum[3] = {0.0, 0.0, 0.0};
    for (int64_t i = 0; i < N; ++i) {
        if (is_fixed_node(P, i)) continue;
        const double li = lam[i];
        const int64_t o = window_offset_a(i, N, n, P->bc, WIN_CENTRED, 0.0);
        const double *wi = w + i * W;
        double dl[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < n; ++k) {
            const int64_t j = grid_index(i + o + k, N, P->bc);
            lam_out[j] += li * wi[k];
            double Nj = 0.0;
            if (p >= 1) {
                if (P->nonlin == NL_ALLEN_CAHN) {
                    Nj = gam * (u[j] - u[j] * u[j] * u[j]);
                    lam_out[j] += li * wi[n + k] * gam * (1.0 - 3.0 * u[j] * u[j]);
                } else if (frozen) {
                    Nj = -gam * (u[j] - u[i]) * g[j];
                    lam_out[j] += li * wi[n + k] * (-gam * g[j]);
                    lam_out[i] += li * wi[n + k] * (gam * g[j]);
                    gbar[j] += li * wi[n + k] * (-gam * (u[j] - u[i]));
                }
            }
            for (int d = 0; d < 3; ++d) {
                const double *dwi = dw + (i * 3 + d) * W;
                dl[d] += li * dwi[k] * u[j];
                if (p >= 1) dl[d] += li * dwi[n + k] * Nj;
            }
        }
        for (int d = 0; d < 3; ++d) gsum[d] += dl[d];
        if (frozen) lam_out[i] += gam * dl[1]; /* c_i = c + g u_i */
    }
    if (frozen) { /* g = own-stencil derivative of u: scatter gbar through D1 rows */
        for (int64_t m = 0; m < N; ++m) {
            const int64_t o = window_offset_a(m, N, n, P->bc, WIN_CENTRED, 0.0);
            const int r = (int)(-o);
            for (int l = 0; l < n; ++l) lam_out[grid_index(m + o + l, N, P->bc)] += gbar[m] * D1d[r * n + l];
        }
    }
    for (int d = 0; d < 3; ++d) grad[d] += gsum[d];
    free(w); free(dw); free(g); free(gbar); free(row_cache);
    return 0;
}

/* Loss of O10: 0.5 * sum_i (uT_i - target_i)^2, and its gradient with respect
 * to the initial state and to (nu, c, delta), by storing every state of the
 * forward run and applying ora_adjoint_step backwards. */
int ora_adjoint_run(const ora_prob *P, const double *u0, const double *target, int64_t steps,
                    double *loss, double *grad_u0, double *grad)
{
    if (check_prob(P) || steps < 0) return -1;
    const int64_t N = P->N;
    double *hist = (double *)malloc(sizeof(double) * (size_t)N * (steps + 1));
    memcpy(hist, u0, sizeof(double) * N);
    for (int64_t s = 0; s < steps; ++s)
        if (ora_run(P, hist + s * N, 1, hist + (s + 1) * N)) { free(hist); return -1; }
    double *lam = (double *)malloc(sizeof(double) * N);
    double *lam2 = (double *)malloc(sizeof(double) * N);
    double l = 0.0;
    for (int64_t j = 0; j < N; ++j) {
        const double d = hist[steps * N + j] - target[j];
        l += 0.5 * d * d;
        lam[j] = d;
    }
    grad[0] = grad[1] = grad[2] = 0.0;
    for (int64_t s = steps - 1; s >= 0; --s) {
        if (ora_adjoint_step(P, hist + s * N, lam, lam2, grad)) { free(hist); free(lam); free(lam2); return -1; }
        double *t = lam; lam = lam2; lam2 = t;
    }
    memcpy(grad_u0, lam, sizeof(double) * N);
    *loss = l;
    free(hist); free(lam); free(lam2);
    return 0;
}
