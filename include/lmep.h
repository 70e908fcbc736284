/*
 * lmep.h -- C ABI of the Local Matrix Exponential Propagator (LMEP) hot path
 * on AMD Instinct MI355X (gfx950), FP64 throughout.
 *
 * The method (Bayona, "Unifying finite differences and semi-Lagrangian schemes
 * via localized matrix exponentials"): for every grid node, form the local
 * operator L on the node's n-point stencil (Sec. 2.1 steps 1-2), take the
 * exponential of the augmented local matrix whose first block row holds
 * e^{dt L}, dt phi1(dt L), dt^2 phi2(dt L) (Sec. 3.1 steps 1-2), harvest the
 * node's row of each block (Sec. 2.1 step 3, Sec. 3.1 step 2) and apply the
 * harvested rows as a banded stencil once per time step (Sec. 3.1 step 3).
 *
 * The PDE is  u_t = -c u_x + nu u_xx - delta u_xxx + react u + N(u)  on a
 * uniform 1-D grid (Sec. 2, problem statement; Remark "No operator splitting";
 * Sec. 3 semi-linear form).  Stencils are centred; next to Dirichlet ends they
 * are the n nearest in-domain nodes and the node's own ("edge") row is
 * harvested (Sec. 2.1 step 3); Neumann ends reflect the stencil evenly.
 *
 * Conventions for every entry point:
 *  - Pointers named d_* are device memory owned by the caller; prob is host
 *    memory.  The plain entry points retain nothing after return (a graph
 *    that lmep_step captures for LMEP_F_GRAPH is replayed and destroyed
 *    within the call); a plan (lmep_plan_create) keeps its scratch buffer and
 *    the pointers of the graphs it captured until lmep_plan_destroy.
 *  - All argument checks run before any device work; on failure the call
 *    returns a negative lmep_status, writes nothing and lmep_last_error()
 *    describes the problem.
 *  - Work is enqueued on hip_stream (a hipStream_t; NULL = default stream)
 *    and is asynchronous.  Errors of earlier asynchronous work surface as
 *    LMEP_ERR_DEVICE.
 *  - The library allocates no device memory.  Temporary storage comes from
 *    the caller's scratch buffer, sized by lmep_scratch_bytes().  The first
 *    call on a device fills a small static table of stencil weights and waits
 *    for it; make that first call outside stream capture.
 *  - No C++ exception crosses this interface.
 */
#ifndef LMEP_H
#define LMEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LMEP_OK = 0,
    LMEP_ERR_ARG = -1,          /* invalid argument (nothing was written)          */
    LMEP_ERR_UNSUPPORTED = -2,  /* valid but not implemented combination           */
    LMEP_ERR_DEVICE = -3,       /* HIP runtime error, now or from earlier work     */
    LMEP_ERR_NONFINITE = -4,    /* LMEP_F_CHECK_FINITE found a NaN / Inf           */
    LMEP_ERR_SCRATCH = -5       /* scratch buffer NULL or smaller than required    */
} lmep_status;

enum { LMEP_BC_PERIODIC = 0, LMEP_BC_DIRICHLET = 1, LMEP_BC_NEUMANN = 2 };

/* Schemes (Sec. 3): LINEAR u+ = W0 u; ETD1 (ETD-s with s = 1); ETD2RK
 * (Cox-Matthews); ETDRK4 (the four-stage scheme of Sec. 3 with
 * alpha, beta, gamma built from phi1..phi3, stationary weights only,
 * n <= 19 on uniform grids).  p = 0, 1, 2, 3 phi-functions. */
enum { LMEP_LINEAR = 0, LMEP_ETD1 = 1, LMEP_ETD2RK = 2, LMEP_ETDRK4 = 3 };

/* Nonlinear terms N(u), g = nl_coef:
 *  BURGERS_FROZEN  u_t + g u u_x = ...: the node's own velocity is frozen into
 *                  its local operator (advection coefficient c + g u_i, so the
 *                  weights are rebuilt every step) and the remainder
 *                  N_j = -g (u_j - u_i) (du/dx)_j enters through W1 (ETD1 only);
 *  KDV             N = -(g/2) d/dx (u^2)  (conservative form of -g u u_x);
 *  ALLEN_CAHN      N = g (u - u^3). */
enum { LMEP_NL_NONE = 0, LMEP_NL_BURGERS_FROZEN = 1, LMEP_NL_KDV = 2, LMEP_NL_ALLEN_CAHN = 3 };

/* Stencil windows (step a1).  CENTRED: o = -(n-1)/2.  UPWIND: the fully
 * one-sided stencils of Sec. 4.1, on the side the flow comes from: the window
 * of node i ends at i (o = -(n-1)) when its advection speed a_i is positive,
 * starts at i (o = 0) when a_i is negative, and is centred when a_i = 0, with
 * a_i = c, or c + g u_i for BURGERS_FROZEN (each node its own side; the
 * derivative in the remainder N_j uses node j's own side).  Either way a
 * Dirichlet grid moves the window to the n nearest in-domain nodes.  A
 * one-sided pure-advection update is stable for Courant numbers |a| dt / h in
 * [(n-3)/2, (n+1)/2] (and at the integers, where it is an exact shift).
 * Its edge-row exponentials cancel heavily, so stationary one-sided tables
 * (no reaction term) and frozen-velocity one-sided windows of n >= 9 points
 * are built by the finite Taylor series in double-double: rows exact to
 * rounding for n up to 15 across that band.  With a reaction term, or under
 * LMEP_OPT_EXP_METHOD = LMEP_EXP_PADE, tables are balanced (a power-of-two
 * diagonal similarity) and built in FP64: ~1e-12 up to n = 9, 5e-11 / 1e-9 /
 * 5e-8 at n = 11 / 13 / 15.  The frozen-velocity remainder differentiates u
 * on one-sided windows, whose end rows grow like 2^n / n: for n >= 13 it
 * amplifies grid-scale perturbations unless the velocity varies little.
 * UPWIND is supported for LINEAR, ETD1 and ETD2RK, one step or several
 * per launch (LMEP_F_PERSISTENT); ETDRK4 and the reverse step return
 * LMEP_ERR_UNSUPPORTED. */
enum { LMEP_WIN_CENTRED = 0, LMEP_WIN_UPWIND = 1 };

/* lmep_step flags */
#define LMEP_F_GRAPH        0x1u  /* capture the step loop in a hipGraph and replay it          */
#define LMEP_F_PERSISTENT   0x2u  /* multi-step launches: each block keeps its tile of nodes,    */
                                  /* with a halo it recomputes, in LDS for up to 8 steps (see   */
                                  /* LMEP_OPT_STEPS_PER_LAUNCH), so                             */
                                  /* HBM is read and written once per launch instead of once    */
                                  /* per step; same result bit for bit as the one-step path.    */
                                  /* Stationary weights: centred or upwind windows.  BURGERS_FROZEN: */
                                  /* the fused finite-Taylor build and step (react = 0,         */
                                  /* LMEP_EXP_AUTO) on Dirichlet or periodic grids, centred or  */
                                  /* upwind windows; other frozen-velocity instances are        */
                                  /* LMEP_ERR_UNSUPPORTED.  Non-uniform instances of at         */
                                  /* most 512 nodes are held whole by one block each (weights   */
                                  /* in registers) for all n_steps (launches of up to 65536     */
                                  /* steps); larger ones are LMEP_ERR_UNSUPPORTED.  So are      */
                                  /* uniform stationary instances with a pointwise or no        */
                                  /* nonlinearity (not ETDRK4) when every instance of their     */
                                  /* kernel group has at most 512 nodes.                        */
#define LMEP_F_CHECK_FINITE 0x4u  /* scan the result; LMEP_ERR_NONFINITE if any entry is not    */
                                  /* finite (synchronises the stream)                            */
#define LMEP_F_PROFILE      0x8u  /* time the weight-build and apply kernels with HIP events    */
                                  /* (synchronises); read back with lmep_profile_last()          */
#define LMEP_F_COUNT        0x10u /* count local matrices and scaling-and-squaring squarings     */
                                  /* (atomics; slows the build; lmep_profile_last())             */

/* One problem instance.  A batch is an array of these; instance k's state
 * occupies d_u[state_off, state_off + N) of every packed state buffer and its
 * weights d_w[weight_off, weight_off + lmep_weight_count(&prob[k])). */
typedef struct {
    int64_t N;          /* grid nodes; N >= n; Neumann also needs N >= (n+1)/2       */
    int32_t n;          /* stencil size: odd, 3..15 with n + p <= 16 (ETDRK4: 3..19)  */
    int32_t bc;         /* LMEP_BC_*                                                  */
    double  h;          /* uniform grid spacing, > 0                                  */
    double  dt;         /* time step, > 0                                             */
    double  c;          /* advection speed                                            */
    double  nu;         /* diffusion coefficient                                      */
    double  delta;      /* dispersion coefficient                                     */
    double  react;      /* linear reaction coefficient (c0 of Thm 2)                  */
    int32_t scheme;     /* LMEP_LINEAR / LMEP_ETD1 / LMEP_ETD2RK / LMEP_ETDRK4        */
    int32_t nonlin;     /* LMEP_NL_*                                                  */
    double  nl_coef;    /* g of the nonlinear term                                    */
    double  bc_left;    /* Dirichlet value held at node 0                             */
    double  bc_right;   /* Dirichlet value held at node N-1                           */
    int64_t state_off;  /* offset (in doubles) of the state in packed state buffers   */
    int64_t weight_off; /* offset (in doubles) of the weights in the weight buffer    */
    int32_t window;     /* LMEP_WIN_* (0 = centred)                                   */
    const double* x;    /* NULL: uniform grid of spacing h.  Otherwise a DEVICE       */
                        /* pointer to the N node coordinates of a non-uniform grid    */
                        /* (strictly increasing; read by lmep_build_weights only, not */
                        /* checked on the host; owned by the caller).  Every node     */
                        /* then gets differentiation matrices on its own window's     */
                        /* coordinates and its own exponential, harvested once        */
                        /* (Sec. 4.3.3).  Supported: Dirichlet ends, centred windows, */
                        /* LINEAR / ETD1 / ETD2RK, nonlinearity NONE or ALLEN_CAHN,   */
                        /* odd n from 3 to 25 with n + p <= 32; anything else is      */
                        /* LMEP_ERR_UNSUPPORTED, as is the reverse step (and          */
                        /* LMEP_F_PERSISTENT for N > 512).  h is then unused.         */
} lmep_problem;

/* Number of doubles of harvested weights one instance needs (kinds = 1 + p =
 * 1, 2, 3 for LINEAR, ETD1, ETD2RK; 6 for ETDRK4):
 *   weights per node (BURGERS_FROZEN, rebuilt every step; non-uniform grids,
 *       built once): kinds * n * N, layout
 *       [kind][k][i]  -- weight k of node i's stencil, kind 0 = W0 (row of
 *       e^{dt L}), 1 = W1 (row of dt phi1(dt L)), 2 = W2 (row of dt phi2(dt L));
 *   stationary operators on uniform grids: kinds * n * n, layout [kind][r][k] -- the harvest of
 *       stencil row r (every node harvests row r = -offset of its stencil).
 *       ETDRK4's kinds are rows of e^{L dt/2}, (dt/2) phi1(L dt/2), e^{L dt},
 *       dt alpha, dt beta and dt gamma with alpha = phi1 - 3 phi2 + 4 phi3,
 *       beta = 2 phi2 - 4 phi3, gamma = 4 phi3 - phi2 (phi_j = phi_j(L dt)).
 * Returns -1 for an invalid problem. */
int64_t lmep_weight_count(const lmep_problem* prob);

/* Bytes of scratch an operation needs: op 0 = lmep_build_weights,
 * 1 = lmep_step, 2 = lmep_adjoint_step.  Returns 0 for invalid arguments. */
size_t lmep_scratch_bytes(const lmep_problem* prob, int32_t count, int32_t op);

/* Build the harvested weights of `count` instances into d_w (steps a1-a6:
 * stencil, local operator, augmented matrix, FP64 Pade scaling-and-squaring
 * exponential per local matrix, harvest).  BURGERS_FROZEN instances on uniform
 * grids with react = 0 take, by default, the same exponential as an exact
 * finite Taylor series instead (the local operator is a polynomial in the
 * nilpotent first-derivative matrix of the window, Sec. 2.1 / Sec. 3.1; see
 * LMEP_OPT_EXP_METHOD).  d_u is read only for BURGERS_FROZEN instances (their
 * frozen velocity) and may be NULL otherwise. */
int lmep_build_weights(const lmep_problem* prob, int32_t count, const double* d_u,
                       double* d_w, void* d_scratch, size_t scratch_bytes, void* hip_stream);

/* Advance every instance n_steps >= 1 steps: d_u_out = (step)^n_steps(d_u_in).
 * d_w must hold the weights of stationary instances (lmep_build_weights);
 * for BURGERS_FROZEN instances the weights are rebuilt every step (into d_w
 * only when LMEP_OPT_FUSE_FROZEN is 0).
 * d_u_in is not modified and must not overlap d_u_out. */
int lmep_step(const lmep_problem* prob, int32_t count, double* d_w, const double* d_u_in,
              double* d_u_out, int32_t n_steps, uint32_t flags, void* d_scratch,
              size_t scratch_bytes, void* hip_stream);

/* For callers that cannot allocate device memory or hand over a workspace
 * (code under stream capture, tight serving loops, harnesses that forbid
 * allocation): lmep_step without the scratch argument.  Same arguments, checks
 * and results, bit for bit, as lmep_step with the same flags.  The scratch is
 * a static array of LMEP_NOALLOC_SCRATCH_BYTES in each device's memory, which
 * the library holds from the first call on that device until the process
 * ends; the call allocates nothing (no hipMalloc, hipFree, hipHostMalloc or
 * other allocating routine) and passes the problem tables to the device
 * through kernel arguments, so nothing in host memory has to outlive it.
 *  - flags: 0 or LMEP_F_PERSISTENT; any other bit is LMEP_ERR_ARG.
 *  - A batch whose lmep_scratch_bytes(prob, count, 1) exceeds
 *    LMEP_NOALLOC_SCRATCH_BYTES returns LMEP_ERR_SCRATCH (the step needs 8
 *    bytes per node of the packed state extent plus about 0.5 KB per instance,
 *    so about 8 million nodes at most).
 *  - Every call on a device uses that device's one array, which keeps the
 *    last call's contents; nothing in it has to start at zero.  Calls ordered
 *    on one stream are safe; calls that overlap on one device (other streams,
 *    or other threads without ordering) race and give wrong results. */
#define LMEP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int lmep_step_noalloc(const lmep_problem* prob, int32_t count, double* d_w, const double* d_u_in,
                      double* d_u_out, int32_t n_steps, uint32_t flags, void* hip_stream);

/* Plans: the grouping, option values and device tables of one batch, made
 * once and reused by many calls, so that a call enqueues kernels only (no
 * host-to-device copy, no host synchronisation) and a step loop captured with
 * LMEP_F_GRAPH is replayed on later calls instead of being captured again.
 *
 * lmep_plan_create checks the batch as the entry point of `op` does (op 1:
 * lmep_step, op 2: lmep_adjoint_step), copies what it needs from prob (prob
 * may be freed afterwards), and uploads the device tables into d_scratch
 * (lmep_scratch_bytes(prob, count, op) bytes, 256-byte aligned) on
 * hip_stream.  The scratch buffer belongs to the plan until lmep_plan_destroy:
 * the caller keeps it allocated and does not write it.
 *  - flags: for op 1, LMEP_F_PERSISTENT or 0 (fixed for the plan); for op 2, 0.
 *  - options: n_options pairs (option, value) of the LMEP_OPT_* below that
 *    override, for this plan only, the process-wide values, which the plan
 *    copies at creation; later lmep_set_option calls do not change it.  NULL
 *    with n_options = 0 takes the process-wide values.
 *  - The plan records an event after its upload; calls on another stream wait
 *    for it on the device.
 * lmep_plan_step and lmep_plan_adjoint_step take the pointers of one call and
 * follow lmep_step and lmep_adjoint_step (same checks, results bit for bit).
 * lmep_plan_step's flags must contain LMEP_F_PERSISTENT exactly when the plan
 * was made with it; with LMEP_F_GRAPH the plan captures the step loop the
 * first time a (d_w, d_u_in, d_u_out, n_steps) combination is seen and replays
 * that graph afterwards (the last four combinations are kept), so the graph
 * keeps those pointers: they must stay valid while the plan lives.
 * A plan is not thread-safe: calls on one plan must not overlap in time.
 * lmep_plan_destroy waits for the plan's last graph launch and frees the
 * plan's host memory and graphs (not the scratch buffer); NULL is ignored. */
typedef struct lmep_plan_s* lmep_plan;
int lmep_plan_create(lmep_plan* plan, const lmep_problem* prob, int32_t count, int32_t op, uint32_t flags,
                     const int32_t* options, int32_t n_options, void* d_scratch, size_t scratch_bytes,
                     void* hip_stream);
int lmep_plan_step(lmep_plan plan, double* d_w, const double* d_u_in, double* d_u_out, int32_t n_steps,
                   uint32_t flags, void* hip_stream);
int lmep_plan_adjoint_step(lmep_plan plan, const double* d_u_k, const double* d_lambda_next, double* d_lambda_k,
                           double* d_grad, void* hip_stream);
int lmep_plan_destroy(lmep_plan plan);

/* Reverse of one LINEAR or ETD1 step (not ETD2RK / ETDRK4 / KDV).  Given the forward
 * state d_u_k = u^k and d_lambda_next = d loss / d u^{k+1}, write
 * d_lambda_k = d loss / d u^k and add this step's parameter derivatives to
 * d_grad[3 * k + {0, 1, 2}] = (d loss/d nu, d loss/d c, d loss/d delta) of
 * instance k.  The weights' dependence on the parameters and on the frozen
 * velocity is taken from the Frechet derivative of each local exponential,
 * read off the block-triangular exponential [[A, E], [0, A]] (FP64 Pade), or,
 * for instances without a reaction term under LMEP_EXP_AUTO, from the
 * derivatives of the exact finite Taylor series of the same exponential (the
 * moments of its symbol shifted by one to three orders).
 * Entries of lambda at Dirichlet end nodes are ignored (those nodes are not
 * updated).  Summation order is fixed, so results are bitwise reproducible. */
int lmep_adjoint_step(const lmep_problem* prob, int32_t count, const double* d_u_k,
                      const double* d_lambda_next, double* d_lambda_k, double* d_grad,
                      void* d_scratch, size_t scratch_bytes, void* hip_stream);

/* Measurements of the last lmep_step calls on this thread: weight-build and
 * apply kernel time of the last LMEP_F_PROFILE call (milliseconds, summed over
 * launches, from HIP events recorded around each launch on the call's stream),
 * and, from the last LMEP_F_COUNT call, the number of local matrices
 * exponentiated and the total number of squarings their scaling-and-squaring
 * took (a node built by the finite Taylor series counts as one matrix with no
 * squarings).  Any pointer may be NULL. */
int lmep_profile_last(double* build_ms, int32_t* build_launches, double* apply_ms,
                      int32_t* apply_launches, int64_t* matrices, int64_t* squarings);

/* Per kernel of the last call on this thread that timed its kernels
 * (LMEP_F_PROFILE, or a reverse step under LMEP_OPT_PROFILE_ADJOINT): returns
 * the number K of distinct kernels it launched and, for 0 <= k < K, writes the
 * kernel's name as a kernel trace shows it without namespace and argument
 * list (e.g. "stepk_kernel<11,1,3,8>", truncated to name_len - 1
 * characters), its time summed over its launches in milliseconds (HIP events
 * recorded on the call's stream around each launch, or, when every step of
 * the call runs a single kernel, one pair around the whole run of its
 * back-to-back launches) and its number of launches.  For k outside [0, K)
 * it writes nothing.  Any pointer may be NULL. */
int32_t lmep_profile_kernel(int32_t k, char* name, size_t name_len, double* ms, int32_t* launches);

/* Thread-local description of the last non-OK status. */
const char* lmep_last_error(void);

/* Process-wide tuning options (read at each lmep_step call).
 *  LMEP_OPT_STEPS_PER_LAUNCH  steps advanced per launch under
 *                             LMEP_F_PERSISTENT: 1, 2, 4, 8 or 16 (default 8).
 *                             More steps mean less HBM traffic but a wider halo
 *                             recomputed by every block.  Frozen-velocity and
 *                             ETDRK4 groups take at most 8 (each kernel group
 *                             of a batch advances its own number per launch).
 *  LMEP_OPT_PROFILE_ADJOINT   1: every lmep_adjoint_step records HIP events
 *                             around its Frechet-derivative kernel(s) and
 *                             around the whole step on its stream, then
 *                             synchronises; lmep_profile_last() reports the
 *                             Frechet kernels as build_ms / build_launches and
 *                             the rest of the step (transposed apply,
 *                             reductions) as apply_ms with apply_launches = 1.
 *                             0 (default): no events, no synchronisation.
 *  LMEP_OPT_FUSE_FROZEN       1 (default): lmep_step advances BURGERS_FROZEN
 *                             instances with one kernel per step that builds
 *                             each node's weights and applies them at once;
 *                             d_w is then not written.  0: build the weights
 *                             into d_w, then apply them (two kernels).  The
 *                             two agree to rounding, not bit for bit (the
 *                             fused kernel sums a node's stencil terms as a
 *                             tree over the lanes).
 *  LMEP_OPT_APPLY_TILE        nodes per block of the one-step apply kernel:
 *                             0 (default) chooses from the group's size (64
 *                             for small non-uniform instances, 256 for small
 *                             groups, 1024 otherwise); 256 or 1024 force that
 *                             tile for every one-step group (non-uniform
 *                             groups also take 64).  Results do not depend on it.
 *  LMEP_OPT_EXP_METHOD        how the per-step weights of BURGERS_FROZEN
 *                             instances are exponentiated.  LMEP_EXP_AUTO
 *                             (default): on a uniform grid with react = 0 the
 *                             window operator dt L is a polynomial of degree
 *                             <= 3 in the window's first-derivative matrix D,
 *                             and D^n = 0, so e^{dt L} and dt phi1(dt L) are
 *                             exact polynomials of degree n - 1 in D; their
 *                             harvested rows are formed from the moments of
 *                             the polynomial (one thread per node, O(n^2)
 *                             work) with no Pade approximant or squaring.
 *                             The expansion is taken about the window node
 *                             nearest the middle of the node's translation
 *                             range, which keeps its FP64 error at or below
 *                             the Pade path's.  Other instances: Pade.
 *                             LMEP_EXP_PADE: Pade scaling-and-squaring for
 *                             every instance.  The two agree to rounding.
 *  LMEP_OPT_TAYLOR_REGION     positions staged per block (= threads) by the
 *                             frozen-velocity multi-step kernel: 0 (default)
 *                             sizes it from the group (about one block per CU
 *                             for small groups, 512 for large ones); a
 *                             multiple of 64 in [128, 512] forces it, raised
 *                             where the halo would leave fewer than 64
 *                             written nodes per block.  Results do not
 *                             depend on it.
 *  LMEP_OPT_MERGE_GROUPS      1: under LMEP_F_PERSISTENT at 8 or 16 steps per
 *                             launch, uniform stationary instances on centred
 *                             windows (ETD schemes, more than 512 nodes) of
 *                             every stencil size share one launch per scheme
 *                             and nonlinearity, their blocks ordered by n
 *                             descending (a group of one size keeps its own
 *                             kernel); 0 (default): one launch per stencil
 *                             size.  Results do not depend on it.
 * lmep_set_option returns LMEP_OK or LMEP_ERR_ARG (unknown option or value);
 * lmep_get_option returns the value or LMEP_ERR_ARG. */
#define LMEP_OPT_STEPS_PER_LAUNCH 1
#define LMEP_OPT_PROFILE_ADJOINT 2
#define LMEP_OPT_FUSE_FROZEN 3
#define LMEP_OPT_APPLY_TILE 4
#define LMEP_OPT_EXP_METHOD 5
#define LMEP_OPT_TAYLOR_REGION 6
#define LMEP_OPT_MERGE_GROUPS 7
#define LMEP_EXP_AUTO 0
#define LMEP_EXP_PADE 1
int lmep_set_option(int32_t option, int32_t value);
int32_t lmep_get_option(int32_t option);

#ifdef __cplusplus
}
#endif
#endif /* LMEP_H */
