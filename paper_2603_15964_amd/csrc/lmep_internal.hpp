// Internal declarations of liblmep: the device-side problem record, the
// scratch layout, and the launchers each kernel file provides to the C-ABI
// layer (lmep_abi.cpp).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lmep {

constexpr int kMaxN = 15;     // largest stencil
constexpr int kMaxM = 16;     // largest local matrix n + p (one 16-lane DPP row)
constexpr int kNumN = 7;      // stencil sizes 3, 5, ..., 15
constexpr int kMaxNWide = 25; // non-uniform grids: largest stencil
constexpr int kMaxMWide = 32; // non-uniform grids: largest local matrix (LDS build)
constexpr int kResidentMaxN = 512;  // non-uniform instances a multi-step block holds whole
constexpr int kResidentMaxSteps = 1 << 16;  // steps of one such launch (longer runs: several)
constexpr int kFdDerivs = 3;  // first, second and third derivative tables
constexpr int kMaxNRk4 = 19;  // uniform grids: ETDRK4 stencils up to 19 points (orders n + 3 <= 22, LDS build)
constexpr int kFdMaxN = 25;   // the finite-difference table covers stencils 3, 5, ..., 25
constexpr int kNumFd = (kFdMaxN - 1) / 2;

// Device-side record of one instance, filled by the host from lmep_problem.
// `item_begin` is the prefix sum of work items (matrices or tiles) over the
// instances of one launch group, so a block finds its instance by a binary
// search.  Kept at 128 bytes.
struct DevProb {
    int64_t N;
    int64_t state_off;
    int64_t weight_off;
    int64_t item_begin;
    int32_t n, bc, scheme, nonlin;
    int32_t p, frozen, index, harvest;  // harvest: what the build writes (HARVEST_*)
    double h, dt, c, nu, delta, react, nl_coef, bc_left, bc_right;
    int32_t window;  // WIN_*
    int32_t each;    // work items of every instance of the table's group when all are equal, else 0
    const double* x;       // node coordinates (non-uniform grids) or nullptr
    double pad2[1];
};
static_assert(sizeof(DevProb) == 160, "DevProb layout");

enum : int { BC_PERIODIC = 0, BC_DIRICHLET = 1, BC_NEUMANN = 2 };
enum : int { SCH_LINEAR = 0, SCH_ETD1 = 1, SCH_ETD2RK = 2, SCH_ETDRK4 = 3 };
// Build parts: the harvested rows W0..Wp of one exponential, or for ETDRK4
// the full step (p = 3 at dt: kinds 2..5 = e^{L dt}, dt alpha, dt beta,
// dt gamma) and the half step (p = 1 at dt/2: kinds 0, 1).
enum : int { HARVEST_PLAIN = 0, HARVEST_RK4_FULL = 1, HARVEST_RK4_HALF = 2 };
enum : int { NL_NONE = 0, NL_BURGERS = 1, NL_KDV = 2, NL_AC = 3 };
// Launch code of the merged multi-step kernel only (never a DevProb value):
// Allen-Cahn where every instance of the launch has coefficient g = 1, so the
// kernel evaluates u - u^3 without the product by g (the same bits).
constexpr int kNlAcUnit = 4;
enum : int { WIN_CENTRED = 0, WIN_UPWIND = 1 };

// Table of finite-difference weights on the centred integer stencil
// x_k = k - (n-1)/2: fd[(n-3)/2][d][a][k] is the weight of node k for the
// (d+1)-th derivative at node a, n = 3, 5, ..., kFdMaxN.  Lives in a static
// device array per device.
constexpr int kFdTableDoubles = kNumFd * kFdDerivs * kFdMaxN * kFdMaxN;
__host__ __device__ inline int fd_index(int n, int d, int a, int k) {
    return ((((n - 3) / 2) * kFdDerivs + d) * kFdMaxN + a) * kFdMaxN + k;
}

// Table of the finite-Taylor build: taylor[(n-3)/2][a][k][j] = k-th derivative
// of the window's Lagrange basis polynomial j at node a of the centred integer
// stencil, divided by k! (row a of D1^k / k!).
constexpr int kTaylorTableDoubles = kNumN * kMaxN * kMaxN * kMaxN;
__host__ __device__ inline int taylor_index(int n, int a, int k, int j) {
    return ((((n - 3) / 2) * kMaxN + a) * kMaxN + k) * kMaxN + j;
}

// ---------------------------------------------------------------- launchers
// Fill the per-device stencil tables (blocking; once per device).
hipError_t fd_table_init(const double** d_table_out);
hipError_t taylor_table_init(const double** d_table_out);
// The finite-Taylor table in double-double: high parts at d_table_out[i],
// low parts at d_table_out[kTaylorTableDoubles + i], same index.
hipError_t taylor_dd_table_init(const double** d_table_out);

// Build weights for one group of instances sharing (n, p).  items = total
// matrices of the group.  stats (nullable, profiling): stats[0] += matrices
// built, stats[1] += squarings performed.  d_u_out (frozen-velocity ETD1
// groups only): fuse the step -- each node's row applies its weights at once
// and writes the node's new value into d_u_out; d_w is then not touched.
hipError_t launch_build(int n, int p, const DevProb* d_probs, int nprob, int64_t items,
                        const double* fd, const double* d_u, double* d_w, unsigned long long* stats,
                        hipStream_t stream, double* d_u_out = nullptr);

// Frozen-velocity ETD1 weights by the finite Taylor series of the exponential
// (react = 0, uniform grid): one thread per node, blocks of kTaylorTile nodes
// of one instance; items = tiles, item_begin = the instance's first tile.
// With d_u_out the step is fused as in launch_build.  stats[0] += nodes built.
// dd: one-sided windows of n >= kTaylorDdMinN points, weights carried in
// double-double from the double-double table (`taylor` is then that table).
constexpr int kTaylorTile = 256;
constexpr int kTaylorDdMinN = 9;
hipError_t launch_build_taylor(int n, const DevProb* d_probs, int nprob, int64_t tiles, const double* fd,
                               const double* taylor, const double* d_u, double* d_w, unsigned long long* stats,
                               hipStream_t stream, double* d_u_out = nullptr, bool dd = false);
// The same fused step, ksteps <= kb steps per launch (Dirichlet or periodic):
// a block stages `reg` positions (kTaylorRegion, or half of it for groups too
// small to fill the GPU otherwise) and writes taylor_stepk_tile(n, kb, reg,
// upwind) nodes; items = tiles of that size per instance.  A step spoils
// n - 1 positions at an open end with centred windows and 2 (n - 1) with
// one-sided ones (the window and the derivative at its positions each reach
// that far to one side).
constexpr int kTaylorRegion = 512;
constexpr int kTaylorMaxKb = 8;  // steps per launch of the frozen-velocity multi-step kernel, at most
__host__ __device__ constexpr int taylor_stepk_reach(int n, bool upwind) { return upwind ? 2 * (n - 1) : n - 1; }
__host__ __device__ constexpr int taylor_stepk_tile(int n, int kb, int reg, bool upwind) {
    return reg - 2 * kb * taylor_stepk_reach(n, upwind);
}
static_assert(taylor_stepk_tile(15, 8, kTaylorRegion, false) >= 256, "halo too wide for the staged region");
static_assert(taylor_stepk_tile(15, 8, kTaylorRegion, true) >= 32, "halo too wide for the staged region");
// (Double-double groups take the one-step kernel at every step instead: at a
// few steps per launch its halo recomputation cost more than the launches.)
hipError_t launch_taylor_stepk(int n, int kb, int ksteps, int reg, const DevProb* d_probs, int nprob, int64_t tiles,
                               const double* fd, const double* taylor, const double* d_u_in, double* d_u_out,
                               unsigned long long* stats, hipStream_t stream);
// Stationary one-sided tables (uniform grid, react = 0, p <= 2) by the finite
// Taylor series in double-double: items = n rows per instance (item_begin =
// the instance's first row); writes the plain table [kind][r][k] with the
// rows of e^{dt L}, dt phi1 and dt phi2.  tdd: the double-double table.
hipError_t launch_build_table_dd(int n, int p, const DevProb* d_probs, int nprob, int64_t items, const double* tdd,
                                 double* d_w, hipStream_t stream);

// Stationary weights by the LDS build (one matrix per wavefront, orders up to
// kMaxMWide): per node on non-uniform grids (p <= 2), and per harvested row of
// a uniform instance whose order n + p exceeds a DPP row (the stationary table
// [kind][r][k]; ETDRK4 parts as in launch_build).  items = nodes or rows.
hipError_t launch_build_wide(int n, int p, const DevProb* d_probs, int nprob, int64_t items, double* d_w,
                             hipStream_t stream);
size_t build_wide_lds_bytes(int n, int p);

// One time step over a group of instances sharing (n, scheme, nonlin,
// per-node weights); ETD2RK's two stages run in one kernel.  d_tile_inst maps
// each block (tile of `tile` nodes, 256 or 1024) to its instance in d_probs,
// whose item_begin is the instance's first tile.
hipError_t launch_apply(int n, int tile, int scheme, int nonlin, bool pernode, const DevProb* d_probs,
                        const int* d_tile_inst, int64_t tiles, const double* fd, const double* d_w,
                        const double* d_u_in, double* d_u_out, hipStream_t stream);
// Several steps per launch for instances of at most kResidentMaxN nodes: one
// block per instance, the whole instance in the block (resident.hip).
// uniform: stationary table weights on a uniform grid (any boundary, pointwise
// or no nonlinearity, n <= kMaxN), else per-node weights of a non-uniform grid
// (Dirichlet).  max_nodes = the group's largest N.
hipError_t launch_resident(int n, int scheme, int nonlin, bool uniform, const DevProb* d_probs, int count,
                           int64_t max_nodes, const double* d_w, const double* d_u_in, double* d_u_out, int ksteps,
                           hipStream_t stream);

// The same for non-uniform grids (stationary per-node weights, n <= kMaxNWide,
// nonlinearity none or Allen-Cahn).
hipError_t launch_apply_nonuniform(int n, int tile, int scheme, int nonlin, const DevProb* d_probs,
                                   const int* d_tile_inst, int64_t tiles, const double* fd, const double* d_w,
                                   const double* d_u_in, double* d_u_out, hipStream_t stream);

// Stationary weights, several steps per launch (stepk.hpp).  A block stages
// kStepRegion consecutive positions of its instance, advances them `ksteps`
// <= kb steps in LDS (kb = 1, 2, 4 or 8) and writes the middle
// stepk_tile(...) of them; the rest is the halo the steps consume (each
// stencil application spoils (n-1)/2 positions at each open end); kb = 16
// for the ETD schemes.
constexpr int kStepRegion = 2048;
constexpr int kStepRk4MaxKb = 8;  // ETDRK4 multi-step launches: at most 8 steps (the stationary ETD kernels 16)
__host__ __device__ constexpr int stepk_apps(int scheme, int nonlin) {
    // stencil applications per step: one per stage, one more per KdV N pass
    return (scheme == SCH_ETDRK4 && nonlin != NL_NONE ? 4 : (scheme == SCH_ETD2RK && nonlin != NL_NONE ? 2 : 1)) *
           (scheme != SCH_LINEAR && nonlin == NL_KDV ? 2 : 1);
}
__host__ __device__ constexpr int stepk_halo(int n, int scheme, int nonlin, int kb) {
    return kb * stepk_apps(scheme, nonlin) * ((n - 1) / 2);
}
__host__ __device__ constexpr int stepk_tile(int n, int scheme, int nonlin, int kb) {
    return kStepRegion - 2 * stepk_halo(n, scheme, nonlin, kb);
}
static_assert(stepk_tile(15, SCH_ETD2RK, NL_KDV, 16) >= 1024, "halo too wide for the staged region");
static_assert(stepk_tile(13, SCH_ETDRK4, NL_KDV, 8) >= 1024, "halo too wide for the staged region");
template <int KB>
hipError_t launch_stepk_depth(int n, int scheme, int nonlin, int ksteps, const DevProb* d_probs,
                              const int* d_tile_inst, int64_t tiles, const double* fd, const double* d_w,
                              const double* d_u_in, double* d_u_out, hipStream_t stream);
template <int KB>
hipError_t launch_stepk_upwind_depth(int side, int n, int scheme, int nonlin, int ksteps, const DevProb* d_probs,
                                     const int* d_tile_inst, int64_t tiles, const double* fd, const double* d_w,
                                     const double* d_u_in, double* d_u_out, hipStream_t stream);
// Block b of a group writes nodes [b' * tile, (b' + 1) * tile) of its instance,
// b' = b - item_begin, tile = stepk_tile(n, scheme, nonlin, kb) -- on
// Dirichlet and Neumann grids the last block [N - tile, N) when N >= tile.
// side: 0 centred windows, 1 one-sided windows ending at the node (c > 0),
// 2 starting at it (c < 0); every instance of a launch has the same side.
hipError_t launch_stepk(int n, int scheme, int nonlin, int kb, int ksteps, const DevProb* d_probs,
                        const int* d_tile_inst, int64_t tiles, const double* fd, const double* d_w,
                        const double* d_u_in, double* d_u_out, hipStream_t stream, int side = 0);
// One launch over instances of several stencil sizes (centred windows, ETD
// schemes, kb = 8 or 16): instance k's blocks write tiles of
// stepk_tile(n_k, ...) nodes; nmax = the largest n (sizes the weight rows'
// dynamic LDS).  Results equal the per-size kernels' bit for bit.
template <int KB>
hipError_t launch_stepk_mixed_depth(int nmax, int scheme, int nonlin, int ksteps, const DevProb* d_probs,
                                    const int* d_tile_inst, int64_t tiles, const double* fd, const double* d_w,
                                    const double* d_u_in, double* d_u_out, hipStream_t stream);
hipError_t launch_stepk_mixed(int nmax, int scheme, int nonlin, int kb, int ksteps, const DevProb* d_probs,
                              const int* d_tile_inst, int64_t tiles, const double* fd, const double* d_w,
                              const double* d_u_in, double* d_u_out, hipStream_t stream);

constexpr int kApplyTileTiny = 64;     // nodes per apply block for small non-uniform instances
constexpr int kApplyTileSmall = 256;   // nodes per apply block for groups with few nodes
constexpr int kApplyTile = 1024;       // nodes per apply block otherwise
constexpr int64_t kSmallGroupNodes = 1 << 20;  // groups below this many nodes use the small tile
constexpr int kAdjTile = 256;     // nodes per block of the reverse-step gathers

// One group (same n and p) of a reverse step.  tile_probs: item_begin =
// prefix of 256-node tiles; node_probs: the same instances with item_begin =
// prefix of nodes.  Scratch arrays are indexed by state_off (ws by
// state_off * ws_stride, dparam by 3 * state_off, part by 3 * tile).
struct AdjointLaunch {
    int n = 0, p = 0;
    const DevProb* tile_probs = nullptr;
    const DevProb* node_probs = nullptr;
    int nprob = 0;
    int64_t tiles = 0, nodes = 0;
    const double* fd = nullptr;
    const double* u = nullptr;
    const double* lam = nullptr;
    double* lam_out = nullptr;
    double* grad = nullptr;
    double* g = nullptr;
    double* ghat = nullptr;
    double* ws = nullptr;
    int ws_stride = 0;
    double* dparam = nullptr;
    double* part = nullptr;
    // set: the whole step by the finite Taylor series (table `taylor`) in one
    // kernel per tile of adj_fused_tile(n) nodes; item_begin = prefix of those tiles
    const double* taylor = nullptr;
    const DevProb* fused_probs = nullptr;
    int64_t fused_tiles = 0;
    bool disp = true;  // some instance of the group has a dispersion term (delta != 0)
    hipEvent_t frechet_begin = nullptr, frechet_end = nullptr;  // recorded around the Frechet kernel if set
};
hipError_t launch_adjoint(const AdjointLaunch& a, hipStream_t stream);
hipError_t launch_adj_fused(const AdjointLaunch& a, hipStream_t stream);
// Nodes per tile of the fused reverse step: a block forms the weights of
// kAdjTile positions, the tile and 2 (n - 1) on each side.
__host__ __device__ constexpr int adj_fused_tile(int n) { return kAdjTile - 4 * (n - 1); }
static_assert(adj_fused_tile(15) >= 128, "fused reverse-step tile");

// Scratch of lmep_step_noalloc (static_scratch.hip): a static array of
// kStaticScratchBytes in every device's memory.  static_scratch() returns the
// current device's address of it (looked up once per device);
// upload_by_args() writes `bytes` (a multiple of 4) of host data to d_dst on
// `stream` through the kernel arguments of small copy kernels, so nothing is
// staged in host memory that would have to outlive the call.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
hipError_t static_scratch(void** d_out);
hipError_t upload_by_args(void* d_dst, const void* host, size_t bytes, hipStream_t stream);

// Finite check: writes 1 into *d_flag if any of the count doubles is not finite.
hipError_t launch_check_finite(const double* d_x, int64_t count, int* d_flag, hipStream_t stream);

}  // namespace lmep
