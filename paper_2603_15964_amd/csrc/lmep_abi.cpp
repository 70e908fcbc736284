// C-ABI of liblmep (declared in include/lmep.h): argument checks, grouping of
// instances by kernel variant, scratch layout, upload of the device problem
// tables, and the launch sequence of each entry point.  A plan
// (lmep_plan_create) keeps the grouping and the uploaded tables of one batch
// for many calls; the plain entry points make a plan for one call.  All
// arithmetic of the method runs in the kernels; this file only plans and
// enqueues.
#include "lmep.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstddef>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "lmep_internal.hpp"

using namespace lmep;

// The Python binding mirrors this layout field by field.
static_assert(LMEP_NOALLOC_SCRATCH_BYTES == kStaticScratchBytes, "static scratch size");
static_assert(offsetof(lmep_problem, window) == 112 && offsetof(lmep_problem, x) == 120 &&
                  sizeof(lmep_problem) == 128,
              "lmep_problem layout");

namespace {

thread_local char t_err[512] = "";
thread_local double t_prof_build_ms = 0.0, t_prof_apply_ms = 0.0;
thread_local int32_t t_prof_build_n = 0, t_prof_apply_n = 0;
thread_local int64_t t_prof_matrices = 0, t_prof_squarings = 0;

// Kernel times of the last profiled call on this thread, per kernel name.
struct KernelTime {
    std::string name;
    double ms = 0.0;
    int32_t launches = 0;
};
thread_local std::vector<KernelTime> t_prof_kernels;

// Tuning options.  The process-wide values (lmep_set_option) are what a plan
// takes unless its creation overrides them; a plan keeps its own copy.
struct Opts {
    int steps_per_launch = 8;   // LMEP_OPT_STEPS_PER_LAUNCH
    int profile_adjoint = 0;    // LMEP_OPT_PROFILE_ADJOINT
    int fuse_frozen = 1;        // LMEP_OPT_FUSE_FROZEN
    int apply_tile = 0;         // LMEP_OPT_APPLY_TILE (0 = by size)
    int exp_method = LMEP_EXP_AUTO;  // LMEP_OPT_EXP_METHOD
    int taylor_region = 0;      // LMEP_OPT_TAYLOR_REGION (0 = by size)
    int merge_groups = 0;       // LMEP_OPT_MERGE_GROUPS
};
std::atomic<int> g_steps_per_launch{8}, g_profile_adjoint{0}, g_fuse_frozen{1}, g_apply_tile{0},
    g_exp_method{LMEP_EXP_AUTO}, g_taylor_region{0}, g_merge_groups{0};

Opts process_opts() {
    Opts o;
    o.steps_per_launch = g_steps_per_launch.load();
    o.profile_adjoint = g_profile_adjoint.load();
    o.fuse_frozen = g_fuse_frozen.load();
    o.apply_tile = g_apply_tile.load();
    o.exp_method = g_exp_method.load();
    o.taylor_region = g_taylor_region.load();
    o.merge_groups = g_merge_groups.load();
    return o;
}

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(t_err, sizeof(t_err), fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(LMEP_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// Validate one option value and store it in o.
int set_opt(Opts& o, int32_t option, int32_t value) {
    switch (option) {
        case LMEP_OPT_STEPS_PER_LAUNCH:
            if (value != 1 && value != 2 && value != 4 && value != 8 && value != 16)
                return fail(LMEP_ERR_ARG, "steps per launch must be 1, 2, 4, 8 or 16, got %d", value);
            o.steps_per_launch = value;
            return LMEP_OK;
        case LMEP_OPT_PROFILE_ADJOINT:
        case LMEP_OPT_FUSE_FROZEN:
            if (value != 0 && value != 1) return fail(LMEP_ERR_ARG, "option %d takes 0 or 1, got %d", option, value);
            (option == LMEP_OPT_PROFILE_ADJOINT ? o.profile_adjoint : o.fuse_frozen) = value;
            return LMEP_OK;
        case LMEP_OPT_EXP_METHOD:
            if (value != LMEP_EXP_AUTO && value != LMEP_EXP_PADE)
                return fail(LMEP_ERR_ARG, "exponential method must be LMEP_EXP_AUTO (0) or LMEP_EXP_PADE (1), got %d",
                            value);
            o.exp_method = value;
            return LMEP_OK;
        case LMEP_OPT_APPLY_TILE:
            if (value != 0 && value != 64 && value != kApplyTileSmall && value != kApplyTile)
                return fail(LMEP_ERR_ARG, "apply tile must be 0, 64, %d or %d, got %d", kApplyTileSmall, kApplyTile,
                            value);
            o.apply_tile = value;
            return LMEP_OK;
        case LMEP_OPT_TAYLOR_REGION:
            if (value != 0 && (value < 128 || value > kTaylorRegion || value % 64 != 0))
                return fail(LMEP_ERR_ARG, "finite-Taylor region must be 0 or a multiple of 64 in [128, %d], got %d",
                            kTaylorRegion, value);
            o.taylor_region = value;
            return LMEP_OK;
        case LMEP_OPT_MERGE_GROUPS:
            if (value != 0 && value != 1) return fail(LMEP_ERR_ARG, "option %d takes 0 or 1, got %d", option, value);
            o.merge_groups = value;
            return LMEP_OK;
        default: return fail(LMEP_ERR_ARG, "unknown option %d", option);
    }
}

int scheme_p(int scheme) {
    return scheme == LMEP_ETDRK4 ? 3 : (scheme == LMEP_ETD2RK ? 2 : (scheme == LMEP_ETD1 ? 1 : 0));
}
int scheme_kinds(int scheme) { return scheme == LMEP_ETDRK4 ? 6 : 1 + scheme_p(scheme); }
bool frozen(const lmep_problem& q) { return q.nonlin == LMEP_NL_BURGERS_FROZEN; }
bool nonuniform(const lmep_problem& q) { return q.x != nullptr; }
bool pernode(const lmep_problem& q) { return frozen(q) || nonuniform(q); }
// Frozen-velocity instances whose weights the finite-Taylor kernel builds: a
// polynomial operator in the first-derivative matrix (uniform grid, no
// reaction term), unless LMEP_OPT_EXP_METHOD asks for Pade.
bool taylor(const lmep_problem& q, const Opts& o) {
    return frozen(q) && !nonuniform(q) && q.react == 0.0 && o.exp_method == LMEP_EXP_AUTO;
}
// One-sided windows whose rows FP64 sums cannot resolve: the finite-Taylor
// build carried in double-double -- every stationary one-sided table (uniform
// grid, no reaction term) and frozen-velocity one-sided windows of
// kTaylorDdMinN or more points -- unless LMEP_OPT_EXP_METHOD asks for Pade.
bool taylor_dd(const lmep_problem& q, const Opts& o) {
    if (q.window != LMEP_WIN_UPWIND || nonuniform(q) || q.react != 0.0 || o.exp_method != LMEP_EXP_AUTO) return false;
    return frozen(q) ? q.n >= kTaylorDdMinN : q.scheme != LMEP_ETDRK4;
}

int64_t weight_count(const lmep_problem& q) {
    const int64_t kinds = scheme_kinds(q.scheme);
    return pernode(q) ? kinds * q.n * q.N : kinds * q.n * q.n;
}

bool finite(double x) { return std::isfinite(x); }

// Checks of one instance (ERR_ARG for malformed input, ERR_UNSUPPORTED for a
// well-formed combination the kernels do not implement).
int check_problem(const lmep_problem& q, int k) {
    const int nmax = nonuniform(q) ? kMaxNWide : (q.scheme == LMEP_ETDRK4 && !frozen(q) ? kMaxNRk4 : kMaxN);
    if (q.n < 3 || q.n > nmax || (q.n % 2) == 0)
        return fail(LMEP_ERR_ARG, "instance %d: stencil size n=%d must be odd, 3..%d", k, q.n, nmax);
    if (q.N < q.n) return fail(LMEP_ERR_ARG, "instance %d: N=%lld < n=%d", k, (long long)q.N, q.n);
    if (!(q.h > 0) || !finite(q.h)) return fail(LMEP_ERR_ARG, "instance %d: grid spacing h must be > 0", k);
    if (!(q.dt > 0) || !finite(q.dt)) return fail(LMEP_ERR_ARG, "instance %d: dt must be > 0", k);
    if (!finite(q.c) || !finite(q.nu) || !finite(q.delta) || !finite(q.react) || !finite(q.nl_coef) ||
        !finite(q.bc_left) || !finite(q.bc_right))
        return fail(LMEP_ERR_ARG, "instance %d: non-finite coefficient", k);
    if (q.bc < 0 || q.bc > 2) return fail(LMEP_ERR_ARG, "instance %d: unknown boundary type %d", k, q.bc);
    if (q.scheme < 0 || q.scheme > 3) return fail(LMEP_ERR_ARG, "instance %d: unknown scheme %d", k, q.scheme);
    if (q.nonlin < 0 || q.nonlin > 3) return fail(LMEP_ERR_ARG, "instance %d: unknown nonlinearity %d", k, q.nonlin);
    if (q.scheme == LMEP_LINEAR && q.nonlin != LMEP_NL_NONE)
        return fail(LMEP_ERR_ARG, "instance %d: LINEAR scheme with a nonlinear term", k);
    if (q.state_off < 0 || q.weight_off < 0) return fail(LMEP_ERR_ARG, "instance %d: negative offset", k);
    // the order of the augmented matrix: a DPP row (16) on uniform grids, the
    // LDS build (32) on non-uniform ones and for uniform ETDRK4 tables
    const int mmax = (nonuniform(q) || q.scheme == LMEP_ETDRK4) ? kMaxMWide : kMaxM;
    if (q.n + scheme_p(q.scheme) > mmax)
        return fail(LMEP_ERR_UNSUPPORTED, "instance %d: n + p = %d exceeds %d", k, q.n + scheme_p(q.scheme), mmax);
    if (frozen(q) && q.scheme != LMEP_ETD1)
        return fail(LMEP_ERR_UNSUPPORTED, "instance %d: frozen-velocity Burgers needs ETD1", k);
    if (q.window != LMEP_WIN_CENTRED && q.window != LMEP_WIN_UPWIND)
        return fail(LMEP_ERR_ARG, "instance %d: unknown window %d", k, q.window);
    if (q.window == LMEP_WIN_UPWIND && q.scheme == LMEP_ETDRK4)
        return fail(LMEP_ERR_UNSUPPORTED, "instance %d: upwind windows cover LINEAR, ETD1 and ETD2RK", k);
    if (nonuniform(q) && (q.bc != LMEP_BC_DIRICHLET || q.window != LMEP_WIN_CENTRED || q.scheme == LMEP_ETDRK4 ||
                          (q.nonlin != LMEP_NL_NONE && q.nonlin != LMEP_NL_ALLEN_CAHN)))
        return fail(LMEP_ERR_UNSUPPORTED,
                    "instance %d: non-uniform grids cover Dirichlet ends, centred windows, LINEAR / ETD1 / ETD2RK "
                    "and pointwise (none / Allen-Cahn) nonlinearity", k);
    return LMEP_OK;
}

// Ranges [off, off + len) of distinct instances must not overlap.
int check_disjoint(std::vector<std::pair<int64_t, int64_t>> r, const char* what) {
    std::sort(r.begin(), r.end());
    for (size_t k = 1; k < r.size(); ++k)
        if (r[k].first < r[k - 1].first + r[k - 1].second)
            return fail(LMEP_ERR_ARG, "%s ranges of two instances overlap", what);
    return LMEP_OK;
}

int check_all(const lmep_problem* prob, int32_t count, bool weights_used) {
    if (!prob || count <= 0) return fail(LMEP_ERR_ARG, "need count >= 1 problems");
    std::vector<std::pair<int64_t, int64_t>> s, w;
    for (int k = 0; k < count; ++k) {
        int rc = check_problem(prob[k], k);
        if (rc) return rc;
        s.emplace_back(prob[k].state_off, prob[k].N);
        w.emplace_back(prob[k].weight_off, weight_count(prob[k]));
    }
    int rc = check_disjoint(s, "state");
    if (rc) return rc;
    return weights_used ? check_disjoint(w, "weight") : LMEP_OK;
}

int64_t state_extent(const lmep_problem* prob, int32_t count) {
    int64_t e = 0;
    for (int k = 0; k < count; ++k) e = std::max(e, prob[k].state_off + prob[k].N);
    return e;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Scratch layout.
struct Layout {
    size_t build_tab = 0, apply_tab = 0, tile_inst = 0, state = 0, flag = 0, total = 0;
    size_t g = 0, ghat = 0, ws = 0, dparam = 0, part = 0;  // reverse step
    int ws_stride = 0;
};

int64_t total_tiles(const lmep_problem* prob, int32_t count, int tile) {
    int64_t t = 0;
    for (int k = 0; k < count; ++k) t += (prob[k].N + tile - 1) / tile;
    return t;
}

// Upper bound on the apply tiles of a batch (non-uniform instances may take
// the 64-node tile, the rest at least the 256-node one).
int64_t max_apply_tiles(const lmep_problem* prob, int32_t count) {
    int64_t t = 0;
    for (int k = 0; k < count; ++k) {
        const int tile = nonuniform(prob[k]) ? kApplyTileTiny : kApplyTileSmall;
        t += (prob[k].N + tile - 1) / tile;
    }
    return t;
}

Layout layout(const lmep_problem* prob, int32_t count, int op) {
    Layout L;
    size_t off = 0;
    const size_t tab = align256(sizeof(DevProb) * (size_t)count);
    L.build_tab = off;
    off += 2 * tab;  // an ETDRK4 instance has two build parts
    L.apply_tab = off;
    off += tab;
    if (op == 1) {
        L.tile_inst = off;
        off += align256(sizeof(int) * (size_t)max_apply_tiles(prob, count));
        L.state = off;
        off += align256(sizeof(double) * (size_t)state_extent(prob, count));
    }
    if (op == 2) {
        const size_t ext = (size_t)state_extent(prob, count);
        int nmax = 3;
        for (int k = 0; k < count; ++k) nmax = std::max(nmax, (int)prob[k].n);
        L.ws_stride = 2 * nmax;
        L.g = off;
        off += align256(sizeof(double) * ext);
        L.ghat = off;
        off += align256(sizeof(double) * ext);
        L.ws = off;
        off += align256(sizeof(double) * ext * (size_t)L.ws_stride);
        L.dparam = off;
        off += align256(sizeof(double) * 3 * ext);
        L.part = off;  // per tile partial sums: 256-node tiles, or the fused kernel's (>= 128 nodes)
        off += align256(sizeof(double) * 3 * (size_t)total_tiles(prob, count, 128));
    }
    L.flag = off;
    off += 256;
    L.total = off;
    return L;
}

// Rows [first, first + count) of a table hold one group, with item_begin the
// prefix of `total` work items: when every instance has the same number of
// items, each row records it and the kernels find a block's instance by a
// division instead of a search.
void mark_each(std::vector<DevProb>& tab, size_t first, size_t count, int64_t total) {
    if (count == 0) return;
    const int64_t each = total / (int64_t)count;
    bool same = each > 0 && each * (int64_t)count == total && each <= INT32_MAX;
    for (size_t k = 0; same && k < count; ++k) same = tab[first + k].item_begin == (int64_t)k * each;
    for (size_t k = 0; k < count; ++k) tab[first + k].each = same ? (int32_t)each : 0;
}

DevProb to_dev(const lmep_problem& q, int index) {
    DevProb d;
    std::memset(&d, 0, sizeof(d));
    d.N = q.N;
    d.state_off = q.state_off;
    d.weight_off = q.weight_off;
    d.n = q.n;
    d.bc = q.bc;
    d.scheme = q.scheme;
    d.nonlin = q.nonlin;
    d.p = scheme_p(q.scheme);
    d.frozen = frozen(q) ? 1 : 0;
    d.index = index;
    d.h = q.h;
    d.dt = q.dt;
    d.c = q.c;
    d.nu = q.nu;
    d.delta = q.delta;
    d.react = q.react;
    d.nl_coef = q.nl_coef;
    d.bc_left = q.bc_left;
    d.bc_right = q.bc_right;
    d.window = q.window;
    d.x = q.x;
    return d;
}

// A launch group: a contiguous slice of a device table whose instances share
// one kernel variant.
struct Group {
    int n = 0, p = 0, scheme = 0, nonlin = 0, tile = 0;
    int reg = 0;             // multi-step finite-Taylor groups: staged positions per block
    int kb = 1;              // steps per launch of the group's multi-step kernel
    bool taylor = false;     // build by finite Taylor series (items = kTaylorTile-node tiles)
    bool dd = false;         // ... carried in double-double (frozen one-sided windows)
    bool ddtable = false;    // stationary one-sided table in double-double (items = rows)
    bool pernode = false;    // weights stored per node (frozen velocity or non-uniform grid)
    bool frozen = false;     // rebuilt every step (frozen velocity)
    bool nonuniform = false; // non-uniform grid: per-node stationary weights
    bool wide = false;       // build groups: the LDS build (non-uniform grids, orders beyond a DPP row)
    bool resident = false;   // non-uniform, several steps per launch, one block per instance
    int64_t max_nodes = 0;
    bool stepk = false;  // stationary multi-step kernel (always for ETDRK4)
    int side = 0;        // stationary windows: 0 centred, 1 one-sided ending at the node (c > 0), 2 starting at it
    bool mixed = false;  // one multi-step launch over several stencil sizes (n = the largest)
    bool unit_g = false;  // merged Allen-Cahn launch whose every instance has g = 1
    int first = 0, count = 0;  // slice of the table
    int64_t items = 0;         // matrices (build) or tiles (apply)
    int64_t nodes = 0;         // nodes of the group's instances
};

// Compute units of the current device (cached per device; 256 on MI355X).
int cu_count() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int c = cache[dev].load();
    if (c <= 0) {
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c <= 0) c = 256;
        cache[dev].store(c);
    }
    return c;
}

// Build groups: keyed by (n, p).  Instances selected by `want`.  frozen_kb > 0:
// finite-Taylor groups advance frozen_kb steps per launch (tiles of
// taylor_stepk_tile(n, frozen_kb) nodes instead of kTaylorTile).
template <class Want>
std::vector<Group> plan_build(const lmep_problem* prob, int32_t count, Want want, std::vector<DevProb>& tab,
                              const Opts& o, int frozen_kb = 0) {
    // one build part per exponential: ETDRK4 needs two (p = 3 at dt, p = 1 at dt/2)
    struct Part {
        int k, harvest;
    };
    // (n, p, kind): kind 0 Pade in DPP rows, 1 the LDS build, 2 finite Taylor,
    // 3 finite Taylor in double-double (frozen velocity), 4 a stationary table
    // in double-double
    std::map<std::tuple<int, int, int>, std::vector<Part>> by;
    // the LDS build for non-uniform grids and for orders beyond a DPP row
    auto kind_of = [&](const lmep_problem& q, int p) {
        if (nonuniform(q) || q.n + p > kMaxM) return 1;
        if (taylor_dd(q, o)) return frozen(q) ? 3 : 4;
        return taylor(q, o) ? 2 : 0;
    };
    for (int k = 0; k < count; ++k) {
        if (!want(prob[k])) continue;
        if (prob[k].scheme == LMEP_ETDRK4) {
            by[{prob[k].n, 3, kind_of(prob[k], 3)}].push_back({k, HARVEST_RK4_FULL});
            by[{prob[k].n, 1, kind_of(prob[k], 1)}].push_back({k, HARVEST_RK4_HALF});
        } else {
            const int p = scheme_p(prob[k].scheme);
            by[{prob[k].n, p, kind_of(prob[k], p)}].push_back({k, HARVEST_PLAIN});
        }
    }
    std::vector<Group> groups;
    for (auto& kv : by) {
        Group g;
        g.n = std::get<0>(kv.first);
        g.p = std::get<1>(kv.first);
        g.wide = std::get<2>(kv.first) == 1;
        g.taylor = std::get<2>(kv.first) == 2 || std::get<2>(kv.first) == 3;
        g.dd = std::get<2>(kv.first) == 3;
        g.ddtable = std::get<2>(kv.first) == 4;
        for (const Part& part : kv.second) g.nodes += prob[part.k].N;
        // double-double groups advance one step per launch (their fused one-step
        // kernel), the others up to kTaylorMaxKb in the multi-step kernel
        const bool multi_taylor = g.taylor && frozen_kb > 0 && !g.dd;
        if (multi_taylor) g.kb = std::min(frozen_kb, kTaylorMaxKb);
        if (multi_taylor) {
            // staged positions per block (= threads): about one block per CU for
            // groups too small to fill the GPU -- a step then costs the latency of
            // one block, not of the two or three an uneven spread puts on some
            // CUs -- and the full region for larger ones
            bool upwind = false;
            for (const Part& part : kv.second) upwind |= prob[part.k].window == LMEP_WIN_UPWIND;
            const int64_t halo = (int64_t)g.kb * taylor_stepk_reach(g.n, upwind);
            const int64_t want_tile = std::max<int64_t>((g.nodes + cu_count() - 1) / cu_count(), 64);
            g.reg = (int)std::min<int64_t>((want_tile + 2 * halo + 63) / 64 * 64, kTaylorRegion);
            // a forced region, raised where it would write fewer than 64 nodes per block
            if (o.taylor_region > 0)
                g.reg = (int)std::min<int64_t>(std::max<int64_t>(o.taylor_region, (64 + 2 * halo + 63) / 64 * 64),
                                               kTaylorRegion);
        }
        g.first = (int)tab.size();
        int64_t items = 0;
        for (const Part& part : kv.second) {
            DevProb d = to_dev(prob[part.k], part.k);
            d.p = g.p;
            d.harvest = part.harvest;
            if (part.harvest == HARVEST_RK4_HALF) d.dt = 0.5 * prob[part.k].dt;
            d.item_begin = items;
            const int64_t tt = multi_taylor ? taylor_stepk_tile(g.n, g.kb, g.reg,
                                                                prob[part.k].window == LMEP_WIN_UPWIND)
                                            : kTaylorTile;
            items += g.taylor ? (prob[part.k].N + tt - 1) / tt
                              : (pernode(prob[part.k]) ? prob[part.k].N : prob[part.k].n);
            tab.push_back(d);
        }
        g.count = (int)kv.second.size();
        g.items = items;
        mark_each(tab, g.first, g.count, items);
        groups.push_back(g);
    }
    return groups;
}

// Apply groups: keyed by kernel variant; also fills the block -> table-row map.
// multi_kb > 0: tiles of the multi-step kernel advancing multi_kb steps per launch.
// Window side of a stationary instance's interior nodes (frozen-velocity and
// non-uniform instances pick theirs per node: 0).
int stationary_side(const lmep_problem& q) {
    if (frozen(q) || nonuniform(q) || q.window != LMEP_WIN_UPWIND || q.c == 0.0) return 0;
    return q.c > 0.0 ? 1 : 2;
}

std::vector<Group> plan_apply(const lmep_problem* prob, int32_t count, std::vector<DevProb>& tab,
                              std::vector<int>& tile_inst, const Opts& o, int multi_kb = 0) {
    // weight kind: 0 stationary table, 1 frozen velocity, 2 non-uniform grid.
    // With LMEP_OPT_MERGE_GROUPS the instances of a multi-step launch at 8 or
    // 16 steps (uniform, stationary, centred, not ETDRK4, more than
    // kResidentMaxN nodes) form one group per scheme and nonlinearity whatever
    // their n (key n = 0), ordered by n descending.
    auto mergeable = [&](const lmep_problem& q) {
        return o.merge_groups != 0 && (multi_kb == 8 || multi_kb == 16) && !frozen(q) && !nonuniform(q) &&
               stationary_side(q) == 0 && q.scheme != LMEP_ETDRK4 && q.N > kResidentMaxN;
    };
    std::map<std::tuple<int, int, int, int, int>, std::vector<int>> by;
    for (int k = 0; k < count; ++k)
        by[{mergeable(prob[k]) ? 0 : prob[k].n, prob[k].scheme, prob[k].nonlin,
            frozen(prob[k]) ? 1 : (nonuniform(prob[k]) ? 2 : 0), stationary_side(prob[k])}]
            .push_back(k);
    std::vector<Group> groups;
    for (auto& kv : by) {
        Group g;
        std::tie(g.n, g.scheme, g.nonlin, std::ignore, g.side) = kv.first;
        if (g.n == 0) {  // several stencil sizes: the largest first (the launch ends on the shortest blocks)
            std::stable_sort(kv.second.begin(), kv.second.end(),
                             [&](int a, int b) { return prob[a].n > prob[b].n; });
            g.n = prob[kv.second.front()].n;
            g.mixed = prob[kv.second.back()].n != g.n;  // one size only: the per-size kernel
        }
        g.pernode = std::get<3>(kv.first) != 0;
        g.frozen = std::get<3>(kv.first) == 1;
        g.nonuniform = std::get<3>(kv.first) == 2;
        g.first = (int)tab.size();
        for (int k : kv.second) g.nodes += prob[k].N;
        for (int k : kv.second) g.max_nodes = std::max(g.max_nodes, prob[k].N);
        g.unit_g = g.mixed && g.nonlin == LMEP_NL_ALLEN_CAHN && g.scheme != LMEP_LINEAR;
        for (int k : kv.second) g.unit_g = g.unit_g && prob[k].nl_coef == 1.0;
        // several steps per launch: whole small instances per block (non-uniform
        // grids always; uniform ones with a stationary table, a pointwise or no
        // nonlinearity and at most kResidentMaxN nodes), else the tiled kernel
        const bool small_uniform = !g.pernode && g.max_nodes <= kResidentMaxN && g.scheme != LMEP_ETDRK4 &&
                                   (g.nonlin == LMEP_NL_NONE || g.nonlin == LMEP_NL_ALLEN_CAHN);
        g.resident = multi_kb > 0 && !g.mixed && (g.nonuniform || small_uniform);
        g.stepk = !g.resident && !g.nonuniform && (multi_kb > 0 || g.scheme == LMEP_ETDRK4);
        if (g.stepk && multi_kb > 0) g.kb = g.scheme == LMEP_ETDRK4 ? std::min(multi_kb, kStepRk4MaxKb) : multi_kb;
        const int64_t avg = g.nodes / (int64_t)kv.second.size();
        const int forced = o.apply_tile;  // 0, 64 (non-uniform groups only), 256 or 1024
        g.tile = g.stepk ? stepk_tile(g.n, g.scheme, g.nonlin, g.kb)
                 : (forced != 0 && (forced != kApplyTileTiny || g.nonuniform))
                     ? forced
                     : (g.nonuniform && avg <= kApplyTileTiny)
                           ? kApplyTileTiny
                           : ((g.nodes < kSmallGroupNodes || avg <= kApplyTileSmall) ? kApplyTileSmall : kApplyTile);
        int64_t tiles = 0;
        for (int k : kv.second) {
            DevProb d = to_dev(prob[k], k);
            d.item_begin = tiles;
            const int64_t tk = g.mixed ? stepk_tile(prob[k].n, g.scheme, g.nonlin, g.kb) : g.tile;
            const int64_t nt = (prob[k].N + tk - 1) / tk;
            for (int64_t t = 0; t < nt; ++t) tile_inst.push_back((int)(tab.size() - g.first));
            tiles += nt;
            tab.push_back(d);
        }
        g.count = (int)kv.second.size();
        g.items = tiles;
        mark_each(tab, g.first, g.count, tiles);
        groups.push_back(g);
    }
    return groups;
}

// Names of the kernels a group launches, as a kernel trace shows them
// (namespace and argument list left out).
std::string bool_s(bool b) { return b ? "true" : "false"; }
std::string build_kernel_name(const Group& g, bool fused, bool multi) {
    char b[96];
    if (g.wide) return "build_wide_kernel";
    const char* dd = g.dd ? "_dd" : "";
    if (g.ddtable) snprintf(b, sizeof(b), "build_table_dd_kernel<%d,%d>", g.n, g.p);
    else if (g.taylor && multi && !g.dd) snprintf(b, sizeof(b), "taylor_stepk_kernel<%d>", g.n);
    else if (g.taylor) snprintf(b, sizeof(b), "build_taylor%s_kernel<%d,%s>", dd, g.n, bool_s(fused).c_str());
    else snprintf(b, sizeof(b), "build_pade_kernel<%d,%d,%s>", g.n, g.p, bool_s(fused).c_str());
    return b;
}
// nonlinearity code of a merged multi-step launch
int mixed_nonlin(const Group& g) { return g.unit_g ? kNlAcUnit : g.nonlin; }
std::string apply_kernel_name(const Group& g) {
    const int kb = g.kb;
    char b[96];
    const int nl = g.scheme == LMEP_LINEAR ? 0 : g.nonlin;
    if (g.stepk && g.scheme == LMEP_ETDRK4) snprintf(b, sizeof(b), "stepk_rk4_kernel<%d,%d,%d>", g.n, g.nonlin, kb);
    else if (g.stepk && g.mixed)
        snprintf(b, sizeof(b), "stepk_mixed_kernel<%d,%d,%d>", g.scheme, g.scheme == LMEP_LINEAR ? 0 : mixed_nonlin(g),
                 kb);
    else if (g.stepk && g.side != 0)
        snprintf(b, sizeof(b), "stepk_upwind_kernel<%d,%d,%d,%d,%d>", g.n, g.scheme, nl, kb, g.side);
    else if (g.stepk) snprintf(b, sizeof(b), "stepk_kernel<%d,%d,%d,%d>", g.n, g.scheme, nl, kb);
    else if (g.resident)
        snprintf(b, sizeof(b), "resident_kernel<%d,%d,%d,%s>", g.n, g.scheme, nl, bool_s(!g.nonuniform).c_str());
    else snprintf(b, sizeof(b), "apply_kernel<%d,%d,%d,%s,%d>", g.n, g.scheme, nl, bool_s(g.pernode).c_str(), g.tile);
    return b;
}

// Host staging for uploads of device tables: a ring of pinned buffers owned by
// the calling thread, each guarded by an event until its copy has been
// consumed, so that consecutive calls do not wait for each other's copies.
struct Staging {
    static constexpr int kSlots = 8;
    struct Slot {
        void* host = nullptr;
        size_t cap = 0;
        hipEvent_t done = nullptr;
        bool pending = false;
    } slot[kSlots];
    int next = 0;
    ~Staging() {
        for (Slot& s : slot) {
            if (s.pending && s.done) (void)hipEventSynchronize(s.done);
            if (s.host) (void)hipHostFree(s.host);
            if (s.done) (void)hipEventDestroy(s.done);
        }
    }
};
thread_local Staging t_stage;

// One host-to-device copy of `bytes` from `image` to d_dst on s.
int upload_image(const void* image, size_t bytes, void* d_dst, hipStream_t s) {
    if (bytes == 0) return LMEP_OK;
    Staging::Slot& st = t_stage.slot[t_stage.next];
    t_stage.next = (t_stage.next + 1) % Staging::kSlots;
    if (!st.done) HIP_TRY(hipEventCreateWithFlags(&st.done, hipEventDisableTiming));
    if (st.pending) {
        HIP_TRY(hipEventSynchronize(st.done));
        st.pending = false;
    }
    if (st.cap < bytes) {
        if (st.host) HIP_TRY(hipHostFree(st.host));
        st.host = nullptr;
        st.cap = 0;
        const size_t cap = std::max<size_t>(bytes, 1 << 16);
        HIP_TRY(hipHostMalloc(&st.host, cap, hipHostMallocDefault));
        st.cap = cap;
    }
    std::memcpy(st.host, image, bytes);
    HIP_TRY(hipMemcpyAsync(d_dst, st.host, bytes, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(st.done, s));
    st.pending = true;
    return LMEP_OK;
}

// Device tables of a call, laid out as in the scratch buffer from offset 0:
// pieces (scratch offset, bytes, data) go into one host image and one copy,
// or, by_args, through kernel arguments (lmep_step_noalloc).
struct Piece {
    size_t off;
    size_t bytes;
    const void* data;
};
int upload_pieces(const std::vector<Piece>& pieces, char* base, hipStream_t s, bool by_args) {
    if (by_args) {
        for (const Piece& p : pieces)
            if (p.bytes) HIP_TRY(upload_by_args(base + p.off, p.data, p.bytes, s));
        return LMEP_OK;
    }
    size_t end = 0;
    for (const Piece& p : pieces)
        if (p.bytes) end = std::max(end, p.off + p.bytes);
    if (end == 0) return LMEP_OK;
    std::vector<char> image(end, 0);
    for (const Piece& p : pieces)
        if (p.bytes) std::memcpy(image.data() + p.off, p.data, p.bytes);
    return upload_image(image.data(), end, base, s);
}

// Scratch checks first (host only), then pick up any pending device error.
int entry_checks(void* d_scratch, size_t scratch_bytes, size_t need) {
    if (!d_scratch || scratch_bytes < need)
        return fail(LMEP_ERR_SCRATCH, "scratch of %zu bytes needed, %zu given", need, d_scratch ? scratch_bytes : 0);
    if (((uintptr_t)d_scratch) % 256 != 0) return fail(LMEP_ERR_ARG, "scratch must be 256-byte aligned");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LMEP_ERR_DEVICE, "earlier device error: %s", hipGetErrorString(e));
    return LMEP_OK;
}

// HIP events bracketing every launch of the profiled kernels, one list per
// kernel name.  All events are created before the first launch so that
// recording them costs the host little and the host stays ahead of the device.
struct Timer {
    bool on = false;
    struct Span {
        int kernel;    // index into names
        bool build;    // weight-build (or fused build + step) launch, else apply
        int launches = 1;  // back-to-back launches of the kernel the span covers
        hipEvent_t a = nullptr, b = nullptr;
    };
    std::vector<std::string> names;
    std::vector<Span> spans;
    size_t used = 0;
    ~Timer() {
        for (Span& sp : spans) {
            if (sp.a) (void)hipEventDestroy(sp.a);
            if (sp.b) (void)hipEventDestroy(sp.b);
        }
    }
    hipError_t reserve(size_t launches) {
        if (!on) return hipSuccess;
        spans.assign(launches, Span{});
        hipError_t e;
        for (Span& sp : spans) {
            if ((e = hipEventCreate(&sp.a)) != hipSuccess) return e;
            if ((e = hipEventCreate(&sp.b)) != hipSuccess) return e;
        }
        return hipSuccess;
    }
    int kernel_index(const std::string& name) {
        for (size_t k = 0; k < names.size(); ++k)
            if (names[k] == name) return (int)k;
        names.push_back(name);
        return (int)names.size() - 1;
    }
    // begin(): returns the span index (or -1 when off); end(idx) records its end
    int begin(const std::string& name, bool build, hipStream_t s, hipError_t& e) {
        e = hipSuccess;
        if (!on) return -1;
        if (used >= spans.size()) {
            e = hipErrorInvalidValue;
            return -1;
        }
        Span& sp = spans[used];
        sp.kernel = kernel_index(name);
        sp.build = build;
        e = hipEventRecord(sp.a, s);
        return (int)used++;
    }
    hipError_t end(int idx, hipStream_t s, int launches = 1) {
        if (!on || idx < 0) return hipSuccess;
        spans[idx].launches = launches;
        return hipEventRecord(spans[idx].b, s);
    }
    // waits for the events; totals into the thread's profile records
    int collect(hipStream_t s) {
        if (!on) return LMEP_OK;
        HIP_TRY(hipStreamSynchronize(s));
        double bms = 0.0, ams = 0.0;
        int32_t bn = 0, an = 0;
        std::vector<KernelTime> per(names.size());
        for (size_t k = 0; k < names.size(); ++k) per[k].name = names[k];
        for (size_t k = 0; k < used; ++k) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, spans[k].a, spans[k].b));
            per[spans[k].kernel].ms += ms;
            per[spans[k].kernel].launches += spans[k].launches;
            if (spans[k].build) {
                bms += ms;
                bn += spans[k].launches;
            } else {
                ams += ms;
                an += spans[k].launches;
            }
        }
        t_prof_build_ms = bms;
        t_prof_apply_ms = ams;
        t_prof_build_n = bn;
        t_prof_apply_n = an;
        t_prof_kernels = per;
        return LMEP_OK;
    }
};

// Stream on which step loops are captured into a graph (the legacy default
// stream cannot be captured); the graph itself is launched on the caller's
// stream.  One per thread, default priority.
struct CaptureStream {
    hipStream_t s = nullptr;
    ~CaptureStream() {
        if (s) (void)hipStreamDestroy(s);
    }
};
thread_local CaptureStream t_capture;

// ------------------------------------------------------------- step plans --
// Everything lmep_step needs besides the pointers of one call: the checked
// batch, the option values, the launch groups and their device tables (their
// place in the scratch buffer given by the layout).
struct StepPlan {
    Opts o;
    bool multi = false;  // LMEP_F_PERSISTENT
    int kb = 1;          // steps per launch
    bool fuse = true;    // frozen-velocity steps in one kernel per launch
    int count = 0;
    std::vector<Group> bgroups, agroups;
    std::vector<DevProb> btab, atab;
    std::vector<int> tile_inst;
    bool all_resident = false;    // every group advances all steps in its first launch
    bool apply_launched = false;  // any apply kernel besides the fused ones
    bool need_taylor = false;
    bool need_dd = false;
    Layout L;
    int64_t ext = 0;
};

int make_step_plan(StepPlan& P, const lmep_problem* prob, int32_t count, bool multi, const Opts& o) {
    int rc = check_all(prob, count, true);
    if (rc) return rc;
    if (multi)
        for (int k = 0; k < count; ++k) {
            if (frozen(prob[k]) && (!taylor(prob[k], o) || prob[k].bc == LMEP_BC_NEUMANN))
                return fail(LMEP_ERR_UNSUPPORTED, "LMEP_F_PERSISTENT with BURGERS_FROZEN (instance %d) needs the "
                            "finite-Taylor build (react = 0, LMEP_EXP_AUTO) on a Dirichlet or periodic grid", k);
            if (nonuniform(prob[k]) && prob[k].N > kResidentMaxN)
                return fail(LMEP_ERR_UNSUPPORTED, "LMEP_F_PERSISTENT on a non-uniform grid needs N <= %d "
                            "(instance %d)", kResidentMaxN, k);
        }
    P.o = o;
    P.multi = multi;
    P.kb = multi ? o.steps_per_launch : 1;
    P.fuse = o.fuse_frozen != 0 || multi;  // the multi-step frozen-velocity kernel is always fused
    P.count = count;
    P.bgroups = plan_build(prob, count, [](const lmep_problem& q) { return frozen(q); }, P.btab, o, multi ? P.kb : 0);
    P.agroups = plan_apply(prob, count, P.atab, P.tile_inst, o, multi ? P.kb : 0);
    for (auto& g : P.bgroups) P.need_taylor |= g.taylor && !g.dd;
    for (auto& g : P.bgroups) P.need_dd |= g.dd;
    P.all_resident = P.bgroups.empty();
    for (auto& g : P.agroups) P.all_resident &= g.resident;
    for (auto& g : P.agroups) P.apply_launched |= !(g.frozen && P.fuse);
    P.L = layout(prob, count, 1);
    P.ext = state_extent(prob, count);
    return LMEP_OK;
}

std::vector<Piece> step_pieces(const StepPlan& P) {
    return {{P.L.build_tab, P.btab.size() * sizeof(DevProb), P.btab.data()},
            {P.L.apply_tab, P.atab.size() * sizeof(DevProb), P.atab.data()},
            {P.L.tile_inst, P.tile_inst.size() * sizeof(int), P.tile_inst.data()}};
}

// Launches of a group for n_steps steps: one per kb steps (the resident
// kernel: one, which runs them all), and the most of any group.
int group_launches(const Group& g, int n_steps) { return g.resident ? 1 : (n_steps + g.kb - 1) / g.kb; }
int step_launches(const StepPlan& P, int n_steps) {
    int l = 1;
    for (auto& g : P.bgroups) l = std::max(l, group_launches(g, n_steps));
    for (auto& g : P.agroups)
        if (!(g.frozen && P.fuse)) l = std::max(l, group_launches(g, n_steps));
    return l;
}

// The launch sequence of n_steps steps (kernels only: capturable).
int enqueue_steps(const StepPlan& P, char* base, const double* fd, const double* tay, const double* tdd, double* d_w,
                  const double* d_u_in, double* d_u_out, int n_steps, unsigned long long* counters, Timer& timer,
                  hipStream_t s) {
    const DevProb* dbt = (const DevProb*)(base + P.L.build_tab);
    const DevProb* dat = (const DevProb*)(base + P.L.apply_tab);
    const int* dti = (const int*)(base + P.L.tile_inst);
    double* bufA = (double*)(base + P.L.state);
    const int launches = step_launches(P, n_steps);
    hipError_t e = hipSuccess;
    // When a step runs a single kernel, its launches follow each other with
    // nothing between them: one pair of events spans them all (events around
    // each launch would add their own cost to short kernels).
    int per_round = (int)P.bgroups.size();
    for (auto& gr : P.agroups) per_round += !(gr.frozen && P.fuse);
    const bool one_span = per_round == 1;
    int span = -1;
    // Round st launches every group that still has steps to go.  Each
    // group's destinations alternate between the scratch state and d_u_out
    // so that its last launch lands in d_u_out and none works in place
    // (groups own disjoint parts of both).
    auto src_of = [&](int st, int lg) -> const double* {
        return (st == 0) ? d_u_in : (((lg - st) % 2 == 0) ? d_u_out : bufA);
    };
    auto dst_of = [&](int st, int lg) -> double* { return ((lg - 1 - st) % 2 == 0) ? d_u_out : bufA; };
    for (int st = 0; st < launches; ++st) {
        // frozen-velocity groups: weights rebuilt, and with fusion applied in
        // the same kernel (their apply groups are then skipped)
        for (auto& gr : P.bgroups) {
            const int lg = group_launches(gr, n_steps), kb = gr.kb;
            if (st >= lg) continue;
            const double* src = src_of(st, lg);
            double* dst = dst_of(st, lg);
            int t = -1;
            if (timer.on && (!one_span || st == 0)) {
                t = timer.begin(build_kernel_name(gr, P.fuse, P.multi), true, s, e);
                HIP_TRY(e);
                if (one_span) span = t;
            }
            const double* tt = gr.dd ? tdd : tay;
            if (gr.taylor && P.multi && !gr.dd)
                HIP_TRY(launch_taylor_stepk(gr.n, kb, std::min(kb, n_steps - st * kb), gr.reg, dbt + gr.first,
                                            gr.count, gr.items, fd, tt, src, dst, counters, s));
            else if (gr.taylor)
                HIP_TRY(launch_build_taylor(gr.n, dbt + gr.first, gr.count, gr.items, fd, tt, src, d_w, counters, s,
                                            P.fuse ? dst : nullptr, gr.dd));
            else
                HIP_TRY(launch_build(gr.n, gr.p, dbt + gr.first, gr.count, gr.items, fd, src, d_w, counters, s,
                                     P.fuse ? dst : nullptr));
            if (!one_span) HIP_TRY(timer.end(t, s));
        }
        int64_t tile0 = 0;
        for (auto& gr : P.agroups) {
            const bool fused = gr.frozen && P.fuse;  // already advanced by its build kernel
            const int lg = group_launches(gr, n_steps), kb = gr.kb;
            if (!fused && st < lg) {
                const double* src = src_of(st, lg);
                double* dst = dst_of(st, lg);
                int t = -1;
                if (timer.on && (!one_span || st == 0)) {
                    t = timer.begin(apply_kernel_name(gr), false, s, e);
                    HIP_TRY(e);
                    if (one_span) span = t;
                }
                if (gr.stepk && gr.mixed)
                    HIP_TRY(launch_stepk_mixed(gr.n, gr.scheme, mixed_nonlin(gr), kb, std::min(kb, n_steps - st * kb),
                                               dat + gr.first, dti + tile0, gr.items, fd, d_w, src, dst, s));
                else if (gr.stepk)
                    HIP_TRY(launch_stepk(gr.n, gr.scheme, gr.nonlin, kb, std::min(kb, n_steps - st * kb),
                                         dat + gr.first, dti + tile0, gr.items, fd, d_w, src, dst, s, gr.side));
                else if (gr.resident) {
                    // in place after the first chunk: a block reads its whole
                    // instance before it writes any of it
                    for (int done = 0; st == 0 && done < n_steps; done += kResidentMaxSteps)
                        HIP_TRY(launch_resident(gr.n, gr.scheme, gr.nonlin, !gr.nonuniform, dat + gr.first, gr.count,
                                                gr.max_nodes,
                                                d_w, done == 0 ? d_u_in : d_u_out, d_u_out,
                                                std::min(kResidentMaxSteps, n_steps - done), s));
                } else if (gr.nonuniform)
                    HIP_TRY(launch_apply_nonuniform(gr.n, gr.tile, gr.scheme, gr.nonlin, dat + gr.first, dti + tile0,
                                                    gr.items, fd, d_w, src, dst, s));
                else
                    HIP_TRY(launch_apply(gr.n, gr.tile, gr.scheme, gr.nonlin, gr.pernode, dat + gr.first,
                                         dti + tile0, gr.items, fd, d_w, src, dst, s));
                if (!one_span) HIP_TRY(timer.end(t, s));
            }
            tile0 += gr.items;
        }
    }
    if (one_span) HIP_TRY(timer.end(span, s, launches));
    return LMEP_OK;
}

// Instantiated graphs of a plan's step loop, keyed by the pointers and the
// step count they were captured with; the oldest is dropped beyond kMax.
struct GraphCache {
    static constexpr size_t kMax = 4;
    struct Entry {
        const void *w, *in, *out;
        int steps;
        hipGraphExec_t exec;
    };
    std::vector<Entry> entries;
    void clear() {
        for (Entry& e : entries) (void)hipGraphExecDestroy(e.exec);
        entries.clear();
    }
    ~GraphCache() { clear(); }
};

// Capture the step loop on this thread's capture stream and instantiate it.
int capture_steps(const StepPlan& P, char* base, const double* fd, const double* tay, const double* tdd, double* d_w,
                  const double* d_u_in, double* d_u_out, int n_steps, hipGraphExec_t* exec) {
    if (!t_capture.s) HIP_TRY(hipStreamCreateWithFlags(&t_capture.s, hipStreamNonBlocking));
    hipStream_t cs = t_capture.s;
    HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    Timer off;
    int rc = enqueue_steps(P, base, fd, tay, tdd, d_w, d_u_in, d_u_out, n_steps, nullptr, off, cs);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &g);
    if (rc) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(LMEP_ERR_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(LMEP_ERR_DEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    return LMEP_OK;
}

// n_steps steps of a planned batch whose tables are in place at `base`.
// cache: graphs kept across calls (plans), or nullptr (captured, replayed and
// destroyed within the call).
int run_step(const StepPlan& P, char* base, double* d_w, const double* d_u_in, double* d_u_out, int n_steps,
             uint32_t flags, hipStream_t s, GraphCache* cache) {
    const double* fd = nullptr;
    const double* tay = nullptr;
    const double* tdd = nullptr;
    HIP_TRY(fd_table_init(&fd));
    if (P.need_taylor) HIP_TRY(taylor_table_init(&tay));
    if (P.need_dd) HIP_TRY(taylor_dd_table_init(&tdd));
    Timer timer;
    timer.on = (flags & LMEP_F_PROFILE) != 0;
    const size_t per_launch = P.bgroups.size() + P.agroups.size();
    HIP_TRY(timer.reserve(per_launch * (size_t)step_launches(P, n_steps)));
    unsigned long long* counters = (flags & LMEP_F_COUNT) ? (unsigned long long*)(base + P.L.flag + 64) : nullptr;
    if (counters) HIP_TRY(hipMemsetAsync(counters, 0, 2 * sizeof(unsigned long long), s));
    int rc;
    if (flags & LMEP_F_GRAPH) {
        hipGraphExec_t exec = nullptr;
        if (cache)
            for (auto& en : cache->entries)
                if (en.w == d_w && en.in == d_u_in && en.out == d_u_out && en.steps == n_steps) exec = en.exec;
        const bool fresh = exec == nullptr;
        if (fresh && (rc = capture_steps(P, base, fd, tay, tdd, d_w, d_u_in, d_u_out, n_steps, &exec))) return rc;
        hipError_t e = hipGraphLaunch(exec, s);
        if (fresh) {
            if (cache) {
                if (cache->entries.size() >= GraphCache::kMax) {
                    (void)hipGraphExecDestroy(cache->entries.front().exec);
                    cache->entries.erase(cache->entries.begin());
                }
                cache->entries.push_back({d_w, d_u_in, d_u_out, n_steps, exec});
            } else {
                (void)hipGraphExecDestroy(exec);
            }
        }
        if (e != hipSuccess) return fail(LMEP_ERR_DEVICE, "graph launch: %s", hipGetErrorString(e));
    } else if ((rc = enqueue_steps(P, base, fd, tay, tdd, d_w, d_u_in, d_u_out, n_steps, counters, timer, s))) {
        return rc;
    }
    if ((rc = timer.collect(s))) return rc;
    if (counters) {
        unsigned long long hc[2] = {0, 0};
        HIP_TRY(hipMemcpyAsync(hc, counters, sizeof(hc), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        t_prof_matrices = (int64_t)hc[0];
        t_prof_squarings = (int64_t)hc[1];
    }
    if (flags & LMEP_F_CHECK_FINITE) {
        int* dflag = (int*)(base + P.L.flag);
        HIP_TRY(hipMemsetAsync(dflag, 0, sizeof(int), s));
        for (const DevProb& d : P.atab) HIP_TRY(launch_check_finite(d_u_out + d.state_off, d.N, dflag, s));
        int hflag = 0;
        HIP_TRY(hipMemcpyAsync(&hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (hflag) return fail(LMEP_ERR_NONFINITE, "non-finite value in the result");
    }
    return LMEP_OK;
}

// Checks of one lmep_step call's pointers and flags (the batch is checked by
// make_step_plan).
int check_step_call(double* d_w, const double* d_u_in, double* d_u_out, int32_t n_steps, uint32_t flags,
                    int64_t ext) {
    if (!d_w || !d_u_in || !d_u_out) return fail(LMEP_ERR_ARG, "NULL weight or state pointer");
    if (n_steps < 1) return fail(LMEP_ERR_ARG, "n_steps must be >= 1");
    if (flags & ~(LMEP_F_GRAPH | LMEP_F_PERSISTENT | LMEP_F_CHECK_FINITE | LMEP_F_PROFILE | LMEP_F_COUNT))
        return fail(LMEP_ERR_ARG, "unknown flag bits 0x%x", flags);
    if ((flags & LMEP_F_GRAPH) && (flags & (LMEP_F_PROFILE | LMEP_F_COUNT)))
        return fail(LMEP_ERR_ARG, "LMEP_F_PROFILE / LMEP_F_COUNT cannot be combined with LMEP_F_GRAPH");
    const char *a = (const char*)d_u_in, *b = (const char*)d_u_out;
    const size_t bytes = sizeof(double) * (size_t)ext;
    if (a < b + bytes && b < a + bytes) return fail(LMEP_ERR_ARG, "d_u_in and d_u_out overlap");
    return LMEP_OK;
}

// lmep_step and lmep_step_noalloc.  noalloc: the scratch is this device's
// static array (d_scratch and scratch_bytes are ignored) and the tables go in
// through kernel arguments.
int step_impl(const lmep_problem* prob, int32_t count, double* d_w, const double* d_u_in, double* d_u_out,
              int32_t n_steps, uint32_t flags, void* d_scratch, size_t scratch_bytes, void* hip_stream,
              bool noalloc) {
    StepPlan P;
    int rc = make_step_plan(P, prob, count, (flags & LMEP_F_PERSISTENT) != 0, process_opts());
    if (rc) return rc;
    if ((rc = check_step_call(d_w, d_u_in, d_u_out, n_steps, flags, P.ext))) return rc;
    if (noalloc) {
        if (P.L.total > kStaticScratchBytes)
            return fail(LMEP_ERR_SCRATCH, "this batch needs %zu bytes of scratch; the static array holds %zu",
                        P.L.total, kStaticScratchBytes);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(LMEP_ERR_DEVICE, "earlier device error: %s", hipGetErrorString(e));
        HIP_TRY(static_scratch(&d_scratch));
    } else if ((rc = entry_checks(d_scratch, scratch_bytes, P.L.total))) {
        return rc;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    char* base = (char*)d_scratch;
    if ((rc = upload_pieces(step_pieces(P), base, s, noalloc))) return rc;
    return run_step(P, base, d_w, d_u_in, d_u_out, n_steps, flags, s, nullptr);
}

// ---------------------------------------------------------- adjoint plans --
struct AdjGroup {
    int n = 0, p = 0, first = 0, cnt = 0;
    int64_t nodes = 0, tiles = 0;
    bool taylor = false;
    bool fused = false;  // whole step in one kernel (finite Taylor, tiles of adj_fused_tile(n) nodes)
    bool disp = false;   // some instance has a dispersion term
    int64_t ftiles = 0;
};
struct AdjPlan {
    Opts o;
    int count = 0;
    std::vector<AdjGroup> groups;
    std::vector<DevProb> nftab, ttab;  // node table then fused-tile table; 256-node tile table
    size_t ntab = 0;                   // node-table entries (first part of nftab)
    bool need_taylor = false;
    Layout L;
    int64_t ext = 0;
};

int make_adj_plan(AdjPlan& P, const lmep_problem* prob, int32_t count, const Opts& o) {
    int rc = check_all(prob, count, false);
    if (rc) return rc;
    for (int k = 0; k < count; ++k) {
        const lmep_problem& q = prob[k];
        if (q.scheme == LMEP_ETD2RK || q.scheme == LMEP_ETDRK4 || q.nonlin == LMEP_NL_KDV ||
            q.window != LMEP_WIN_CENTRED || nonuniform(q))
            return fail(LMEP_ERR_UNSUPPORTED,
                        "instance %d: the reverse step covers LINEAR and ETD1 without KdV, centred windows, "
                        "uniform grids", k);
    }
    P.o = o;
    P.count = count;
    // groups by (n, p, method): a node table and a tile table with the same
    // instance order; instances without a reaction term take the finite
    // Taylor series unless LMEP_OPT_EXP_METHOD asks for Pade
    const bool auto_method = o.exp_method == LMEP_EXP_AUTO;
    std::map<std::tuple<int, int, int>, std::vector<int>> by;
    for (int k = 0; k < count; ++k)
        by[{prob[k].n, scheme_p(prob[k].scheme), (auto_method && prob[k].react == 0.0) ? 1 : 0}].push_back(k);
    std::vector<DevProb> ntab, ftab;
    for (auto& kv : by) {
        AdjGroup g;
        g.n = std::get<0>(kv.first);
        g.p = std::get<1>(kv.first);
        g.first = (int)ntab.size();
        g.cnt = (int)kv.second.size();
        g.taylor = std::get<2>(kv.first) == 1;
        g.fused = g.taylor;
        P.need_taylor |= g.taylor;
        for (int k : kv.second) {
            DevProb d = to_dev(prob[k], k);
            d.item_begin = g.nodes;
            ntab.push_back(d);
            d.item_begin = g.tiles;  // tile tables are searched from the group's first tile
            P.ttab.push_back(d);
            d.item_begin = g.ftiles;
            ftab.push_back(d);
            g.nodes += prob[k].N;
            g.disp |= prob[k].delta != 0.0;
            g.tiles += (prob[k].N + kAdjTile - 1) / kAdjTile;
            g.ftiles += (prob[k].N + adj_fused_tile(g.n) - 1) / adj_fused_tile(g.n);
        }
        mark_each(ntab, g.first, g.cnt, g.nodes);
        mark_each(P.ttab, g.first, g.cnt, g.tiles);
        mark_each(ftab, g.first, g.cnt, g.ftiles);
        P.groups.push_back(g);
    }
    P.ntab = ntab.size();
    P.nftab = ntab;
    P.nftab.insert(P.nftab.end(), ftab.begin(), ftab.end());
    P.L = layout(prob, count, 2);
    P.ext = state_extent(prob, count);
    return LMEP_OK;
}

std::vector<Piece> adj_pieces(const AdjPlan& P) {
    return {{P.L.build_tab, P.nftab.size() * sizeof(DevProb), P.nftab.data()},
            {P.L.apply_tab, P.ttab.size() * sizeof(DevProb), P.ttab.data()}};
}

int check_adj_call(const double* d_u_k, const double* d_lambda_next, double* d_lambda_k, double* d_grad,
                   int64_t ext) {
    if (!d_u_k || !d_lambda_next || !d_lambda_k || !d_grad) return fail(LMEP_ERR_ARG, "NULL pointer argument");
    const char *a = (const char*)d_lambda_next, *b = (const char*)d_lambda_k;
    const size_t bytes = sizeof(double) * (size_t)ext;
    if (a < b + bytes && b < a + bytes) return fail(LMEP_ERR_ARG, "d_lambda_next and d_lambda_k overlap");
    return LMEP_OK;
}

int run_adjoint(const AdjPlan& P, char* base, const double* d_u_k, const double* d_lambda_next, double* d_lambda_k,
                double* d_grad, hipStream_t s) {
    const double* fd = nullptr;
    const double* tay = nullptr;
    HIP_TRY(fd_table_init(&fd));
    if (P.need_taylor) HIP_TRY(taylor_table_init(&tay));
    const DevProb* dn = (const DevProb*)(base + P.L.build_tab);
    const DevProb* df = dn + P.ntab;
    const DevProb* dtt = (const DevProb*)(base + P.L.apply_tab);
    // optional profiling: events around each group's per-node kernel and around the whole step
    const bool prof = P.o.profile_adjoint != 0;
    std::vector<hipEvent_t> ev;
    auto make_event = [&](hipEvent_t* e) -> hipError_t {
        hipError_t r = hipEventCreate(e);
        if (r == hipSuccess) ev.push_back(*e);
        return r;
    };
    struct Cleanup {
        std::vector<hipEvent_t>& ev;
        ~Cleanup() {
            for (hipEvent_t e : ev) (void)hipEventDestroy(e);
        }
    } cleanup{ev};
    hipEvent_t all_a = nullptr, all_b = nullptr;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> per(P.groups.size(), {nullptr, nullptr});
    if (prof) {
        HIP_TRY(make_event(&all_a));
        HIP_TRY(make_event(&all_b));
        for (auto& pe : per) {
            HIP_TRY(make_event(&pe.first));
            HIP_TRY(make_event(&pe.second));
        }
        HIP_TRY(hipEventRecord(all_a, s));
    }
    int64_t part_base = 0;
    for (size_t gi = 0; gi < P.groups.size(); ++gi) {
        const AdjGroup& g = P.groups[gi];
        AdjointLaunch a;
        a.n = g.n;
        a.p = g.p;
        a.node_probs = dn + g.first;
        a.tile_probs = dtt + g.first;
        a.nprob = g.cnt;
        a.tiles = g.tiles;
        a.nodes = g.nodes;
        a.fd = fd;
        a.u = d_u_k;
        a.lam = d_lambda_next;
        a.lam_out = d_lambda_k;
        a.grad = d_grad;
        a.g = (double*)(base + P.L.g);
        a.ghat = (double*)(base + P.L.ghat);
        a.ws = (double*)(base + P.L.ws);
        a.ws_stride = P.L.ws_stride;
        a.dparam = (double*)(base + P.L.dparam);
        // per-tile partial sums: the group's own rows of the partial-sum array
        a.part = (double*)(base + P.L.part) + 3 * part_base;
        a.taylor = g.taylor ? tay : nullptr;
        if (g.fused) {
            a.fused_probs = df + g.first;
            a.fused_tiles = g.ftiles;
            a.disp = g.disp;
        }
        if (prof) {
            a.frechet_begin = per[gi].first;
            a.frechet_end = per[gi].second;
        }
        HIP_TRY(launch_adjoint(a, s));
        part_base += g.fused ? g.ftiles : g.tiles;
    }
    if (prof) {
        HIP_TRY(hipEventRecord(all_b, s));
        HIP_TRY(hipStreamSynchronize(s));
        double fms = 0.0;
        std::vector<KernelTime> kt;
        for (size_t gi = 0; gi < P.groups.size(); ++gi) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, per[gi].first, per[gi].second));
            fms += ms;
            char nm[64];
            if (P.groups[gi].fused)
                snprintf(nm, sizeof(nm), "adj_fused_kernel<%d,%d,%s>", P.groups[gi].n, P.groups[gi].p,
                         P.groups[gi].disp ? "true" : "false");
            else
                snprintf(nm, sizeof(nm), "adj_frechet_kernel<%d,%d>", P.groups[gi].n, P.groups[gi].p);
            bool found = false;
            for (auto& k : kt)
                if (k.name == nm) {
                    k.ms += ms;
                    k.launches += 1;
                    found = true;
                }
            if (!found) kt.push_back({nm, (double)ms, 1});
        }
        float all = 0.f;
        HIP_TRY(hipEventElapsedTime(&all, all_a, all_b));
        t_prof_build_ms = fms;
        t_prof_build_n = (int32_t)P.groups.size();
        t_prof_apply_ms = (double)all - fms;
        t_prof_apply_n = 1;
        t_prof_kernels = kt;
    }
    return LMEP_OK;
}

}  // namespace

// A plan: one batch's checked problems, launch groups and option values, its
// device tables uploaded once into the caller's scratch buffer, and the graphs
// captured for it.
struct lmep_plan_s {
    int op = 0;
    char* base = nullptr;
    hipEvent_t ready = nullptr;        // recorded after the table upload
    hipStream_t created_on = nullptr;  // stream of the upload
    std::vector<hipStream_t> waited;   // other streams made to wait for `ready`
    hipEvent_t last = nullptr;         // recorded after each graph launch
    bool launched_graph = false;
    StepPlan step;
    AdjPlan adj;
    GraphCache graphs;
};

namespace {
// Order work on stream s after the plan's table upload.
int plan_order(lmep_plan_s* P, hipStream_t s) {
    if (s == P->created_on) return LMEP_OK;
    for (hipStream_t w : P->waited)
        if (w == s) return LMEP_OK;
    HIP_TRY(hipStreamWaitEvent(s, P->ready, 0));
    P->waited.push_back(s);
    return LMEP_OK;
}
}  // namespace

extern "C" {

int64_t lmep_weight_count(const lmep_problem* prob) {
    if (!prob || check_problem(*prob, 0)) return -1;
    return weight_count(*prob);
}

size_t lmep_scratch_bytes(const lmep_problem* prob, int32_t count, int32_t op) {
    if (op < 0 || op > 2 || check_all(prob, count, false)) return 0;
    return layout(prob, count, op).total;
}

const char* lmep_last_error(void) { return t_err; }

int lmep_set_option(int32_t option, int32_t value) {
    Opts o = process_opts();
    int rc = set_opt(o, option, value);
    if (rc) return rc;
    g_steps_per_launch.store(o.steps_per_launch);
    g_profile_adjoint.store(o.profile_adjoint);
    g_fuse_frozen.store(o.fuse_frozen);
    g_apply_tile.store(o.apply_tile);
    g_exp_method.store(o.exp_method);
    g_taylor_region.store(o.taylor_region);
    g_merge_groups.store(o.merge_groups);
    return LMEP_OK;
}

int32_t lmep_get_option(int32_t option) {
    const Opts o = process_opts();
    switch (option) {
        case LMEP_OPT_STEPS_PER_LAUNCH: return o.steps_per_launch;
        case LMEP_OPT_PROFILE_ADJOINT: return o.profile_adjoint;
        case LMEP_OPT_FUSE_FROZEN: return o.fuse_frozen;
        case LMEP_OPT_APPLY_TILE: return o.apply_tile;
        case LMEP_OPT_EXP_METHOD: return o.exp_method;
        case LMEP_OPT_TAYLOR_REGION: return o.taylor_region;
        case LMEP_OPT_MERGE_GROUPS: return o.merge_groups;
        default: return fail(LMEP_ERR_ARG, "unknown option %d", option);
    }
}

int lmep_profile_last(double* build_ms, int32_t* build_launches, double* apply_ms, int32_t* apply_launches,
                      int64_t* matrices, int64_t* squarings) {
    if (build_ms) *build_ms = t_prof_build_ms;
    if (build_launches) *build_launches = t_prof_build_n;
    if (apply_ms) *apply_ms = t_prof_apply_ms;
    if (apply_launches) *apply_launches = t_prof_apply_n;
    if (matrices) *matrices = t_prof_matrices;
    if (squarings) *squarings = t_prof_squarings;
    return LMEP_OK;
}

int32_t lmep_profile_kernel(int32_t k, char* name, size_t name_len, double* ms, int32_t* launches) {
    const int32_t count = (int32_t)t_prof_kernels.size();
    if (k < 0 || k >= count) return count;
    const KernelTime& kt = t_prof_kernels[k];
    if (name && name_len > 0) snprintf(name, name_len, "%s", kt.name.c_str());
    if (ms) *ms = kt.ms;
    if (launches) *launches = kt.launches;
    return count;
}

int lmep_build_weights(const lmep_problem* prob, int32_t count, const double* d_u, double* d_w, void* d_scratch,
                       size_t scratch_bytes, void* hip_stream) {
    int rc = check_all(prob, count, true);
    if (rc) return rc;
    if (!d_w) return fail(LMEP_ERR_ARG, "d_w is NULL");
    for (int k = 0; k < count; ++k)
        if (frozen(prob[k]) && !d_u) return fail(LMEP_ERR_ARG, "instance %d needs d_u (frozen velocity)", k);
    const Layout L = layout(prob, count, 0);
    if ((rc = entry_checks(d_scratch, scratch_bytes, L.total))) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    const double* fd = nullptr;
    HIP_TRY(fd_table_init(&fd));
    std::vector<DevProb> btab;
    const double* tay = nullptr;
    const Opts o = process_opts();
    auto groups = plan_build(prob, count, [](const lmep_problem&) { return true; }, btab, o);
    char* base = (char*)d_scratch;
    if ((rc = upload_pieces({{L.build_tab, btab.size() * sizeof(DevProb), btab.data()}}, base, s, false))) return rc;
    const DevProb* dtab = (const DevProb*)(base + L.build_tab);
    const double* tdd = nullptr;
    for (auto& g : groups) {
        if (g.taylor && !g.dd && !tay) HIP_TRY(taylor_table_init(&tay));
        if ((g.dd || g.ddtable) && !tdd) HIP_TRY(taylor_dd_table_init(&tdd));
        if (g.wide)
            HIP_TRY(launch_build_wide(g.n, g.p, dtab + g.first, g.count, g.items, d_w, s));
        else if (g.ddtable)
            HIP_TRY(launch_build_table_dd(g.n, g.p, dtab + g.first, g.count, g.items, tdd, d_w, s));
        else if (g.taylor)
            HIP_TRY(launch_build_taylor(g.n, dtab + g.first, g.count, g.items, fd, g.dd ? tdd : tay, d_u, d_w,
                                        nullptr, s, nullptr, g.dd));
        else
            HIP_TRY(launch_build(g.n, g.p, dtab + g.first, g.count, g.items, fd, d_u, d_w, nullptr, s));
    }
    return LMEP_OK;
}

int lmep_step(const lmep_problem* prob, int32_t count, double* d_w, const double* d_u_in, double* d_u_out,
              int32_t n_steps, uint32_t flags, void* d_scratch, size_t scratch_bytes, void* hip_stream) {
    return step_impl(prob, count, d_w, d_u_in, d_u_out, n_steps, flags, d_scratch, scratch_bytes, hip_stream, false);
}

int lmep_step_noalloc(const lmep_problem* prob, int32_t count, double* d_w, const double* d_u_in, double* d_u_out,
                      int32_t n_steps, uint32_t flags, void* hip_stream) {
    if (flags & ~LMEP_F_PERSISTENT)
        return fail(LMEP_ERR_ARG, "lmep_step_noalloc takes LMEP_F_PERSISTENT only, got flags 0x%x", flags);
    return step_impl(prob, count, d_w, d_u_in, d_u_out, n_steps, flags, nullptr, 0, hip_stream, true);
}

int lmep_adjoint_step(const lmep_problem* prob, int32_t count, const double* d_u_k, const double* d_lambda_next,
                      double* d_lambda_k, double* d_grad, void* d_scratch, size_t scratch_bytes, void* hip_stream) {
    AdjPlan P;
    int rc = make_adj_plan(P, prob, count, process_opts());
    if (rc) return rc;
    if ((rc = check_adj_call(d_u_k, d_lambda_next, d_lambda_k, d_grad, P.ext))) return rc;
    if ((rc = entry_checks(d_scratch, scratch_bytes, P.L.total))) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    char* base = (char*)d_scratch;
    if ((rc = upload_pieces(adj_pieces(P), base, s, false))) return rc;
    return run_adjoint(P, base, d_u_k, d_lambda_next, d_lambda_k, d_grad, s);
}

int lmep_plan_create(lmep_plan* plan, const lmep_problem* prob, int32_t count, int32_t op, uint32_t flags,
                     const int32_t* options, int32_t n_options, void* d_scratch, size_t scratch_bytes,
                     void* hip_stream) {
    if (!plan) return fail(LMEP_ERR_ARG, "plan is NULL");
    *plan = nullptr;
    if (op != 1 && op != 2) return fail(LMEP_ERR_ARG, "plans cover op 1 (lmep_step) and 2 (lmep_adjoint_step)");
    if (n_options < 0 || (n_options > 0 && !options)) return fail(LMEP_ERR_ARG, "bad option list");
    Opts o = process_opts();
    for (int k = 0; k < n_options; ++k) {
        int rc = set_opt(o, options[2 * k], options[2 * k + 1]);
        if (rc) return rc;
    }
    if (op == 1 && (flags & ~LMEP_F_PERSISTENT))
        return fail(LMEP_ERR_ARG, "a step plan takes LMEP_F_PERSISTENT or 0 at creation, got 0x%x", flags);
    if (op == 2 && flags) return fail(LMEP_ERR_ARG, "an adjoint plan takes no flags, got 0x%x", flags);
    lmep_plan_s* P = new (std::nothrow) lmep_plan_s;
    if (!P) return fail(LMEP_ERR_ARG, "out of host memory");
    P->op = op;
    int rc = op == 1 ? make_step_plan(P->step, prob, count, (flags & LMEP_F_PERSISTENT) != 0, o)
                     : make_adj_plan(P->adj, prob, count, o);
    const size_t need = op == 1 ? P->step.L.total : P->adj.L.total;
    if (!rc) rc = entry_checks(d_scratch, scratch_bytes, need);
    const double* fd = nullptr;
    hipError_t e = hipSuccess;
    if (!rc && (e = fd_table_init(&fd)) != hipSuccess) rc = fail(LMEP_ERR_DEVICE, "stencil table: %s", hipGetErrorString(e));
    hipStream_t s = (hipStream_t)hip_stream;
    P->base = (char*)d_scratch;
    P->created_on = s;
    if (!rc) rc = upload_pieces(op == 1 ? step_pieces(P->step) : adj_pieces(P->adj), P->base, s, false);
    if (!rc && (e = hipEventCreateWithFlags(&P->ready, hipEventDisableTiming)) != hipSuccess)
        rc = fail(LMEP_ERR_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    if (!rc && (e = hipEventRecord(P->ready, s)) != hipSuccess)
        rc = fail(LMEP_ERR_DEVICE, "hipEventRecord: %s", hipGetErrorString(e));
    if (!rc && (e = hipEventCreateWithFlags(&P->last, hipEventDisableTiming)) != hipSuccess)
        rc = fail(LMEP_ERR_DEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    if (rc) {
        if (P->ready) (void)hipEventDestroy(P->ready);
        if (P->last) (void)hipEventDestroy(P->last);
        delete P;
        return rc;
    }
    *plan = P;
    return LMEP_OK;
}

int lmep_plan_step(lmep_plan plan, double* d_w, const double* d_u_in, double* d_u_out, int32_t n_steps,
                   uint32_t flags, void* hip_stream) {
    if (!plan || plan->op != 1) return fail(LMEP_ERR_ARG, "not a step plan");
    const StepPlan& P = plan->step;
    int rc = check_step_call(d_w, d_u_in, d_u_out, n_steps, flags, P.ext);
    if (rc) return rc;
    if (((flags & LMEP_F_PERSISTENT) != 0) != P.multi)
        return fail(LMEP_ERR_ARG, "LMEP_F_PERSISTENT must be given exactly when the plan was made with it");
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LMEP_ERR_DEVICE, "earlier device error: %s", hipGetErrorString(e));
    hipStream_t s = (hipStream_t)hip_stream;
    if ((rc = plan_order(plan, s))) return rc;
    rc = run_step(P, plan->base, d_w, d_u_in, d_u_out, n_steps, flags, s, &plan->graphs);
    if (!rc && (flags & LMEP_F_GRAPH)) {
        HIP_TRY(hipEventRecord(plan->last, s));
        plan->launched_graph = true;
    }
    return rc;
}

int lmep_plan_adjoint_step(lmep_plan plan, const double* d_u_k, const double* d_lambda_next, double* d_lambda_k,
                           double* d_grad, void* hip_stream) {
    if (!plan || plan->op != 2) return fail(LMEP_ERR_ARG, "not an adjoint plan");
    int rc = check_adj_call(d_u_k, d_lambda_next, d_lambda_k, d_grad, plan->adj.ext);
    if (rc) return rc;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(LMEP_ERR_DEVICE, "earlier device error: %s", hipGetErrorString(e));
    hipStream_t s = (hipStream_t)hip_stream;
    if ((rc = plan_order(plan, s))) return rc;
    return run_adjoint(plan->adj, plan->base, d_u_k, d_lambda_next, d_lambda_k, d_grad, s);
}

int lmep_plan_destroy(lmep_plan plan) {
    if (!plan) return LMEP_OK;
    int rc = LMEP_OK;
    // graph executions still in flight finish before their graphs go
    if (plan->launched_graph && hipEventSynchronize(plan->last) != hipSuccess)
        rc = fail(LMEP_ERR_DEVICE, "waiting for the plan's last graph launch failed");
    plan->graphs.clear();
    if (plan->ready) (void)hipEventDestroy(plan->ready);
    if (plan->last) (void)hipEventDestroy(plan->last);
    delete plan;
    return rc;
}

}  // extern "C"
