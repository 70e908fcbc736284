// C-ABI of liblmep (declared in include/lmep.h): argument checks, grouping of
// instances by kernel variant, scratch layout, upload of the device problem
// tables, and the launch sequence of each entry point.  All arithmetic of the
// method runs in the kernels; this file only plans and enqueues.
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
std::atomic<int> t_steps_per_launch{8};  // LMEP_OPT_STEPS_PER_LAUNCH, process-wide
std::atomic<int> t_profile_adjoint{0};   // LMEP_OPT_PROFILE_ADJOINT, process-wide
std::atomic<int> t_fuse_frozen{1};       // LMEP_OPT_FUSE_FROZEN, process-wide
std::atomic<int> t_apply_tile{0};        // LMEP_OPT_APPLY_TILE, process-wide (0 = by size)
std::atomic<int> t_exp_method{LMEP_EXP_AUTO};  // LMEP_OPT_EXP_METHOD, process-wide

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
bool taylor(const lmep_problem& q) {
    return frozen(q) && !nonuniform(q) && q.react == 0.0 && t_exp_method.load() == LMEP_EXP_AUTO;
}

int64_t weight_count(const lmep_problem& q) {
    const int64_t kinds = scheme_kinds(q.scheme);
    return pernode(q) ? kinds * q.n * q.N : kinds * q.n * q.n;
}

bool finite(double x) { return std::isfinite(x); }

// Checks of one instance (ERR_ARG for malformed input, ERR_UNSUPPORTED for a
// well-formed combination the kernels do not implement).
int check_problem(const lmep_problem& q, int k) {
    const int nmax = nonuniform(q) ? kMaxNWide : kMaxN;
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
    if (q.n + scheme_p(q.scheme) > (nonuniform(q) ? kMaxMWide : kMaxM))
        return fail(LMEP_ERR_UNSUPPORTED, "instance %d: n + p = %d exceeds %d", k, q.n + scheme_p(q.scheme),
                    nonuniform(q) ? kMaxMWide : kMaxM);
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
    bool taylor = false;     // build by finite Taylor series (items = kTaylorTile-node tiles)
    bool pernode = false;    // weights stored per node (frozen velocity or non-uniform grid)
    bool frozen = false;     // rebuilt every step (frozen velocity)
    bool nonuniform = false; // non-uniform grid: wide build, per-node stationary weights
    bool resident = false;   // non-uniform, several steps per launch, one block per instance
    int64_t max_nodes = 0;
    bool stepk = false;  // stationary multi-step kernel (always for ETDRK4)
    int first = 0, count = 0;  // slice of the table
    int64_t items = 0;         // matrices (build) or tiles (apply)
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
                              int frozen_kb = 0) {
    // one build part per exponential: ETDRK4 needs two (p = 3 at dt, p = 1 at dt/2)
    struct Part {
        int k, harvest;
    };
    // (n, p, kind): kind 0 Pade on a uniform grid, 1 non-uniform grid, 2 finite Taylor
    std::map<std::tuple<int, int, int>, std::vector<Part>> by;
    for (int k = 0; k < count; ++k) {
        if (!want(prob[k])) continue;
        const int kind = nonuniform(prob[k]) ? 1 : (taylor(prob[k]) ? 2 : 0);
        if (prob[k].scheme == LMEP_ETDRK4) {
            by[{prob[k].n, 3, kind}].push_back({k, HARVEST_RK4_FULL});
            by[{prob[k].n, 1, kind}].push_back({k, HARVEST_RK4_HALF});
        } else {
            by[{prob[k].n, scheme_p(prob[k].scheme), kind}].push_back({k, HARVEST_PLAIN});
        }
    }
    std::vector<Group> groups;
    for (auto& kv : by) {
        Group g;
        g.n = std::get<0>(kv.first);
        g.p = std::get<1>(kv.first);
        g.nonuniform = std::get<2>(kv.first) == 1;
        g.taylor = std::get<2>(kv.first) == 2;
        if (g.taylor && frozen_kb > 0) {
            // staged positions per block (= threads): about one block per CU for
            // groups too small to fill the GPU -- a step then costs the latency of
            // one block, not of the two or three an uneven spread puts on some
            // CUs -- and the full region for larger ones
            int64_t nodes = 0;
            bool upwind = false;
            for (const Part& part : kv.second) {
                nodes += prob[part.k].N;
                upwind |= prob[part.k].window == LMEP_WIN_UPWIND;
            }
            const int64_t halo = (int64_t)frozen_kb * taylor_stepk_reach(g.n, upwind);
            const int64_t want_tile = std::max<int64_t>((nodes + cu_count() - 1) / cu_count(), 64);
            g.reg = (int)std::min<int64_t>((want_tile + 2 * halo + 63) / 64 * 64, kTaylorRegion);
        }
        g.first = (int)tab.size();
        int64_t items = 0;
        for (const Part& part : kv.second) {
            DevProb d = to_dev(prob[part.k], part.k);
            d.p = g.p;
            d.harvest = part.harvest;
            if (part.harvest == HARVEST_RK4_HALF) d.dt = 0.5 * prob[part.k].dt;
            d.item_begin = items;
            const int64_t tt = frozen_kb > 0 ? taylor_stepk_tile(g.n, frozen_kb, g.reg,
                                                                 prob[part.k].window == LMEP_WIN_UPWIND)
                                             : kTaylorTile;
            items += g.taylor ? (prob[part.k].N + tt - 1) / tt
                              : (pernode(prob[part.k]) ? prob[part.k].N : prob[part.k].n);
            tab.push_back(d);
        }
        g.count = (int)kv.second.size();
        g.items = items;
        groups.push_back(g);
    }
    return groups;
}

// Apply groups: keyed by kernel variant; also fills the block -> table-row map.
// multi_kb > 0: tiles of the multi-step kernel advancing multi_kb steps per launch.
std::vector<Group> plan_apply(const lmep_problem* prob, int32_t count, std::vector<DevProb>& tab,
                              std::vector<int>& tile_inst, int multi_kb = 0) {
    // weight kind: 0 stationary table, 1 frozen velocity, 2 non-uniform grid
    std::map<std::tuple<int, int, int, int>, std::vector<int>> by;
    for (int k = 0; k < count; ++k)
        by[{prob[k].n, prob[k].scheme, prob[k].nonlin, frozen(prob[k]) ? 1 : (nonuniform(prob[k]) ? 2 : 0)}]
            .push_back(k);
    std::vector<Group> groups;
    for (auto& kv : by) {
        Group g;
        std::tie(g.n, g.scheme, g.nonlin, std::ignore) = kv.first;
        g.pernode = std::get<3>(kv.first) != 0;
        g.frozen = std::get<3>(kv.first) == 1;
        g.nonuniform = std::get<3>(kv.first) == 2;
        g.first = (int)tab.size();
        int64_t nodes = 0;
        for (int k : kv.second) nodes += prob[k].N;
        g.stepk = !g.nonuniform && (multi_kb > 0 || g.scheme == LMEP_ETDRK4);
        g.resident = g.nonuniform && multi_kb > 0;
        for (int k : kv.second) g.max_nodes = std::max(g.max_nodes, prob[k].N);
        const int64_t avg = nodes / (int64_t)kv.second.size();
        const int forced = t_apply_tile.load();  // 0, 64 (non-uniform groups only), 256 or 1024
        g.tile = g.stepk ? stepk_tile(g.n, g.scheme, g.nonlin, multi_kb > 0 ? multi_kb : 1)
                 : (forced != 0 && (forced != kApplyTileTiny || g.nonuniform))
                     ? forced
                     : (g.nonuniform && avg <= kApplyTileTiny)
                           ? kApplyTileTiny
                           : ((nodes < kSmallGroupNodes || avg <= kApplyTileSmall) ? kApplyTileSmall : kApplyTile);
        int64_t tiles = 0;
        for (int k : kv.second) {
            DevProb d = to_dev(prob[k], k);
            d.item_begin = tiles;
            const int64_t nt = (prob[k].N + g.tile - 1) / g.tile;
            for (int64_t t = 0; t < nt; ++t) tile_inst.push_back((int)(tab.size() - g.first));
            tiles += nt;
            tab.push_back(d);
        }
        g.count = (int)kv.second.size();
        g.items = tiles;
        groups.push_back(g);
    }
    return groups;
}

// Host staging for the device tables: pinned memory owned by the calling
// thread, reused across calls; an event guards reuse until the previous copy
// has been consumed.
struct Staging {
    void* host = nullptr;
    size_t cap = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
    ~Staging() {
        if (pending && done) hipEventSynchronize(done);
        if (host) hipHostFree(host);
        if (done) hipEventDestroy(done);
    }
};
thread_local Staging t_stage;

// by_args: write the tables through kernel arguments (upload_by_args) instead,
// which needs no pinned host buffer (lmep_step_noalloc).
int upload(const std::vector<DevProb>& a, const std::vector<DevProb>& b, void* d_a, void* d_b, hipStream_t s,
           const std::vector<int>* c = nullptr, void* d_c = nullptr, bool by_args = false) {
    const size_t na = a.size() * sizeof(DevProb), nb = b.size() * sizeof(DevProb);
    const size_t nc = c ? c->size() * sizeof(int) : 0;
    if (by_args) {
        if (na) HIP_TRY(upload_by_args(d_a, a.data(), na, s));
        if (nb) HIP_TRY(upload_by_args(d_b, b.data(), nb, s));
        if (nc) HIP_TRY(upload_by_args(d_c, c->data(), nc, s));
        return LMEP_OK;
    }
    Staging& st = t_stage;
    if (!st.done) HIP_TRY(hipEventCreateWithFlags(&st.done, hipEventDisableTiming));
    if (st.pending) {
        HIP_TRY(hipEventSynchronize(st.done));
        st.pending = false;
    }
    if (st.cap < na + nb + nc) {
        if (st.host) HIP_TRY(hipHostFree(st.host));
        st.host = nullptr;
        st.cap = 0;
        const size_t cap = std::max<size_t>(na + nb + nc, 1 << 16);
        HIP_TRY(hipHostMalloc(&st.host, cap, hipHostMallocDefault));
        st.cap = cap;
    }
    char* h = (char*)st.host;
    if (na) std::memcpy(h, a.data(), na);
    if (nb) std::memcpy(h + na, b.data(), nb);
    if (nc) std::memcpy(h + na + nb, c->data(), nc);
    if (na) HIP_TRY(hipMemcpyAsync(d_a, h, na, hipMemcpyHostToDevice, s));
    if (nb) HIP_TRY(hipMemcpyAsync(d_b, h + na, nb, hipMemcpyHostToDevice, s));
    if (nc) HIP_TRY(hipMemcpyAsync(d_c, h + na + nb, nc, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(st.done, s));
    st.pending = true;
    return LMEP_OK;
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

// HIP events bracketing every build and apply launch (LMEP_F_PROFILE).  All
// events are created before the first launch so that recording them costs
// the host little and the host stays ahead of the device.
struct Timer {
    bool on = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> build, apply;
    size_t nb = 0, na = 0;
    ~Timer() {
        for (auto& v : {&build, &apply})
            for (auto& ev : *v) {
                if (ev.first) hipEventDestroy(ev.first);
                if (ev.second) hipEventDestroy(ev.second);
            }
    }
    hipError_t reserve(size_t builds, size_t applies) {
        if (!on) return hipSuccess;
        build.assign(builds, {nullptr, nullptr});
        apply.assign(applies, {nullptr, nullptr});
        hipError_t e;
        for (auto& v : {&build, &apply})
            for (auto& ev : *v) {
                if ((e = hipEventCreate(&ev.first)) != hipSuccess) return e;
                if ((e = hipEventCreate(&ev.second)) != hipSuccess) return e;
            }
        return hipSuccess;
    }
    hipError_t mark(bool is_build, hipStream_t s, bool begin) {
        if (!on) return hipSuccess;
        auto& v = is_build ? build : apply;
        size_t& k = is_build ? nb : na;
        if (k >= v.size()) return hipErrorInvalidValue;
        if (begin) return hipEventRecord(v[k].first, s);
        return hipEventRecord(v[k++].second, s);
    }
};

// Stream on which step loops are captured into a graph (the legacy default
// stream cannot be captured); the graph itself is launched on the caller's
// stream.  One per thread, default priority.
struct CaptureStream {
    hipStream_t s = nullptr;
    ~CaptureStream() {
        if (s) hipStreamDestroy(s);
    }
};
thread_local CaptureStream t_capture;

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
    if (option == LMEP_OPT_STEPS_PER_LAUNCH) {
        if (value != 1 && value != 2 && value != 4 && value != 8)
            return fail(LMEP_ERR_ARG, "steps per launch must be 1, 2, 4 or 8, got %d", value);
        t_steps_per_launch.store(value);
        return LMEP_OK;
    }
    if (option == LMEP_OPT_PROFILE_ADJOINT || option == LMEP_OPT_FUSE_FROZEN) {
        if (value != 0 && value != 1) return fail(LMEP_ERR_ARG, "option %d takes 0 or 1, got %d", option, value);
        (option == LMEP_OPT_PROFILE_ADJOINT ? t_profile_adjoint : t_fuse_frozen).store(value);
        return LMEP_OK;
    }
    if (option == LMEP_OPT_EXP_METHOD) {
        if (value != LMEP_EXP_AUTO && value != LMEP_EXP_PADE)
            return fail(LMEP_ERR_ARG, "exponential method must be LMEP_EXP_AUTO (0) or LMEP_EXP_PADE (1), got %d",
                        value);
        t_exp_method.store(value);
        return LMEP_OK;
    }
    if (option == LMEP_OPT_APPLY_TILE) {
        if (value != 0 && value != 64 && value != kApplyTileSmall && value != kApplyTile)
            return fail(LMEP_ERR_ARG, "apply tile must be 0, 64, %d or %d, got %d", kApplyTileSmall, kApplyTile, value);
        t_apply_tile.store(value);
        return LMEP_OK;
    }
    return fail(LMEP_ERR_ARG, "unknown option %d", option);
}

int32_t lmep_get_option(int32_t option) {
    if (option == LMEP_OPT_STEPS_PER_LAUNCH) return t_steps_per_launch.load();
    if (option == LMEP_OPT_PROFILE_ADJOINT) return t_profile_adjoint.load();
    if (option == LMEP_OPT_FUSE_FROZEN) return t_fuse_frozen.load();
    if (option == LMEP_OPT_APPLY_TILE) return t_apply_tile.load();
    if (option == LMEP_OPT_EXP_METHOD) return t_exp_method.load();
    return fail(LMEP_ERR_ARG, "unknown option %d", option);
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
    std::vector<DevProb> btab, none;
    const double* tay = nullptr;
    auto groups = plan_build(prob, count, [](const lmep_problem&) { return true; }, btab);
    char* base = (char*)d_scratch;
    if ((rc = upload(btab, none, base + L.build_tab, nullptr, s))) return rc;
    const DevProb* dtab = (const DevProb*)(base + L.build_tab);
    for (auto& g : groups) {
        if (g.taylor && !tay) HIP_TRY(taylor_table_init(&tay));
        if (g.nonuniform)
            HIP_TRY(launch_build_wide(g.n, g.p, dtab + g.first, g.count, g.items, d_w, s));
        else if (g.taylor)
            HIP_TRY(launch_build_taylor(g.n, dtab + g.first, g.count, g.items, fd, tay, d_u, d_w, nullptr, s));
        else
            HIP_TRY(launch_build(g.n, g.p, dtab + g.first, g.count, g.items, fd, d_u, d_w, nullptr, s));
    }
    return LMEP_OK;
}

}  // extern "C"

namespace {

// lmep_step and lmep_step_noalloc.  noalloc: the scratch is this device's
// static array (d_scratch and scratch_bytes are ignored) and the tables go in
// through kernel arguments.
int step_impl(const lmep_problem* prob, int32_t count, double* d_w, const double* d_u_in, double* d_u_out,
              int32_t n_steps, uint32_t flags, void* d_scratch, size_t scratch_bytes, void* hip_stream,
              bool noalloc) {
    int rc = check_all(prob, count, true);
    if (rc) return rc;
    if (!d_w || !d_u_in || !d_u_out) return fail(LMEP_ERR_ARG, "NULL weight or state pointer");
    if (n_steps < 1) return fail(LMEP_ERR_ARG, "n_steps must be >= 1");
    if (flags & ~(LMEP_F_GRAPH | LMEP_F_PERSISTENT | LMEP_F_CHECK_FINITE | LMEP_F_PROFILE | LMEP_F_COUNT))
        return fail(LMEP_ERR_ARG, "unknown flag bits 0x%x", flags);
    const bool multi = (flags & LMEP_F_PERSISTENT) != 0;
    if (multi)
        for (int k = 0; k < count; ++k) {
            if (frozen(prob[k]) && (!taylor(prob[k]) || prob[k].bc == LMEP_BC_NEUMANN))
                return fail(LMEP_ERR_UNSUPPORTED, "LMEP_F_PERSISTENT with BURGERS_FROZEN (instance %d) needs the "
                            "finite-Taylor build (react = 0, LMEP_EXP_AUTO) on a Dirichlet or periodic grid", k);
            if (prob[k].window != LMEP_WIN_CENTRED && !frozen(prob[k]))
                return fail(LMEP_ERR_UNSUPPORTED, "LMEP_F_PERSISTENT with stationary weights needs centred windows "
                            "(instance %d)", k);
            if (nonuniform(prob[k]) && prob[k].N > kResidentMaxN)
                return fail(LMEP_ERR_UNSUPPORTED, "LMEP_F_PERSISTENT on a non-uniform grid needs N <= %d "
                            "(instance %d)", kResidentMaxN, k);
        }
    if ((flags & LMEP_F_GRAPH) && (flags & (LMEP_F_PROFILE | LMEP_F_COUNT)))
        return fail(LMEP_ERR_ARG, "LMEP_F_PROFILE / LMEP_F_COUNT cannot be combined with LMEP_F_GRAPH");
    const int64_t ext = state_extent(prob, count);
    {
        const char *a = (const char*)d_u_in, *b = (const char*)d_u_out;
        const size_t bytes = sizeof(double) * (size_t)ext;
        if (a < b + bytes && b < a + bytes) return fail(LMEP_ERR_ARG, "d_u_in and d_u_out overlap");
    }
    const Layout L = layout(prob, count, 1);
    if (noalloc) {
        if (L.total > kStaticScratchBytes)
            return fail(LMEP_ERR_SCRATCH, "this batch needs %zu bytes of scratch; the static array holds %zu",
                        L.total, kStaticScratchBytes);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(LMEP_ERR_DEVICE, "earlier device error: %s", hipGetErrorString(e));
        HIP_TRY(static_scratch(&d_scratch));
    } else if ((rc = entry_checks(d_scratch, scratch_bytes, L.total))) {
        return rc;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    const double* fd = nullptr;
    HIP_TRY(fd_table_init(&fd));

    std::vector<DevProb> btab, atab;
    std::vector<int> tile_inst;
    const int kb = multi ? t_steps_per_launch.load() : 1;
    auto bgroups = plan_build(prob, count, [](const lmep_problem& q) { return frozen(q); }, btab, multi ? kb : 0);
    const double* tay = nullptr;
    for (auto& gr : bgroups)
        if (gr.taylor && !tay) HIP_TRY(taylor_table_init(&tay));
    auto agroups = plan_apply(prob, count, atab, tile_inst, multi ? kb : 0);
    // resident groups (small non-uniform instances) advance all n_steps from
    // d_u_in to d_u_out in the first iteration; when nothing else is in the
    // batch that iteration is all there is
    bool all_resident = bgroups.empty();
    for (auto& gr : agroups) all_resident &= gr.resident;
    const int launches = all_resident ? 1 : (n_steps + kb - 1) / kb;  // apply launches per group
    char* base = (char*)d_scratch;
    if ((rc = upload(btab, atab, base + L.build_tab, base + L.apply_tab, s, &tile_inst, base + L.tile_inst,
                     noalloc)))
        return rc;
    const DevProb* dbt = (const DevProb*)(base + L.build_tab);
    const DevProb* dat = (const DevProb*)(base + L.apply_tab);
    const int* dti = (const int*)(base + L.tile_inst);
    double* bufA = (double*)(base + L.state);

    Timer timer;
    timer.on = (flags & LMEP_F_PROFILE) != 0;
    HIP_TRY(timer.reserve(bgroups.empty() ? 0 : (size_t)launches, (size_t)launches));
    unsigned long long* counters = (flags & LMEP_F_COUNT) ? (unsigned long long*)(base + L.flag + 64) : nullptr;
    if (counters) HIP_TRY(hipMemsetAsync(counters, 0, 2 * sizeof(unsigned long long), s));
    const bool graph = (flags & LMEP_F_GRAPH) != 0;
    hipGraph_t g = nullptr;
    hipGraphExec_t ge = nullptr;
    hipStream_t launch_stream = s;
    if (graph) {
        if (!t_capture.s) HIP_TRY(hipStreamCreateWithFlags(&t_capture.s, hipStreamNonBlocking));
        s = t_capture.s;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    }

    // frozen-velocity groups under LMEP_F_PERSISTENT always take the fused multi-step kernel
    const bool fuse = t_fuse_frozen.load() != 0 || multi;
    bool apply_launched = false;  // any apply kernel besides the fused ones
    for (auto& gr : agroups) apply_launched |= !(gr.frozen && fuse);
    auto enqueue = [&]() -> int {
        // destinations alternate between the scratch state and d_u_out so that
        // the last step lands in d_u_out and no step works in place
        for (int st = 0; st < launches; ++st) {
            const double* src = (st == 0) ? d_u_in : (((launches - st) % 2 == 0) ? d_u_out : bufA);
            double* dst = ((launches - 1 - st) % 2 == 0) ? d_u_out : bufA;
            if (!bgroups.empty()) {
                // frozen-velocity groups: weights rebuilt, and with fusion applied
                // in the same kernel (their apply groups are then skipped)
                HIP_TRY(timer.mark(true, s, true));
                for (auto& gr : bgroups) {
                    if (gr.taylor && multi)
                        HIP_TRY(launch_taylor_stepk(gr.n, kb, std::min(kb, n_steps - st * kb), gr.reg, dbt + gr.first,
                                                    gr.count, gr.items, fd, tay, src, dst, counters, s));
                    else if (gr.taylor)
                        HIP_TRY(launch_build_taylor(gr.n, dbt + gr.first, gr.count, gr.items, fd, tay, src, d_w,
                                                    counters, s, fuse ? dst : nullptr));
                    else
                        HIP_TRY(launch_build(gr.n, gr.p, dbt + gr.first, gr.count, gr.items, fd, src, d_w, counters,
                                             s, fuse ? dst : nullptr));
                }
                HIP_TRY(timer.mark(true, s, false));
            }
            if (apply_launched) HIP_TRY(timer.mark(false, s, true));
            int64_t tile0 = 0;
            for (auto& gr : agroups) {
                const bool fused = gr.frozen && fuse;  // already advanced by its build kernel
                if (!fused && gr.stepk)
                    HIP_TRY(launch_stepk(gr.n, gr.scheme, gr.nonlin, kb, std::min(kb, n_steps - st * kb),
                                         dat + gr.first, dti + tile0, gr.items, fd, d_w, src, dst, s));
                else if (gr.resident) {
                    // in place after the first chunk: a block reads its whole
                    // instance before it writes any of it
                    for (int done = 0; st == 0 && done < n_steps; done += kResidentMaxSteps)
                        HIP_TRY(launch_resident(gr.n, gr.scheme, gr.nonlin, dat + gr.first, gr.count, gr.max_nodes,
                                                d_w, done == 0 ? d_u_in : d_u_out, d_u_out,
                                                std::min(kResidentMaxSteps, n_steps - done), s));
                }
                else if (gr.nonuniform)
                    HIP_TRY(launch_apply_nonuniform(gr.n, gr.tile, gr.scheme, gr.nonlin, dat + gr.first, dti + tile0,
                                                    gr.items, fd, d_w, src, dst, s));
                else if (!fused)
                    HIP_TRY(launch_apply(gr.n, gr.tile, gr.scheme, gr.nonlin, gr.pernode, dat + gr.first,
                                         dti + tile0, gr.items, fd, d_w, src, dst, s));
                tile0 += gr.items;
            }
            if (apply_launched) HIP_TRY(timer.mark(false, s, false));
        }
        return LMEP_OK;
    };
    rc = enqueue();
    if (graph) {
        hipError_t e = hipStreamEndCapture(s, &g);
        if (rc) {
            if (g) hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(LMEP_ERR_DEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
        s = launch_stream;
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (e == hipSuccess) e = hipGraphLaunch(ge, s);
        if (ge) hipGraphExecDestroy(ge);
        hipGraphDestroy(g);
        if (e != hipSuccess) return fail(LMEP_ERR_DEVICE, "graph launch: %s", hipGetErrorString(e));
    } else if (rc) {
        return rc;
    }

    if (timer.on) {
        HIP_TRY(hipStreamSynchronize(s));
        double bms = 0.0, ams = 0.0;
        for (size_t k = 0; k < timer.nb; ++k) {
            const auto& ev = timer.build[k];
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev.first, ev.second));
            bms += ms;
        }
        for (size_t k = 0; k < timer.na; ++k) {
            const auto& ev = timer.apply[k];
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, ev.first, ev.second));
            ams += ms;
        }
        t_prof_build_ms = bms;
        t_prof_apply_ms = ams;
        t_prof_build_n = (int32_t)timer.nb;
        t_prof_apply_n = (int32_t)timer.na;
    }
    if (counters) {
        unsigned long long hc[2] = {0, 0};
        HIP_TRY(hipMemcpyAsync(hc, counters, sizeof(hc), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        t_prof_matrices = (int64_t)hc[0];
        t_prof_squarings = (int64_t)hc[1];
    }

    if (flags & LMEP_F_CHECK_FINITE) {
        int* dflag = (int*)(base + L.flag);
        HIP_TRY(hipMemsetAsync(dflag, 0, sizeof(int), s));
        for (int k = 0; k < count; ++k)
            HIP_TRY(launch_check_finite(d_u_out + prob[k].state_off, prob[k].N, dflag, s));
        int hflag = 0;
        HIP_TRY(hipMemcpyAsync(&hflag, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (hflag) return fail(LMEP_ERR_NONFINITE, "non-finite value in the result");
    }
    return LMEP_OK;
}

}  // namespace

extern "C" {

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
    if (!d_u_k || !d_lambda_next || !d_lambda_k || !d_grad) return fail(LMEP_ERR_ARG, "NULL pointer argument");
    const int64_t ext = state_extent(prob, count);
    {
        const char *a = (const char*)d_lambda_next, *b = (const char*)d_lambda_k;
        const size_t bytes = sizeof(double) * (size_t)ext;
        if (a < b + bytes && b < a + bytes) return fail(LMEP_ERR_ARG, "d_lambda_next and d_lambda_k overlap");
    }
    const Layout L = layout(prob, count, 2);
    if ((rc = entry_checks(d_scratch, scratch_bytes, L.total))) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    const double* fd = nullptr;
    HIP_TRY(fd_table_init(&fd));

    // groups by (n, p, method): a node table and a tile table with the same
    // instance order; instances without a reaction term take the finite
    // Taylor series unless LMEP_OPT_EXP_METHOD asks for Pade
    const bool auto_method = t_exp_method.load() == LMEP_EXP_AUTO;
    std::map<std::tuple<int, int, int>, std::vector<int>> by;
    for (int k = 0; k < count; ++k)
        by[{prob[k].n, scheme_p(prob[k].scheme), (auto_method && prob[k].react == 0.0) ? 1 : 0}].push_back(k);
    std::vector<DevProb> ntab, ttab, ftab;
    struct G {
        int n, p, first, cnt;
        int64_t nodes, tiles;
        bool taylor;
        bool fused = false;  // whole step in one kernel (finite Taylor, tiles of adj_fused_tile(n) nodes)
        int64_t ftiles = 0;
    };
    std::vector<G> groups;
    const double* tay = nullptr;
    int64_t tile_base = 0;
    for (auto& kv : by) {
        G g{std::get<0>(kv.first), std::get<1>(kv.first), (int)ntab.size(), (int)kv.second.size(), 0, 0,
            std::get<2>(kv.first) == 1};
        if (g.taylor && !tay) HIP_TRY(taylor_table_init(&tay));
        g.fused = g.taylor;
        for (int k : kv.second) {
            DevProb d = to_dev(prob[k], k);
            d.item_begin = g.nodes;
            ntab.push_back(d);
            d.item_begin = tile_base + g.tiles;  // global tile index: rows of the partial-sum array
            ttab.push_back(d);
            d.item_begin = g.ftiles;
            ftab.push_back(d);
            g.nodes += prob[k].N;
            g.tiles += (prob[k].N + kAdjTile - 1) / kAdjTile;
            g.ftiles += (prob[k].N + adj_fused_tile(g.n) - 1) / adj_fused_tile(g.n);
        }
        // tile tables are searched from the group's first tile
        for (int q = g.first; q < g.first + g.cnt; ++q) ttab[q].item_begin -= tile_base;
        groups.push_back(g);
        tile_base += g.tiles;
    }
    char* base = (char*)d_scratch;
    // the build-table region holds two tables per instance: node table, then fused-tile table
    std::vector<DevProb> nftab(ntab);
    nftab.insert(nftab.end(), ftab.begin(), ftab.end());
    if ((rc = upload(nftab, ttab, base + L.build_tab, base + L.apply_tab, s))) return rc;
    const DevProb* dn = (const DevProb*)(base + L.build_tab);
    const DevProb* df = dn + ntab.size();
    const DevProb* dtt = (const DevProb*)(base + L.apply_tab);
    // optional profiling: events around each group's Frechet kernel and around the whole step
    Timer timer;
    timer.on = t_profile_adjoint.load() != 0;
    HIP_TRY(timer.reserve(groups.size(), 1));
    HIP_TRY(timer.mark(false, s, true));
    int64_t part_base = 0;
    for (auto& g : groups) {
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
        a.g = (double*)(base + L.g);
        a.ghat = (double*)(base + L.ghat);
        a.ws = (double*)(base + L.ws);
        a.ws_stride = L.ws_stride;
        a.dparam = (double*)(base + L.dparam);
        a.part = (double*)(base + L.part) + 3 * part_base;
        a.taylor = g.taylor ? tay : nullptr;
        if (g.fused) {
            a.fused_probs = df + g.first;
            a.fused_tiles = g.ftiles;
        }
        if (timer.on) {
            a.frechet_begin = timer.build[timer.nb].first;
            a.frechet_end = timer.build[timer.nb].second;
            ++timer.nb;
        }
        HIP_TRY(launch_adjoint(a, s));
        part_base += g.fused ? g.ftiles : g.tiles;
    }
    HIP_TRY(timer.mark(false, s, false));
    if (timer.on) {
        HIP_TRY(hipStreamSynchronize(s));
        double fms = 0.0;
        for (size_t k = 0; k < timer.nb; ++k) {
            float ms = 0.f;
            HIP_TRY(hipEventElapsedTime(&ms, timer.build[k].first, timer.build[k].second));
            fms += ms;
        }
        float all = 0.f;
        HIP_TRY(hipEventElapsedTime(&all, timer.apply[0].first, timer.apply[0].second));
        t_prof_build_ms = fms;
        t_prof_build_n = (int32_t)timer.nb;
        t_prof_apply_ms = (double)all - fms;
        t_prof_apply_n = 1;
    }
    return LMEP_OK;
}

}  // extern "C"
