// Banded apply for stationary weights, up to KB time steps per launch.
//
// The update is the one of apply.hip (LINEAR, ETD1 or ETD2RK with no,
// Allen-Cahn or KdV nonlinearity; Sec. 3.1 step 3 and Sec. 4), organised so
// that several steps cost one pass over HBM:
//  * a block stages kStepRegion consecutive positions of its instance, runs its
//    steps in LDS and writes back the middle TILE of them.  Each stencil
//    application spoils R = (n-1)/2 values at each open end of the region, so
//    the halo on each side is KB * (applications per step) * R.  Halo values
//    are recomputed, never exchanged, so no block waits for another, and
//    global traffic is 16 bytes per node per launch;
//  * a thread owns V consecutive positions and reads the window of V + n - 1
//    values it needs from LDS once per array (register blocking).  One padding
//    slot after every 8 doubles spreads a 16-lane group's windows over all
//    banks and, because V = 8, makes every window read a constant offset from
//    the thread's base;
//  * the pointwise Allen-Cahn term is formed on the fly from the state window;
//    KdV's derivative term gets a pass of its own;
//  * the interior row's weights live in registers; blocks that reach a
//    Dirichlet end redo the nodes next to it with their own clamped row in a
//    short extra pass, and blocks that reach a Neumann end give halo
//    positions their mirror node's value;
//  * on Dirichlet and Neumann grids the last block of an instance is moved
//    back to end at node N - 1 (it rewrites part of its neighbour's tile with
//    the same values): the clamped windows next to an end reach n - 1 nodes
//    inwards, and a tile starting there would not hold what they depend on.
// One-sided (upwind) windows of a stationary operator are the same kernel
// with the interior window ending (SIDE 1, c > 0) or starting (SIDE 2, c < 0)
// at the node: every application then spoils n - 1 positions on the upstream
// side only, so the whole halo sits upstream of the tile, and the Dirichlet
// pass covers the n - 1 clamped nodes at the upstream end and the held
// downstream end.
// Every value is formed by the same expression, in the same order, as in the
// one-step apply kernel, so the two give bitwise identical states.
#pragma once
#include "lmep_device.hpp"

namespace lmep {
namespace {

constexpr int NT = 256;
constexpr int V = 8;               // positions per thread and pass
constexpr int LR = kStepRegion;    // staged positions per block
static_assert(LR == NT * V, "one pass per thread covers the region");
constexpr int MARGIN = 16;         // unused slots before and after the region (>= R)
constexpr int LP = (LR + 2 * MARGIN) + (LR + 2 * MARGIN) / 8;  // padded length of one array

// LDS slot of region position q, -MARGIN <= q < LR + MARGIN.
__device__ __forceinline__ int phys(int q) { return (q + MARGIN) + ((q + MARGIN) >> 3); }
// Slot of position p0 - MARGIN + c for p0 a multiple of 8 and c >= 0: a
// constant offset from phys(p0 - MARGIN).
__host__ __device__ constexpr int rel(int c) { return c + (c >> 3); }
__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Node whose value sits at unwrapped position j.  Neumann ends reflect evenly
// about 0 and N-1; repeated reflection is periodic with period 2(N-1), which
// only grids narrower than the halo need.
__device__ __forceinline__ int64_t node_of(int64_t j, int64_t N, int bc) {
    if (bc == BC_NEUMANN) {
        if (j >= 0 && j <= N - 1) return j;
        const int64_t P2 = 2 * (N - 1);
        if (j < 0 && j >= -(N - 1)) return -j;
        if (j > N - 1 && j <= P2) return P2 - j;
        int64_t m = j % P2;
        if (m < 0) m += P2;
        return m > N - 1 ? P2 - m : m;
    }
    return map_index(j, N, bc);
}

template <int NL>
__device__ __forceinline__ double pointwise_N(double x, double g) {
    if constexpr (NL == kNlAcUnit) return x - x * x * x;  // g = 1: the same value
    else return g * (x - x * x * x);
}

// Interior window of a SIDE: offset O (stencil i + O .. i + O + n - 1), row
// RI = -O, and the nodes the Dirichlet pass redoes (EC of them).
template <int NN, int SIDE>
struct Win {
    static constexpr int O = SIDE == 0 ? -((NN - 1) / 2) : (SIDE == 1 ? -(NN - 1) : 0);
    static constexpr int RI = -O;
    static constexpr int EC = SIDE == 0 ? NN - 1 : NN;
    static_assert(-O <= MARGIN && NN - 1 + O <= MARGIN, "window reads must stay inside the margins");
};

template <int NN, int SCH, int NL, int KB>
struct Shape {
    static constexpr int R = (NN - 1) / 2;
    static constexpr int PP = (SCH == SCH_ETD2RK) ? 2 : (SCH == SCH_ETD1 ? 1 : 0);
    static constexpr bool HAS_N = (PP > 0) && (NL != NL_NONE);
    static constexpr bool DERIV = HAS_N && (NL == NL_KDV);  // N is itself a stencil
    static constexpr bool RK2N = (SCH == SCH_ETD2RK) && HAS_N;
    static constexpr int HALO = stepk_halo(NN, SCH, NL, KB);
    static constexpr int TILE = stepk_tile(NN, SCH, NL, KB);
    // arrays: state, first stage (the next state without RK2N), then
    //   KdV:              N(u) (+ N(a) with ETD2RK; its second stage reads no u
    //                     and writes the next state over the old one),
    //   pointwise ETD2RK: the next state (its second stage reads u for N(u)).
    static constexpr int NBUF = 2 + (DERIV ? (RK2N ? 2 : 1) : (RK2N ? 1 : 0));
    static_assert(R <= MARGIN, "window reads must stay inside the margins");
    static_assert(TILE > 0 && HALO % 1 == 0, "tile");
};

// The kernel body.  lds: S::NBUF * LP doubles; sw: (PP + 1) n^2; sD1: n^2 when
// the nonlinearity differentiates (the caller's shared arrays).
template <int NN, int SCH, int NL, int KB, int SIDE>
__device__ __forceinline__ void stepk_body(const DevProb& P, const double* __restrict__ fd,
                                           const double* __restrict__ w, const double* __restrict__ u_in,
                                           double* __restrict__ u_out, int ksteps, double* lds, double* sw,
                                           double* sD1) {
    using S = Shape<NN, SCH, NL, KB>;
    using Wn = Win<NN, SIDE>;
    constexpr int R = S::R, PP = S::PP, W = V + NN - 1;
    constexpr int O = Wn::O, RI = Wn::RI;
    // halo before the tile: (applications) x (reach of a window to the left)
    constexpr int LHALO = KB * stepk_apps(SCH, NL) * RI;
    const int tid = threadIdx.x;
    const int64_t N = P.N;
    const int bc = P.bc;
    const int64_t tb = ((int64_t)blockIdx.x - P.item_begin) * S::TILE;  // the block's own tile
    const int64_t t0 = (bc != BC_PERIODIC && N >= S::TILE && tb > N - S::TILE) ? N - S::TILE : tb;
    const int64_t base = t0 - LHALO;  // unwrapped position of region index 0
    const double g = P.nl_coef;
    // does the region reach an end of the grid?  (block-uniform)
    const bool at_end = base < NN || base + LR > N - NN;
    const bool dir = (bc == BC_DIRICHLET) && at_end;
    const bool neu = (bc == BC_NEUMANN) && at_end;

    for (int q = tid; q < (PP + 1) * NN * NN; q += NT) sw[q] = w[P.weight_off + q];
    if constexpr (S::DERIV) {
        const double ih = 1.0 / P.h;
        for (int q = tid; q < NN * NN; q += NT) sD1[q] = fd[fd_index(NN, 0, q / NN, q % NN)] * ih;
    }
    {
        const double* __restrict__ u = u_in + P.state_off;
        double v[V];
#pragma unroll
        for (int t = 0; t < V; ++t) {
            int64_t j = node_of(base + tid + t * NT, N, bc);
            j = j < 0 ? 0 : (j > N - 1 ? N - 1 : j);
            v[t] = u[j];
        }
#pragma unroll
        for (int t = 0; t < V; ++t) lds[phys(tid + t * NT)] = v[t];
    }
    __syncthreads();

    // interior-row weights of each kind, read from global memory at a
    // block-uniform address, so they live in scalar registers and leave the
    // vector registers to the windows
    double Wc[PP + 1][NN];
#pragma unroll
    for (int kd = 0; kd <= PP; ++kd)
#pragma unroll
        for (int k = 0; k < NN; ++k) Wc[kd][k] = w[P.weight_off + (kd * NN + RI) * NN + k];
    double D1c[S::DERIV ? NN : 1];
    if constexpr (S::DERIV) {
#pragma unroll
        for (int k = 0; k < NN; ++k) D1c[k] = sD1[RI * NN + k];
    }

    const int p0 = tid * V;                   // this thread's first position
    const int wb = phys(p0 - MARGIN);         // slot base of its windows
    const int ob = wb + rel(MARGIN);          // slot base of its own positions
    // window value j (position p0 + O + j) of array a
    auto wread = [&](const double* __restrict__ a, int j) { return a[wb + rel(MARGIN + O + j)]; };
    auto own = [&](const double* __restrict__ a, int v) { return a[ob + rel(v) - rel(0)]; };
    // one-sided rows: slot of the first node of the window of node i
    auto edge_win = [&](int64_t i, int64_t off) { return clampi((int)(i + off - base), -MARGIN, LR + MARGIN - NN); };

    // KdV: N = -(g/2) D1 (u u) over the region
    auto deriv_N = [&](const double* __restrict__ src, double* __restrict__ dst) {
        double x[W];
#pragma unroll
        for (int j = 0; j < W; ++j) x[j] = wread(src, j);
        double o[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < NN; ++k) acc += D1c[k] * x[v + k] * x[v + k];
            o[v] = -0.5 * g * acc;
        }
#pragma unroll
        for (int v = 0; v < V; ++v) dst[ob + rel(v) - rel(0)] = o[v];
    };

    // N at window entry j of the state array su (pointwise) or from sn (KdV)
    auto n_at = [&](const double* __restrict__ su, const double* __restrict__ sn, double xu, int slot) -> double {
        if constexpr (S::DERIV) return sn[slot];
        else return pointwise_N<NL>(xu, g);
    };

    // N(a) - N(u) at a slot; KdV reads both from their arrays and never u itself
    auto n_diff = [&](const double* __restrict__ su, const double* __restrict__ snu, const double* __restrict__ sa,
                      const double* __restrict__ sna, int slot) -> double {
        if constexpr (S::DERIV) return sna[slot] - snu[slot];
        else return pointwise_N<NL>(sa[slot], g) - pointwise_N<NL>(su[slot], g);
    };

    // First stage (the whole step for LINEAR / ETD1): dst = W0 . u (+ W1 . N),
    // the two sums interleaved term by term.
    auto stage_a = [&](const double* __restrict__ su, const double* __restrict__ sn, double* __restrict__ dst) {
        double xu[W];
        double xn[S::HAS_N ? W : 1];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            xu[j] = wread(su, j);
            if constexpr (S::HAS_N) xn[j] = n_at(su, sn, xu[j], wb + rel(MARGIN + O + j));
        }
        double o[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < NN; ++k) {
                acc += Wc[0][k] * xu[v + k];
                if constexpr (S::HAS_N) acc += Wc[1][k] * xn[v + k];
            }
            o[v] = acc;
        }
#pragma unroll
        for (int v = 0; v < V; ++v) dst[ob + rel(v) - rel(0)] = o[v];
    };

    // Second ETD2RK stage: dst = a + W2 . (N(a) - N(u))
    auto stage_b = [&](const double* __restrict__ su, const double* __restrict__ snu, const double* __restrict__ sa,
                       const double* __restrict__ sna, double* __restrict__ dst) {
        double d[W];
#pragma unroll
        for (int j = 0; j < W; ++j) d[j] = n_diff(su, snu, sa, sna, wb + rel(MARGIN + O + j));
        double o[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            double acc = own(sa, v);
#pragma unroll
            for (int k = 0; k < NN; ++k) acc += Wc[PP][k] * d[v + k];
            o[v] = acc;
        }
#pragma unroll
        for (int v = 0; v < V; ++v) dst[ob + rel(v) - rel(0)] = o[v];
    };

    // Dirichlet: after a pass has written every position with the interior
    // row, blocks that reach an end redo the nodes whose window is clamped
    // with their own row (and hold the end nodes).  Centred: node e of the
    // 2R such nodes is e (e < R) or N - 1 - (e - R); one-sided: the n - 1
    // nodes at the upstream end, then the downstream end node.
    auto edge_node = [&](int e, int64_t& i, int& q) -> bool {
        if constexpr (SIDE == 0) i = e < R ? (int64_t)e : N - 1 - (e - R);
        else if constexpr (SIDE == 1) i = e < NN - 1 ? (int64_t)e : N - 1;
        else i = e < NN - 1 ? N - 1 - e : 0;
        q = (int)(i - base);
        return i - base >= 0 && i - base < LR;
    };
    auto edge_N = [&](const double* __restrict__ src, double* __restrict__ dst) {
        if (!dir) return;
        __syncthreads();
        for (int e = tid; e < Wn::EC; e += NT) {
            int64_t i;
            int q;
            if (!edge_node(e, i, q)) continue;
            const int64_t off = window_offset(i, N, NN, bc, P.window, P.c);
            const int rr = (int)(-off);
            const int b0 = edge_win(i, off);
            double acc = 0.0;
            for (int k = 0; k < NN; ++k) {
                const double y = src[phys(b0 + k)];
                acc += sD1[rr * NN + k] * y * y;
            }
            dst[phys(q)] = -0.5 * g * acc;
        }
    };
    auto edge_a = [&](const double* __restrict__ su, const double* __restrict__ sn, double* __restrict__ dst) {
        if (!dir) return;
        __syncthreads();
        for (int e = tid; e < Wn::EC; e += NT) {
            int64_t i;
            int q;
            if (!edge_node(e, i, q)) continue;
            if (i == 0 || i == N - 1) {
                dst[phys(q)] = (i == 0) ? P.bc_left : P.bc_right;
                continue;
            }
            const int64_t off = window_offset(i, N, NN, bc, P.window, P.c);
            const int rr = (int)(-off);
            const int b0 = edge_win(i, off);
            double acc = 0.0;
            for (int k = 0; k < NN; ++k) {
                const double y = su[phys(b0 + k)];
                acc += sw[rr * NN + k] * y;
                if constexpr (S::HAS_N) acc += sw[(NN + rr) * NN + k] * n_at(su, sn, y, phys(b0 + k));
            }
            dst[phys(q)] = acc;
        }
    };
    auto edge_b = [&](const double* __restrict__ su, const double* __restrict__ snu, const double* __restrict__ sa,
                      const double* __restrict__ sna, double* __restrict__ dst) {
        if (!dir) return;
        __syncthreads();
        for (int e = tid; e < Wn::EC; e += NT) {
            int64_t i;
            int q;
            if (!edge_node(e, i, q)) continue;
            double acc = sa[phys(q)];
            if (i != 0 && i != N - 1) {  // the first stage holds the end values
                const int64_t off = window_offset(i, N, NN, bc, P.window, P.c);
                const int rr = (int)(-off);
                const int b0 = edge_win(i, off);
                for (int k = 0; k < NN; ++k) acc += sw[(PP * NN + rr) * NN + k] * n_diff(su, snu, sa, sna, phys(b0 + k));
            }
            dst[phys(q)] = acc;
        }
    };

    // Neumann: positions beyond an end take their mirror node's value.  Only
    // out-of-domain positions are written and only in-domain ones are read.
    auto reflect = [&](double* __restrict__ buf) {
        if (!neu) return;
        for (int q = tid; q < LR; q += NT) {
            const int64_t j = base + q;
            if (j < 0 || j > N - 1) {
                const int64_t m = node_of(j, N, bc);
                buf[phys(q)] = buf[phys(clampi((int)(m - base), 0, LR - 1))];
            }
        }
    };
    // KdV's N at a mirrored position is the mirror node's value, as for u
    auto finish_N = [&](double* __restrict__ buf) {
        if (neu) {
            __syncthreads();
            reflect(buf);
        }
    };

    double* cur = lds;           // state
    double* sa = lds + LP;       // first stage (the next state without RK2N)
    double* snu = S::DERIV ? lds + 2 * LP : nullptr;
    double* sna = (S::DERIV && S::RK2N) ? lds + 3 * LP : nullptr;
    double* nxt = S::RK2N ? (S::DERIV ? cur : lds + 2 * LP) : nullptr;
    for (int st = 0; st < ksteps; ++st) {
        if constexpr (S::DERIV) {
            deriv_N(cur, snu);
            edge_N(cur, snu);
            finish_N(snu);
            __syncthreads();
        }
        stage_a(cur, snu, sa);
        edge_a(cur, snu, sa);
        __syncthreads();
        if (neu) {  // block-uniform: only blocks that reach a Neumann end mirror
            reflect(sa);
            __syncthreads();
        }
        if constexpr (S::RK2N) {
            if constexpr (S::DERIV) {
                deriv_N(sa, sna);
                edge_N(sa, sna);
                finish_N(sna);
                __syncthreads();
            }
            stage_b(cur, snu, sa, sna, nxt);
            edge_b(cur, snu, sa, sna, nxt);
            __syncthreads();
            if (neu) {
                reflect(nxt);
                __syncthreads();
            }
            if constexpr (!S::DERIV) {
                double* t = cur;
                cur = nxt;
                nxt = t;
            }
        } else {
            double* t = cur;
            cur = sa;
            sa = t;
        }
    }

    double* __restrict__ out = u_out + P.state_off;
    for (int q = tid; q < S::TILE; q += NT) {
        const int64_t i = t0 + q;
        if (i < N) out[i] = cur[phys(q + LHALO)];
    }
}

template <int NN, int SCH, int NL, int KB>
__global__ __launch_bounds__(NT) void stepk_kernel(const DevProb* __restrict__ probs, const int* __restrict__ tile_inst,
                                                   const double* __restrict__ fd, const double* __restrict__ w,
                                                   const double* __restrict__ u_in, double* __restrict__ u_out,
                                                   int ksteps) {
    using S = Shape<NN, SCH, NL, KB>;
    __shared__ double lds[S::NBUF * LP];
    __shared__ double sw[(S::PP + 1) * NN * NN];
    __shared__ double sD1[S::DERIV ? NN * NN : 1];
    stepk_body<NN, SCH, NL, KB, 0>(probs[tile_inst[blockIdx.x]], fd, w, u_in, u_out, ksteps, lds, sw, sD1);
}
// one-sided windows: SIDE 1 (c > 0, window ends at the node), 2 (c < 0)
template <int NN, int SCH, int NL, int KB, int SIDE>
__global__ __launch_bounds__(NT) void stepk_upwind_kernel(const DevProb* __restrict__ probs,
                                                          const int* __restrict__ tile_inst,
                                                          const double* __restrict__ fd, const double* __restrict__ w,
                                                          const double* __restrict__ u_in, double* __restrict__ u_out,
                                                          int ksteps) {
    using S = Shape<NN, SCH, NL, KB>;
    __shared__ double lds[S::NBUF * LP];
    __shared__ double sw[(S::PP + 1) * NN * NN];
    __shared__ double sD1[S::DERIV ? NN * NN : 1];
    stepk_body<NN, SCH, NL, KB, SIDE>(probs[tile_inst[blockIdx.x]], fd, w, u_in, u_out, ksteps, lds, sw, sD1);
}

// Several stencil sizes in one launch (centred windows): each block runs the
// body of its instance's n, the blocks of larger stencils first (the host
// orders the instances so), so that the launch ends on the shortest blocks.
// The weight and derivative rows sit in dynamic LDS sized for the launch's
// largest n; the staged state is the same size for every n.
template <int SCH, int NL, int KB>
__global__ __launch_bounds__(NT) void stepk_mixed_kernel(const DevProb* __restrict__ probs,
                                                         const int* __restrict__ tile_inst,
                                                         const double* __restrict__ fd, const double* __restrict__ w,
                                                         const double* __restrict__ u_in, double* __restrict__ u_out,
                                                         int ksteps, int nmax) {
    using S = Shape<3, SCH, NL, KB>;  // NBUF does not depend on n
    __shared__ double lds[S::NBUF * LP];
    extern __shared__ double dyn[];
    const DevProb& P = probs[tile_inst[blockIdx.x]];
    double* sw = dyn;
    double* sD1 = dyn + (S::PP + 1) * nmax * nmax;
    switch (P.n) {
        case 3: stepk_body<3, SCH, NL, KB, 0>(P, fd, w, u_in, u_out, ksteps, lds, sw, sD1); break;
        case 5: stepk_body<5, SCH, NL, KB, 0>(P, fd, w, u_in, u_out, ksteps, lds, sw, sD1); break;
        case 7: stepk_body<7, SCH, NL, KB, 0>(P, fd, w, u_in, u_out, ksteps, lds, sw, sD1); break;
        case 9: stepk_body<9, SCH, NL, KB, 0>(P, fd, w, u_in, u_out, ksteps, lds, sw, sD1); break;
        case 11: stepk_body<11, SCH, NL, KB, 0>(P, fd, w, u_in, u_out, ksteps, lds, sw, sD1); break;
        case 13: stepk_body<13, SCH, NL, KB, 0>(P, fd, w, u_in, u_out, ksteps, lds, sw, sD1); break;
        case 15: stepk_body<15, SCH, NL, KB, 0>(P, fd, w, u_in, u_out, ksteps, lds, sw, sD1); break;
        default: break;
    }
}

template <int SCH, int NL, int KB>
hipError_t go_mixed(int nmax, const DevProb* p, const int* ti, int64_t tiles, const double* fd, const double* w,
                    const double* ui, double* uo, int ksteps, hipStream_t s) {
    using S = Shape<3, SCH, NL, KB>;
    const size_t dyn = sizeof(double) * ((S::PP + 1) * nmax * nmax + (S::DERIV ? nmax * nmax : 0));
    hipLaunchKernelGGL((stepk_mixed_kernel<SCH, NL, KB>), dim3((unsigned)tiles), dim3(NT), dyn, s, p, ti, fd, w, ui,
                       uo, ksteps, nmax);
    return hipGetLastError();
}

template <int KB>
hipError_t dispatch_mixed(int nmax, int scheme, int nonlin, const DevProb* p, const int* ti, int64_t tiles,
                          const double* fd, const double* w, const double* ui, double* uo, int ksteps, hipStream_t s) {
    if (nmax < 3 || nmax > kMaxN || nmax % 2 == 0) return hipErrorInvalidValue;
    if (scheme == SCH_LINEAR) return go_mixed<SCH_LINEAR, NL_NONE, KB>(nmax, p, ti, tiles, fd, w, ui, uo, ksteps, s);
    if (scheme != SCH_ETD1 && scheme != SCH_ETD2RK) return hipErrorInvalidValue;
    const bool rk2 = scheme == SCH_ETD2RK;
    switch (nonlin) {
        case NL_NONE:
            return rk2 ? go_mixed<SCH_ETD2RK, NL_NONE, KB>(nmax, p, ti, tiles, fd, w, ui, uo, ksteps, s)
                       : go_mixed<SCH_ETD1, NL_NONE, KB>(nmax, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case NL_AC:
            return rk2 ? go_mixed<SCH_ETD2RK, NL_AC, KB>(nmax, p, ti, tiles, fd, w, ui, uo, ksteps, s)
                       : go_mixed<SCH_ETD1, NL_AC, KB>(nmax, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case NL_KDV:
            return rk2 ? go_mixed<SCH_ETD2RK, NL_KDV, KB>(nmax, p, ti, tiles, fd, w, ui, uo, ksteps, s)
                       : go_mixed<SCH_ETD1, NL_KDV, KB>(nmax, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case kNlAcUnit:
            return rk2 ? go_mixed<SCH_ETD2RK, kNlAcUnit, KB>(nmax, p, ti, tiles, fd, w, ui, uo, ksteps, s)
                       : go_mixed<SCH_ETD1, kNlAcUnit, KB>(nmax, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        default: return hipErrorInvalidValue;
    }
}

template <int NN, int SCH, int NL, int KB, int SIDE>
hipError_t go(const DevProb* p, const int* ti, int64_t tiles, const double* fd, const double* w, const double* ui,
              double* uo, int ksteps, hipStream_t s) {
    if constexpr (SIDE == 0)
        hipLaunchKernelGGL((stepk_kernel<NN, SCH, NL, KB>), dim3((unsigned)tiles), dim3(NT), 0, s, p, ti, fd, w, ui,
                           uo, ksteps);
    else
        hipLaunchKernelGGL((stepk_upwind_kernel<NN, SCH, NL, KB, SIDE>), dim3((unsigned)tiles), dim3(NT), 0, s, p, ti,
                           fd, w, ui, uo, ksteps);
    return hipGetLastError();
}

template <int NN, int KB, int SIDE>
hipError_t dispatch(int scheme, int nonlin, const DevProb* p, const int* ti, int64_t tiles, const double* fd,
                    const double* w, const double* ui, double* uo, int ksteps, hipStream_t s) {
    if (scheme == SCH_LINEAR) return go<NN, SCH_LINEAR, NL_NONE, KB, SIDE>(p, ti, tiles, fd, w, ui, uo, ksteps, s);
    if (scheme != SCH_ETD1 && scheme != SCH_ETD2RK) return hipErrorInvalidValue;
    const bool rk2 = scheme == SCH_ETD2RK;
    switch (nonlin) {
        case NL_NONE:
            return rk2 ? go<NN, SCH_ETD2RK, NL_NONE, KB, SIDE>(p, ti, tiles, fd, w, ui, uo, ksteps, s)
                       : go<NN, SCH_ETD1, NL_NONE, KB, SIDE>(p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case NL_AC:
            return rk2 ? go<NN, SCH_ETD2RK, NL_AC, KB, SIDE>(p, ti, tiles, fd, w, ui, uo, ksteps, s)
                       : go<NN, SCH_ETD1, NL_AC, KB, SIDE>(p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case NL_KDV:
            return rk2 ? go<NN, SCH_ETD2RK, NL_KDV, KB, SIDE>(p, ti, tiles, fd, w, ui, uo, ksteps, s)
                       : go<NN, SCH_ETD1, NL_KDV, KB, SIDE>(p, ti, tiles, fd, w, ui, uo, ksteps, s);
        default: return hipErrorInvalidValue;
    }
}

template <int KB, int SIDE>
hipError_t dispatch_n(int n, int scheme, int nonlin, const DevProb* p, const int* ti, int64_t tiles, const double* fd,
                      const double* w, const double* ui, double* uo, int ksteps, hipStream_t s) {
    switch (n) {
        case 3: return dispatch<3, KB, SIDE>(scheme, nonlin, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case 5: return dispatch<5, KB, SIDE>(scheme, nonlin, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case 7: return dispatch<7, KB, SIDE>(scheme, nonlin, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case 9: return dispatch<9, KB, SIDE>(scheme, nonlin, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case 11: return dispatch<11, KB, SIDE>(scheme, nonlin, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case 13: return dispatch<13, KB, SIDE>(scheme, nonlin, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case 15: return dispatch<15, KB, SIDE>(scheme, nonlin, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace lmep
