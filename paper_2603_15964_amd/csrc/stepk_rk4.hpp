// ETDRK4 for stationary weights, up to KB steps per launch (the scheme's
// stages a, b, c and final update of Sec. 3, each operator replaced by its
// harvested local row, Sec. 3.1 step 3):
//   a  = E2 u + P2 N(u)
//   b  = E2 u + P2 N(a)
//   c  = E2 a + P2 (2 N(b) - N(u))
//   u+ = E u + A N(u) + B (N(a) + N(b)) + C N(c)
// with E2, P2 the rows of e^{L dt/2}, (dt/2) phi1(L dt/2) and E, A, B, C the
// rows of e^{L dt}, dt alpha, dt beta, dt gamma (weight kinds 0..5).
//
// Same organisation as stepk.hpp: a block stages kStepRegion positions,
// advances them KB steps in LDS and writes the middle tile; every stage costs
// (n-1)/2 positions of halo per side (twice that with KdV's derivative term,
// which gets passes of its own).  Allen-Cahn: N is formed on the fly, four
// arrays (u, a, b, c) and N(a) + N(b) stored over a once c exists.  KdV: six
// arrays, stages written over dead ones.  Dirichlet end rows, Neumann
// mirrors and the placement of an instance's last block as in stepk.hpp.  E2 and P2 stay in registers; E, A, B, C are read
// from LDS in the final pass.
#pragma once
#include "stepk.hpp"

namespace lmep {
namespace {

template <int NN, int NL, int KB>
struct ShapeRK4 {
    static constexpr int R = (NN - 1) / 2;
    static constexpr bool HAS_N = (NL != NL_NONE);
    static constexpr bool DERIV = (NL == NL_KDV);
    static constexpr int HALO = stepk_halo(NN, SCH_ETDRK4, NL, KB);
    static constexpr int TILE = stepk_tile(NN, SCH_ETDRK4, NL, KB);
    static constexpr int NBUF = !HAS_N ? 2 : (DERIV ? 6 : 4);
    static_assert(NN <= kMaxNRk4, "ETDRK4 stencils up to kMaxNRk4 points");
    static_assert(R <= MARGIN && TILE > 0, "shape");
};

template <int NN, int NL, int KB>
__global__ __launch_bounds__(NT) void stepk_rk4_kernel(const DevProb* __restrict__ probs,
                                                       const int* __restrict__ tile_inst,
                                                       const double* __restrict__ fd, const double* __restrict__ w,
                                                       const double* __restrict__ u_in, double* __restrict__ u_out,
                                                       int ksteps) {
    using S = ShapeRK4<NN, NL, KB>;
    constexpr int R = S::R, W = V + NN - 1, NK = 6;
    __shared__ double lds[S::NBUF * LP];
    __shared__ double sw[NK * NN * NN];
    __shared__ double sD1[S::DERIV ? NN * NN : 1];

    const int tid = threadIdx.x;
    const DevProb& P = probs[tile_inst[blockIdx.x]];
    const int64_t N = P.N;
    const int bc = P.bc;
    // the last block of a Dirichlet or Neumann instance ends at node N - 1 (see stepk.hpp)
    const int64_t own = ((int64_t)blockIdx.x - P.item_begin) * S::TILE;
    const int64_t t0 = (bc != BC_PERIODIC && N >= S::TILE && own > N - S::TILE) ? N - S::TILE : own;
    const int64_t base = t0 - S::HALO;
    const double g = P.nl_coef;
    const bool at_end = base < NN || base + LR > N - NN;
    const bool dir = (bc == BC_DIRICHLET) && at_end;
    const bool neu = (bc == BC_NEUMANN) && at_end;

    for (int q = tid; q < NK * NN * NN; q += NT) sw[q] = w[P.weight_off + q];
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

    double E2[NN], P2[NN];  // half-step rows (centre row), used three times per step
#pragma unroll
    for (int k = 0; k < NN; ++k) {
        E2[k] = sw[(0 * NN + R) * NN + k];
        P2[k] = sw[(1 * NN + R) * NN + k];
    }
    double D1c[S::DERIV ? NN : 1];
    if constexpr (S::DERIV) {
#pragma unroll
        for (int k = 0; k < NN; ++k) D1c[k] = sD1[R * NN + k];
    }

    const int p0 = tid * V;
    const int wb = phys(p0 - MARGIN);
    const int ob = wb + rel(MARGIN);
    auto wslot = [&](int j) { return wb + rel(MARGIN - R + j); };  // slot of window entry j
    auto oslot = [&](int v) { return ob + rel(v) - rel(0); };       // slot of own position v
    auto edge_win = [&](int64_t i, int64_t off) { return clampi((int)(i + off - base), -MARGIN, LR + MARGIN - NN); };
    auto nval = [&](double x) { return pointwise_N<NL>(x, g); };

    // ---- passes over the whole region -------------------------------------
    // KdV: dst = -(g/2) D1 (x x)
    auto deriv_N = [&](const double* __restrict__ src, double* __restrict__ dst) {
        double x[W];
#pragma unroll
        for (int j = 0; j < W; ++j) x[j] = src[wslot(j)];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < NN; ++k) acc += D1c[k] * x[v + k] * x[v + k];
            dst[oslot(v)] = -0.5 * g * acc;
        }
    };
    // dst = E2 . x + P2 . y, with y_j given by yf(slot of j)
    auto half_stage = [&](const double* __restrict__ x, auto yf, double* __restrict__ dst) {
        double xs[W], ys[W];
#pragma unroll
        for (int j = 0; j < W; ++j) {
            xs[j] = x[wslot(j)];
            ys[j] = yf(wslot(j));
        }
#pragma unroll
        for (int v = 0; v < V; ++v) {
            double acc = 0.0;
#pragma unroll
            for (int k = 0; k < NN; ++k) {
                acc += E2[k] * xs[v + k];
                acc += P2[k] * ys[v + k];
            }
            dst[oslot(v)] = acc;
        }
    };
    // o += row(kind) . f over the window, f_j given by f(slot of j)
    auto add_term = [&](double (&o)[V], int kind, auto f) {
        double wk[NN], xs[W];
#pragma unroll
        for (int k = 0; k < NN; ++k) wk[k] = sw[(kind * NN + R) * NN + k];
#pragma unroll
        for (int j = 0; j < W; ++j) xs[j] = f(wslot(j));
#pragma unroll
        for (int v = 0; v < V; ++v)
#pragma unroll
            for (int k = 0; k < NN; ++k) o[v] += wk[k] * xs[v + k];
    };

    // ---- Dirichlet: nodes with one-sided windows, own rows; ends held --------
    auto edge_node = [&](int e, int64_t& i, int& q) -> bool {
        i = e < R ? (int64_t)e : N - 1 - (e - R);
        q = (int)(i - base);
        return i - base >= 0 && i - base < LR;
    };
    // own-row version of a stage: dst[i] = sum over the node's own window of
    // the term function tf(rr, k, slot)
    auto edge_fix = [&](double* __restrict__ dst, auto tf) {
        if (!dir) return;
        __syncthreads();
        for (int e = tid; e < 2 * R; e += NT) {
            int64_t i;
            int q;
            if (!edge_node(e, i, q)) continue;
            if (i == 0 || i == N - 1) {
                dst[phys(q)] = (i == 0) ? P.bc_left : P.bc_right;
                continue;
            }
            const int64_t off = window_offset(i, N, NN, bc);
            const int rr = (int)(-off);
            const int b0 = edge_win(i, off);
            double acc = 0.0;
            for (int k = 0; k < NN; ++k) acc += tf(rr, k, phys(b0 + k));
            dst[phys(q)] = acc;
        }
    };
    auto edge_N = [&](const double* __restrict__ src, double* __restrict__ dst) {
        if (!dir) return;
        __syncthreads();
        for (int e = tid; e < 2 * R; e += NT) {
            int64_t i;
            int q;
            if (!edge_node(e, i, q)) continue;
            const int64_t off = window_offset(i, N, NN, bc);
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
    auto reflect = [&](double* __restrict__ buf) {
        if (!neu) return;
        __syncthreads();
        for (int q = tid; q < LR; q += NT) {
            const int64_t j = base + q;
            if (j < 0 || j > N - 1) {
                const int64_t m = node_of(j, N, bc);
                buf[phys(q)] = buf[phys(clampi((int)(m - base), 0, LR - 1))];
            }
        }
    };
    auto swk = [&](int kind, int rr, int k) { return sw[(kind * NN + rr) * NN + k]; };
    // a finished array: own rows at Dirichlet ends, mirrors at Neumann ends
    auto finish = [&](double* __restrict__ dst, auto tf) {
        edge_fix(dst, tf);
        reflect(dst);
        __syncthreads();
    };
    auto finish_N = [&](const double* __restrict__ src, double* __restrict__ dst) {
        edge_N(src, dst);
        reflect(dst);
        __syncthreads();
    };

    // the arrays rotate as offsets into lds, not as stored pointers: pointers
    // kept in an array and reassigned across steps lose their LDS address
    // space and turn every access into a flat one
    int bo[S::NBUF];
#pragma unroll
    for (int b = 0; b < S::NBUF; ++b) bo[b] = b * LP;

    for (int st = 0; st < ksteps; ++st) {
        double* U = lds + bo[0];
        if constexpr (!S::HAS_N) {
            // no nonlinearity: u+ = E u
            double o[V];
#pragma unroll
            for (int v = 0; v < V; ++v) o[v] = 0.0;
            add_term(o, 2, [&](int s) { return U[s]; });
#pragma unroll
            for (int v = 0; v < V; ++v) lds[bo[1] + oslot(v)] = o[v];
            finish(lds + bo[1], [&](int rr, int k, int s) { return swk(2, rr, k) * U[s]; });
            const int t = bo[0];
            bo[0] = bo[1];
            bo[1] = t;
        } else if constexpr (!S::DERIV) {
            double *A1 = lds + bo[1], *A2 = lds + bo[2], *A3 = lds + bo[3];
            // a = E2 u + P2 N(u)
            half_stage(U, [&](int s) { return nval(U[s]); }, A1);
            finish(A1, [&](int rr, int k, int s) { return swk(0, rr, k) * U[s] + swk(1, rr, k) * nval(U[s]); });
            // b = E2 u + P2 N(a)
            half_stage(U, [&](int s) { return nval(A1[s]); }, A2);
            finish(A2, [&](int rr, int k, int s) { return swk(0, rr, k) * U[s] + swk(1, rr, k) * nval(A1[s]); });
            // c = E2 a + P2 (2 N(b) - N(u))
            half_stage(A1, [&](int s) { return 2.0 * nval(A2[s]) - nval(U[s]); }, A3);
            finish(A3, [&](int rr, int k, int s) {
                return swk(0, rr, k) * A1[s] + swk(1, rr, k) * (2.0 * nval(A2[s]) - nval(U[s]));
            });
            // N(a) + N(b) over a (pointwise, own positions only)
#pragma unroll
            for (int v = 0; v < V; ++v) A1[oslot(v)] = nval(A1[oslot(v)]) + nval(A2[oslot(v)]);
            __syncthreads();
            // u+ = E u + A N(u) + B (N(a) + N(b)) + C N(c), into A2
            double o[V];
#pragma unroll
            for (int v = 0; v < V; ++v) o[v] = 0.0;
            add_term(o, 2, [&](int s) { return U[s]; });
            add_term(o, 3, [&](int s) { return nval(U[s]); });
            add_term(o, 4, [&](int s) { return A1[s]; });
            add_term(o, 5, [&](int s) { return nval(A3[s]); });
#pragma unroll
            for (int v = 0; v < V; ++v) A2[oslot(v)] = o[v];
            finish(A2, [&](int rr, int k, int s) {
                return swk(2, rr, k) * U[s] + swk(3, rr, k) * nval(U[s]) + swk(4, rr, k) * A1[s] +
                       swk(5, rr, k) * nval(A3[s]);
            });
            const int o0 = bo[0], o1 = bo[1], o2 = bo[2], o3 = bo[3];
            bo[0] = o2;  // u+ (in A2)
            bo[1] = o0;  // old u
            bo[2] = o1;  // A1
            bo[3] = o3;  // A3
        } else {
            double *NU = lds + bo[1], *A1 = lds + bo[2], *NA = lds + bo[3], *B1 = lds + bo[4], *NB = lds + bo[5];
            deriv_N(U, NU);
            finish_N(U, NU);
            // a = E2 u + P2 N(u)
            half_stage(U, [&](int s) { return NU[s]; }, A1);
            finish(A1, [&](int rr, int k, int s) { return swk(0, rr, k) * U[s] + swk(1, rr, k) * NU[s]; });
            deriv_N(A1, NA);
            finish_N(A1, NA);
            // b = E2 u + P2 N(a)
            half_stage(U, [&](int s) { return NA[s]; }, B1);
            finish(B1, [&](int rr, int k, int s) { return swk(0, rr, k) * U[s] + swk(1, rr, k) * NA[s]; });
            deriv_N(B1, NB);
            finish_N(B1, NB);
            // c = E2 a + P2 (2 N(b) - N(u)), over b (no longer read)
            half_stage(A1, [&](int s) { return 2.0 * NB[s] - NU[s]; }, B1);
            finish(B1, [&](int rr, int k, int s) { return swk(0, rr, k) * A1[s] + swk(1, rr, k) * (2.0 * NB[s] - NU[s]); });
            // N(a) + N(b) over N(a); N(c) over a
#pragma unroll
            for (int v = 0; v < V; ++v) NA[oslot(v)] = NA[oslot(v)] + NB[oslot(v)];
            deriv_N(B1, A1);
            finish_N(B1, A1);
            // u+ = E u + A N(u) + B (N(a) + N(b)) + C N(c), into N(b)
            double o[V];
#pragma unroll
            for (int v = 0; v < V; ++v) o[v] = 0.0;
            add_term(o, 2, [&](int s) { return U[s]; });
            add_term(o, 3, [&](int s) { return NU[s]; });
            add_term(o, 4, [&](int s) { return NA[s]; });
            add_term(o, 5, [&](int s) { return A1[s]; });
#pragma unroll
            for (int v = 0; v < V; ++v) NB[oslot(v)] = o[v];
            finish(NB, [&](int rr, int k, int s) {
                return swk(2, rr, k) * U[s] + swk(3, rr, k) * NU[s] + swk(4, rr, k) * NA[s] + swk(5, rr, k) * A1[s];
            });
            const int o0 = bo[0];
            bo[0] = bo[5];  // u+ (in N(b))
            bo[5] = o0;
        }
    }

    double* __restrict__ out = u_out + P.state_off;
    for (int q = tid; q < S::TILE; q += NT) {
        const int64_t i = t0 + q;
        if (i < N) out[i] = lds[bo[0] + phys(q + S::HALO)];
    }
}

template <int NN, int NL, int KB>
hipError_t go_rk4(const DevProb* p, const int* ti, int64_t tiles, const double* fd, const double* w,
                  const double* ui, double* uo, int ksteps, hipStream_t s) {
    hipLaunchKernelGGL((stepk_rk4_kernel<NN, NL, KB>), dim3((unsigned)tiles), dim3(NT), 0, s, p, ti, fd, w, ui, uo,
                       ksteps);
    return hipGetLastError();
}

template <int NN, int KB>
hipError_t dispatch_rk4(int nonlin, const DevProb* p, const int* ti, int64_t tiles, const double* fd, const double* w,
                        const double* ui, double* uo, int ksteps, hipStream_t s) {
    if constexpr (NN > kMaxNRk4) {
        return hipErrorInvalidValue;
    } else {
        switch (nonlin) {
            case NL_NONE: return go_rk4<NN, NL_NONE, KB>(p, ti, tiles, fd, w, ui, uo, ksteps, s);
            case NL_AC: return go_rk4<NN, NL_AC, KB>(p, ti, tiles, fd, w, ui, uo, ksteps, s);
            case NL_KDV: return go_rk4<NN, NL_KDV, KB>(p, ti, tiles, fd, w, ui, uo, ksteps, s);
            default: return hipErrorInvalidValue;
        }
    }
}

template <int KB>
hipError_t dispatch_n_rk4(int n, int nonlin, const DevProb* p, const int* ti, int64_t tiles, const double* fd,
                          const double* w, const double* ui, double* uo, int ksteps, hipStream_t s) {
    switch (n) {
        case 3: return dispatch_rk4<3, KB>(nonlin, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case 5: return dispatch_rk4<5, KB>(nonlin, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case 7: return dispatch_rk4<7, KB>(nonlin, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case 9: return dispatch_rk4<9, KB>(nonlin, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case 11: return dispatch_rk4<11, KB>(nonlin, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case 13: return dispatch_rk4<13, KB>(nonlin, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case 15: return dispatch_rk4<15, KB>(nonlin, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case 17: return dispatch_rk4<17, KB>(nonlin, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        case 19: return dispatch_rk4<19, KB>(nonlin, p, ti, tiles, fd, w, ui, uo, ksteps, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace
}  // namespace lmep
