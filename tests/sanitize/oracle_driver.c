/* The oracle under the sanitizers: weights, runs and reverse steps of small
 * problems of every kind it covers (schemes, nonlinearities, boundaries,
 * windows, non-uniform grids, stencils from 3 to 19 points), plus rejected
 * ones.  Exits 0 when every call returned what its arguments call for. */
#include <stdio.h>
#include <stdlib.h>

#include "lmep_oracle.c"

static int fails = 0;
#define EXPECT(c) do { if (!(c)) { fprintf(stderr, "line %d: %s\n", __LINE__, #c); ++fails; } } while (0)

static ora_prob make(int64_t N, int n, int bc, int scheme, int nonlin, int window) {
    ora_prob p;
    memset(&p, 0, sizeof(p));
    p.N = N; p.n = n; p.bc = bc; p.h = 0.05; p.dt = 0.01; p.c = 0.7; p.nu = 0.01;
    p.scheme = scheme; p.nonlin = nonlin; p.nl_coef = nonlin ? 0.5 : 0.0; p.window = window;
    p.bc_left = 0.1; p.bc_right = -0.1;
    return p;
}

static int kinds(int scheme) { return scheme == SCH_ETDRK4 ? 6 : 1 + scheme_p(scheme); }

int main(void) {
    int ok_calls = 0;
    for (int n = 3; n <= 19; n += 4)
        for (int scheme = 0; scheme <= 3; ++scheme)
            for (int nonlin = 0; nonlin <= 3; ++nonlin)
                for (int bc = 0; bc <= 2; ++bc)
                    for (int window = 0; window <= 1; ++window) {
                        if (scheme == SCH_LINEAR && nonlin) continue;
                        if (nonlin == NL_BURGERS_FROZEN && scheme != SCH_ETD1) continue;
                        const int64_t N = n + 9;
                        ora_prob p = make(N, n, bc, scheme, nonlin, window);
                        double *u = malloc(sizeof(double) * N), *v = malloc(sizeof(double) * N);
                        double *w = malloc(sizeof(double) * N * kinds(scheme) * n);
                        for (int64_t i = 0; i < N; ++i) u[i] = 0.3 * sin(0.4 * (double)i) + 0.05;
                        const int rb = ora_build_weights(&p, u, w);
                        const int rr = ora_run(&p, u, 3, v);
                        EXPECT(rb == rr);
                        if (rb == 0) {  /* values may grow (unstable combinations are allowed here) */
                            ++ok_calls;
                            if ((scheme == SCH_LINEAR || scheme == SCH_ETD1) && window == WIN_CENTRED &&
                                nonlin != NL_KDV) {
                                double grad[3];
                                const int ra = ora_adjoint_step(&p, u, u, v, grad);
                                EXPECT(ra == 0 || ra == -1);
                            }
                        }
                        free(u); free(v); free(w);
                    }
    EXPECT(ok_calls > 100);
    /* a non-uniform (Chebyshev) grid */
    {
        const int64_t N = 40;
        double x[40], u[40], v[40];
        for (int i = 0; i < N; ++i) { x[i] = -cos(M_PI * i / (N - 1)); u[i] = 0.5 * x[i]; }
        ora_prob p = make(N, 21, BC_DIRICHLET, SCH_ETD1, NL_ALLEN_CAHN, WIN_CENTRED);
        p.x = x; p.dt = 1e-4;
        double *w = malloc(sizeof(double) * N * 2 * 21);
        EXPECT(ora_build_weights(&p, u, w) == 0);
        EXPECT(ora_run(&p, u, 2, v) == 0);
        free(w);
    }
    /* rejected problems */
    {
        double u[20], v[20];
        for (int i = 0; i < 20; ++i) u[i] = 0.0;
        ora_prob p = make(20, 4, BC_PERIODIC, SCH_ETD1, NL_NONE, WIN_CENTRED);
        EXPECT(ora_run(&p, u, 1, v) != 0);
        p = make(5, 9, BC_PERIODIC, SCH_ETD1, NL_NONE, WIN_CENTRED);
        EXPECT(ora_run(&p, u, 1, v) != 0);
    }
    if (fails) fprintf(stderr, "%d check(s) failed\n", fails);
    else printf("oracle: all checks passed (%d problems)\n", ok_calls);
    return fails ? 1 : 0;
}
