// Host paths of the C ABI under the sanitizers: weight counts, scratch sizes,
// options, and every entry point with arguments the host checks reject (or,
// for well-formed batches, the device error of a machine without a GPU).
// Exits 0 when every call returned a status of the expected kind.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "lmep.h"

static int fails = 0;
#define EXPECT(cond)                                                            \
    do {                                                                        \
        if (!(cond)) {                                                          \
            std::fprintf(stderr, "line %d: %s (%s)\n", __LINE__, #cond, lmep_last_error()); \
            ++fails;                                                            \
        }                                                                       \
    } while (0)

static lmep_problem base(int n, int scheme, int nonlin, int bc, int window, int64_t N) {
    lmep_problem p;
    std::memset(&p, 0, sizeof(p));
    p.N = N;
    p.n = n;
    p.bc = bc;
    p.h = 0.01;
    p.dt = 1e-4;
    p.c = 0.5;
    p.nu = 1e-3;
    p.scheme = scheme;
    p.nonlin = nonlin;
    p.nl_coef = nonlin ? 1.0 : 0.0;
    p.window = window;
    return p;
}

int main() {
    // weight counts and scratch sizes over the supported combinations
    std::vector<lmep_problem> batch;
    int64_t soff = 0, woff = 0;
    for (int n = 3; n <= 15; n += 2)
        for (int scheme = 0; scheme <= 3; ++scheme)
            for (int nonlin = 0; nonlin <= 3; ++nonlin)
                for (int bc = 0; bc <= 2; ++bc)
                    for (int window = 0; window <= 1; ++window) {
                        if (scheme == 0 && nonlin != 0) continue;
                        if (nonlin == 1 && scheme != 1) continue;
                        if (window == 1 && scheme == 3) continue;
                        if (n + (scheme == 3 ? 3 : scheme) > 16) continue;
                        lmep_problem p = base(n, scheme, nonlin, bc, window, 40 + 7 * n);
                        const int64_t wc = lmep_weight_count(&p);
                        EXPECT(wc > 0);
                        p.state_off = soff;
                        p.weight_off = woff;
                        soff += p.N;
                        woff += wc;
                        batch.push_back(p);
                    }
    const int32_t cnt = (int32_t)batch.size();
    for (int op = 0; op <= 2; ++op) {
        const size_t b = lmep_scratch_bytes(batch.data(), cnt, op);
        (void)b;  // op 2 refuses batches the reverse step does not cover (0)
    }
    EXPECT(lmep_scratch_bytes(batch.data(), cnt, 1) > 0);
    EXPECT(lmep_scratch_bytes(nullptr, 0, 1) == 0);

    // options
    EXPECT(lmep_set_option(LMEP_OPT_STEPS_PER_LAUNCH, 16) == LMEP_OK);
    EXPECT(lmep_get_option(LMEP_OPT_STEPS_PER_LAUNCH) == 16);
    EXPECT(lmep_set_option(LMEP_OPT_STEPS_PER_LAUNCH, 3) == LMEP_ERR_ARG);
    EXPECT(lmep_set_option(LMEP_OPT_STEPS_PER_LAUNCH, 8) == LMEP_OK);
    EXPECT(lmep_set_option(LMEP_OPT_TAYLOR_REGION, 320) == LMEP_OK);
    EXPECT(lmep_set_option(LMEP_OPT_TAYLOR_REGION, 100) == LMEP_ERR_ARG);
    EXPECT(lmep_set_option(LMEP_OPT_TAYLOR_REGION, 0) == LMEP_OK);
    EXPECT(lmep_set_option(99, 1) == LMEP_ERR_ARG);
    EXPECT(lmep_get_option(99) == LMEP_ERR_ARG);

    // malformed instances and calls are rejected before any device work
    double* fake = reinterpret_cast<double*>(0x1000);
    std::vector<char> host_scratch(1);
    lmep_problem bad = base(4, 1, 3, 0, 0, 100);  // even n
    EXPECT(lmep_step(&bad, 1, fake, fake, fake + 512, 1, 0, host_scratch.data(), 1, nullptr) == LMEP_ERR_ARG);
    bad = base(9, 1, 3, 0, 2, 100);  // unknown window
    EXPECT(lmep_build_weights(&bad, 1, fake, fake, host_scratch.data(), 1, nullptr) == LMEP_ERR_ARG);
    bad = base(9, 3, 3, 0, 1, 100);  // ETDRK4 on upwind windows
    EXPECT(lmep_step(&bad, 1, fake, fake, fake + 512, 1, 0, host_scratch.data(), 1 << 20, nullptr) ==
           LMEP_ERR_UNSUPPORTED);
    lmep_problem two[2] = {base(9, 1, 3, 0, 0, 100), base(9, 1, 3, 0, 0, 100)};
    two[1].state_off = 50;  // overlapping states
    two[1].weight_off = 2 * 9 * 9;
    EXPECT(lmep_step(two, 2, fake, fake, fake + 512, 1, 0, host_scratch.data(), 1 << 20, nullptr) == LMEP_ERR_ARG);
    EXPECT(lmep_step(batch.data(), cnt, fake, fake, fake, 1, 0, host_scratch.data(), 1 << 30, nullptr) ==
           LMEP_ERR_ARG);  // in place
    EXPECT(lmep_step(batch.data(), cnt, fake, fake, fake + (1 << 20), 1, 0, host_scratch.data(), 1, nullptr) ==
           LMEP_ERR_SCRATCH);
    EXPECT(lmep_step(batch.data(), cnt, fake, fake, fake + (1 << 20), 1, 0x100, host_scratch.data(), 1 << 30,
                     nullptr) == LMEP_ERR_ARG);  // unknown flag
    EXPECT(lmep_step_noalloc(batch.data(), cnt, fake, fake, fake + (1 << 20), 1, LMEP_F_GRAPH, nullptr) ==
           LMEP_ERR_ARG);
    lmep_problem adj = base(9, 2, 3, 0, 0, 100);  // the reverse step covers LINEAR and ETD1 only
    EXPECT(lmep_adjoint_step(&adj, 1, fake, fake, fake + 512, fake + 1024, host_scratch.data(), 1 << 20, nullptr) ==
           LMEP_ERR_UNSUPPORTED);
    lmep_plan plan = nullptr;
    EXPECT(lmep_plan_create(&plan, &bad, 1, 1, 0, nullptr, 0, host_scratch.data(), 1 << 20, nullptr) ==
           LMEP_ERR_UNSUPPORTED);
    EXPECT(plan == nullptr);
    const int32_t opts[2] = {LMEP_OPT_STEPS_PER_LAUNCH, 5};
    lmep_problem ok1 = base(9, 1, 3, 0, 0, 100);
    EXPECT(lmep_plan_create(&plan, &ok1, 1, 1, 0, opts, 1, host_scratch.data(), 1 << 20, nullptr) == LMEP_ERR_ARG);
    EXPECT(lmep_plan_create(&plan, &ok1, 1, 7, 0, nullptr, 0, host_scratch.data(), 1 << 20, nullptr) == LMEP_ERR_ARG);
    (void)lmep_plan_destroy(nullptr);

    // well-formed calls reach the device and fail there (no GPU here)
    const size_t need = lmep_scratch_bytes(&ok1, 1, 1);
    std::vector<char> big(need + 512);
    char* aligned = big.data() + (256 - reinterpret_cast<uintptr_t>(big.data()) % 256) % 256;
    const int rc = lmep_step(&ok1, 1, fake, fake, fake + 512, 3, 0, aligned, need, nullptr);
    EXPECT(rc == LMEP_ERR_DEVICE || rc == LMEP_OK);
    char name[64];
    double ms = 0;
    int32_t launches = 0;
    (void)lmep_profile_kernel(0, name, sizeof(name), &ms, &launches);
    if (fails) std::fprintf(stderr, "%d check(s) failed\n", fails);
    else std::printf("abi host paths: all checks passed\n");
    return fails ? 1 : 0;
}
