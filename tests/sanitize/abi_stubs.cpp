// Stand-ins for the library's kernel launchers and device tables, so that the
// C-ABI host code can be built for the CPU with address and undefined-behaviour
// sanitizers and its host paths (argument checks, plans, scratch layouts,
// options, error strings) exercised without a GPU.  Every stand-in reports a
// device error; none is reached by a call that the host checks reject.
#include "lmep_internal.hpp"

namespace lmep {

hipError_t launch_apply(int, int, int, int, bool, const DevProb*, const int*, int64_t, const double*, const double*,
                        const double*, double*, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_build(int, int, const DevProb*, int, int64_t, const double*, const double*, double*,
                        unsigned long long*, hipStream_t, double*) { return hipErrorInvalidValue; }
hipError_t launch_stepk(int, int, int, int, int, const DevProb*, const int*, int64_t, const double*, const double*,
                        const double*, double*, hipStream_t, int) { return hipErrorInvalidValue; }
hipError_t launch_stepk_mixed(int, int, int, int, int, const DevProb*, const int*, int64_t, const double*,
                              const double*, const double*, double*, hipStream_t) { return hipErrorInvalidValue; }
hipError_t fd_table_init(const double**) { return hipErrorInvalidValue; }
hipError_t taylor_table_init(const double**) { return hipErrorInvalidValue; }
hipError_t taylor_dd_table_init(const double**) { return hipErrorInvalidValue; }
hipError_t launch_adjoint(const AdjointLaunch&, hipStream_t) { return hipErrorInvalidValue; }
hipError_t static_scratch(void**) { return hipErrorInvalidValue; }
hipError_t upload_by_args(void*, const void*, size_t, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_resident(int, int, int, bool, const DevProb*, int, int64_t, const double*, const double*, double*,
                           int, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_build_wide(int, int, const DevProb*, int, int64_t, double*, hipStream_t) {
    return hipErrorInvalidValue;
}
hipError_t launch_build_taylor(int, const DevProb*, int, int64_t, const double*, const double*, const double*, double*,
                               unsigned long long*, hipStream_t, double*, bool) { return hipErrorInvalidValue; }
hipError_t launch_check_finite(const double*, int64_t, int*, hipStream_t) { return hipErrorInvalidValue; }
hipError_t launch_taylor_stepk(int, int, int, int, const DevProb*, int, int64_t, const double*, const double*,
                               const double*, double*, unsigned long long*, hipStream_t) {
    return hipErrorInvalidValue;
}
hipError_t launch_build_table_dd(int, int, const DevProb*, int, int64_t, const double*, double*, hipStream_t) {
    return hipErrorInvalidValue;
}
hipError_t launch_apply_nonuniform(int, int, int, int, const DevProb*, const int*, int64_t, const double*,
                                   const double*, const double*, double*, hipStream_t) {
    return hipErrorInvalidValue;
}

}  // namespace lmep
