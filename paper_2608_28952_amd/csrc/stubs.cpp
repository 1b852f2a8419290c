// stubs.cpp -- entry points declared in include/jacobi.h whose drivers are
// not built yet; they fail loudly with a clear error.
#include "jx_common.hpp"

extern "C" {

size_t jacobi_eig_batched_workspace(int, const int *, int, const jacobi_opts *) { return 0; }

int jacobi_eig_batched(int, const int *, const int64_t *, int, const void *, double *, double *,
                       const double *, void *, size_t, const jacobi_opts *, jacobi_info *info,
                       jacobi_stream_t) {
    jx::set_error("jacobi_eig_batched: not available in this build");
    if (info) info->status = 3;
    return 3;
}
}
