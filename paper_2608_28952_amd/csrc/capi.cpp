// capi.cpp -- the extern "C" surface of libjacobi.so (include/jacobi.h):
// argument checks, defaults, error text, and dispatch to the drivers.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <string>
#include <vector>

#include "jx_common.hpp"
#include "jx_host.hpp"

namespace jx {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }
const char *last_error() { return g_last_error.c_str(); }

static jacobi_opts resolve(const jacobi_opts *o) {
    jacobi_opts r;
    jacobi_opts_default(&r);
    if (o) r = *o;
    if (!(r.tol > 0.0)) r.tol = 0.0;  // per-routine default
    if (r.max_sweeps <= 0) r.max_sweeps = 60;
    return r;
}

template <class F>
static int guarded(jacobi_info *info, F &&f) {
    g_last_error.clear();
    try {
        return f();
    } catch (const HipFail &) {
        if (info) info->status = 3;
        return 3;
    }
}

}  // namespace jx

using namespace jx;

extern "C" {

int jacobi_opts_default(jacobi_opts *o) {
    if (!o) return -1;
    o->tol = 0.0;
    o->max_sweeps = 60;
    o->block = 0;
    o->ordering = JACOBI_ORDER_ROUND_ROBIN_SORTED;
    o->precision = JACOBI_PREC_FP64;
    o->inner_max_sweeps = 1;
    o->refine = -1;
    o->sort = 1;
    o->want_vectors = 1;
    o->threshold = 0;
    o->precondition = -1;
    o->pivot = 0;
    return 0;
}

const char *jacobi_last_error(void) { return jx::last_error(); }

int jacobi_init(void) {
    g_last_error.clear();
    try {
        (void)device_ctx();
        (void)noalloc_setup();
        return 0;
    } catch (const HipFail &) {
        return 3;
    }
}

size_t jacobi_eig_workspace(int n, const jacobi_opts *o) {
    if (n <= 1) return 256;
    jacobi_opts r = resolve(o);
    if (r.block == 1) return n <= 1024 ? scalar_workspace(n) : 0;
    if (r.block != 0 && r.block != 32 && r.block != 64) return 0;
    return plan_eig(n, r).total;
}

int jacobi_eig(int n, const double *dA, int lda, char uplo, double *dW, double *dQ, int ldq,
               const double *dQ0, int ldq0, void *dWork, size_t workBytes, const jacobi_opts *opts,
               jacobi_info *info, jacobi_stream_t stream) {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    jacobi_opts o = resolve(opts);
    if (info) *info = jacobi_info{};
    auto fail = [&](int code, const char *msg) {
        set_error(msg);
        if (info) info->status = code;
        return code;
    };
    if (n < 0) return fail(-1, "n < 0");
    if (n > 0 && !dA) return fail(-2, "dA is NULL");
    if (lda < (n > 1 ? n : 1)) return fail(-3, "lda < n");
    if (uplo != 'U' && uplo != 'u' && uplo != 'L' && uplo != 'l') return fail(-4, "uplo must be 'U' or 'L'");
    if (n > 0 && !dW) return fail(-5, "dW is NULL");
    if (o.want_vectors && n > 0 && !dQ) return fail(-6, "dQ is NULL but vectors were requested");
    if (o.want_vectors && ldq < (n > 1 ? n : 1)) return fail(-7, "ldq < n");
    if (dQ0 && ldq0 < (n > 1 ? n : 1)) return fail(-9, "ldq0 < n");
    if (o.block != 0 && o.block != 1 && o.block != 32 && o.block != 64)
        return fail(-12, "opts->block must be 0, 1, 32 or 64");
    if (o.ordering != JACOBI_ORDER_ROUND_ROBIN && o.ordering != JACOBI_ORDER_ANTIDIAG &&
        o.ordering != JACOBI_ORDER_ROUND_ROBIN_SORTED)
        return fail(-12, "opts->ordering invalid");
    if (o.precision != JACOBI_PREC_FP64 && o.precision != JACOBI_PREC_MIXED_FP32)
        return fail(-12, "opts->precision must be JACOBI_PREC_FP64 or JACOBI_PREC_MIXED_FP32");
    if (o.block == 1 && (n > 1024 || o.precision != JACOBI_PREC_FP64))
        return fail(-12, "opts->block = 1 (scalar Jacobi) takes n <= 1024 and JACOBI_PREC_FP64");
    if (o.block == 1 && dQ0) return fail(-8, "no warm start with opts->block = 1");
    if (o.threshold != 0 && (o.threshold != 1 || o.block != 1))
        return fail(-12, "opts->threshold = 1 (relative) needs opts->block = 1");
    if (o.pivot != 0 && (o.pivot != 1 || o.block == 1))
        return fail(-12, "opts->pivot = 1 needs a blocked solve (opts->block 0, 32 or 64)");
    if (n == 0) {
        if (info) info->status = 0;
        return 0;
    }
    return guarded(info, [&]() -> int {
        if (n > 1 && o.block == 1) {
            const int rc = run_eig_scalar(n, dA, lda, uplo, dW, o.want_vectors ? dQ : nullptr, ldq, dWork, workBytes,
                                          o, info, s);
            if (rc == -100) set_error("workspace too small");
            if (info) info->status = rc;
            return rc;
        }
        if (n == 1) {  // W = A, Q = 1
            JX_HIP(hipMemcpyAsync(dW, dA, sizeof(double), hipMemcpyDeviceToDevice, s));
            if (o.want_vectors) {
                double one = 1.0;
                if (dQ0) JX_HIP(hipMemcpyAsync(dQ, dQ0, sizeof(double), hipMemcpyDeviceToDevice, s));
                else JX_HIP(hipMemcpyAsync(dQ, &one, sizeof(double), hipMemcpyHostToDevice, s));
            }
            JX_HIP(hipStreamSynchronize(s));
            double a = 0.0;
            JX_HIP(hipMemcpy(&a, dA, sizeof(double), hipMemcpyDeviceToHost));
            const int st = std::isfinite(a) ? 0 : 2;
            if (info) info->status = st;
            return st;
        }
        const int rc = run_eig(n, dA, lda, uplo, dW, o.want_vectors ? dQ : nullptr, ldq, dQ0, ldq0, dWork, workBytes,
                               o, info, s);
        if (rc == -100) set_error("workspace too small");
        if (info) info->status = rc;
        return rc;
    });
}

size_t jacobi_svd_workspace(int m, int n, const jacobi_opts *o) {
    if (n <= 0 || m < n) return 256;
    jacobi_opts r = resolve(o);
    if (r.block != 0 && r.block != 32 && r.block != 64) return 0;
    return plan_svd(m, n, r).total;
}

int jacobi_svd(int m, int n, const double *dG, int ldg, double *dS, double *dU, int ldu, double *dV, int ldv,
               void *dWork, size_t workBytes, const jacobi_opts *opts, jacobi_info *info, jacobi_stream_t stream) {
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    jacobi_opts o = resolve(opts);
    if (info) *info = jacobi_info{};
    auto fail = [&](int code, const char *msg) {
        set_error(msg);
        if (info) info->status = code;
        return code;
    };
    if (n < 0) return fail(-2, "n < 0");
    if (m < n) return fail(-1, "m < n");
    if (n > 0 && !dG) return fail(-3, "dG is NULL");
    if (ldg < (m > 1 ? m : 1)) return fail(-4, "ldg < m");
    if (n > 0 && !dS) return fail(-5, "dS is NULL");
    if (o.want_vectors && n > 0 && (!dU || !dV)) return fail(-6, "dU / dV NULL but vectors were requested");
    if (o.want_vectors && ldu < (m > 1 ? m : 1)) return fail(-7, "ldu < m");
    if (o.want_vectors && ldv < (n > 1 ? n : 1)) return fail(-9, "ldv < n");
    if (o.block != 0 && o.block != 32 && o.block != 64) return fail(-12, "opts->block must be 0, 32 or 64");
    if (o.ordering != JACOBI_ORDER_ROUND_ROBIN && o.ordering != JACOBI_ORDER_ANTIDIAG &&
        o.ordering != JACOBI_ORDER_ROUND_ROBIN_SORTED)
        return fail(-12, "opts->ordering invalid");
    if (o.precision != JACOBI_PREC_FP64 && o.precision != JACOBI_PREC_MIXED_FP32)
        return fail(-12, "opts->precision must be JACOBI_PREC_FP64 or JACOBI_PREC_MIXED_FP32");
    if (o.threshold != 0) return fail(-12, "opts->threshold must be 0 for the SVD");
    if (o.pivot != 0) return fail(-12, "opts->pivot must be 0 for the SVD");
    if (n == 0) {
        if (info) info->status = 0;
        return 0;
    }
    return guarded(info, [&]() -> int {
        const int rc = run_svd(m, n, dG, ldg, dS, o.want_vectors ? dU : nullptr, ldu, o.want_vectors ? dV : nullptr,
                               ldv, dWork, workBytes, o, info, s);
        if (rc == -100) set_error("workspace too small");
        if (info) info->status = rc;
        return rc;
    });
}

int jacobi_schedule(int N, int ordering, int *hPairs, int *hSizes) {
    if (N < 2 || (N & 1)) return -1;
    if (ordering != JACOBI_ORDER_ROUND_ROBIN && ordering != JACOBI_ORDER_ANTIDIAG) return -2;
    if (!hPairs) return -3;
    std::vector<int> pairs, sizes;
    const int R = make_schedule(N, ordering, pairs, sizes);
    for (size_t i = 0; i < pairs.size(); ++i) hPairs[i] = pairs[i];
    if (hSizes)
        for (int r = 0; r < R; ++r) hSizes[r] = sizes[r];
    return R;
}

int jacobi_subproblem_solve(int count, int m2, const double *dAhat, double *dV, double *dD,
                            int inner_sweeps, jacobi_stream_t stream) {
    if (count < 0) return -1;
    if (m2 != 32 && m2 != 64 && m2 != 128) return -2;
    if (count > 0 && (!dAhat || !dV || !dD)) return -3;
    if (count == 0) return 0;
    return guarded(nullptr, [&]() -> int {
        return run_subproblem(count, m2, dAhat, dV, dD, inner_sweeps, reinterpret_cast<hipStream_t>(stream));
    });
}

static int block_step(int n, int b, double *dA, double *dQ, int npairs, const int *hPairs, const double *dV,
                      const double *dD, bool f32, jacobi_stream_t stream) {
    if (b != 32 && b != 64) return -2;
    if (n <= 0 || n % (2 * b) || n % 128) return -1;
    if (npairs != n / (2 * b)) return -5;
    if (!dA || !hPairs || !dV || !dD) return -3;
    std::vector<char> seen(n / b, 0);
    for (int k = 0; k < npairs; ++k) {
        const int I = hPairs[2 * k], J = hPairs[2 * k + 1];
        if (I < 0 || J >= n / b || I >= J || seen[I] || seen[J]) return -6;
        seen[I] = seen[J] = 1;
    }
    return guarded(nullptr, [&]() -> int {
        return run_block_step(n, b, dA, dQ, npairs, hPairs, dV, dD, f32, reinterpret_cast<hipStream_t>(stream));
    });
}

int jacobi_pivot_step(int n, int b, double *dA, int npairs, const int *hPairs, double *dV, int *dPerm,
                      jacobi_stream_t stream) {
    if (b != 32 && b != 64) return -2;
    if (n <= 0 || n % (2 * b) || n % 128) return -1;
    if (!dA) return -3;
    if (npairs != n / (2 * b)) return -4;
    if (!hPairs) return -5;
    std::vector<char> seen(n / b, 0);
    for (int k = 0; k < npairs; ++k) {
        const int I = hPairs[2 * k], J = hPairs[2 * k + 1];
        if (I < 0 || J >= n / b || I >= J || seen[I] || seen[J]) return -5;
        seen[I] = seen[J] = 1;
    }
    if (!dV) return -6;
    return guarded(nullptr, [&]() -> int {
        return run_pivot_step(n, b, dA, npairs, hPairs, dV, dPerm, reinterpret_cast<hipStream_t>(stream));
    });
}

int jacobi_qr(int m, int n, const double *dG, int ldg, double *dQ, int ldq, double *dR, int ldr,
              jacobi_stream_t stream) {
    if (n < 1) return -2;
    if (m < n) return -1;
    if (!dG) return -3;
    if (ldg < m) return -4;
    if (!dQ) return -5;
    if (ldq < m) return -6;
    if (!dR) return -7;
    if (ldr < n) return -8;
    return guarded(nullptr, [&]() -> int {
        return run_qr(m, n, dG, ldg, dQ, ldq, dR, ldr, reinterpret_cast<hipStream_t>(stream));
    });
}

int jacobi_gram_blocks(int m, int n, int b, const double *dG, int ldg, int npairs, const int *hPairs, int fp32,
                       double *dAhat, jacobi_stream_t stream) {
    if (b != 32 && b != 64) return -3;
    if (n <= 0 || n % b) return -2;
    if (m < n) return -1;
    if (!dG) return -4;
    if (ldg < m) return -5;
    if (npairs < 0) return -6;
    if (npairs > 0 && !hPairs) return -7;
    for (int k = 0; k < npairs; ++k) {
        const int I = hPairs[2 * k], J = hPairs[2 * k + 1];
        if (I < 0 || J < 0 || I >= n / b || J >= n / b || I == J) return -7;
    }
    if (npairs > 0 && !dAhat) return -9;
    if (npairs == 0) return 0;
    return guarded(nullptr, [&]() -> int {
        return run_gram_blocks(m, n, b, dG, ldg, npairs, hPairs, fp32 != 0, dAhat,
                               reinterpret_cast<hipStream_t>(stream));
    });
}

int jacobi_block_step(int n, int b, double *dA, double *dQ, int npairs, const int *hPairs,
                      const double *dV, const double *dD, jacobi_stream_t stream) {
    return block_step(n, b, dA, dQ, npairs, hPairs, dV, dD, false, stream);
}

int jacobi_block_step32(int n, int b, double *dA, double *dQ, int npairs, const int *hPairs,
                        const double *dV, const double *dD, jacobi_stream_t stream) {
    return block_step(n, b, dA, dQ, npairs, hPairs, dV, dD, true, stream);
}

}  // extern "C"
