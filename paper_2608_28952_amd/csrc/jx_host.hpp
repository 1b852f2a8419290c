// jx_host.hpp -- host-side helpers shared by the drivers of libjacobi.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <mutex>
#include <vector>

#include "jx_common.hpp"

namespace jx {

// Sub-allocations of one device workspace, each aligned to 256 bytes.
struct WorkspaceBuilder {
    size_t off = 0;
    size_t add(size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    }
    size_t total() const { return off > 0 ? off : 256; }
};

// Library-owned device memory for calls that pass no workspace.
struct DeviceBuffer {
    char *ptr = nullptr;
    void alloc(size_t bytes) {
        void *p = nullptr;
        JX_HIP(hipMalloc(&p, bytes));
        ptr = static_cast<char *>(p);
    }
    ~DeviceBuffer() {
        if (ptr) (void)hipFree(ptr);
    }
};

// Per-device context (ctx.cpp), created on first use on a device and kept
// until the process ends: the second stream of the sweeps, events ordering
// the two streams, pinned host memory for the scalars read back per sweep.
// One solve at a time uses it: the drivers hold `mu` for the whole call.
struct DeviceCtx {
    static constexpr int NEV = 4;
    static constexpr size_t PINNED_BYTES = 4096;
    int device = 0;
    std::mutex mu;
    hipStream_t side = nullptr;
    hipEvent_t ev[NEV] = {};
    char *pinned = nullptr;
};
DeviceCtx &device_ctx();  // the current device's context (created on first use)
// Device address of the current device's static scratch array of the
// no-allocation entry point (looked up once per device).
void *noalloc_setup();

struct EigPlan {
    int n, npad, b, N, H, R;
    bool vectors, refine, mixed, need_q, temps, sorted, pivot;
    size_t off_ablk, off_q, off_v, off_flags, off_pairs, off_force, off_tiles, off_qmask, off_side, off_smap, off_xcopy, off_copy0, off_partial,
        off_scal, off_w, off_rank, off_a0, off_t1, off_t2, off_ablk32, off_q32, off_v32, off_ablk2, off_inv;
    size_t total;
};

struct SvdPlan {
    int m, n, mpad, npad, b, N, H, R, nchunks;
    bool vectors, refine, mixed;
    size_t off_g, off_v, off_vhat, off_flags, off_pairs, off_force, off_partial, off_ahat, off_meas,
        off_cnt, off_sigma, off_rank, off_g0, off_t1, off_t2, off_g32, off_v32, off_vhat32;
    bool qr;  // QR preprocessing (then the buffers below)
    size_t off_qb1, off_ra, off_rb, off_rc, off_x, off_ux, off_vx, off_rinv, off_tp, off_qscal, off_probe, off_inner,
        inner_bytes;
    size_t total;
};

EigPlan plan_eig(int n, const jacobi_opts &o);
SvdPlan plan_svd(int m, int n, const jacobi_opts &o);
int run_svd(int m, int n, const double *dG, int ldg, double *dS, double *dU, int ldu, double *dV, int ldv,
            void *dWork, size_t workBytes, const jacobi_opts &o, jacobi_info *info, hipStream_t s);
int make_schedule(int N, int ordering, std::vector<int> &pairs, std::vector<int> &sizes);
int run_eig(int n, const double *dA, int lda, char uplo, double *dW, double *dQ, int ldq,
            const double *dQ0, int ldq0, void *dWork, size_t workBytes, const jacobi_opts &o,
            jacobi_info *info, hipStream_t s);
size_t scalar_workspace(int n);
int run_eig_scalar(int n, const double *dA, int lda, char uplo, double *dW, double *dQ, int ldq, void *dWork,
                   size_t workBytes, const jacobi_opts &o, jacobi_info *info, hipStream_t s);
int run_subproblem(int count, int m2, const double *dAhat, double *dV, double *dD, int inner,
                   hipStream_t s);
int run_qr(int m, int n, const double *dG, int ldg, double *dQ, int ldq, double *dR, int ldr, hipStream_t s);
int run_gram_blocks(int m, int n, int b, const double *dG, int ldg, int npairs, const int *hPairs, bool f32,
                    double *dAhat, hipStream_t s);
// f32: the same step by the FP32 kernels (inputs rounded, results widened)
int run_pivot_step(int n, int b, double *dA, int npairs, const int *hPairs, double *dV, int *dPerm, hipStream_t s);
int run_block_step(int n, int b, double *dA, double *dQ, int npairs, const int *hPairs,
                   const double *dV, const double *dD, bool f32, hipStream_t s);

}  // namespace jx
