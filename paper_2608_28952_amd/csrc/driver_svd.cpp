// driver_svd.cpp -- host orchestration of the one-sided block Jacobi SVD
// (Alg. 6, §6) on one GPU.
//
// Per sweep, per round r of the pair schedule (N/2 disjoint column-block pairs):
//   Gram   A_hat_p = G(:,[I,J])^T G(:,[I,J]) (eq. SVD_subproblem), row-chunked
//   K1     subproblem kernel on A_hat_p (skip when every column pair of the
//          block is already orthogonal to tol) -> V_hat_p
//   K2'    G(:,[I,J]) <- G(:,[I,J]) V_hat_p and V(:,[I,J]) <- V(:,[I,J]) V_hat_p
// The sweeps stop when a whole sweep rotates no pair ("the columns of G are
// nearly orthogonal").  Then Sigma = column norms, U = G Sigma^+, sorted by
// descending sigma.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "jx_common.hpp"
#include "jx_host.hpp"
#include "jx_prof.hpp"

namespace jx {

void launch_copy_rect(int m, int n, const double *src, int lds_, double *dst, int ldd, int mpad, int npad,
                      hipStream_t s);

static int svd_block(int n) { return n > 512 ? 64 : 32; }

SvdPlan plan_svd(int m, int n, const jacobi_opts &o) {
    SvdPlan p{};
    p.m = m;
    p.n = n;
    p.b = o.block > 0 ? o.block : svd_block(n);
    const int unit = std::max(2 * p.b, 128);
    p.npad = std::max(unit, (n + unit - 1) / unit * unit);
    p.nchunks = std::max(1, std::min(32, (m + 1023) / 1024));
    const int rows = std::max(128, ((m + p.nchunks - 1) / p.nchunks + 127) / 128 * 128);
    p.mpad = rows * p.nchunks;
    p.N = p.npad / p.b;
    p.H = p.N / 2;
    p.R = (o.ordering == JACOBI_ORDER_ANTIDIAG) ? p.N : p.N - 1;
    p.vectors = o.want_vectors != 0;
    p.mixed = o.precision != JACOBI_PREC_FP64;
    p.refine = p.mixed || o.refine == 1 || (o.refine < 0 && n >= 256);
    const size_t m2sq = (size_t)(2 * p.b) * (2 * p.b);
    WorkspaceBuilder wb;
    p.off_g = wb.add(sizeof(double) * (size_t)p.mpad * p.npad);
    p.off_v = wb.add(sizeof(double) * (size_t)p.npad * p.npad);
    // one V_hat and one flag set per round of a sweep: the V update of round
    // r runs later, on a second stream (run_svd)
    p.off_vhat = wb.add(sizeof(double) * (size_t)p.R * p.H * m2sq);
    p.off_flags = wb.add(sizeof(int) * (size_t)p.R * p.H);
    p.off_pairs = wb.add(sizeof(int) * 2 * (size_t)p.R * p.H);
    p.off_force = wb.add(sizeof(int) * (size_t)p.R * p.H);
    p.off_partial = wb.add(sizeof(double) * (size_t)p.H * p.nchunks * m2sq);
    p.off_ahat = wb.add(sizeof(double) * p.H * m2sq);
    p.off_meas = wb.add(sizeof(double) * (size_t)p.R * p.H);
    p.off_cnt = wb.add(sizeof(int) * 4);
    p.off_sigma = wb.add(sizeof(double) * p.npad);
    p.off_rank = wb.add(sizeof(int) * p.npad);
    if (p.mixed) {
        p.off_g32 = wb.add(sizeof(float) * (size_t)p.mpad * p.npad);
        p.off_v32 = wb.add(sizeof(float) * (size_t)p.npad * p.npad);
        p.off_vhat32 = wb.add(sizeof(float) * (size_t)p.R * p.H * m2sq);
    }
    if (p.refine) {
        p.off_g0 = wb.add(sizeof(double) * (size_t)p.mpad * p.npad);
        p.off_t1 = wb.add(sizeof(double) * (size_t)p.npad * p.npad);
        p.off_t2 = wb.add(sizeof(double) * (size_t)p.npad * p.npad);
    }
    p.total = wb.total();
    return p;
}

// Rounds padded to N/2 pairs (see the eigensolver driver).
void padded_rounds_pub(int N, int ordering, std::vector<int> &pairs, std::vector<int> &force);

// The second stream of a solve and its two events (ordering within one
// device only, so no system-scope fence).
struct SideStream {
    hipStream_t sq = nullptr;
    hipEvent_t ev_go = nullptr, ev_done = nullptr;
    SideStream() {
        JX_HIP(hipStreamCreateWithFlags(&sq, hipStreamNonBlocking));
        const unsigned fl = hipEventDisableTiming | hipEventDisableSystemFence;
        JX_HIP(hipEventCreateWithFlags(&ev_go, fl));
        JX_HIP(hipEventCreateWithFlags(&ev_done, fl));
    }
    ~SideStream() {
        if (sq) (void)hipStreamSynchronize(sq);
        if (ev_go) (void)hipEventDestroy(ev_go);
        if (ev_done) (void)hipEventDestroy(ev_done);
        if (sq) (void)hipStreamDestroy(sq);
    }
    SideStream(const SideStream &) = delete;
    SideStream &operator=(const SideStream &) = delete;
};

int run_svd(int m, int n, const double *dG, int ldg, double *dS, double *dU, int ldu, double *dV, int ldv,
            void *dWork, size_t workBytes, const jacobi_opts &o, jacobi_info *info, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    jacobi_info inf{};
    SvdPlan p = plan_svd(m, n, o);
    DeviceBuffer own;
    char *ws = static_cast<char *>(dWork);
    if (!ws) {
        own.alloc(p.total);
        ws = own.ptr;
    } else if (workBytes < p.total) {
        return -100;
    }
    double *G = reinterpret_cast<double *>(ws + p.off_g);
    double *V = reinterpret_cast<double *>(ws + p.off_v);
    double *Vh = reinterpret_cast<double *>(ws + p.off_vhat);
    int *flags = reinterpret_cast<int *>(ws + p.off_flags);
    int *pairs = reinterpret_cast<int *>(ws + p.off_pairs);
    int *force = reinterpret_cast<int *>(ws + p.off_force);
    double *partial = reinterpret_cast<double *>(ws + p.off_partial);
    double *ahat = reinterpret_cast<double *>(ws + p.off_ahat);
    double *meas = reinterpret_cast<double *>(ws + p.off_meas);
    int *cnt = reinterpret_cast<int *>(ws + p.off_cnt);
    double *sigma = reinterpret_cast<double *>(ws + p.off_sigma);
    int *rank = reinterpret_cast<int *>(ws + p.off_rank);

    std::vector<int> hp, hf;
    padded_rounds_pub(p.N, o.ordering, hp, hf);
    const bool any_force = std::any_of(hf.begin(), hf.end(), [](int v) { return v != 0; });
    JX_HIP(hipMemcpyAsync(pairs, hp.data(), sizeof(int) * hp.size(), hipMemcpyHostToDevice, s));
    JX_HIP(hipMemcpyAsync(force, hf.data(), sizeof(int) * hf.size(), hipMemcpyHostToDevice, s));
    launch_copy_rect(m, n, dG, ldg, G, p.mpad, p.mpad, p.npad, s);
    launch_set_identity(p.npad, p.npad, V, p.npad, s);
    double *G0 = nullptr, *T1 = nullptr, *T2 = nullptr;
    if (p.refine) {
        G0 = reinterpret_cast<double *>(ws + p.off_g0);
        T1 = reinterpret_cast<double *>(ws + p.off_t1);
        T2 = reinterpret_cast<double *>(ws + p.off_t2);
        JX_HIP(hipMemcpyAsync(G0, G, sizeof(double) * (size_t)p.mpad * p.npad, hipMemcpyDeviceToDevice, s));
    }
    const double tol = o.tol > 0.0 ? o.tol : std::sqrt((double)m) * 2.220446049250313e-16;
    const int m2 = 2 * p.b;
    struct PinnedInt {
        int *ptr = nullptr;
        PinnedInt() { JX_HIP(hipHostMalloc(reinterpret_cast<void **>(&ptr), sizeof(int) * 4, hipHostMallocDefault)); }
        ~PinnedInt() { if (ptr) (void)hipHostFree(ptr); }
    } hcnt;
    std::vector<double> hmeas((size_t)p.R * p.H);
    const bool verbose = std::getenv("JACOBI_VERBOSE") != nullptr;

    float *G32 = p.mixed ? reinterpret_cast<float *>(ws + p.off_g32) : nullptr;
    float *V32 = p.mixed ? reinterpret_cast<float *>(ws + p.off_v32) : nullptr;
    float *Vh32 = p.mixed ? reinterpret_cast<float *>(ws + p.off_vhat32) : nullptr;
    bool f32 = false;
    int sweeps = 0, sweeps32 = 0, status = 1;
    double last_meas = 0.0;
    // V is read only after a sweep, so each round's V update runs on a second
    // stream, on at most CUs - H CUs, once the next round's Gram blocks are
    // done: beside that round's subproblems, which hold H CUs.  Round r keeps
    // its own V_hat and flags for it; the solve's stream joins once a sweep.
    SideStream side;
    const size_t m2sq = (size_t)m2 * m2;
    auto vhat_r = [&](int r) { return Vh + (size_t)r * p.H * m2sq; };
    auto vhat32_r = [&](int r) { return Vh32 + (size_t)r * p.H * m2sq; };
    auto flags_r = [&](int r) { return flags + (size_t)r * p.H; };
    auto update_v = [&](int r) {  // after round r's subproblems and round r + 1's Gram blocks
        JX_HIP(hipEventRecord(side.ev_go, s));
        JX_HIP(hipStreamWaitEvent(side.sq, side.ev_go, 0));
        const int *pr = pairs + (size_t)2 * r * p.H;
        ProfScope ps(PROF_UPDATE_Q, side.sq, (double)p.H * 2.0 * p.npad * m2 * m2,
                     (double)p.H * 2.0 * p.npad * m2 * (f32 ? sizeof(float) : sizeof(double)));
        if (f32) launch_update_q32(p.b, p.H, pr, V32, p.npad, p.npad, vhat32_r(r), flags_r(r), side.sq, p.H);
        else launch_update_q(p.b, p.H, pr, V, p.npad, p.npad, vhat_r(r), flags_r(r), side.sq, p.H);
    };
    auto sweep_once = [&]() -> int {  // returns rotated pair count
        JX_HIP(hipMemsetAsync(cnt, 0, sizeof(int), s));
        for (int r = 0; r < p.R; ++r) {
            const int *pr = pairs + (size_t)2 * r * p.H;
            {
                ProfScope ps(PROF_GRAM, s, (double)p.H * 2.0 * p.mpad * m2 * m2,
                             (double)p.H * p.mpad * m2 * (f32 ? sizeof(float) : sizeof(double)));
                if (f32)
                    launch_gram32(p.b, p.H, pr, G32, p.mpad, p.mpad, p.nchunks, reinterpret_cast<float *>(partial),
                                  ahat, s);
                else launch_gram(p.b, p.H, pr, G, p.mpad, p.mpad, p.nchunks, partial, ahat, s);
            }
            if (r > 0) update_v(r - 1);
            SubArgs a{};
            a.mode = SUB_GRAM;
            a.m2 = m2;
            a.count = p.H;
            a.pairs = pr;
            a.ahat = ahat;
            a.vout = vhat_r(r);
            a.flags = flags_r(r);
            a.skip_thr = tol;
            a.inner_sweeps = o.inner_max_sweeps;
            a.inner_off = meas + (size_t)r * p.H;
            a.force_skip = any_force ? force + (size_t)r * p.H : nullptr;
            a.rot_count = cnt;
            if (f32) a.vout32 = vhat32_r(r);
            {
                ProfScope ps(PROF_SUBPROBLEM, s, 0.0, 0.0);
                launch_subproblem(a, s);
            }
            {
                ProfScope ps(PROF_UPDATE_Q, s, (double)p.H * 2.0 * p.mpad * m2 * m2,
                             (double)p.H * 2.0 * p.mpad * m2 * (f32 ? sizeof(float) : sizeof(double)));
                if (f32) launch_update_q32(p.b, p.H, pr, G32, p.mpad, p.mpad, vhat32_r(r), flags_r(r), s);
                else launch_update_q(p.b, p.H, pr, G, p.mpad, p.mpad, vhat_r(r), flags_r(r), s);
            }
        }
        update_v(p.R - 1);
        JX_HIP(hipEventRecord(side.ev_done, side.sq));
        JX_HIP(hipStreamWaitEvent(s, side.ev_done, 0));
        JX_HIP(hipMemcpyAsync(hcnt.ptr, cnt, sizeof(int), hipMemcpyDeviceToHost, s));
        JX_HIP(hipMemcpyAsync(hmeas.data(), meas, sizeof(double) * hmeas.size(), hipMemcpyDeviceToHost, s));
        JX_HIP(hipStreamSynchronize(s));
        last_meas = 0.0;
        for (size_t i = 0; i < hmeas.size(); ++i)
            if (!any_force || !hf[i]) last_meas = std::max(last_meas, hmeas[i]);
        if (verbose)
            std::fprintf(stderr, "[jacobi_svd] sweep %d %s rotated pairs %d max cos %.3e\n", sweeps,
                         f32 ? "fp32" : "fp64", hcnt.ptr[0], last_meas);
        return hcnt.ptr[0];
    };
    // cond(G) estimated from the column norms of the FP32 iterate (max / min
    // over the nonzero columns), which approach the singular values as the
    // columns become orthogonal.
    std::vector<double> hnorm(n);
    auto cond32 = [&]() -> double {
        launch_col_norms32(m, n, G32, p.mpad, sigma, s);
        JX_HIP(hipMemcpyAsync(hnorm.data(), sigma, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        JX_HIP(hipStreamSynchronize(s));
        double mx = 0.0, mn = HUGE_VAL;
        for (int j = 0; j < n; ++j) {
            mx = std::max(mx, hnorm[j]);
            if (hnorm[j] > 0.0) mn = std::min(mn, hnorm[j]);
        }
        return mn < HUGE_VAL ? mx / mn : 1.0;
    };
    // Sweeps until a sweep rotates no pair (stop <= 0) or the largest relative
    // cosine drops to stop.  Returns 0, 1 (cap), 2 (non-finite), 4 (the FP32
    // phase stagnates or has no more to gain).
    auto phase = [&](double stop, int cap) -> int {
        double prev = -1.0;
        for (;;) {
            if (sweeps >= cap) return 1;
            const int rot = sweep_once();
            ++sweeps;
            if (f32) ++sweeps32;
            if (!std::isfinite(last_meas)) return 2;
            if (rot == 0 || (stop > 0.0 && last_meas <= stop)) return 0;
            if (f32 && prev >= 0.0 && last_meas < 1e-3 && last_meas > 0.5 * prev) return 4;
            // V from the FP32 phase is accurate to about u32 = 2^-24, so G0 V
            // gives the columns of the smallest singular values cosines of
            // about u32 cond(G) again (3.2 u32 cond(G) measured at cond =
            // 1e6): FP32 sweeps below that level are repeated in FP64.  The
            // phase ends once the largest cosine is within 2 u32 cond(G).
            if (f32 && last_meas <= 2.0 * 0x1p-24 * cond32()) return 4;
            prev = last_meas;
        }
    };
    // V <- V (3 I - V^T V) / 2, G = G0 V in FP64 from the original
    auto recompute = [&]() {
        const int np = p.npad;
        launch_gemm_f64('T', 'N', np, np, np, 1.0, V, np, V, np, 0.0, T1, np, s);
        JX_HIP(hipMemcpyAsync(T2, V, sizeof(double) * (size_t)np * np, hipMemcpyDeviceToDevice, s));
        launch_gemm_f64('N', 'N', np, np, np, -0.5, V, np, T1, np, 1.5, T2, np, s);
        JX_HIP(hipMemcpyAsync(V, T2, sizeof(double) * (size_t)np * np, hipMemcpyDeviceToDevice, s));
        launch_gemm_f64('N', 'N', p.mpad, np, np, 1.0, G0, p.mpad, V, np, 0.0, G, p.mpad, s);
    };
    const double switch_cos = 1e-5;
    if (p.mixed) {
        launch_cast_to_f32((size_t)p.mpad * p.npad, G, G32, s);
        launch_set_identity32(p.npad, V32, p.npad, s);
        f32 = true;
        status = phase(switch_cos, o.max_sweeps);
        f32 = false;
        if (status != 2) {
            launch_cast_to_f64((size_t)p.npad * p.npad, V32, V, s);
            recompute();
            status = phase(0.0, o.max_sweeps + 8);
        }
    } else {
        status = phase(0.0, o.max_sweeps);
    }
    if (status == 0 && p.refine) {
        recompute();
        status = phase(0.0, o.max_sweeps + 12);
    }
    if (status != 2) {
        launch_col_norms(m, n, G, p.mpad, sigma, s);
        if (o.sort) {
            launch_rank(n, sigma, -1, rank, s);
        } else {
            std::vector<int> id(n);
            for (int i = 0; i < n; ++i) id[i] = i;
            JX_HIP(hipMemcpyAsync(rank, id.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
        }
        launch_scatter_values(n, sigma, rank, dS, s);
        if (p.vectors) {
            if (dU) launch_scale_scatter(m, n, G, p.mpad, sigma, rank, dU, ldu, s);
            if (dV) launch_scatter_columns(n, n, V, p.npad, rank, dV, ldv, s);
        }
        JX_HIP(hipStreamSynchronize(s));
    }
    inf.status = status;
    inf.sweeps = sweeps;
    inf.sweeps_by_prec[1] = sweeps32;
    inf.sweeps_by_prec[2] = sweeps - sweeps32;
    inf.off_rel = last_meas;
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return status;
}

}  // namespace jx
