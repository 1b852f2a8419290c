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

// Largest relative cosine at which the SVD sweeps refine V inside the
// quadratic phase, and the decrease the last sweep must show (run_svd).
constexpr double EARLY_REFINE_COS = 1e-6;
constexpr double EARLY_REFINE_DROP = 1e-2;

static int svd_block(int n) { return n > 512 ? 64 : 32; }

SvdPlan plan_svd(int m, int n, const jacobi_opts &o) {
    SvdPlan p{};
    p.m = m;
    p.n = n;
    p.b = o.block > 0 ? o.block : svd_block(n);
    const int unit = std::max(2 * p.b, 128);
    p.npad = std::max(unit, (n + unit - 1) / unit * unit);
    p.N = p.npad / p.b;
    p.H = p.N / 2;
    // Gram row chunks: chunks of up to 1024 rows, more (down to 128 rows) when
    // the pairs alone give too few workgroups (about 256 fill the chip)
    const int fill = std::min((256 + p.H - 1) / p.H, (m + 127) / 128);
    p.nchunks = std::max(1, std::min(32, std::max((m + 1023) / 1024, fill)));
    const int rows = std::max(128, ((m + p.nchunks - 1) / p.nchunks + 127) / 128 * 128);
    p.mpad = rows * p.nchunks;
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
    // QR preprocessing (§6): G = Q R, one-sided Jacobi on R^T (n x n) by a
    // nested plain solve, U = Q V_R.  Default on; the plain solve's buffers
    // above stay reserved for the fallback when the Gram matrix is not
    // numerically positive definite or a singular value is zero.
    p.qr = o.precondition != 0 && n >= 2;
    if (p.qr) {
        const size_t np2 = sizeof(double) * (size_t)p.npad * p.npad;
        p.off_qb1 = wb.add(sizeof(double) * (size_t)p.mpad * p.npad);
        p.off_ra = wb.add(np2);
        p.off_rb = wb.add(np2);
        p.off_rc = wb.add(np2);
        p.off_x = wb.add(np2);
        p.off_ux = wb.add(np2);
        p.off_vx = wb.add(np2);
        p.off_rinv = wb.add(sizeof(double) * (size_t)p.npad * 128);
        p.off_tp = wb.add(sizeof(double) * (size_t)std::max(p.mpad, p.npad) * 128);
        p.off_qscal = wb.add(sizeof(double) * ((size_t)p.npad + 8));
        p.off_probe = wb.add(sizeof(double) * ((2 * (size_t)p.npad + (size_t)p.mpad) * 128 + 136));
        jacobi_opts oi = o;
        oi.precondition = 0;
        p.inner_bytes = plan_svd(n, n, oi).total;
        p.off_inner = wb.add(p.inner_bytes);
    }
    p.total = wb.total();
    return p;
}

// Rounds padded to N/2 pairs (see the eigensolver driver).
void padded_rounds_pub(int N, int ordering, std::vector<int> &pairs, std::vector<int> &force);

// The second stream of a solve and its two events: those of the device
// context (ordering within one device only, so no system-scope fence).
struct SideStream {
    hipStream_t sq = nullptr;
    hipEvent_t ev_go = nullptr, ev_done = nullptr;
    explicit SideStream(DeviceCtx &c) : sq(c.side), ev_go(c.ev[0]), ev_done(c.ev[1]) {}
    ~SideStream() {
        if (sq) (void)hipStreamSynchronize(sq);
    }
    SideStream(const SideStream &) = delete;
    SideStream &operator=(const SideStream &) = delete;
};

// ---------------------------------------------------------------------------
// QR preprocessing (§6, "Preprocessing with QR")
// ---------------------------------------------------------------------------

// One CholeskyQR pass on the padded src (mpad x npad, the leading n columns
// real, the rest zero): W = src^T src (+ shift I), W = R^T R by blocked
// Cholesky (128-blocks: the diagonal block factored and inverted in one
// workgroup, its block row R_kj = R_kk^{-T} W_kj and the trailing update by
// FP64 MFMA GEMMs), then, if dst, dst = src R^{-1} by block columns (panel j:
// src_j - dst_{<j} R_{<j,j}, times R_jj^{-1}).  R is written to Rout
// (npad x npad, zero below the diagonal, identity on the padding).  Returns
// false if a pivot was not positive and finite.
struct QrScratch {
    double *rinv;   // npad x 128: the inverted diagonal blocks, block k at rinv + k 128^2
    double *tp;     // max(mpad, npad) x 128 panel temporary
    double *scal;   // npad + 8 doubles: partial sums, then scalars
    int *flag;
};

static bool chol_qr_pass(int mpad, int n, int npad, const double *src, double *dst, double *Rout, double shift,
                         const QrScratch &q, hipStream_t s) {
    constexpr int B = 128;
    launch_gemm_f64('T', 'N', npad, npad, mpad, 1.0, src, mpad, src, mpad, 0.0, Rout, npad, s);
    launch_unit_pad_diag(n, npad, Rout, npad, s);
    if (shift > 0.0) launch_shift_diag(n, shift, Rout, npad, s);
    launch_fill_int(q.flag, 1, 0, s);
    for (int k0 = 0; k0 < npad; k0 += B) {
        double *rinv = q.rinv + (size_t)(k0 / B) * B * B;
        launch_chol_diag(Rout, npad, k0, rinv, q.flag, s);
        const int rest = npad - k0 - B;
        if (rest <= 0) break;
        double *wrow = Rout + (size_t)(k0 + B) * npad + k0;  // W(k0:k0+B, k0+B:npad)
        // R_kj = R_kk^{-T} W_kj into the panel temporary, then back in place
        launch_gemm_f64('T', 'N', B, rest, B, 1.0, rinv, B, wrow, npad, 0.0, q.tp, B, s);
        JX_HIP(hipMemcpy2DAsync(wrow, sizeof(double) * npad, q.tp, sizeof(double) * B, sizeof(double) * B, rest,
                                hipMemcpyDeviceToDevice, s));
        // trailing W_jj' -= R_kj^T R_kj'
        double *trail = Rout + (size_t)(k0 + B) * npad + k0 + B;
        launch_gemm_f64('T', 'N', rest, rest, B, -1.0, wrow, npad, wrow, npad, 1.0, trail, npad, s);
    }
    launch_zero_lower(npad, Rout, npad, s);
    int hflag = 0;
    JX_HIP(hipMemcpyAsync(&hflag, q.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    JX_HIP(hipStreamSynchronize(s));
    if (hflag) return false;
    if (dst) {
        JX_HIP(hipMemcpyAsync(dst, src, sizeof(double) * (size_t)mpad * npad, hipMemcpyDeviceToDevice, s));
        for (int j = 0; j < npad / B; ++j) {
            double *dj = dst + (size_t)j * B * mpad;
            if (j > 0)
                launch_gemm_f64('N', 'N', mpad, B, B * j, -1.0, dst, mpad, Rout + (size_t)j * B * npad, npad, 1.0, dj,
                                mpad, s);
            launch_gemm_f64('N', 'N', mpad, B, B, 1.0, dj, mpad, q.rinv + (size_t)j * B * B, B, 0.0, q.tp, mpad, s);
            JX_HIP(hipMemcpyAsync(dj, q.tp, sizeof(double) * (size_t)mpad * B, hipMemcpyDeviceToDevice, s));
        }
    }
    return true;
}

// CholeskyQR2 with a safeguard: R_1 from the first pass, Q_1 = G R_1^{-1},
// then the second pass on Q_1; R = R_2 R_1.  The first pass is repeated with
// the shift 11 (m n + n (n + 1)) u ||G||_F^2 (shifted CholeskyQR, Fukaya et al.
// 2020), followed by CholeskyQR2 on its Q_1, when its Cholesky meets a pivot
// that is not positive and finite, or when the diagonal of R_1 spans more than
// 1e7 (cond(G) near u^{-1/2}: the unshifted Gram matrix has lost the small
// singular values).  src/dst: the padded G copy and a second mpad x npad
// buffer; on return *qout is the buffer holding Q (when want_q) and `rs`
// the factors in the order they were made (R = rs.back() ... rs.front()).
// Returns false when a pass fails even so.
// max |r_ii| / min |r_ii| over the leading n diagonal entries of R (a lower
// bound of its condition number); infinite for a zero or non-finite entry.
static double diag_span(int n, const double *R, int ldr, const QrScratch &q, hipStream_t s) {
    launch_diag_of(n, R, ldr, q.scal, s);
    std::vector<double> d(n);
    JX_HIP(hipMemcpyAsync(d.data(), q.scal, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    JX_HIP(hipStreamSynchronize(s));
    double mx = 0.0, mn = HUGE_VAL;
    for (double v : d) {
        if (!std::isfinite(v)) return HUGE_VAL;
        mx = std::max(mx, std::fabs(v));
        mn = std::min(mn, std::fabs(v));
    }
    return mn > 0.0 ? mx / mn : HUGE_VAL;
}

// Backward error of the factorization on a fixed probe block X (n x 128):
// ||G X - Q (R X)||_F / ||G X||_F with R X = R_last (... (R_1 X)).  The
// explicitly inverted diagonal blocks of the panel solves lose accuracy with
// their own condition, e.g. for (nearly) dependent columns inside one block;
// the probe sees such a factorization's error at the cost of a few thin
// GEMMs.  G: a fresh padded copy of the input (mpad x npad); probe: (2 npad
// + mpad) x 128 + 136 doubles.
static double qr_probe_error(int mpad, int n, int npad, const double *G, const double *Q,
                             const std::vector<double *> &rs, double *probe, const QrScratch &q, hipStream_t s) {
    constexpr int C = 128;
    double *X = probe, *Y = probe + (size_t)npad * C, *GX = probe + 2 * (size_t)npad * C;
    double *part = GX + (size_t)mpad * C;  // C column partials, then the two sums
    launch_fill_probe(n, npad, C, X, s);
    launch_gemm_f64('N', 'N', mpad, C, npad, 1.0, G, mpad, X, npad, 0.0, GX, mpad, s);
    for (double *R : rs) {  // X <- R X, the first factor first
        launch_gemm_f64('N', 'N', npad, C, npad, 1.0, R, npad, X, npad, 0.0, Y, npad, s);
        std::swap(X, Y);
    }
    // Q (R X) into the free half of the tile buffer, then the difference
    launch_gemm_f64('N', 'N', mpad, C, npad, 1.0, Q, mpad, X, npad, 0.0, q.tp, mpad, s);
    launch_diff_frob2(mpad, C, GX, q.tp, mpad, part, part + C, s);
    launch_frob2(mpad, C, GX, mpad, part, part + C + 1, s);
    double h[2] = {0.0, 0.0};
    JX_HIP(hipMemcpyAsync(h, part + C, sizeof(h), hipMemcpyDeviceToHost, s));
    JX_HIP(hipStreamSynchronize(s));
    return h[1] > 0.0 ? std::sqrt(h[0] / h[1]) : 0.0;
}

static bool cholesky_qr2(int m, int n, int mpad, int npad, double *src, double *dst, double *const Rbuf[3],
                         const QrScratch &q, bool want_q, double **qout, std::vector<double *> &rs, hipStream_t s) {
    rs.clear();
    double *cur = src, *nxt = dst;
    bool shifted = !chol_qr_pass(mpad, n, npad, cur, nxt, Rbuf[0], 0.0, q, s);
    if (!shifted) shifted = !(diag_span(n, Rbuf[0], npad, q, s) <= 1e7);
    if (shifted) {  // (restarts from G: the unshifted pass above wrote only R_1 and Q_1)
        launch_frob2(m, n, cur, mpad, q.scal, q.scal + npad, s);
        double fro2 = 0.0;
        JX_HIP(hipMemcpyAsync(&fro2, q.scal + npad, sizeof(double), hipMemcpyDeviceToHost, s));
        JX_HIP(hipStreamSynchronize(s));
        const double shift = 11.0 * ((double)m * n + (double)n * (n + 1)) * 2.220446049250313e-16 * fro2;
        if (!std::isfinite(shift) || !chol_qr_pass(mpad, n, npad, cur, nxt, Rbuf[0], shift, q, s)) return false;
        rs.push_back(Rbuf[0]);
        std::swap(cur, nxt);
        if (!chol_qr_pass(mpad, n, npad, cur, nxt, Rbuf[1], 0.0, q, s)) return false;
        rs.push_back(Rbuf[1]);
    } else {
        rs.push_back(Rbuf[0]);
    }
    std::swap(cur, nxt);
    double *Rl = Rbuf[rs.size()];
    if (!chol_qr_pass(mpad, n, npad, cur, want_q ? nxt : nullptr, Rl, 0.0, q, s)) return false;
    rs.push_back(Rl);
    // the last pass starts from a Q_1 with orthonormal columns to a few
    // digits, so its R is close to I; a diagonal spanning more than 10 means
    // Q_1 was (numerically) rank deficient and the factorization is not to
    // be trusted
    if (diag_span(n, Rl, npad, q, s) > 10.0) return false;
    *qout = nxt;
    return true;
}

// QR_FALLBACK: not used (the plain solve runs instead), else the solve's status.
constexpr int QR_FALLBACK = -1000;
static int svd_qr(const SvdPlan &p, char *ws, const double *dG, int ldg, double *dS, double *dU, int ldu,
                  double *dV, int ldv, const jacobi_opts &o, jacobi_info &inf, hipStream_t s) {
    const int m = p.m, n = p.n, mpad = p.mpad, npad = p.npad;
    double *Gc = reinterpret_cast<double *>(ws + p.off_g);
    double *B1 = reinterpret_cast<double *>(ws + p.off_qb1);
    double *Ra = reinterpret_cast<double *>(ws + p.off_ra);
    double *Rb = reinterpret_cast<double *>(ws + p.off_rb);
    double *Rc = reinterpret_cast<double *>(ws + p.off_rc);
    double *X = reinterpret_cast<double *>(ws + p.off_x);
    double *Ux = reinterpret_cast<double *>(ws + p.off_ux);
    double *Vx = reinterpret_cast<double *>(ws + p.off_vx);
    QrScratch q{reinterpret_cast<double *>(ws + p.off_rinv), reinterpret_cast<double *>(ws + p.off_tp),
                reinterpret_cast<double *>(ws + p.off_qscal),
                reinterpret_cast<int *>(ws + p.off_qscal + sizeof(double) * ((size_t)npad + 6))};
    const bool vec = p.vectors;
    launch_copy_rect(m, n, dG, ldg, Gc, mpad, mpad, npad, s);
    std::vector<double *> Rs;
    double *Rbuf[3] = {Ra, Rb, Rc};
    double *Qf = nullptr;
    if (!cholesky_qr2(m, n, mpad, npad, Gc, B1, Rbuf, q, true, &Qf, Rs, s)) return QR_FALLBACK;
    double *cur = Qf == Gc ? B1 : Gc;  // the other big buffer (free)
    launch_copy_rect(m, n, dG, ldg, cur, mpad, mpad, npad, s);
    if (!(qr_probe_error(mpad, n, npad, cur, Qf, Rs, reinterpret_cast<double *>(ws + p.off_probe), q, s) <= 1e-13))
        return QR_FALLBACK;
    // X = R^T = R_1^T R_2^T ... (the last factor applied last)
    launch_gemm_f64('T', 'T', npad, npad, npad, 1.0, Rs[0], npad, Rs[1], npad, 0.0, X, npad, s);
    if (Rs.size() == 3) {  // X <- X R_3^T, into R_1's buffer (no longer needed)
        launch_gemm_f64('N', 'T', npad, npad, npad, 1.0, X, npad, Rs[2], npad, 0.0, Rs[0], npad, s);
        std::swap(X, Rs[0]);
    }
    // one-sided Jacobi on R^T: R^T V_R = U_R Sigma, so G = Q R = (Q V_R) Sigma U_R^T
    jacobi_opts oi = o;
    oi.precondition = 0;
    if (vec) {
        JX_HIP(hipMemsetAsync(Ux, 0, sizeof(double) * (size_t)npad * npad, s));
        JX_HIP(hipMemsetAsync(Vx, 0, sizeof(double) * (size_t)npad * npad, s));
    }
    jacobi_info ii{};
    const int st = run_svd(n, n, X, npad, dS, vec ? Ux : nullptr, npad, vec ? Vx : nullptr, npad,
                           ws + p.off_inner, p.inner_bytes, oi, &ii, s);
    if (st < 0 || st >= 2) return st;  // argument / workspace errors, non-finite, HIP error
    inf = ii;
    if (!vec) return st;  // 0, or 1 (not converged: the last iterate's values)
    // a zero singular value leaves a zero column in U_R: the plain solve
    // handles that case (its V is an accumulated rotation)
    std::vector<double> hs(n);
    JX_HIP(hipMemcpyAsync(hs.data(), dS, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    JX_HIP(hipStreamSynchronize(s));
    if (*std::min_element(hs.begin(), hs.end()) <= 0.0) return QR_FALLBACK;
    // U = Q V_R (FP64 MFMA), its leading m x n part to dU
    launch_gemm_f64('N', 'N', mpad, npad, npad, 1.0, Qf, mpad, Vx, npad, 0.0, cur, mpad, s);
    launch_copy_rect(m, n, cur, mpad, dU, ldu, m, n, s);
    // V = U_R, the normalised columns of R^T V_R: orthogonal only to about
    // u cond(G); Newton-Schulz steps V <- V (3 I - V^T V) / 2 until one starts
    // from ||V^T V - I||_F <= 1e-8 (each squares the deviation; the residual
    // changes by sigma_i |dv_i| = O(u ||G||))
    double *T1 = Rb, *T2 = Rc;
    for (int it = 0; it < 5; ++it) {
        launch_gemm_f64('T', 'N', npad, npad, npad, 1.0, Ux, npad, Ux, npad, 0.0, T1, npad, s);
        launch_dev_identity(n, T1, npad, q.scal, q.scal + npad, s);
        double dev2 = 0.0;
        JX_HIP(hipMemcpyAsync(&dev2, q.scal + npad, sizeof(double), hipMemcpyDeviceToHost, s));
        JX_HIP(hipStreamSynchronize(s));
        if (!(dev2 <= 1e-2)) return QR_FALLBACK;  // too far from orthogonal for the iteration
        if (dev2 <= 1e-30) break;
        JX_HIP(hipMemcpyAsync(T2, Ux, sizeof(double) * (size_t)npad * npad, hipMemcpyDeviceToDevice, s));
        launch_gemm_f64('N', 'N', npad, npad, npad, -0.5, Ux, npad, T1, npad, 1.5, T2, npad, s);
        std::swap(Ux, T2);
        if (dev2 <= 1e-16) break;
    }
    launch_copy_rect(n, n, Ux, npad, dV, ldv, n, n, s);
    JX_HIP(hipStreamSynchronize(s));
    return st;
}

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
    {
        // a non-finite entry: status 2 before any sweep (the sweeps' largest
        // relative cosine is a max that would pass over a NaN)
        double *part = reinterpret_cast<double *>(ws + p.off_sigma);
        double *out = reinterpret_cast<double *>(ws + p.off_meas);
        launch_count_nonfinite(m, n, dG, ldg, part, out, s);
        double bad = 0.0;
        JX_HIP(hipMemcpyAsync(&bad, out, sizeof(double), hipMemcpyDeviceToHost, s));
        JX_HIP(hipStreamSynchronize(s));
        if (bad != 0.0) {
            inf.status = 2;
            inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (info) *info = inf;
            return 2;
        }
    }
    if (p.qr) {
        const int rc = svd_qr(p, ws, dG, ldg, dS, dU, ldu, dV, ldv, o, inf, s);
        if (rc != QR_FALLBACK) {
            inf.status = rc;
            inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (info) *info = inf;
            return rc;
        }
        inf = jacobi_info{};
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
    padded_rounds_pub(p.N, o.ordering == JACOBI_ORDER_ANTIDIAG ? JACOBI_ORDER_ANTIDIAG : JACOBI_ORDER_ROUND_ROBIN, hp,
                      hf);
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
    DeviceCtx &ctx = device_ctx();
    std::lock_guard<std::mutex> lk(ctx.mu);
    struct {
        int *ptr;
    } hcnt{reinterpret_cast<int *>(ctx.pinned)};
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
    SideStream side(ctx);
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
    // phase stagnates or has no more to gain), 5 (early > 0: a sweep in the
    // quadratic phase left the largest cosine at or below early, having cut
    // it by at least EARLY_REFINE_DROP).
    auto phase = [&](double stop, int cap, double early = 0.0) -> int {
        double prev = -1.0;
        for (;;) {
            if (sweeps >= cap) return 1;
            const int rot = sweep_once();
            ++sweeps;
            if (f32) ++sweeps32;
            if (!std::isfinite(last_meas)) return 2;
            if (rot == 0 || (stop > 0.0 && last_meas <= stop)) return 0;
            if (early > 0.0 && prev > 0.0 && sweeps < cap && last_meas <= early &&
                last_meas <= EARLY_REFINE_DROP * prev)
                return 5;
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
    // V <- V (3 I - V^T V) / 2 (ns times), G = G0 V in FP64 from the original.
    // After the FP32 phase V is orthogonal to about 1e-6; one step leaves
    // 1e-12, which G0 V turns into cosines of about cond(G) 1e-12 (1.4e-6 at
    // cond = 1e6, in the way of the later refinement), so the switch takes two.
    auto recompute = [&](int ns) {
        const int np = p.npad;
        for (int k = 0; k < ns; ++k) {
            launch_gemm_f64('T', 'N', np, np, np, 1.0, V, np, V, np, 0.0, T1, np, s);
            JX_HIP(hipMemcpyAsync(T2, V, sizeof(double) * (size_t)np * np, hipMemcpyDeviceToDevice, s));
            launch_gemm_f64('N', 'N', np, np, np, -0.5, V, np, T1, np, 1.5, T2, np, s);
            JX_HIP(hipMemcpyAsync(V, T2, sizeof(double) * (size_t)np * np, hipMemcpyDeviceToDevice, s));
        }
        launch_gemm_f64('N', 'N', p.mpad, np, np, 1.0, G0, p.mpad, V, np, 0.0, G, p.mpad, s);
    };
    const double switch_cos = 1e-5;
    // Sweeps to convergence with the refinement inside the quadratic phase.
    // Convergence is a sweep that rotates no pair; refined after it, the
    // recomputed G = G0 V carries cosines of rounding size above tol, which
    // take one more rotating sweep and one more check sweep.  Refined once a
    // sweep has left the largest cosine at or below EARLY_REFINE_COS (and cut
    // it by 100x: the quadratic phase), the sweep that finishes the
    // convergence also absorbs that rounding.  If more than two sweeps
    // follow, the refinement is repeated at the end.
    bool early_refined = false;
    auto to_conv = [&](int cap) {
        status = phase(0.0, cap, p.refine ? EARLY_REFINE_COS : 0.0);
        if (status == 5) {
            const int before = sweeps;
            recompute(1);
            status = phase(0.0, cap + 12);
            early_refined = status == 0 && sweeps - before <= 2;
        }
    };
    if (p.mixed) {
        launch_cast_to_f32((size_t)p.mpad * p.npad, G, G32, s);
        launch_set_identity32(p.npad, V32, p.npad, s);
        f32 = true;
        status = phase(switch_cos, o.max_sweeps);
        f32 = false;
        if (status != 2) {
            launch_cast_to_f64((size_t)p.npad * p.npad, V32, V, s);
            recompute(2);
            to_conv(o.max_sweeps + 8);
        }
    } else {
        to_conv(o.max_sweeps);
    }
    if (status == 0 && p.refine && !early_refined) {
        recompute(1);
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

// Gram blocks of one round on explicit data (kernel-level test hook): G (m x n,
// column-major, n a multiple of b) is copied into the SVD's padded layout (rows
// in the same row chunks as a solve of this size), rounded to FP32 when f32,
// and ahat[p] = [G_I G_J]^T [G_I G_J] (2b x 2b) for each listed pair.
int run_gram_blocks(int m, int n, int b, const double *dG, int ldg, int npairs, const int *hPairs, bool f32,
                    double *dAhat, hipStream_t s) {
    jacobi_opts o;
    jacobi_opts_default(&o);
    o.block = b;
    const SvdPlan p = plan_svd(m, n, o);
    const size_t m2sq = (size_t)(2 * b) * (2 * b);
    WorkspaceBuilder wb;
    const size_t o_g = wb.add(sizeof(double) * (size_t)p.mpad * p.npad);
    const size_t o_g32 = f32 ? wb.add(sizeof(float) * (size_t)p.mpad * p.npad) : 0;
    const size_t o_pr = wb.add(sizeof(int) * 2 * (size_t)npairs);
    const size_t o_part = wb.add(sizeof(double) * (size_t)npairs * p.nchunks * m2sq);
    DeviceBuffer buf;
    buf.alloc(wb.total());
    double *G = reinterpret_cast<double *>(buf.ptr + o_g);
    int *pairs = reinterpret_cast<int *>(buf.ptr + o_pr);
    JX_HIP(hipMemcpyAsync(pairs, hPairs, sizeof(int) * 2 * npairs, hipMemcpyHostToDevice, s));
    launch_copy_rect(m, n, dG, ldg, G, p.mpad, p.mpad, p.npad, s);
    if (f32) {
        float *G32 = reinterpret_cast<float *>(buf.ptr + o_g32);
        launch_cast_to_f32((size_t)p.mpad * p.npad, G, G32, s);
        launch_gram32(b, npairs, pairs, G32, p.mpad, p.mpad, p.nchunks, reinterpret_cast<float *>(buf.ptr + o_part),
                      dAhat, s);
    } else {
        launch_gram(b, npairs, pairs, G, p.mpad, p.mpad, p.nchunks, reinterpret_cast<double *>(buf.ptr + o_part),
                    dAhat, s);
    }
    JX_HIP(hipStreamSynchronize(s));
    return 0;
}

// The reduced QR of the SVD's preprocessing on explicit data (test hook):
// G (m x n) = Q (m x n) R (n x n upper, positive diagonal) by the same passes
// as the solve (CholeskyQR2, shifted first pass when needed).  Returns 0, or
// 1 when the Cholesky factorization failed.
int run_qr(int m, int n, const double *dG, int ldg, double *dQ, int ldq, double *dR, int ldr, hipStream_t s) {
    jacobi_opts o;
    jacobi_opts_default(&o);
    const SvdPlan p = plan_svd(m, n, o);
    const int mpad = p.mpad, npad = p.npad;
    const size_t big = sizeof(double) * (size_t)mpad * npad, sq = sizeof(double) * (size_t)npad * npad;
    WorkspaceBuilder wb;
    const size_t o_g = wb.add(big), o_b = wb.add(big), o_ra = wb.add(sq), o_rb = wb.add(sq), o_rc = wb.add(sq),
                 o_r = wb.add(sq), o_ri = wb.add(sizeof(double) * (size_t)npad * 128),
                 o_tp = wb.add(sizeof(double) * (size_t)std::max(mpad, npad) * 128),
                 o_sc = wb.add(sizeof(double) * ((size_t)npad + 8)),
                 o_pr = wb.add(sizeof(double) * ((2 * (size_t)npad + (size_t)mpad) * 128 + 136));
    DeviceBuffer buf;
    buf.alloc(wb.total());
    auto D = [&](size_t off) { return reinterpret_cast<double *>(buf.ptr + off); };
    QrScratch q{D(o_ri), D(o_tp), D(o_sc), reinterpret_cast<int *>(buf.ptr + o_sc + sizeof(double) * ((size_t)npad + 6))};
    launch_copy_rect(m, n, dG, ldg, D(o_g), mpad, mpad, npad, s);
    std::vector<double *> Rs;
    double *Rbuf[3] = {D(o_ra), D(o_rb), D(o_rc)};
    double *Qf = nullptr;
    if (!cholesky_qr2(m, n, mpad, npad, D(o_g), D(o_b), Rbuf, q, true, &Qf, Rs, s)) return 1;
    double *Gf = Qf == D(o_g) ? D(o_b) : D(o_g);
    launch_copy_rect(m, n, dG, ldg, Gf, mpad, mpad, npad, s);
    if (!(qr_probe_error(mpad, n, npad, Gf, Qf, Rs, D(o_pr), q, s) <= 1e-13)) return 1;
    // R = R_last ... R_1
    double *R = D(o_r);
    launch_gemm_f64('N', 'N', npad, npad, npad, 1.0, Rs[1], npad, Rs[0], npad, 0.0, R, npad, s);
    if (Rs.size() == 3) {
        launch_gemm_f64('N', 'N', npad, npad, npad, 1.0, Rs[2], npad, R, npad, 0.0, Rs[0], npad, s);
        R = Rs[0];
    }
    launch_copy_rect(m, n, Qf, mpad, dQ, ldq, m, n, s);
    launch_copy_rect(n, n, R, npad, dR, ldr, n, n, s);
    JX_HIP(hipStreamSynchronize(s));
    return 0;
}

}  // namespace jx
