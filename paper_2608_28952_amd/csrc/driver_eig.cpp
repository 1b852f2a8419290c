// driver_eig.cpp -- host orchestration of the blocked two-sided Jacobi
// eigensolver (Alg. 1 run as Alg. 2, §3, on one GPU).
//
// Per sweep, per round r of the pair schedule (N/2 disjoint block pairs):
//   K1  subproblem kernel: A_hat = A([I,J],[I,J]) -> V_hat, D_hat written back
//   K2  fused tile update: A[p,q] <- V_p^T A[p,q] V_q for every p < q
//   K2' Q(:, [I,J]) <- Q(:, [I,J]) V_hat
// then Xi(A) (eq. Omega_A) is summed on the GPU and read back once per sweep.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "jx_common.hpp"
#include "jx_host.hpp"
#include "jx_prof.hpp"

namespace jx {

// ---------------------------------------------------------------------------
// Pair schedules
// ---------------------------------------------------------------------------

// Round-robin for even N: round K (0 .. N-2) pairs every I, J in 1 .. N-1 with
// I + J = K (mod N-1) (Alg. 3's group K over the odd count N-1), and the index
// left without a partner (2 I = K mod N-1) with N.  Pairs returned 0-based.
static void schedule_rr(int N, std::vector<int> &pairs, std::vector<int> &sizes) {
    const int M = N - 1;
    pairs.clear();
    sizes.assign(M, N / 2);
    for (int K = 0; K < M; ++K) {
        for (int I = 1; I <= M; ++I) {
            int J = ((K - I) % M + M) % M;  // I + J = K (mod M), J in 0 .. M-1
            if (J == 0) J = M;
            if (J == I) {
                pairs.push_back(I - 1);
                pairs.push_back(N - 1);
            } else if (I < J) {
                pairs.push_back(I - 1);
                pairs.push_back(J - 1);
            }
        }
    }
}

// Alg. 3 (§3): group K holds the (I, J), I < J, with I + J = K (mod N).
static void schedule_antidiag(int N, std::vector<int> &pairs, std::vector<int> &sizes) {
    pairs.clear();
    sizes.assign(N, 0);
    for (int K = 0; K < N; ++K) {
        for (int I = 1; I <= N; ++I) {
            int J = ((K - I) % N + N) % N;
            if (J == 0) J = N;
            if (I < J) {
                pairs.push_back(I - 1);
                pairs.push_back(J - 1);
                ++sizes[K];
            }
        }
    }
}

int make_schedule(int N, int ordering, std::vector<int> &pairs, std::vector<int> &sizes) {
    if (N < 2 || (N & 1)) return -1;
    if (ordering == JACOBI_ORDER_ANTIDIAG) {
        schedule_antidiag(N, pairs, sizes);
        return N;
    }
    schedule_rr(N, pairs, sizes);
    return N - 1;
}

// Rounds padded to N/2 pairs: a group of Alg. 3 with N/2 - 1 pairs leaves two
// indices idle; they form a placeholder pair that is never rotated.
static void padded_rounds(int N, int ordering, std::vector<int> &pairs, std::vector<int> &force) {
    std::vector<int> raw, sizes;
    const int R = make_schedule(N, ordering, raw, sizes);
    const int H = N / 2;
    pairs.assign((size_t)R * H * 2, 0);
    force.assign((size_t)R * H, 0);
    size_t base = 0;
    for (int r = 0; r < R; ++r) {
        std::vector<char> used(N, 0);
        for (int k = 0; k < sizes[r]; ++k) {
            const int I = raw[2 * (base + k)], J = raw[2 * (base + k) + 1];
            pairs[2 * ((size_t)r * H + k)] = I;
            pairs[2 * ((size_t)r * H + k) + 1] = J;
            used[I] = used[J] = 1;
        }
        int k = sizes[r];
        std::vector<int> idle;
        for (int i = 0; i < N; ++i)
            if (!used[i]) idle.push_back(i);
        for (size_t t = 0; t + 1 < idle.size(); t += 2, ++k) {
            pairs[2 * ((size_t)r * H + k)] = idle[t];
            pairs[2 * ((size_t)r * H + k) + 1] = idle[t + 1];
            force[(size_t)r * H + k] = 1;
        }
        base += sizes[r];
    }
}

void padded_rounds_pub(int N, int ordering, std::vector<int> &pairs, std::vector<int> &force) {
    padded_rounds(N, ordering, pairs, force);
}

// ---------------------------------------------------------------------------
// Plan and workspace
// ---------------------------------------------------------------------------

static int default_block(int n) { return n > 512 ? 64 : 32; }

// Sweeps after which the subproblems are solved to convergence (see phase()).
constexpr int INNER_ESCALATE = 30;
// Relative off-norm at which the FP64 sweeps refine Q inside the quadratic
// phase (run_eig): low enough that one sweep usually follows (as after a
// refinement at convergence, so Q keeps that orthogonality), high enough
// that this sweep is one the solve needs anyway.  More than
// EARLY_REFINE_SWEEPS sweeps after it, and the refinement is repeated at
// the end.
constexpr double EARLY_REFINE = 1e-8;
constexpr int EARLY_REFINE_SWEEPS = 2;
// The refinement is moved into the quadratic phase only when the last sweep
// cut the off-norm by this factor: under linear convergence (clusters of
// equal eigenvalues) more sweeps remain, and the refinement waits for the
// end (an exactly clustered spectrum at n = 256, refined early at 4e-9 in a
// run of 0.4x decreases, stalled near 7e-11 for 50 sweeps).
constexpr double EARLY_REFINE_DROP = 1e-2;

// V_hat / flag buffers of consecutive rounds (see EigState)
constexpr int NVBUF = 3;

EigPlan plan_eig(int n, const jacobi_opts &o) {
    EigPlan p{};
    p.n = n;
    p.b = o.block > 0 ? o.block : default_block(n);
    const int unit = std::max(2 * p.b, 128);
    p.npad = std::max(unit, (n + unit - 1) / unit * unit);
    p.N = p.npad / p.b;
    p.H = p.N / 2;
    p.R = (o.ordering == JACOBI_ORDER_ANTIDIAG) ? p.N : p.N - 1;
    p.vectors = o.want_vectors != 0;
    p.mixed = o.precision != JACOBI_PREC_FP64;
    // the mixed ladder always ends with the FP64 recomputation from the
    // original matrix, which needs Q even for eigenvalues only
    p.refine = p.mixed || (p.vectors && (o.refine == 1 || (o.refine < 0 && n >= 256)));
    p.need_q = p.vectors || p.mixed;
    // three npad x npad FP64 temporaries: the original matrix and two GEMM
    // results for the refinement, and for a warm start's Q0^T A Q0 (a start
    // is used whenever Q is kept), so no call allocates beside its workspace
    p.temps = p.refine || p.need_q;
    const size_t npad = p.npad, nb = (size_t)p.N * (p.N + 1) / 2;
    const size_t m2sq = (size_t)(2 * p.b) * (2 * p.b);
    WorkspaceBuilder wb;
    p.off_ablk = wb.add(sizeof(double) * nb * p.b * p.b);
    p.off_q = p.need_q ? wb.add(sizeof(double) * npad * npad) : 0;
    if (p.mixed) {
        p.off_ablk32 = wb.add(sizeof(float) * nb * p.b * p.b);
        p.off_q32 = wb.add(sizeof(float) * npad * npad);
        p.off_v32 = wb.add(sizeof(float) * NVBUF * p.H * m2sq);
    }
    p.off_v = wb.add(sizeof(double) * NVBUF * p.H * m2sq);
    p.off_flags = wb.add(sizeof(int) * NVBUF * p.H);
    p.off_pairs = wb.add(sizeof(int) * 2 * (size_t)p.R * p.H);
    p.off_force = wb.add(sizeof(int) * (size_t)p.R * p.H);
    p.off_tiles = wb.add(sizeof(int) * (size_t)p.R * p.H * (p.H - 1));  // per round, critical tiles first
    p.off_qmask = wb.add(sizeof(int) * (size_t)p.R * p.H);               // per critical tile: its next-round blocks
    p.off_side = wb.add(sizeof(double) * 8 * (size_t)p.H * p.b * p.b);   // their originals, 2 rounds (FP64 or FP32)
    p.off_smap = wb.add(sizeof(int) * 4 * ((size_t)p.R * p.H * (p.H - 1) / 2 + 1));  // where a tile's blocks are copied
    p.off_xcopy = wb.add(sizeof(int) * 8 * (size_t)p.R * p.H);          // other copies per round
    p.off_copy0 = wb.add(sizeof(int) * 8 * (size_t)p.H);                // copies before a sweep's round 0
    p.sorted = o.ordering == JACOBI_ORDER_ROUND_ROBIN_SORTED;
    p.pivot = o.pivot == 1;
    if (p.sorted) {  // re-sorting between sweeps: a second block storage and the inverse permutation
        p.off_ablk2 = wb.add(sizeof(double) * nb * p.b * p.b);
        p.off_inv = wb.add(sizeof(int) * npad);
    }
    p.off_partial = wb.add(sizeof(double) * 2 * nb);
    p.off_scal = wb.add(sizeof(double) * 8);
    p.off_w = wb.add(sizeof(double) * npad);
    p.off_rank = wb.add(sizeof(int) * npad);
    if (p.temps) {
        p.off_a0 = wb.add(sizeof(double) * npad * npad);
        p.off_t1 = wb.add(sizeof(double) * npad * npad);
        p.off_t2 = wb.add(sizeof(double) * npad * npad);
    }
    p.total = wb.total();
    return p;
}

// ---------------------------------------------------------------------------
// Sweeps
// ---------------------------------------------------------------------------

struct EigState {
    const EigPlan &p;
    char *ws;
    hipStream_t s;
    double *ablk, *Q, *V, *partial, *scal;
    int *flags, *pairs, *force, *tiles, *qmask, *smap, *xcopy, *copy0;
    int ncopy0 = 0;
    std::vector<int> nxcopy;
    char *side;  // two rounds' copies of the critical blocks' originals
    float *ablk32 = nullptr, *Q32 = nullptr, *V32 = nullptr;
    bool f32 = false;  // current phase works on the FP32 copies
    double *h_scal;  // pinned
    int inner;
    double tol;
    int any_force;
    // second stream for the rest of the tile updates and the Q updates,
    // which overlap the next round's subproblem solves.  The V_hat / flag
    // buffers rotate over NVBUF = 3 rounds: round r + 3's subproblem kernel
    // (which rewrites buffer r mod 3) follows round r + 2's critical tiles on
    // s, which wait for round r + 1's rest tiles on sq, which follow round r's
    // Q update on sq; so no round reuses a buffer that is still read.
    hipStream_t sq = nullptr;
    hipEvent_t ev_v = nullptr;   // critical tiles of the last round done (on s)
    hipEvent_t ev_q = nullptr;   // Q update of the last round done (on sq)
    bool q_pending = false;
    // per round: the first ncrit[r] tiles of its list hold the blocks the next
    // round's subproblems read (qmask: which of their four blocks); those
    // blocks are done first, the rest of every tile on sq beside the next
    // round's subproblems
    std::vector<int> ncrit;
    hipEvent_t ev_rest = nullptr;  // rest tiles of the last round done (on sq)
    bool rest_pending = false;
    // profiling: skip flags of every round copied to pinned host memory
    int *h_flaglog = nullptr;
    int flog_cap = 0, flog_count = 0, flog_base = 0;

    // copies of round r's critical blocks' originals (4 blocks per critical
    // tile), in the current precision; rounds alternate between two buffers
    void *sidebuf(int r) const {
        return side + (size_t)(r & 1) * 4 * p.H * p.b * p.b * (f32 ? sizeof(float) : sizeof(double));
    }
    double *Vbuf(int r) const { return V + (size_t)(r % NVBUF) * p.H * (2 * p.b) * (2 * p.b); }
    float *Vbuf32(int r) const { return V32 + (size_t)(r % NVBUF) * p.H * (2 * p.b) * (2 * p.b); }
    int *Fbuf(int r) const { return flags + (size_t)(r % NVBUF) * p.H; }

    // Re-sorting (ordering JACOBI_ORDER_ROUND_ROBIN_SORTED): the indices are
    // permuted so that the diagonal is ascending, A <- P^T A P and Q <- Q P
    // (an exact permutation), before a sweep.  Block (I, J) then holds
    // indices whose current diagonal values are close together, so nearly
    // equal eigenvalues meet inside one subproblem, which the inner solve
    // separates, instead of only in the pair of their two blocks once a
    // sweep.  Padding indices keep their places.
    double *ablk2 = nullptr, *qspare = nullptr, *wdiag = nullptr;
    int *rank = nullptr, *inv = nullptr;
    void resort() {
        const size_t nab = (size_t)p.N * (p.N + 1) / 2 * p.b * p.b;
        if (f32) launch_extract_diag32(p.npad, p.b, ablk32, wdiag, s);
        else launch_extract_diag(p.npad, p.b, ablk, wdiag, s);
        launch_rank(p.n, wdiag, +1, rank, s);
        launch_inverse_perm(p.n, p.npad, rank, inv, s);
        if (f32) {
            launch_permute_sym32(p.npad, p.b, inv, ablk32, reinterpret_cast<float *>(ablk2), s);
            JX_HIP(hipMemcpyAsync(ablk32, ablk2, sizeof(float) * nab, hipMemcpyDeviceToDevice, s));
        } else {  // the permuted copy becomes A's storage (the two buffers trade places)
            launch_permute_sym(p.npad, p.b, inv, ablk, ablk2, s);
            std::swap(ablk, ablk2);
        }
        if (p.need_q) {
            const size_t nq = (size_t)p.npad * p.npad;
            if (f32) {
                float *sp = reinterpret_cast<float *>(qspare);
                launch_permute_cols32(p.npad, p.npad, inv, Q32, p.npad, sp, p.npad, s);
                JX_HIP(hipMemcpyAsync(Q32, sp, sizeof(float) * nq, hipMemcpyDeviceToDevice, s));
            } else {
                launch_permute_cols(p.npad, p.npad, inv, Q, p.npad, qspare, p.npad, s);
                JX_HIP(hipMemcpyAsync(Q, qspare, sizeof(double) * nq, hipMemcpyDeviceToDevice, s));
            }
        }
    }

    // {Xi(A)^2, sum of squared diagonal}
    void norms(double &off2, double &dia2) {
        if (f32) launch_block_norms32(p.npad, p.b, ablk32, partial, scal, s);
        else launch_block_norms(p.npad, p.b, ablk, partial, scal, s);
        JX_HIP(hipMemcpyAsync(h_scal, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        JX_HIP(hipStreamSynchronize(s));
        off2 = h_scal[0];
        dia2 = h_scal[1];
    }

    void sweep(double skip_thr) {
        const int m2 = 2 * p.b;
        const int ntiles = p.H * (p.H - 1) / 2;
        // algorithmic work of a rotated subproblem per inner sweep: m2 (m2 - 1) / 2
        // scalar rotations, each applied to two rows and two columns of the
        // full m2 x m2 A_hat and to two columns of V_hat, 6 flops per entry
        // pair: 18 m2 flops per rotation (18.7 MFLOP at m2 = 128).  Bytes:
        // the three blocks of the pair read and written, V_hat written.
        const double k1_flops = (double)p.H * std::max(1, inner) * (m2 * (m2 - 1) / 2.0) * 18.0 * m2;
        const double k1_bytes = (double)p.H * (6.0 * p.b * p.b + (double)m2 * m2) * sizeof(double);
        // round 0's critical blocks as they stand (later rounds' copies are
        // written by the round before, as it produces those blocks)
        if (f32) launch_copy_blocks32(p.b, ablk32, copy0, ncopy0, sidebuf(0), s);
        else launch_copy_blocks(p.b, ablk, copy0, ncopy0, sidebuf(0), s);
        for (int r = 0; r < p.R; ++r) {
            const int *pr = pairs + (size_t)2 * r * p.H;
            SubArgs a{};
            a.mode = SUB_EIG;
            a.m2 = m2;
            a.count = p.H;
            a.pairs = pr;
            a.ablk = ablk;
            a.vout = Vbuf(r);
            a.flags = Fbuf(r);
            a.skip_thr = skip_thr;
            a.inner_sweeps = inner;
            a.force_skip = any_force ? force + (size_t)r * p.H : nullptr;
            if (f32) {
                a.ablk32 = ablk32;
                a.vout32 = Vbuf32(r);
            }
            // flags of this round land in the profiler's flag log at `slot`
            const int slot_next = (h_flaglog && flog_count < flog_cap) ? flog_base + flog_count * p.H : -1;
            {
                ProfScope ps(PROF_SUBPROBLEM, s, k1_flops / p.H, k1_bytes / p.H, slot_next, p.H, m2);
                launch_subproblem(a, s);
            }
            if (p.pivot && !f32) {  // V_hat <- V_hat P, D_hat <- P^T D_hat P before any tile reads them
                PivotArgs pa{};
                pa.count = p.H;
                pa.m2 = m2;
                pa.pairs = pr;
                pa.ablk = ablk;
                pa.V = Vbuf(r);
                pa.flags = Fbuf(r);
                launch_pivot(pa, s);
            }
            int slot = -1;
            if (h_flaglog && flog_count < flog_cap) {
                JX_HIP(hipMemcpyAsync(h_flaglog + (size_t)flog_count * p.H, Fbuf(r), sizeof(int) * p.H,
                                      hipMemcpyDeviceToHost, s));
                slot = flog_base + flog_count * p.H;
                ++flog_count;
            }
            // Tile updates.  The blocks that round r + 1's subproblems read
            // (qm: some quadrants of the first nc tiles) are computed here, on
            // s, their originals saved to `side`; the rest of every tile runs
            // on sq on at most CUs - H CUs, beside round r + 1's subproblems,
            // and must be done before round r + 1's tiles (which also reuse
            // `side`).
            const int *tl = tiles + (size_t)2 * r * ntiles;
            const int *qm = qmask + (size_t)r * p.H;
            const int nc = ncrit[r];
            // b = 64: the rest of the tiles and the Q update share one
            // persistent launch (no tail of idle CUs between the two)
            const bool fuse = p.b == 64;
            if (rest_pending) {
                JX_HIP(hipStreamWaitEvent(s, ev_rest, 0));
                rest_pending = false;
            }
            {
                {
                    // one block of a tile: 3/8 of its products (b = 64), 3/4 (b = 32)
                    ProfScope ps(PROF_UPDATE_A, s, (p.b == 64 ? 0.375 : 0.75) * nc / ntiles, 0.0, slot, p.H, m2);
                    void *sd = sidebuf(r);
                    if (f32) launch_update_a32(p.b, p.H, pr, ablk32, Vbuf32(r), Fbuf(r), tl, nc, s, UA_QUAD, qm, nc, sd);
                    else launch_update_a(p.b, p.H, pr, ablk, Vbuf(r), Fbuf(r), tl, nc, s, UA_QUAD, qm, nc, sd);
                }
                JX_HIP(hipEventRecord(ev_v, s));
                JX_HIP(hipStreamWaitEvent(sq, ev_v, 0));
                // this round's tiles also write the copies of the next round's
                // critical blocks; blocks they do not produce are copied after them
                void *sd = sidebuf(r), *sn = r + 1 < p.R ? sidebuf(r + 1) : nullptr;
                const int *sm = smap + 4 * (size_t)r * ntiles;
                if (fuse) {  // the rest of the tiles and the Q update in one launch
                    ProfScope ps(PROF_UPDATE_AQ, sq, p.need_q ? (double)p.npad : 0.0, 0.0, slot, p.H, m2);
                    if (f32)
                        launch_update_aq32(p.b, p.H, pr, ablk32, Vbuf32(r), Fbuf(r), tl, ntiles, qm, nc, sd, sn, sm,
                                           p.need_q ? Q32 : nullptr, p.npad, p.npad, p.H, sq);
                    else
                        launch_update_aq(p.b, p.H, pr, ablk, Vbuf(r), Fbuf(r), tl, ntiles, qm, nc, sd, sn, sm,
                                         p.need_q ? Q : nullptr, p.npad, p.npad, p.H, sq);
                } else {
                    ProfScope ps(PROF_UPDATE_A_REST, sq, 1.0, 0.0, slot, p.H, m2);
                    if (f32)
                        launch_update_a32(p.b, p.H, pr, ablk32, Vbuf32(r), Fbuf(r), tl, ntiles, sq, p.H, qm, nc, sd,
                                          sn, sm);
                    else
                        launch_update_a(p.b, p.H, pr, ablk, Vbuf(r), Fbuf(r), tl, ntiles, sq, p.H, qm, nc, sd, sn, sm);
                }
                if (sn && nxcopy[r] > 0) {
                    if (f32) launch_copy_blocks32(p.b, ablk32, xcopy + (size_t)8 * r * p.H, nxcopy[r], sn, sq);
                    else launch_copy_blocks(p.b, ablk, xcopy + (size_t)8 * r * p.H, nxcopy[r], sn, sq);
                }
                JX_HIP(hipEventRecord(ev_rest, sq));
                rest_pending = true;
            }
            if (p.need_q && !fuse) {
                hipStream_t qs = sq ? sq : s;
                {
                    ProfScope ps(PROF_UPDATE_Q, qs, (double)p.npad, 0.0, slot, p.H, m2);
                    // beside the next round's subproblems: leave them their CUs
                    const int reserve = sq ? p.H : 0;
                    if (f32) launch_update_q32(p.b, p.H, pr, Q32, p.npad, p.npad, Vbuf32(r), Fbuf(r), qs, reserve);
                    else launch_update_q(p.b, p.H, pr, Q, p.npad, p.npad, Vbuf(r), Fbuf(r), qs, reserve);
                }
            }
            if (sq && p.need_q) {
                JX_HIP(hipEventRecord(ev_q, sq));
                q_pending = true;
            }
        }
        // A and Q complete before anyone reads them (norms, refinement, output)
        if (rest_pending) {
            JX_HIP(hipStreamWaitEvent(s, ev_rest, 0));
            rest_pending = false;
        }
        if (q_pending) {
            JX_HIP(hipStreamWaitEvent(s, ev_q, 0));
            q_pending = false;
        }
    }

    // the device context's second stream and events (ordering between the
    // two streams of one device only: the kernels' own completion makes
    // their writes visible device-wide, so no system-scope fence)
    void use_streams(DeviceCtx &c) {
        sq = c.side;
        ev_v = c.ev[0];
        ev_q = c.ev[1];
        ev_rest = c.ev[2];
    }
    ~EigState() {
        if (sq) (void)hipStreamSynchronize(sq);
    }
};

// FP64 GEMM with profiling record.
static void gemm_p(char ta, char tb, int M, int N, int K, double alpha, const double *A, int lda,
                   const double *B, int ldb, double beta, double *C, int ldc, hipStream_t s) {
    ProfScope ps(PROF_GEMM, s, 2.0 * M * (double)N * K,
                 sizeof(double) * ((double)M * K + (double)K * N + (beta != 0.0 ? 2.0 : 1.0) * M * N));
    launch_gemm_f64(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
}

static bool finite(double x) { return std::isfinite(x); }

int run_eig(int n, const double *dA, int lda, char uplo, double *dW, double *dQ, int ldq,
            const double *dQ0, int ldq0, void *dWork, size_t workBytes, const jacobi_opts &o,
            jacobi_info *info, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    jacobi_info inf{};
    EigPlan p = plan_eig(n, o);
    DeviceBuffer own;
    char *ws = static_cast<char *>(dWork);
    if (!ws) {
        own.alloc(p.total);
        ws = own.ptr;
    } else if (workBytes < p.total) {
        return -100;
    }
    DeviceCtx &ctx = device_ctx();
    std::lock_guard<std::mutex> lk(ctx.mu);

    EigState st{p, ws, s};
    st.ablk = reinterpret_cast<double *>(ws + p.off_ablk);
    st.Q = p.need_q ? reinterpret_cast<double *>(ws + p.off_q) : nullptr;
    if (p.mixed) {
        st.ablk32 = reinterpret_cast<float *>(ws + p.off_ablk32);
        st.Q32 = reinterpret_cast<float *>(ws + p.off_q32);
        st.V32 = reinterpret_cast<float *>(ws + p.off_v32);
    }
    st.V = reinterpret_cast<double *>(ws + p.off_v);
    st.flags = reinterpret_cast<int *>(ws + p.off_flags);
    st.pairs = reinterpret_cast<int *>(ws + p.off_pairs);
    st.force = reinterpret_cast<int *>(ws + p.off_force);
    st.tiles = reinterpret_cast<int *>(ws + p.off_tiles);
    st.qmask = reinterpret_cast<int *>(ws + p.off_qmask);
    st.side = ws + p.off_side;
    st.smap = reinterpret_cast<int *>(ws + p.off_smap);
    st.xcopy = reinterpret_cast<int *>(ws + p.off_xcopy);
    st.copy0 = reinterpret_cast<int *>(ws + p.off_copy0);
    st.partial = reinterpret_cast<double *>(ws + p.off_partial);
    st.scal = reinterpret_cast<double *>(ws + p.off_scal);
    st.h_scal = reinterpret_cast<double *>(ctx.pinned);
    st.inner = o.inner_max_sweeps;
    st.tol = o.tol > 0.0 ? o.tol : 1e-14;
    st.use_streams(ctx);
    if (p.sorted) {
        st.ablk2 = reinterpret_cast<double *>(ws + p.off_ablk2);
        st.inv = reinterpret_cast<int *>(ws + p.off_inv);
        st.wdiag = reinterpret_cast<double *>(ws + p.off_w);
        st.rank = reinterpret_cast<int *>(ws + p.off_rank);
        st.qspare = p.temps ? reinterpret_cast<double *>(ws + p.off_t1) : nullptr;
    }
    struct PinnedInts {
        int *ptr = nullptr;
        ~PinnedInts() { if (ptr) (void)hipHostFree(ptr); }
    } flaglog;
    if (prof_on()) {
        st.flog_cap = (o.max_sweeps + 8) * p.R;
        JX_HIP(hipHostMalloc(reinterpret_cast<void **>(&flaglog.ptr), sizeof(int) * (size_t)st.flog_cap * p.H,
                             hipHostMallocDefault));
        st.h_flaglog = flaglog.ptr;
        st.flog_base = prof_flag_base();
    }

    // schedule and tile list (host -> device once per call)
    std::vector<int> hp, hf;
    padded_rounds(p.N, o.ordering == JACOBI_ORDER_ANTIDIAG ? JACOBI_ORDER_ANTIDIAG : JACOBI_ORDER_ROUND_ROBIN, hp, hf);
    st.any_force = std::any_of(hf.begin(), hf.end(), [](int v) { return v != 0; }) ? 1 : 0;
    // tile lists: per round, the critical tiles first (tile (p, q) of round r
    // holds block (I', J') of a pair of round r + 1 (cyclically) when I' is in
    // pair p and J' in pair q), then the others in (p, q) order.  qmask of a
    // critical tile: bit 2 h + c for each such block, h its row block within
    // pair p (0: the pair's first block) and c its column block within pair q.
    std::vector<int> ht, hq((size_t)p.R * p.H, 0);
    st.ncrit.assign(p.R, 0);
    {
        std::vector<int> pos(p.N, 0), half(p.N, 0);
        std::vector<int> crit((size_t)p.H * p.H);
        for (int r = 0; r < p.R; ++r) {
            for (int k = 0; k < p.H; ++k) {
                pos[hp[2 * ((size_t)r * p.H + k)]] = k;
                pos[hp[2 * ((size_t)r * p.H + k) + 1]] = k;
                half[hp[2 * ((size_t)r * p.H + k)]] = 0;
                half[hp[2 * ((size_t)r * p.H + k) + 1]] = 1;
            }
            std::fill(crit.begin(), crit.end(), -1);
            const int rn = (r + 1) % p.R;
            for (int k = 0; k < p.H; ++k) {
                const int I = hp[2 * ((size_t)rn * p.H + k)], J = hp[2 * ((size_t)rn * p.H + k) + 1];
                const int a = pos[I], b = pos[J];
                if (a == b) continue;  // a block of a round-r pair: written by the subproblem kernel
                const int lo = std::min(a, b), hi = std::max(a, b);
                const int h = a < b ? half[I] : half[J], c = a < b ? half[J] : half[I];
                int &ci = crit[(size_t)lo * p.H + hi];
                if (ci < 0) {
                    ci = st.ncrit[r]++;
                    ht.push_back(lo);
                    ht.push_back(hi);
                }
                hq[(size_t)r * p.H + ci] |= 1 << (2 * h + c);
            }
            for (int a = 0; a < p.H; ++a)
                for (int b = a + 1; b < p.H; ++b)
                    if (crit[(size_t)a * p.H + b] < 0) { ht.push_back(a); ht.push_back(b); }
        }
    }
    JX_HIP(hipMemcpyAsync(st.pairs, hp.data(), sizeof(int) * hp.size(), hipMemcpyHostToDevice, s));
    JX_HIP(hipMemcpyAsync(st.force, hf.data(), sizeof(int) * hf.size(), hipMemcpyHostToDevice, s));
    if (!ht.empty())
        JX_HIP(hipMemcpyAsync(st.tiles, ht.data(), sizeof(int) * ht.size(), hipMemcpyHostToDevice, s));
    JX_HIP(hipMemcpyAsync(st.qmask, hq.data(), sizeof(int) * hq.size(), hipMemcpyHostToDevice, s));
    // Copies of the critical blocks' originals (the critical kernel reads
    // them, and writes the blocks in place).  Round r + 1's critical blocks
    // are pairs of round r + 2, so within a sweep round r's tiles produce
    // them: smap[r][tile][quad] names the slot (4 ci + quad of the next
    // round's critical tile ci) the quadrant's new value is also written to
    // (-1: none).  A block outside round r's tiles (a placeholder pair of
    // round r, never rotated) is copied after them (xcopy); round 0's
    // blocks are copied at each sweep's start (copy0).
    {
        const int ntiles = p.H * (p.H - 1) / 2;
        std::vector<int> hsm(4 * ((size_t)p.R * ntiles + 1), -1), hx((size_t)8 * p.R * p.H, 0), hc0;
        st.nxcopy.assign(p.R, 0);
        std::vector<int> pos(p.N, 0), half(p.N, 0), tix((size_t)p.H * p.H, -1);
        auto block_of = [&](int rr, int ci, int quad) {  // (row, column) block of quadrant quad of crit tile ci
            const int lo = ht[2 * ((size_t)rr * ntiles + ci)], hi = ht[2 * ((size_t)rr * ntiles + ci) + 1];
            return std::make_pair(hp[2 * ((size_t)rr * p.H + lo) + (quad >> 1)],
                                  hp[2 * ((size_t)rr * p.H + hi) + (quad & 1)]);
        };
        for (int r = 0; r + 1 < p.R; ++r) {
            for (int k = 0; k < p.H; ++k) {
                pos[hp[2 * ((size_t)r * p.H + k)]] = k;
                pos[hp[2 * ((size_t)r * p.H + k) + 1]] = k;
                half[hp[2 * ((size_t)r * p.H + k)]] = 0;
                half[hp[2 * ((size_t)r * p.H + k) + 1]] = 1;
            }
            for (int i = 0; i < ntiles; ++i)
                tix[(size_t)ht[2 * ((size_t)r * ntiles + i)] * p.H + ht[2 * ((size_t)r * ntiles + i) + 1]] = i;
            const int rn = r + 1;
            for (int ci = 0; ci < st.ncrit[rn]; ++ci)
                for (int quad = 0; quad < 4; ++quad) {
                    if (!((hq[(size_t)rn * p.H + ci] >> quad) & 1)) continue;
                    const auto bl = block_of(rn, ci, quad);
                    const int X = bl.first, Y = bl.second, slot = 4 * ci + quad;
                    const int a = pos[X], b = pos[Y];
                    if (a != b) {
                        const int i = tix[(size_t)std::min(a, b) * p.H + std::max(a, b)];
                        const int h2 = a < b ? half[X] : half[Y], c2 = a < b ? half[Y] : half[X];
                        const int q2 = 2 * h2 + c2;
                        hsm[4 * ((size_t)r * ntiles + i) + q2] = slot;
                    } else {
                        int &n = st.nxcopy[r];
                        hx[(size_t)8 * r * p.H + 2 * n] = (int)ublk(std::min(X, Y), std::max(X, Y));
                        hx[(size_t)8 * r * p.H + 2 * n + 1] = slot;
                        ++n;
                    }
                }
        }
        for (int ci = 0; ci < st.ncrit[0]; ++ci)
            for (int quad = 0; quad < 4; ++quad) {
                if (!((hq[ci] >> quad) & 1)) continue;
                const auto bl = block_of(0, ci, quad);
                hc0.push_back((int)ublk(std::min(bl.first, bl.second), std::max(bl.first, bl.second)));
                hc0.push_back(4 * ci + quad);
            }
        st.ncopy0 = (int)hc0.size() / 2;
        JX_HIP(hipMemcpyAsync(st.smap, hsm.data(), sizeof(int) * hsm.size(), hipMemcpyHostToDevice, s));
        JX_HIP(hipMemcpyAsync(st.xcopy, hx.data(), sizeof(int) * hx.size(), hipMemcpyHostToDevice, s));
        if (!hc0.empty())
            JX_HIP(hipMemcpyAsync(st.copy0, hc0.data(), sizeof(int) * hc0.size(), hipMemcpyHostToDevice, s));
        JX_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
    }

    // A -> upper block storage; Q = I or Q0 (then A <- Q0^T A Q0)
    double *A0 = p.temps ? reinterpret_cast<double *>(ws + p.off_a0) : nullptr;
    double *T1 = p.temps ? reinterpret_cast<double *>(ws + p.off_t1) : nullptr;
    double *T2 = p.temps ? reinterpret_cast<double *>(ws + p.off_t2) : nullptr;
    if (p.refine || (dQ0 && p.need_q)) launch_full_from_triangle(n, p.npad, dA, lda, uplo, A0, s);
    if (dQ0 && p.need_q) {  // A <- Q0^T A Q0 (FP64 MFMA GEMMs), Q = Q0
        launch_copy_pad(n, p.npad, dQ0, ldq0, st.Q, p.npad, s);
        gemm_p('N', 'N', p.npad, p.npad, p.npad, 1.0, A0, p.npad, st.Q, p.npad, 0.0, T1, p.npad, s);
        gemm_p('T', 'N', p.npad, p.npad, p.npad, 1.0, st.Q, p.npad, T1, p.npad, 0.0, T2, p.npad, s);
        launch_pack_sym(p.npad, p.npad, p.b, T2, p.npad, 'U', st.ablk, s);
    } else {
        launch_pack_sym(n, p.npad, p.b, dA, lda, uplo, st.ablk, s);
        if (p.need_q) launch_set_identity(p.npad, p.npad, st.Q, p.npad, s);
    }

    double off2, dia2;
    st.norms(off2, dia2);
    const double fro0 = std::sqrt(off2 + dia2);
    int status = 1;
    if (!finite(off2) || !finite(dia2)) status = 2;
    const double tol = o.tol > 0.0 ? o.tol : 1e-14;
    const double skip_thr = tol * fro0 * std::sqrt(2.0 / ((double)p.N * (p.N - 1)));
    int sweeps = 0, sweeps32 = 0;
    const bool verbose = std::getenv("JACOBI_VERBOSE") != nullptr;
    // Sweeps until Xi(A) <= stop * ||A||_F.  Returns 0 (reached), 1 (cap),
    // 2 (non-finite), 4 (FP32 phase slows down: less than 2x decrease per sweep
    // below 1e-3), 5 (early > 0: the quadratic phase has reached
    // Xi(A) <= early ||A||_F, the last sweep having cut the off-norm by at
    // least EARLY_REFINE_DROP).
    auto phase = [&](double stop, int cap, double early = 0.0) -> int {
        double prev = -1.0;
        for (;;) {
            if (verbose)
                std::fprintf(stderr, "[jacobi_eig] sweep %d %s off/||A||_F = %.3e\n", sweeps, st.f32 ? "fp32" : "fp64",
                             fro0 > 0 ? std::sqrt(off2) / fro0 : 0.0);
            if (!finite(off2) || !finite(dia2)) return 2;
            const double rel = fro0 > 0 ? std::sqrt(off2) / fro0 : 0.0;
            if (rel <= stop) return 0;
            // End of the FP32 phase once a sweep no longer halves the off-norm.
            // Slow convergence here means eigenvalues close together or near
            // FP32 resolution, which the FP64 phase must resolve anyway: on a
            // graded spectrum (|lambda| from 1 down to 1e-8, n = 4096) FP32
            // sweeps on to 1e-5 (a 0.8 ratio test) left 12 FP64 sweeps where
            // plain FP64 needs 8 from that point: 30 sweeps in all against 27.
            if (st.f32 && prev >= 0.0 && rel < 1e-3 && rel > 0.5 * prev) return 4;
            if (sweeps >= cap) return 1;
            if (early > 0.0 && prev > 0.0 && rel <= early && rel <= EARLY_REFINE_DROP * prev) return 5;
            prev = rel;
            // Approximate inner solves converge only linearly on (nearly)
            // repeated eigenvalues: an exactly clustered spectrum took 53-56
            // sweeps at n = 256 and 1024, 10 with inner solves to
            // convergence.  After INNER_ESCALATE sweeps the remaining ones
            // solve each subproblem to convergence.
            if (sweeps >= INNER_ESCALATE && st.inner > 0) st.inner = 0;
            if (p.sorted) st.resort();
            st.sweep(skip_thr);
            ++sweeps;
            if (st.f32) ++sweeps32;
            st.norms(off2, dia2);
        }
    };
    // Orthogonality refinement and recomputation from the original matrix:
    // Q <- Q (3 I - Q^T Q) / 2, A1 = Q^T A0 Q in FP64, A1 -> block storage.
    const double switch_rel = 1e-5;
    auto recompute = [&]() {
        const int np = p.npad;
        gemm_p('T', 'N', np, np, np, 1.0, st.Q, np, st.Q, np, 0.0, T1, np, s);    // M = Q^T Q
        JX_HIP(hipMemcpyAsync(T2, st.Q, sizeof(double) * (size_t)np * np, hipMemcpyDeviceToDevice, s));
        gemm_p('N', 'N', np, np, np, -0.5, st.Q, np, T1, np, 1.5, T2, np, s);     // 1.5 Q - 0.5 Q M
        JX_HIP(hipMemcpyAsync(st.Q, T2, sizeof(double) * (size_t)np * np, hipMemcpyDeviceToDevice, s));
        gemm_p('N', 'N', np, np, np, 1.0, A0, np, st.Q, np, 0.0, T1, np, s);      // A0 Q
        gemm_p('T', 'N', np, np, np, 1.0, st.Q, np, T1, np, 0.0, T2, np, s);      // Q^T A0 Q
        launch_pack_sym(np, np, p.b, T2, np, 'U', st.ablk, s);
        st.norms(off2, dia2);
    };
    bool early_refined = false;
    // Sweeps to tol with the orthogonality refinement inside the quadratic
    // phase: once Xi(A) <= EARLY_REFINE ||A||_F after a sweep that cut it by
    // EARLY_REFINE_DROP (and before the sweep cap), Q is refined and A_1 =
    // Q^T A_0 Q recomputed, then the sweeps finish.  The recomputed A_1
    // carries rounding of about n u ||A||_F (1.8e-13 at n = 4096), above tol,
    // so a refinement after convergence costs one more full sweep; here the
    // last sweep of the quadratic phase absorbs it.  If more than
    // EARLY_REFINE_SWEEPS sweeps follow, the refinement is repeated at the
    // end.  `fresh`: A_1 has just been recomputed (the precision switch);
    // already in the quadratic phase, that recomputation is the refinement.
    auto to_tol = [&](int cap, bool fresh) {
        const int s0 = sweeps;
        if (fresh && fro0 > 0.0 && std::sqrt(off2) <= EARLY_REFINE * fro0) {
            status = phase(tol, cap);
            early_refined = status == 0 && sweeps - s0 <= EARLY_REFINE_SWEEPS;
            return;
        }
        status = phase(tol, cap, EARLY_REFINE);
        if (status == 5) {
            const int before = sweeps;
            recompute();
            status = phase(tol, cap + 12);
            early_refined = status == 0 && sweeps - before <= EARLY_REFINE_SWEEPS;
        }
    };
    if (status != 2) {
        if (p.mixed) {
            // FP32 sweeps (subproblems still solved in FP64) to off <= 1e-5 or stagnation
            const size_t nab = (size_t)p.N * (p.N + 1) / 2 * p.b * p.b;
            launch_cast_to_f32(nab, st.ablk, st.ablk32, s);
            launch_cast_to_f32((size_t)p.npad * p.npad, st.Q, st.Q32, s);
            st.f32 = true;
            st.norms(off2, dia2);
            status = phase(switch_rel, o.max_sweeps);
            st.f32 = false;
            if (status != 2) {
                launch_cast_to_f64((size_t)p.npad * p.npad, st.Q32, st.Q, s);
                recompute();
                to_tol(o.max_sweeps + 8, true);
            }
        } else if (p.refine) {
            to_tol(o.max_sweeps, false);
        } else {
            status = phase(tol, o.max_sweeps);
        }
        // final orthogonality refinement: the sweeps after it rotate by angles of
        // the size of Q's orthogonality error and mostly skip.  Below order
        // 256 with the automatic setting, Q's orthogonality is measured first
        // (||Q^T Q - I||_F from one GEMM) and refined only above 2e-13.
        bool refine_now = status == 0 && p.refine && !early_refined;
        if (status == 0 && !p.refine && p.vectors && o.refine < 0 && p.temps) {
            const int np = p.npad;
            gemm_p('T', 'N', np, np, np, 1.0, st.Q, np, st.Q, np, 0.0, T1, np, s);
            launch_dev_identity(n, T1, np, T2, T2 + np, s);
            double dev2 = 0.0;
            JX_HIP(hipMemcpyAsync(&dev2, T2 + np, sizeof(double), hipMemcpyDeviceToHost, s));
            JX_HIP(hipStreamSynchronize(s));
            if (!(dev2 <= 4e-26)) {
                launch_full_from_triangle(n, p.npad, dA, lda, uplo, A0, s);
                refine_now = true;
            }
        }
        if (refine_now) {
            recompute();
            status = phase(tol, o.max_sweeps + 12);
        }
    }

    // eigenvalues (first n diagonal entries), sorted; Q columns permuted alike
    double *w = reinterpret_cast<double *>(ws + p.off_w);
    int *rank = reinterpret_cast<int *>(ws + p.off_rank);
    if (status != 2) {
        launch_extract_diag(p.npad, p.b, st.ablk, w, s);
        if (o.sort) {
            launch_rank(n, w, +1, rank, s);
        } else {
            std::vector<int> id(n);
            for (int i = 0; i < n; ++i) id[i] = i;
            JX_HIP(hipMemcpyAsync(rank, id.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
        }
        launch_scatter_values(n, w, rank, dW, s);
        if (p.vectors && dQ) launch_scatter_columns(n, n, st.Q, p.npad, rank, dQ, ldq, s);
        JX_HIP(hipStreamSynchronize(s));
    }
    if (st.h_flaglog) {
        JX_HIP(hipStreamSynchronize(s));
        prof_add_flags(std::vector<int>(st.h_flaglog, st.h_flaglog + (size_t)st.flog_count * p.H));
    }
    inf.status = status;
    inf.sweeps = sweeps;
    inf.sweeps_by_prec[1] = sweeps32;
    inf.sweeps_by_prec[2] = sweeps - sweeps32;
    inf.off_rel = fro0 > 0 ? std::sqrt(off2) / fro0 : 0.0;
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return status;
}

// ---------------------------------------------------------------------------
// b = 1: scalar two-sided Jacobi (Alg. 1 with b = 1) in round-robin order
// ---------------------------------------------------------------------------

// Orders from which a round runs over n/2 workgroups (one launch per round);
// below, every sweep runs in one persistent workgroup.
constexpr int SCALAR_MULTI_MIN = 128;
// Orders from which eigenvector solves end with an orthogonality refinement
// (Newton-Schulz on Q, A_1 = Q^T A_0 Q recomputed, sweeps to the tolerance).
constexpr int SCALAR_REFINE_MIN = 256;

size_t scalar_workspace(int n) {
    const int ne = n + (n & 1);
    WorkspaceBuilder wb;
    wb.add(sizeof(double) * (size_t)n * n);        // A
    wb.add(sizeof(double) * (size_t)n * n);        // Q
    wb.add(sizeof(int) * (size_t)ne * (ne - 1));   // pairs
    wb.add(sizeof(double) * 4);                    // sweeps, off-norm, ||A||_F
    wb.add(sizeof(double) * n);                    // diagonal
    wb.add(sizeof(int) * n);                       // ranks
    if (n >= SCALAR_MULTI_MIN) {
        wb.add(sizeof(double) * (size_t)n * n);    // the second copy of A (rounds alternate)
        wb.add(sizeof(int) * 4);                   // rotations of a sweep
    }
    if (n >= SCALAR_REFINE_MIN) {
        wb.add(sizeof(double) * (size_t)n * n);    // A_0 (refinement)
        wb.add(sizeof(double) * (size_t)n * n);    // GEMM temporary
        wb.add(sizeof(double) * ((size_t)n + 8));  // reduction partials
    }
    return wb.total();
}

int run_eig_scalar(int n, const double *dA, int lda, char uplo, double *dW, double *dQ, int ldq, void *dWork,
                   size_t workBytes, const jacobi_opts &o, jacobi_info *info, hipStream_t s) {
    const auto t0 = std::chrono::steady_clock::now();
    const int ne = n + (n & 1);
    const size_t total = scalar_workspace(n);
    DeviceBuffer own;
    char *ws = static_cast<char *>(dWork);
    if (!ws) {
        own.alloc(total);
        ws = own.ptr;
    } else if (workBytes < total) {
        return -100;
    }
    WorkspaceBuilder wb;
    double *A = reinterpret_cast<double *>(ws + wb.add(sizeof(double) * (size_t)n * n));
    double *Q = reinterpret_cast<double *>(ws + wb.add(sizeof(double) * (size_t)n * n));
    int *pairs = reinterpret_cast<int *>(ws + wb.add(sizeof(int) * (size_t)ne * (ne - 1)));
    double *out = reinterpret_cast<double *>(ws + wb.add(sizeof(double) * 4));
    double *w = reinterpret_cast<double *>(ws + wb.add(sizeof(double) * n));
    int *rank = reinterpret_cast<int *>(ws + wb.add(sizeof(int) * n));
    const bool multi = n >= SCALAR_MULTI_MIN;
    double *A2 = multi ? reinterpret_cast<double *>(ws + wb.add(sizeof(double) * (size_t)n * n)) : nullptr;
    int *rot = multi ? reinterpret_cast<int *>(ws + wb.add(sizeof(int) * 4)) : nullptr;
    const bool big = n >= SCALAR_REFINE_MIN;
    double *A0 = big ? reinterpret_cast<double *>(ws + wb.add(sizeof(double) * (size_t)n * n)) : nullptr;
    double *T1 = big ? reinterpret_cast<double *>(ws + wb.add(sizeof(double) * (size_t)n * n)) : nullptr;
    double *part = big ? reinterpret_cast<double *>(ws + wb.add(sizeof(double) * ((size_t)n + 8))) : nullptr;
    std::vector<int> hp, hs;
    make_schedule(ne, JACOBI_ORDER_ROUND_ROBIN, hp, hs);
    JX_HIP(hipMemcpyAsync(pairs, hp.data(), sizeof(int) * hp.size(), hipMemcpyHostToDevice, s));
    launch_sym_full(n, dA, lda, uplo, A, s);
    const bool vec = o.want_vectors && dQ;
    if (vec) launch_set_identity(n, n, Q, n, s);
    const bool rel = o.threshold == 1;
    const double tol = o.tol > 0.0 ? o.tol : (rel ? 2.220446049250313e-16 : 1e-14);
    double h[4] = {0.0, 0.0, 0.0, 0.0};  // sweeps, Xi(A), ||A||_F, rotations of the last sweep
    if (!multi) {
        launch_scalar_rr(n, ne, pairs, A, vec ? Q : nullptr, tol, o.max_sweeps, rel ? 1 : 0, out, s);
        JX_HIP(hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, s));
        JX_HIP(hipStreamSynchronize(s));
    } else {
        // one launch per round; the rounds alternate between A and A2
        DeviceCtx &ctx = device_ctx();
        std::lock_guard<std::mutex> lk(ctx.mu);  // its pinned scalars
        double *hs2 = reinterpret_cast<double *>(ctx.pinned);
        launch_scalar_norms(n, A, out, s);
        JX_HIP(hipMemcpyAsync(hs2, out, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
        JX_HIP(hipStreamSynchronize(s));
        double off2 = hs2[0];
        const double fro = std::sqrt(hs2[1]);
        // absolute mode: pairs with |a_pq| <= tol ||A||_F / sqrt(n (n - 1))
        // are not rotated, so a sweep that rotates none meets the stop test
        const double skip = tol * fro / std::sqrt((double)n * (n - 1));
        int sw = 0, rotated = 1;
        double *cur = A, *nxt = A2;
        const int H = ne / 2;
        auto sweeps_to = [&](int cap) {
            rotated = 1;
            while (sw < cap && off2 == off2 && (rel ? rotated > 0 : std::sqrt(off2) > tol * fro)) {
                launch_fill_int(rot, 1, 0, s);
                for (int r = 0; r < ne - 1; ++r) {
                    launch_scalar_round(n, ne, pairs + (size_t)2 * r * H, cur, nxt, vec ? Q : nullptr, tol,
                                        rel ? 1 : 0, skip, rot, s);
                    std::swap(cur, nxt);
                }
                ++sw;
                launch_scalar_norms(n, cur, out, s);
                JX_HIP(hipMemcpyAsync(hs2, out, sizeof(double), hipMemcpyDeviceToHost, s));
                JX_HIP(hipMemcpyAsync(hs2 + 2, rot, sizeof(int), hipMemcpyDeviceToHost, s));
                JX_HIP(hipStreamSynchronize(s));
                off2 = hs2[0];
                rotated = *reinterpret_cast<int *>(hs2 + 2);
            }
        };
        if (big) JX_HIP(hipMemcpyAsync(A0, A, sizeof(double) * (size_t)n * n, hipMemcpyDeviceToDevice, s));
        sweeps_to(o.max_sweeps);
        // Orthogonality refinement (absolute mode with vectors, n >= 256,
        // unless opts.refine = 0): the rotations' rounding leaves Q^T Q - I
        // growing with n.  Newton-Schulz steps Q <- Q (3 I - Q^T Q) / 2 until
        // one starts from ||Q^T Q - I||_F^2 <= 1e-16, then A_1 = Q^T A_0 Q
        // (symmetrised) replaces A and the sweeps continue to the tolerance.
        const bool refine = big && vec && !rel && o.refine != 0 && off2 == off2 && std::sqrt(off2) <= tol * fro;
        if (refine) {
            for (int it = 0; it < 4; ++it) {
                launch_gemm_f64('T', 'N', n, n, n, 1.0, Q, n, Q, n, 0.0, T1, n, s);
                launch_dev_identity(n, T1, n, part, part + n, s);
                double dev2 = 0.0;
                JX_HIP(hipMemcpyAsync(&dev2, part + n, sizeof(double), hipMemcpyDeviceToHost, s));
                JX_HIP(hipStreamSynchronize(s));
                if (!(dev2 > 1e-30)) break;
                JX_HIP(hipMemcpyAsync(nxt, Q, sizeof(double) * (size_t)n * n, hipMemcpyDeviceToDevice, s));
                launch_gemm_f64('N', 'N', n, n, n, -0.5, Q, n, T1, n, 1.5, nxt, n, s);
                JX_HIP(hipMemcpyAsync(Q, nxt, sizeof(double) * (size_t)n * n, hipMemcpyDeviceToDevice, s));
                if (dev2 <= 1e-16) break;
            }
            launch_gemm_f64('N', 'N', n, n, n, 1.0, A0, n, Q, n, 0.0, T1, n, s);
            launch_gemm_f64('T', 'N', n, n, n, 1.0, Q, n, T1, n, 0.0, nxt, n, s);
            launch_sym_full(n, nxt, n, 'U', cur, s);
            launch_scalar_norms(n, cur, out, s);
            JX_HIP(hipMemcpyAsync(hs2, out, sizeof(double), hipMemcpyDeviceToHost, s));
            JX_HIP(hipStreamSynchronize(s));
            off2 = hs2[0];
            sweeps_to(sw + o.max_sweeps);
        }
        if (cur != A) JX_HIP(hipMemcpyAsync(A, cur, sizeof(double) * (size_t)n * n, hipMemcpyDeviceToDevice, s));
        h[0] = sw;
        h[1] = std::sqrt(off2);
        h[2] = fro;
        h[3] = rotated;
    }
    const int sweeps = (int)h[0];
    const bool done = rel ? h[3] == 0.0 : h[1] <= tol * h[2];
    int status = (std::isfinite(h[1]) && std::isfinite(h[2])) ? (done ? 0 : 1) : 2;
    if (status != 2) {
        launch_diag_of(n, A, n, w, s);
        if (o.sort) {
            launch_rank(n, w, +1, rank, s);
        } else {
            std::vector<int> id(n);
            for (int i = 0; i < n; ++i) id[i] = i;
            JX_HIP(hipMemcpyAsync(rank, id.data(), sizeof(int) * n, hipMemcpyHostToDevice, s));
        }
        launch_scatter_values(n, w, rank, dW, s);
        if (vec) launch_scatter_columns(n, n, Q, n, rank, dQ, ldq, s);
        JX_HIP(hipStreamSynchronize(s));
    }
    jacobi_info inf{};
    inf.status = status;
    inf.sweeps = sweeps;
    inf.sweeps_by_prec[2] = sweeps;
    inf.off_rel = h[2] > 0.0 ? h[1] / h[2] : 0.0;
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return status;
}

// ---------------------------------------------------------------------------
// Kernel-level entry points for tests
// ---------------------------------------------------------------------------

int run_subproblem(int count, int m2, const double *dAhat, double *dV, double *dD, int inner,
                   hipStream_t s) {
    SubArgs a{};
    a.mode = SUB_PLAIN;
    a.m2 = m2;
    a.count = count;
    a.ahat = dAhat;
    a.vout = dV;
    a.dout = dD;
    a.inner_sweeps = inner;
    launch_subproblem(a, s);
    JX_HIP(hipStreamSynchronize(s));
    return 0;
}

int run_pivot_step(int n, int b, double *dA, int npairs, const int *hPairs, double *dV, int *dPerm,
                   hipStream_t s) {
    const int N = n / b, m2 = 2 * b;
    const size_t nb = (size_t)N * (N + 1) / 2;
    DeviceBuffer buf;
    WorkspaceBuilder wb;
    const size_t o_ab = wb.add(sizeof(double) * nb * b * b);
    const size_t o_v = wb.add(sizeof(double) * (size_t)npairs * m2 * m2);
    const size_t o_p = wb.add(sizeof(int) * 2 * (size_t)npairs);
    buf.alloc(wb.total());
    double *ablk = reinterpret_cast<double *>(buf.ptr + o_ab);
    double *V = reinterpret_cast<double *>(buf.ptr + o_v);
    int *pairs = reinterpret_cast<int *>(buf.ptr + o_p);
    JX_HIP(hipMemcpyAsync(pairs, hPairs, sizeof(int) * 2 * npairs, hipMemcpyHostToDevice, s));
    launch_pack_sym(n, n, b, dA, n, 'U', ablk, s);
    launch_vperm_from_colmajor(npairs, m2, dV, V, s);
    PivotArgs pa{};
    pa.count = npairs;
    pa.m2 = m2;
    pa.pairs = pairs;
    pa.ablk = ablk;
    pa.V = V;
    pa.perm_out = dPerm;
    launch_pivot(pa, s);
    launch_colmajor_from_vperm(npairs, m2, V, dV, s);
    launch_unpack_sym(n, b, ablk, dA, n, s);
    JX_HIP(hipStreamSynchronize(s));
    return 0;
}

int run_block_step(int n, int b, double *dA, double *dQ, int npairs, const int *hPairs,
                   const double *dV, const double *dD, bool f32, hipStream_t s) {
    const int N = n / b, H = N / 2, m2 = 2 * b;
    const size_t nb = (size_t)N * (N + 1) / 2;
    DeviceBuffer buf;
    WorkspaceBuilder wb;
    const size_t o_ab = wb.add(sizeof(double) * nb * b * b);
    const size_t o_v = wb.add(sizeof(double) * (size_t)H * m2 * m2);
    const size_t o_f = wb.add(sizeof(int) * H);
    const size_t o_p = wb.add(sizeof(int) * 2 * H);
    const size_t o_t = wb.add(sizeof(int) * (size_t)H * (H - 1) + sizeof(int));
    const size_t o_m = wb.add(sizeof(int) * (size_t)H * (H - 1) / 2 + sizeof(int));
    const size_t o_s = wb.add(sizeof(double) * 4 * (size_t)b * b * (H * (H - 1) / 2 + 1));
    const size_t o_l = wb.add(sizeof(int) * 8 * (size_t)(H * (H - 1) / 2 + 1));
    // FP32 copies of A's blocks, V_hat (vperm32 order) and Q
    const size_t o_a32 = f32 ? wb.add(sizeof(float) * nb * b * b) : 0;
    const size_t o_v32 = f32 ? wb.add(sizeof(float) * (size_t)H * m2 * m2) : 0;
    const size_t o_q32 = f32 && dQ ? wb.add(sizeof(float) * (size_t)n * n) : 0;
    buf.alloc(wb.total());
    double *ablk = reinterpret_cast<double *>(buf.ptr + o_ab);
    double *V = reinterpret_cast<double *>(buf.ptr + o_v);
    int *flags = reinterpret_cast<int *>(buf.ptr + o_f);
    int *pairs = reinterpret_cast<int *>(buf.ptr + o_p);
    int *tiles = reinterpret_cast<int *>(buf.ptr + o_t);
    int *qmask = reinterpret_cast<int *>(buf.ptr + o_m);
    void *side = buf.ptr + o_s;
    // The sweep's two-phase tile update: the first half of the tiles take
    // the part of critical tiles (masks cycling through one block of either
    // column half and two opposite blocks), then the bounded kernel does the
    // rest of those and every other tile whole.
    std::vector<int> ht, hq;
    for (int a = 0; a < H; ++a)
        for (int c = a + 1; c < H; ++c) { ht.push_back(a); ht.push_back(c); }
    const int ntiles = (int)ht.size() / 2, nq = (ntiles + 1) / 2;
    const int pattern[6] = {1, 2, 4, 8, 9, 6};
    for (int i = 0; i < nq; ++i) hq.push_back(pattern[i % 6]);
    (void)npairs;
    JX_HIP(hipMemcpyAsync(pairs, hPairs, sizeof(int) * 2 * H, hipMemcpyHostToDevice, s));
    if (!ht.empty()) JX_HIP(hipMemcpyAsync(tiles, ht.data(), sizeof(int) * ht.size(), hipMemcpyHostToDevice, s));
    if (!hq.empty()) JX_HIP(hipMemcpyAsync(qmask, hq.data(), sizeof(int) * hq.size(), hipMemcpyHostToDevice, s));
    JX_HIP(hipMemsetAsync(flags, 0, sizeof(int) * H, s));
    launch_pack_sym(n, n, b, dA, n, 'U', ablk, s);
    launch_vperm_from_colmajor(H, m2, dV, V, s);
    launch_write_pair_blocks(H, b, pairs, dD, ablk, s);
    // copies of the critical blocks' originals, which the critical kernel reads
    std::vector<int> hl;
    for (int i = 0; i < nq; ++i)
        for (int quad = 0; quad < 4; ++quad) {
            if (!((hq[i] >> quad) & 1)) continue;
            const int X = hPairs[2 * ht[2 * i] + (quad >> 1)], Y = hPairs[2 * ht[2 * i + 1] + (quad & 1)];
            hl.push_back((int)ublk(std::min(X, Y), std::max(X, Y)));
            hl.push_back(4 * i + quad);
        }
    int *lst = reinterpret_cast<int *>(buf.ptr + o_l);
    if (!hl.empty()) JX_HIP(hipMemcpyAsync(lst, hl.data(), sizeof(int) * hl.size(), hipMemcpyHostToDevice, s));
    if (f32) {
        float *a32 = reinterpret_cast<float *>(buf.ptr + o_a32);
        float *v32 = reinterpret_cast<float *>(buf.ptr + o_v32);
        launch_cast_to_f32(nb * b * b, ablk, a32, s);
        launch_vperm32_from_colmajor(H, m2, dV, v32, s);
        launch_copy_blocks32(b, a32, lst, (int)hl.size() / 2, side, s);
        launch_update_a32(b, H, pairs, a32, v32, flags, tiles, nq, s, UA_QUAD, qmask, nq, side);
        launch_update_a32(b, H, pairs, a32, v32, flags, tiles, ntiles, s, 1, qmask, nq, side);
        if (dQ) {
            float *q32 = reinterpret_cast<float *>(buf.ptr + o_q32);
            launch_cast_to_f32((size_t)n * n, dQ, q32, s);
            launch_update_q32(b, H, pairs, q32, n, n, v32, flags, s);
            launch_cast_to_f64((size_t)n * n, q32, dQ, s);
        }
        launch_cast_to_f64(nb * b * b, a32, ablk, s);
    } else {
        launch_copy_blocks(b, ablk, lst, (int)hl.size() / 2, side, s);
        launch_update_a(b, H, pairs, ablk, V, flags, tiles, nq, s, UA_QUAD, qmask, nq, side);
        launch_update_a(b, H, pairs, ablk, V, flags, tiles, ntiles, s, 1, qmask, nq, side);
        if (dQ) launch_update_q(b, H, pairs, dQ, n, n, V, flags, s);
    }
    launch_unpack_sym(n, b, ablk, dA, n, s);
    JX_HIP(hipStreamSynchronize(s));
    return 0;
}

}  // namespace jx
