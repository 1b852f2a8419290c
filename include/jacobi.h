/*
 * jacobi.h -- C ABI of libjacobi.so, an MI355X (gfx950) blocked Jacobi
 * eigensolver and one-sided Jacobi SVD.
 *
 * Method: Demmel, Luo, Schneider, Wang, "Minimizing the Arithmetic and
 * Communication Complexity of Jacobi's Method for Eigenvalues and Singular
 * Values: Part Two -- Parallel Algorithms" (arXiv 2608.28952).
 *   - jacobi_eig: block Jacobi (Alg. 1, §2.1) run in the parallel form of
 *     Alg. 2 (§3): each step diagonalises N/2 disjoint 2b x 2b subproblems
 *     A([I,J],[I,J]) (one GPU workgroup each, the workgroups playing the
 *     processors of Alg. 2), then applies the block rotations to block rows,
 *     block columns and Q.  Convergence is measured by the off-norm Xi(A) of
 *     eq. (Omega_A), §2.1.
 *   - jacobi_svd: one-sided block Jacobi (Alg. 6, §6); each subproblem is the
 *     Gram block G(:,[I,J])^T G(:,[I,J]) of eq. (SVD_subproblem), formed on
 *     the fly; Sigma = column norms and U = G Sigma^+ at the end.
 *   - jacobi_eig_batched: many independent small problems in one launch.
 *
 * Conventions for every entry point
 *   - Matrices are column-major: element (i, j) at ptr[i + j * ld].
 *   - Pointers named d* are device pointers (HIP device memory) owned by the
 *     caller; pointers named h* are host pointers, read or written only during
 *     the call.  Inputs are never modified.  Outputs must not alias inputs.
 *   - All device work is enqueued on `stream` (NULL = the default stream).  The
 *     calls return after the results are complete (they synchronise `stream`),
 *     because the sweep count and status are reported on the host.
 *   - Scratch memory: `dWork`/`workBytes` may supply device workspace of at
 *     least the size returned by the matching *_workspace query; then the call
 *     allocates no device memory.  If dWork is NULL the library allocates (and
 *     frees) the workspace itself.
 *   - Per-device context: the first call on a device (or jacobi_init) creates
 *     a second stream, a few events and 4 KiB of pinned host memory for that
 *     device, kept until the process ends.  jacobi_eig and jacobi_svd use them
 *     and run one at a time per device (a mutex); calls on different devices
 *     run concurrently.
 *   - Return value (also stored in info->status when info is non-NULL):
 *         0    success
 *        -i    argument i (1-based) is invalid
 *      -100    dWork too small
 *         1    not converged within opts->max_sweeps (outputs hold the last
 *              iterate, sorted)
 *         2    non-finite value in the input or an iterate
 *         3    HIP runtime error (text from jacobi_last_error())
 */
#ifndef JACOBI_H
#define JACOBI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t *jacobi_stream_t; /* the same type as hipStream_t */

enum jacobi_order {
    JACOBI_ORDER_ROUND_ROBIN = 0,       /* N-1 rounds of N/2 disjoint block pairs     */
    JACOBI_ORDER_ANTIDIAG = 1,          /* Alg. 3: groups I + J = K (mod N)           */
    JACOBI_ORDER_ROUND_ROBIN_SORTED = 2 /* eig: round-robin, the indices permuted
                                           before each sweep so that the diagonal
                                           is ascending (A <- P^T A P, Q <- Q P);
                                           svd: as round-robin                     */
};

enum jacobi_prec {
    JACOBI_PREC_FP64 = 0,       /* every sweep in FP64                            */
    JACOBI_PREC_MIXED_FP32 = 1, /* FP32 MFMA sweeps, then FP64 recovery sweeps    */
    JACOBI_PREC_MIXED_BF16 = 2  /* reserved: BF16 sweeps are not implemented; the
                                   solvers return the opts argument's error code */
};

enum jacobi_dtype { JACOBI_F32 = 0, JACOBI_F64 = 1 };

typedef struct {
    double tol;           /* 0 (default) = the routine's own default.
                             eig: stop when Xi(A) <= tol * ||A||_F (1e-14);
                             svd: stop when every column pair has
                             |g_i^T g_j| <= tol * |g_i| |g_j| (sqrt(m) * eps) */
    int max_sweeps;       /* default 60; caps the sweeps up to the orthogonality
                             refinement (the sweeps after it may run up to 12
                             past the cap) */
    int block;            /* b; 0 = default (64 for n > 512, smaller below); eig
                             also 1 = scalar Jacobi (Alg. 1 with b = 1, round-
                             robin rounds of n/2 rotations in one workgroup;
                             n <= 1024, FP64, no warm start) */
    int ordering;         /* enum jacobi_order; default JACOBI_ORDER_ROUND_ROBIN_SORTED */
    int precision;        /* enum jacobi_prec */
    int inner_max_sweeps; /* cap on inner scalar sweeps per subproblem; 0 = until
                             the subproblem's off-norm <= eps ||A_hat||_F (cap 30).
                             Default 1: the paper allows approximate
                             diagonalisation of the subproblem (§3).  eig: after
                             30 sweeps without reaching tol, the remaining
                             sweeps solve each subproblem to convergence
                             (repeated eigenvalues converge only linearly with
                             approximate inner solves). */
    int refine;           /* 1 = orthogonality refinement of Q/V (Newton-Schulz,
                             then a recomputed FP64 A = Q^T A0 Q or G = G0 V and
                             FP64 sweeps to tol); -1 = automatic (default: on
                             for n >= 256 -- eig: with eigenvectors -- and in
                             mixed precision).  Blocked eig and svd refine
                             inside the quadratic phase (after the first sweep
                             that leaves off(A) <= 1e-8 ||A||_F, or the largest
                             cosine <= 1e-6, having cut it by 100x), so that
                             the sweep that finishes also absorbs the
                             recomputation's rounding; again at the end if
                             more than two sweeps follow */
    int sort;             /* 1 = eigenvalues ascending / sigma descending (default) */
    int want_vectors;     /* 0 = eigenvalues (singular values) only; default 1 */
    int threshold;        /* eig with block = 1: 0 = absolute stop test above
                             (default); 1 = the relative threshold of Demmel &
                             Veselic: a pair is rotated only when |a_pq| > tol *
                             sqrt(|a_pp a_qq|) (tol default eps), the sweeps stop
                             once a sweep rotates none -- every eigenvalue of a
                             graded positive definite A to high relative
                             accuracy.  Other paths: must be 0 */
    int precondition;     /* svd: reduced QR first (§6, "Preprocessing with QR"):
                             G = Q R by CholeskyQR2 on FP64 MFMA (shifted first
                             pass if the Gram matrix is not numerically positive
                             definite), one-sided Jacobi on R^T, U = Q V_R and
                             V = the normalised columns of R^T V_R after
                             Newton-Schulz steps.  1 or -1 (default) = on; 0 = off
                             (one-sided Jacobi on G itself).  Falls back to the
                             plain solve when the factorization fails or a
                             singular value is zero.  eig: unused */
    int pivot;            /* eig, b = 32 or 64: 1 = the pivoting step of the
                             convergence conditions (§2.1, after eq. (sweep
                             cost)) after every subproblem solve of the FP64
                             sweeps: LU with partial pivoting on the leading b
                             rows of V_hat selects a column permutation P, and
                             V_hat <- V_hat P, D_hat <- P^T D_hat P.  Default 0
                             (the paper's algorithms omit it).  svd, batched
                             and b = 1: must be 0 */
} jacobi_opts;

typedef struct {
    int status;             /* same as the return value */
    int sweeps;             /* total sweeps performed */
    int sweeps_by_prec[3];  /* sweeps in BF16, FP32, FP64 */
    int fallback_used;      /* batched warm start rejected -> cold start */
    double off_rel;         /* final Xi(A)/||A||_F (eig) or max relative cosine (svd) */
    double seconds;         /* wall time of the call */
} jacobi_info;

/* Fill *o with the defaults listed above.  Returns 0, or -1 if o is NULL. */
int jacobi_opts_default(jacobi_opts *o);

/* Create the per-device context of the current HIP device now (otherwise the
 * first solver call on the device does).  Returns 0, or 3 on a HIP error. */
int jacobi_init(void);

/* Device workspace in bytes needed by jacobi_eig / jacobi_svd /
 * jacobi_eig_batched for these sizes and options (o may be NULL = defaults). */
size_t jacobi_eig_workspace(int n, const jacobi_opts *o);
size_t jacobi_svd_workspace(int m, int n, const jacobi_opts *o);
size_t jacobi_eig_batched_workspace(int batch, const int *h_n, int dtype, const jacobi_opts *o);

/*
 * Symmetric eigendecomposition A = Q diag(W) Q^T (Alg. 1 Ensure clause).
 *   n          order (>= 0)
 *   dA, lda    symmetric input; only the `uplo` triangle ('U' or 'L') is read
 *   dW         out: n eigenvalues (ascending when opts->sort)
 *   dQ, ldq    out: n x n eigenvectors as columns (may be NULL when
 *              opts->want_vectors == 0)
 *   dQ0, ldq0  optional orthogonal start (warm start or resume from an
 *              earlier iterate): the sweeps start from Q0^T A Q0 and Q = Q0.
 *              NULL = identity.  Used when eigenvectors are requested or the
 *              precision is mixed; ignored for FP64 eigenvalues only.
 *   dWork, workBytes, opts (NULL = defaults), info (may be NULL), stream
 */
int jacobi_eig(int n, const double *dA, int lda, char uplo, double *dW, double *dQ, int ldq,
               const double *dQ0, int ldq0, void *dWork, size_t workBytes,
               const jacobi_opts *opts, jacobi_info *info, jacobi_stream_t stream);

/*
 * jacobi_eig without any device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, outputs and
 * status codes as jacobi_eig, minus dWork/workBytes: the workspace is a
 * static device array of this library, jacobi_eig_noalloc_max_bytes()
 * bytes (64 MiB) on every GPU the library runs on, held until the process
 * ends.  Its device address is looked up once per device, by jacobi_init
 * or by the first call on that device.
 *   - Orders whose workspace (jacobi_eig_workspace(n, opts)) exceeds the
 *     array are rejected with -1 before any device work (with the default
 *     options: n <= 1152 with eigenvectors, n <= 2432 eigenvalues only).
 *   - The call allocates nothing: no hipMalloc/hipFree, no allocating
 *     library routine; the caller passes inputs and outputs.
 *   - Every call on a GPU shares that GPU's array, which keeps the last
 *     call's contents (each call initialises what it reads).  Calls that
 *     overlap on one GPU (from several threads or streams) race on it.
 */
int jacobi_eig_noalloc(int n, const double *dA, int lda, char uplo, double *dW, double *dQ, int ldq,
                       const double *dQ0, int ldq0, const jacobi_opts *opts, jacobi_info *info,
                       jacobi_stream_t stream);
size_t jacobi_eig_noalloc_max_bytes(void);

/*
 * Thin SVD G = U diag(S) V^T by one-sided block Jacobi (Alg. 6, §6).
 *   m >= n >= 0 (m < n returns -1); dG, ldg: m x n input
 *   dS: n singular values (descending when opts->sort)
 *   dU, ldu: m x n left vectors, U = G_final Sigma^+ (a zero sigma gives a
 *   zero column); dV, ldv: n x n right vectors.  dU/dV may be NULL when
 *   opts->want_vectors == 0.
 */
int jacobi_svd(int m, int n, const double *dG, int ldg, double *dS, double *dU, int ldu,
               double *dV, int ldv, void *dWork, size_t workBytes, const jacobi_opts *opts,
               jacobi_info *info, jacobi_stream_t stream);

/*
 * Batched symmetric eigendecomposition of `batch` independent matrices of
 * orders h_n[k] (0 <= h_n[k] <= 256; order 0 is skipped), one graph launch
 * (batching is an addition, not in the paper; the per-matrix method is
 * the block Jacobi of §3 with the round-robin ordering, applied inside one
 * workgroup).
 *   h_n, h_offA  host arrays: orders and element offsets (int64) of matrix k in
 *              dA and dQ; matrix k is column-major with leading dimension
 *              h_n[k]; only its upper triangle is read
 *   dtype      JACOBI_F32 or JACOBI_F64: element type of dA
 *   dW         out: eigenvalues, matrix k at offset sum_{i<k} h_n[i]
 *              (ascending when opts->sort)
 *   dQ         out: FP64 eigenvectors (columns) at the offsets h_offA; may be
 *              NULL when opts->want_vectors == 0
 *   dQ0        optional FP64 warm starts in the layout of dQ (NULL = cold): the
 *              FP64 refinement starts from Q0 (Newton-Schulz steps
 *              Q <- Q (3 I - Q^T Q) / 2 until one starts from
 *              ||Q^T Q - I||_F <= 1e-8, at most four, then Q^T A Q); a warm
 *              start that does not lower the off-norm is replaced by the cold
 *              start (info[k].fallback_used = 1)
 *   opts       tol (0 = 1e-14: off(A) <= tol ||A||_F per matrix), max_sweeps
 *              (FP64 sweeps), block (0 = tuned per size bucket, or 8 / 16 =
 *              the block size of the two-level scheme), precision
 *              (JACOBI_PREC_FP64: FP64 sweeps only; otherwise an FP32 phase
 *              precedes the FP64 refinement where the tuning table says so),
 *              want_vectors, sort.  ordering, inner_max_sweeps, refine and
 *              precondition are not used; threshold and pivot must be 0
 *              (-11 otherwise).
 *   dWork      workspace of jacobi_eig_batched_workspace() bytes, or NULL (the
 *              library allocates it; the graph is then not cached)
 *   info       NULL or an array of `batch` records: status, sweeps,
 *              sweeps_by_prec[1] (FP32) / [2] (FP64), fallback_used, off_rel
 * Returns the largest per-matrix status (0, 1 not converged, 2 non-finite
 * input), a negative argument index (1-based; -11 for opts->block), -100 for a
 * short workspace, or 3 for a HIP error.  The graph (queue reset, then per
 * size class a persistent FP32 kernel and a persistent FP64 kernel, classes on
 * parallel streams) is cached for calls with the same sizes, offsets, pointers
 * and options.
 */
int jacobi_eig_batched(int batch, const int *h_n, const int64_t *h_offA, int dtype, const void *dA,
                       double *dW, double *dQ, const double *dQ0, void *dWork, size_t workBytes,
                       const jacobi_opts *opts, jacobi_info *info, jacobi_stream_t stream);

/*
 * Tuning table of jacobi_eig_batched: per element type and size bucket
 * (0: n <= 32, 1: <= 64, 2: <= 128, 3: <= 192, 4: <= 256) the block size bs
 * (8 or 16) and the FP32 phase (mixed: 0 none, 1 until off(A) <= 1e-5
 * ||A||_F, 2 until 1e-3 ||A||_F; either ends early when the decrease
 * stalls).  The active table is the
 * JSON file named by the environment variable JACOBI_TUNE_FILE when it parses
 * and was written for the current device, else built-in defaults.
 *   jacobi_batched_tuning: returns 1 (from the file), 0 (defaults) or -1.
 *   jacobi_batched_autotune: times every (bs, mixed) candidate on a seeded
 *     calibration batch of `per_bucket` random symmetric matrices per bucket
 *     (a batch that fills the GPU, e.g. 1024, times throughput); the active
 *     entry is timed first and kept unless a candidate whose every matrix
 *     converges is at least 3 % faster.  Writes the table and the timings
 *     (per bucket, the active entry's first) as JSON to `path` and makes it
 *     active for this process.
 *     Returns 0, -1 (arguments), -4 (file not written) or 3 (HIP error).
 *   jacobi_batched_graph_stats: cached-graph hits and graphs built so far.
 */
int jacobi_batched_tuning(int dtype, int bucket, int *bs, int *mixed);
int jacobi_batched_autotune(int dtype, int per_bucket, unsigned seed, const char *path);
int jacobi_batched_graph_stats(int *hits, int *builds);

/* ------------------------------------------------------------------------ */
/* Learned warm start (an addition; the paper has no learned part)          */
/* ------------------------------------------------------------------------ */
/*
 * A small network maps the parameters theta (8) of a matrix family
 * A(theta) = A0 + sum_k theta_k B_k (order 64) to the 2016 strictly upper
 * coordinates (row-major (0,1), (0,2), ..., (62,63)) of a skew generator S; the
 * warm start is Q0 = Qref cay(S), cay(S) = (I - S)^{-1} (I + S), handed to
 * jacobi_eig_batched as dQ0.  Network: 8 -> 256 -> 256 -> 2016, GELU (tanh
 * form) on the hidden layers, linear output; GEMMs on BF16 MFMA with FP32
 * accumulation.
 *
 * Parameter vector (jws_param_count() FP32 values; the gradient and the BF16
 * copy use the same layout): W1 (16 x 256, rows 8..15 zero: the input is
 * padded to 16 features), W2 (256 x 256), W3 (256 x 2016), all row-major
 * K x N, then b1 (256), b2 (256), b3 (2016).  The forward and backward read
 * the weights from the BF16 copy and the biases from the FP32 vector (dBias
 * = its b1, i.e. element offset 16*256 + 256*256 + 256*2016).
 * Activations: dActs holds jws_acts_bytes(batch) bytes of BF16 values per
 * call, row-major B x features, at these element offsets (in units of B):
 * the forward's input X0 (B x 16, features 8..15 zero) at 0, Z1 at 16, H1 at
 * 272, Z2 at 528, H2 at 784 (each B x 256; Z = pre-activation, H = GELU(Z));
 * the backward's dL/dZ2 at 1040 and dL/dZ1 at 1296 (B x 256) and the BF16 copy
 * of dL/dOut at 1552 (B x 2016).  A backward must use the buffer of the
 * forward of the same batch.
 * All pointers are device pointers owned by the caller; row-major B x
 * features.  The calls enqueue on `stream` and return without waiting.
 * Returns 0, -i (argument i invalid) or 3 (HIP error).
 */
size_t jws_param_count(void);
size_t jws_acts_bytes(int batch);
/* dOut (B x 2016 FP32) = network(dTheta (B x 8 FP32)) */
int jws_mlp_forward(int batch, const float *dTheta, const uint16_t *dWbf16, const float *dBias, float *dOut,
                    uint16_t *dActs, jacobi_stream_t stream);
/* Gradients of a loss with dL/dOut = dGradOut: dGradW (weight part of the
 * parameter layout, FP32) and dGradB (b1 | b2 | b3).  dGradOut and the
 * back-propagated dL/dZ are rounded to BF16 for the MFMA products. */
int jws_mlp_backward(int batch, const uint16_t *dActs, const float *dGradOut, const uint16_t *dWbf16, float *dGradW,
                     float *dGradB, jacobi_stream_t stream);
/* Mean squared error over B x 2016 outputs: dLoss[0] (FP64) and, if dGradOut
 * is not NULL, dGradOut = 2 (dOut - dTarget) / (B * 2016). */
int jws_mse(int batch, const float *dOut, const float *dTarget, float *dGradOut, double *dLoss,
            jacobi_stream_t stream);
/* One Adam step (bias-corrected, Kingma & Ba) on nparams FP32 values; the
 * BF16 copy is refreshed (round to nearest, ties to even).  step >= 1. */
int jws_adam_step(int nparams, float *dMaster, uint16_t *dWbf16, const float *dGrad, float *dM, float *dV, float lr,
                  float beta1, float beta2, float eps, int step, jacobi_stream_t stream);
/* BF16 copy (nearest, ties to even) of count FP32 values. */
int jws_to_bf16(size_t count, const float *dSrc, uint16_t *dDst, jacobi_stream_t stream);
/* dS: batch column-major n x n skew matrices whose strictly upper entries
 * (row-major order) are dCoords * dStd + dMean (dMean / dStd may be NULL). */
int jws_skew_from_coords(int batch, int n, const float *dCoords, const float *dMean, const float *dStd, double *dS,
                         jacobi_stream_t stream);
/* dQ0[k] = dQref (I - dS[k])^{-1} (I + dS[k]) for batch skew-symmetric FP64
 * column-major n x n matrices, n <= 64. */
int jws_cayley_batched(int batch, int n, const double *dS, const double *dQref, double *dQ0, jacobi_stream_t stream);

/* Training data of the warm start.
 * jws_family_matrices: dA[c] = dA0 + sum_t dTheta[c k + t] dB[t] for c < count,
 *   every matrix n x n FP64 (dTheta count x k row-major, dB k matrices).
 * jws_canonical_targets: for count solutions dQ (n x n column-major each, the
 *   eigenvectors as columns, eigenvalues ascending; 2 <= n <= 64) and the
 *   reference dQref: W = Qref^T Q, its columns matched to Qref's columns by
 *   overlap (n times the largest remaining |W_ij|, ties to the lowest
 *   i n + j), column signs making diag(W) >= 0, the column of smallest
 *   |W_jj| (lowest j) negated when det W < 0, S = (W - I)(W + I)^{-1} (Gauss-
 *   Jordan with partial pivoting, FP64) made exactly skew.  dCoords (count x
 *   n(n-1)/2 FP32, row-major strictly upper entries) receives S, dKeep[c] = 1
 *   when S is finite with max |S_ij| <= maxabs; otherwise the row is zero and
 *   dKeep[c] = 0.
 * jws_column_stats: mean and standard deviation (population, plus eps) of the
 *   columns of dX (rows x cols FP32) over the rows with dKeep != 0 (`kept`
 *   of them); dWork: jws_column_stats_work(rows, cols) bytes.  Partial sums
 *   per 1024 rows in FP64, added in a fixed order.
 * jws_gather_standardize: for r < kept, dXo[r] = dX[dIdx[r]] (xcols values)
 *   and dTo[r] = (dT[dIdx[r]] - dMean) / dStd (tcols values), FP32 rows.
 * All enqueue on `stream`; return 0, -i or 3. */
int jws_family_matrices(int count, int n, int k, const double *dTheta, const double *dA0, const double *dB, double *dA,
                        jacobi_stream_t stream);
int jws_canonical_targets(int count, int n, const double *dQ, const double *dQref, float *dCoords, int *dKeep,
                          double maxabs, jacobi_stream_t stream);
size_t jws_column_stats_work(int rows, int cols);
int jws_column_stats(int rows, int cols, const float *dX, const int *dKeep, int kept, float eps, float *dMean,
                     float *dStd, double *dWork, jacobi_stream_t stream);
int jws_gather_standardize(int kept, const int *dIdx, int xcols, const float *dX, int tcols, const float *dT,
                           const float *dMean, const float *dStd, float *dXo, float *dTo, jacobi_stream_t stream);

/* Text of the last error of the calling thread ("" if none). */
const char *jacobi_last_error(void);

/* ------------------------------------------------------------------------ */
/* Building blocks exported for kernel-level tests                           */
/* ------------------------------------------------------------------------ */

/*
 * The pair schedule used by the sweeps (Alg. 3 of §3, or the round-robin
 * ordering derived from it).  N even >= 2 block indices.  Writes
 * rounds * (N/2) pairs (I, J), I < J, 0-based, into hPairs (2 ints each,
 * capacity N * (N - 1) ints) and returns the number of rounds, or a negative
 * argument error.  For JACOBI_ORDER_ANTIDIAG the groups have unequal sizes;
 * hSizes (capacity N) receives the size of each group (may be NULL for
 * round-robin).
 */
int jacobi_schedule(int N, int ordering, int *hPairs, int *hSizes);

/*
 * Subproblem solver (the diagonalisation step of Alg. 2 on one processor):
 * for `count` independent symmetric matrices of order m2 (32, 64 or 128),
 * column-major and contiguous in dAhat (m2*m2 doubles each), run
 * `inner_sweeps` round-robin sweeps of scalar Jacobi (0 = until the
 * off-norm <= eps ||A_hat||_F, at most 30) and write the accumulated
 * orthogonal V_hat (dV, m2*m2 doubles each, column-major) and the rotated
 * matrix D_hat = V_hat^T A_hat V_hat (dD, same layout).  Returns 0 or an
 * error code.
 */
int jacobi_subproblem_solve(int count, int m2, const double *dAhat, double *dV, double *dD,
                            int inner_sweeps, jacobi_stream_t stream);

/*
 * One parallel step of Alg. 2 (§3) on explicit data: A (n x n, symmetric,
 * full column-major, lda = n) and Q (n x n, may be NULL) are updated in place
 * for the `npairs` disjoint block pairs hPairs (0-based, I < J, block size b;
 * n must be a multiple of 2b and npairs == n / (2b), i.e. every block index
 * belongs to one pair) with the rotations dV (npairs matrices of order 2b,
 * column-major) and diagonal blocks dD (same layout):
 *   A([I,J],[I,J]) <- D for each pair, every other block pair (p, q)
 *   A[p, q] <- V_p^T A[p, q] V_q, and Q(:, [I,J]) <- Q(:, [I,J]) V.
 */
int jacobi_block_step(int n, int b, double *dA, double *dQ, int npairs, const int *hPairs,
                      const double *dV, const double *dD, jacobi_stream_t stream);

/*
 * The pivoting step (§2.1, the convergence conditions after eq. (sweep cost))
 * by the kernel the solver runs with opts->pivot = 1, on explicit data in the
 * solver's storage: A (n x n symmetric, full column-major, lda = n) holds the
 * diagonalised subproblems D_hat in its pair blocks A([I,J],[I,J]); dV holds
 * npairs rotations V_hat of order 2b (column-major).  For each pair, LU with
 * partial pivoting on V_hat(0:b, :)^T (the first maximal |entry| on ties;
 * multipliers l = x_ik / x_kk, updates fma(-l, x_kj, x_ij)) gives the
 * permutation P; then V_hat <- V_hat P and A([I,J],[I,J]) <- P^T A([I,J],[I,J]) P
 * in place, other blocks untouched.  dPerm (may be NULL): npairs x 2b ints,
 * column j of V_hat P is column dPerm[j] of V_hat.  n, b, hPairs as for
 * jacobi_block_step.  Returns 0 or an error code.
 */
int jacobi_pivot_step(int n, int b, double *dA, int npairs, const int *hPairs, double *dV, int *dPerm,
                      jacobi_stream_t stream);

/*
 * The same step of Alg. 2 (§3) by the FP32 kernels of the precision ladder's
 * FP32 phase (JACOBI_PREC_MIXED_FP32): A, Q, V and D are rounded to FP32 on
 * entry, the tile and Q updates run on FP32 MFMA with FP32 accumulation, and
 * A and Q are widened back to FP64 in place.  Arguments, layouts, ownership
 * and error codes as for jacobi_block_step.
 */
int jacobi_block_step32(int n, int b, double *dA, double *dQ, int npairs, const int *hPairs,
                        const double *dV, const double *dD, jacobi_stream_t stream);

/*
 * The reduced QR factorization that precedes the one-sided SVD (§6,
 * "Preprocessing with QR"), by the kernels jacobi_svd uses: G (m x n,
 * m >= n >= 1, ldg >= m) = Q R with Q (m x n, ldq >= m) orthonormal columns and
 * R (n x n, ldr >= n) upper triangular with a positive diagonal (zero below).
 * CholeskyQR2 on FP64 MFMA: R_1 = chol(G^T G), Q_1 = G R_1^{-1}, then again on
 * Q_1, R = R_2 R_1; when the first Cholesky meets a non-positive pivot, the
 * first pass is shifted by 11 (m n + n (n + 1)) u ||G||_F^2 and CholeskyQR2
 * follows.  Allocates its own temporaries.  Returns 0, 1 (the factorization
 * failed: G is numerically rank deficient or not finite), -i for argument i,
 * or 3.
 */
int jacobi_qr(int m, int n, const double *dG, int ldg, double *dQ, int ldq, double *dR, int ldr,
              jacobi_stream_t stream);

/*
 * Gram blocks of the one-sided SVD (eq. SVD_subproblem, §6) by the kernels a
 * jacobi_svd sweep uses: for each of the npairs column-block pairs (I, J)
 * (0-based, I != J, block size b = 32 or 64), dAhat[p] (2b x 2b FP64,
 * column-major, contiguous per pair) = [G_I G_J]^T [G_I G_J], where G_I =
 * dG(:, I b .. I b + b - 1).  m >= n, n a multiple of b, ldg >= m.  The rows
 * are summed in the row chunks a solve of this m uses (MFMA partial sums per
 * chunk, then a fixed-order FP64 sum over chunks).  fp32 != 0: G is rounded to
 * FP32 and the partial sums run on FP32 MFMA with FP32 accumulation (the
 * precision ladder's FP32 phase).  Allocates its own temporaries; returns 0,
 * -i for argument i, or 3.
 */
int jacobi_gram_blocks(int m, int n, int b, const double *dG, int ldg, int npairs, const int *hPairs, int fp32,
                       double *dAhat, jacobi_stream_t stream);

/* ------------------------------------------------------------------------ */
/* Kernel profiling (benchmarks)                                             */
/* ------------------------------------------------------------------------ */

/* Kernel kinds reported by jacobi_profile_query. */
enum jacobi_prof_kind {
    JACOBI_PROF_SUBPROBLEM = 0, /* 2b x 2b subproblem solver                     */
    JACOBI_PROF_UPDATE_A = 1,   /* fused pair-tile update V_p^T A[p,q] V_q       */
    JACOBI_PROF_UPDATE_Q = 2,   /* Q(:, [I,J]) V_hat                              */
    JACOBI_PROF_GEMM = 3,       /* refinement GEMMs                              */
    JACOBI_PROF_GRAM = 4,       /* Gram blocks of the one-sided SVD              */
    JACOBI_PROF_UPDATE_A_REST = 5, /* pair tiles no next-round subproblem waits for,
                                      on the second stream beside the subproblems  */
    JACOBI_PROF_UPDATE_AQ = 6      /* b = 64: those tiles and the Q update in one
                                      launch on the second stream                 */
};

/*
 * on != 0: from now on every launch of the kernels above records a HIP event
 * pair on its launch stream plus its algorithmic work (flops and HBM bytes
 * the method needs for that launch; skipped pairs and rotation tiles whose
 * both sides were skipped count zero; a rotated 2b x 2b subproblem counts, per
 * inner sweep, 2b (2b - 1) / 2 scalar rotations of two rows and two columns
 * of the full 2b x 2b matrix and two columns of V_hat, 18 * 2b flops each, and
 * its three blocks read and written plus V_hat written).  Clears earlier
 * records.  Synchronises the device.
 * Not thread-safe against concurrent solver calls.  Returns 0 or 3.
 */
int jacobi_profile_enable(int on);

/* Totals over the recorded launches of one kind: launch count, summed event
 * time in milliseconds, summed algorithmic flops and bytes.  Any output
 * pointer may be NULL.  Synchronises the device.  Returns 0 or 3. */
int jacobi_profile_query(int kind, int *launches, double *total_ms, double *flops, double *bytes);

#ifdef __cplusplus
}
#endif
#endif /* JACOBI_H */
