/*
 * jacobi_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU reference for what the GPU library
 * computes.  Only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load this file's shared object.  The product path never
 * calls it and shares no code, header, table or helper with it.
 *
 * Method source: Demmel, Luo, Schneider, Wang, "Minimizing the Arithmetic and
 * Communication Complexity of Jacobi's Method for Eigenvalues and Singular
 * Values: Part Two -- Parallel Algorithms" (arXiv 2608.28952).
 *
 *   ora_eig            scalar cyclic Jacobi (the b = 1 case of Alg. 1, §2.1;
 *                      one 2x2 rotation per off-diagonal pair as described in
 *                      §1).  Stop test on the off-norm Xi(A) of eq. (Omega_A),
 *                      §2.1, summed directly.
 *   ora_svd            one-sided Jacobi SVD (Alg. 6, §6) with b = 1, i.e. the
 *                      Hestenes method, followed by Sigma = column norms and
 *                      U = G Sigma^+ (the last two steps of Alg. 6).
 *   ora_antidiag_list  Alg. 3 (index list generator, "cyclic by anti-diagonals").
 *   ora_rr_list        round-robin ordering for an even number of indices,
 *                      derived from Alg. 3 on N-1 indices (see below).
 *   ora_block_step     one parallel step of Alg. 2 (§3): the block row/column
 *                      update formulas applied to A and Q, and the replacement
 *                      of A([I,J],[I,J]) by D, in long double.
 *   ora_check_*        long-double invariants: off-norm, ||A - Q D Q^T||_F,
 *                      ||Q^T Q - I||_F, SVD residuals.
 *   ora_cayley         Cayley map W = (I - S)^{-1} (I + S) by Gaussian
 *                      elimination with partial pivoting, long double.
 *   ora_lupp_cols      the pivoting step of block Jacobi (§2.1, the
 *                      convergence conditions after eq. (sweep cost)): LU with
 *                      partial pivoting applied to the leading rows of the
 *                      subproblem's rotation, giving the column permutation
 *                      P of the update V_hat <- V_hat P.
 *
 * The 2x2 rotation used by ora_eig / ora_svd is the textbook symmetric Schur
 * decomposition (Golub & Van Loan, Matrix Computations, §8.5.2; Rutishauser
 * 1966): for the pivot block [[app, apq], [apq, aqq]],
 *     theta = (aqq - app) / (2 apq),
 *     t     = sgn(theta) / (|theta| + sqrt(1 + theta^2)),  sgn(0) = +1,
 *     c     = 1 / sqrt(1 + t^2),  s = t c,
 * and J = [[c, s], [-s, c]] on columns (p, q) gives J^T A J with a zero (p, q)
 * entry and diagonal app - t apq, aqq + t apq.  Each such rotation lowers the
 * squared off-norm by exactly 2 apq^2 (§1).
 *
 * Storage: column-major, element (i, j) of an n x n matrix at [i + j * ld].
 * Return codes: 0 ok, 1 not converged within max_sweeps, 2 non-finite input
 * or iterate, negative = invalid argument.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IDX(i, j, ld) ((size_t)(i) + (size_t)(j) * (size_t)(ld))

/* ------------------------------------------------------------------------ */
/* Orderings                                                                 */
/* ------------------------------------------------------------------------ */

/*
 * Alg. 3 (§3): for K = 0 .. P-1 (P = number of block indices, called sqrt(P)
 * in the paper), group K holds every (I, J), 1 <= I < J <= P, with
 * I + J = K (mod P).  Output: pairs written 0-based as (I-1, J-1) into
 * `pairs` (2 ints each), group sizes into `sizes` (P entries).
 * Returns the total number of pairs, P (P - 1) / 2.
 */
int ora_antidiag_list(int P, int *pairs, int *sizes)
{
    int total = 0;
    if (P < 2) return 0;
    for (int K = 0; K < P; ++K) {
        int cnt = 0;
        /* for each I the one J in 1 .. P with I + J = K mod P; kept if J > I
         * (the pairs of the group in increasing I) */
        for (int I = 1; I <= P - 1; ++I) {
            int J = ((K - I) % P + P) % P;
            if (J == 0) J = P;
            if (J > I) {
                pairs[2 * total] = I - 1;
                pairs[2 * total + 1] = J - 1;
                ++total;
                ++cnt;
            }
        }
        sizes[K] = cnt;
    }
    return total;
}

/*
 * Round-robin ordering for an even count N of indices: N - 1 rounds of N / 2
 * disjoint pairs covering every unordered pair once.  Round K (K = 0 .. N-2)
 * is Alg. 3's group K taken over the odd count M = N - 1 of indices
 * 1 .. M (pairs with I + J = K mod M), plus the one index I* of 1 .. M left
 * idle by that group (2 I* = K mod M) paired with index N.  For odd N this is
 * Alg. 3 itself (N rounds, one index idle per round).  Pairs are written
 * 0-based, each as (smaller, larger); sizes[K] receives the round size.
 * Returns the number of rounds.
 */
int ora_rr_list(int N, int *pairs, int *sizes)
{
    if (N < 2) return 0;
    if (N % 2 == 1) {
        ora_antidiag_list(N, pairs, sizes);
        return N;
    }
    int M = N - 1, total = 0;
    for (int K = 0; K < M; ++K) {
        int cnt = 0;
        for (int I = 1; I <= M - 1; ++I) {  /* the one J in 1 .. M with I + J = K mod M */
            int J = ((K - I) % M + M) % M;
            if (J == 0) J = M;
            if (J > I) {
                pairs[2 * total] = I - 1;
                pairs[2 * total + 1] = J - 1;
                ++total;
                ++cnt;
            }
        }
        for (int I = 1; I <= M; ++I)
            if ((2 * I) % M == K % M) {
                pairs[2 * total] = I - 1;
                pairs[2 * total + 1] = N - 1;
                ++total;
                ++cnt;
            }
        sizes[K] = cnt;
    }
    return M;
}

/* ------------------------------------------------------------------------ */
/* Scalar two-sided Jacobi                                                   */
/* ------------------------------------------------------------------------ */

/* eq. (Omega_A): Xi(A) = sqrt(sum_{i != j} a_ij^2), summed directly. */
double ora_offnorm(int n, const double *A, int lda)
{
    double s = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            if (i != j) s += A[IDX(i, j, lda)] * A[IDX(i, j, lda)];
    return sqrt(s);
}

static double frob(int n, const double *A, int lda)
{
    double s = 0.0;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) s += A[IDX(i, j, lda)] * A[IDX(i, j, lda)];
    return sqrt(s);
}

/* The symmetric Schur 2x2 of the header comment. */
static void schur2(double app, double aqq, double apq, double *c, double *s, double *t)
{
    double theta = (aqq - app) / (2.0 * apq);
    double sg = theta >= 0.0 ? 1.0 : -1.0;
    double tt;
    if (fabs(theta) > 1e150) /* 1 + theta^2 would overflow: t ~ 1/(2 theta) */
        tt = 0.5 / theta;
    else
        tt = sg / (fabs(theta) + sqrt(1.0 + theta * theta));
    *t = tt;
    *c = 1.0 / sqrt(1.0 + tt * tt);
    *s = tt * (*c);
}

/*
 * Rotate the pair (p, q) of the symmetric n x n matrix A (full storage) and
 * the columns p, q of Q (if non-NULL): A <- J^T A J, Q <- Q J.
 */
static void rotate_pair(int n, double *A, int lda, double *Q, int ldq, int p, int q,
                        double c, double s, double t)
{
    double apq = A[IDX(p, q, lda)];
    for (int k = 0; k < n; ++k) {
        if (k == p || k == q) continue;
        double akp = A[IDX(k, p, lda)], akq = A[IDX(k, q, lda)];
        double nkp = c * akp - s * akq;
        double nkq = s * akp + c * akq;
        A[IDX(k, p, lda)] = nkp;
        A[IDX(p, k, lda)] = nkp;
        A[IDX(k, q, lda)] = nkq;
        A[IDX(q, k, lda)] = nkq;
    }
    A[IDX(p, p, lda)] -= t * apq;
    A[IDX(q, q, lda)] += t * apq;
    A[IDX(p, q, lda)] = 0.0;
    A[IDX(q, p, lda)] = 0.0;
    if (Q) {
        for (int k = 0; k < n; ++k) {
            double qkp = Q[IDX(k, p, ldq)], qkq = Q[IDX(k, q, ldq)];
            Q[IDX(k, p, ldq)] = c * qkp - s * qkq;
            Q[IDX(k, q, ldq)] = s * qkp + c * qkq;
        }
    }
}

static int all_finite(int m, int n, const double *A, int lda)
{
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i)
            if (!isfinite(A[IDX(i, j, lda)])) return 0;
    return 1;
}

/* Stable ascending (dir = +1) or descending (dir = -1) index sort by key. */
static void sort_index(int n, const double *key, int *perm, int dir)
{
    for (int i = 0; i < n; ++i) perm[i] = i;
    /* insertion sort: plain and stable */
    for (int i = 1; i < n; ++i) {
        int v = perm[i];
        int j = i - 1;
        while (j >= 0 && (dir > 0 ? key[perm[j]] > key[v] : key[perm[j]] < key[v])) {
            perm[j + 1] = perm[j];
            --j;
        }
        perm[j + 1] = v;
    }
}

/*
 * Scalar cyclic Jacobi eigensolver (Alg. 1 with b = 1).
 *
 *   n, A, lda   symmetric input (full storage read; only used, never written)
 *   W           out: n eigenvalues, ascending (stable by index on ties)
 *   Q, ldq      out: n x n eigenvectors, columns permuted like W (may be NULL)
 *   Q0, ldq0    optional start: iterate from Q0^T A Q0 with Q = Q0 (NULL = I)
 *   tol         stop when Xi(A) <= tol * ||A_0||_F (checked before each sweep)
 *   max_sweeps  sweep cap
 *   order       0 = row-cyclic (p < q lexicographic), 1 = round-robin rounds
 *               (ora_rr_list on the n scalar indices)
 *   nthreads    > 1 with order 1: the disjoint rotations of a round are
 *               applied in parallel (§3: disjoint transformations commute)
 *   max_rot     > 0: stop (status 1) once this many rotations were applied
 *               (bounds the work for timing samples); 0 = no cap
 *   check_rot   if non-NULL, every rotation checks the identity
 *               off^2(after) = off^2(before) - 2 apq^2 (§1) and the largest
 *               relative deviation is stored here (O(n^2) per rotation).
 *   sweeps_out, rot_out  sweeps performed, rotations applied
 *   relative    0: the stop test above, every nonzero a_pq rotated.  1: the
 *               relative threshold of Demmel & Veselic (cited in §1): pair
 *               (p, q) is rotated only when |a_pq| > tol sqrt(|a_pp a_qq|),
 *               and the sweeps stop when a sweep rotates no pair (for a
 *               positive definite A this computes every eigenvalue to high
 *               relative accuracy).
 */
static int rotate_it(double app, double aqq, double apq, double tol, int relative)
{
    if (apq == 0.0) return 0;
    return relative ? fabs(apq) > tol * sqrt(fabs(app * aqq)) : 1;
}
int ora_eig(int n, const double *A_in, int lda, double *W, double *Q, int ldq,
            const double *Q0, int ldq0, double tol, int max_sweeps, int order,
            int nthreads, long long max_rot, double *check_rot, int *sweeps_out,
            long long *rot_out, int relative)
{
    if (n < 0) return -1;
    if (lda < (n > 1 ? n : 1)) return -3;
    if (Q && ldq < (n > 1 ? n : 1)) return -6;
    if (sweeps_out) *sweeps_out = 0;
    if (rot_out) *rot_out = 0;
    if (check_rot) *check_rot = 0.0;
    if (n == 0) return 0;
    if (!all_finite(n, n, A_in, lda)) return 2;

    double *A = (double *)malloc(sizeof(double) * (size_t)n * n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) A[IDX(i, j, n)] = A_in[IDX(i, j, lda)];
    double *Qw = NULL;
    if (Q) {
        Qw = (double *)calloc((size_t)n * n, sizeof(double));
        if (Q0) {
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) Qw[IDX(i, j, n)] = Q0[IDX(i, j, ldq0)];
        } else {
            for (int i = 0; i < n; ++i) Qw[IDX(i, i, n)] = 1.0;
        }
    }
    if (Q0) { /* A <- Q0^T A Q0, plain triple loops */
        double *T = (double *)calloc((size_t)n * n, sizeof(double));
        for (int j = 0; j < n; ++j)
            for (int k = 0; k < n; ++k) {
                double qkj = Q0[IDX(k, j, ldq0)];
                for (int i = 0; i < n; ++i) T[IDX(i, j, n)] += A[IDX(i, k, n)] * qkj;
            }
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) {
                double s = 0.0;
                for (int k = 0; k < n; ++k) s += Q0[IDX(k, i, ldq0)] * T[IDX(k, j, n)];
                A[IDX(i, j, n)] = s;
            }
        for (int j = 0; j < n; ++j) /* symmetrize the rounding of the product */
            for (int i = j + 1; i < n; ++i) {
                double v = 0.5 * (A[IDX(i, j, n)] + A[IDX(j, i, n)]);
                A[IDX(i, j, n)] = v;
                A[IDX(j, i, n)] = v;
            }
        free(T);
    }

    double fro0 = frob(n, A_in, lda);
    int *rr_pairs = NULL, *rr_sizes = NULL, rounds = 0;
    if (order == 1 && n >= 2) {
        rr_pairs = (int *)malloc(sizeof(int) * (size_t)n * (n - 1));
        rr_sizes = (int *)malloc(sizeof(int) * (size_t)(n + 1));
        rounds = ora_rr_list(n, rr_pairs, rr_sizes);
    }
    int status = 1, sweeps = 0;
    long long nrot = 0;
    double worst = 0.0;

    long long rot_before = -1;
    for (;;) {
        double off = ora_offnorm(n, A, n);
        if (!isfinite(off)) { status = 2; break; }
        if (!relative && off <= tol * fro0) { status = 0; break; }
        if (relative && nrot == rot_before) { status = 0; break; }  /* the last sweep rotated nothing */
        if (sweeps >= max_sweeps) { status = 1; break; }
        if (max_rot > 0 && nrot >= max_rot) { status = 1; break; }
        rot_before = nrot;
        if (order == 0) {
            for (int p = 0; p < n - 1; ++p)
                for (int q = p + 1; q < n; ++q) {
                    double apq = A[IDX(p, q, n)];
                    if (!rotate_it(A[IDX(p, p, n)], A[IDX(q, q, n)], apq, tol, relative)) continue;
                    if (max_rot > 0 && nrot >= max_rot) break;
                    double c, s, t, before = 0.0;
                    if (check_rot) before = ora_offnorm(n, A, n);
                    schur2(A[IDX(p, p, n)], A[IDX(q, q, n)], apq, &c, &s, &t);
                    rotate_pair(n, A, n, Qw, n, p, q, c, s, t);
                    ++nrot;
                    if (check_rot) {
                        double after = ora_offnorm(n, A, n);
                        double d = fabs(before * before - after * after - 2.0 * apq * apq);
                        double rel = d / (before * before > 0 ? before * before : 1.0);
                        if (rel > worst) worst = rel;
                    }
                }
        } else {
            int base = 0;
            for (int K = 0; K < rounds; ++K) {
                if (max_rot > 0 && nrot >= max_rot) break;
                int np = rr_sizes[K];
                const int *pr = rr_pairs + 2 * base;
                base += np;
                if (nthreads <= 1) {
                    for (int k = 0; k < np; ++k) {
                        int p = pr[2 * k], q = pr[2 * k + 1];
                        double apq = A[IDX(p, q, n)];
                        if (!rotate_it(A[IDX(p, p, n)], A[IDX(q, q, n)], apq, tol, relative)) continue;
                        double c, s, t, before = 0.0;
                        if (check_rot) before = ora_offnorm(n, A, n);
                        schur2(A[IDX(p, p, n)], A[IDX(q, q, n)], apq, &c, &s, &t);
                        rotate_pair(n, A, n, Qw, n, p, q, c, s, t);
                        ++nrot;
                        if (check_rot) {
                            double after = ora_offnorm(n, A, n);
                            double d = fabs(before * before - after * after - 2.0 * apq * apq);
                            double rel = d / (before * before > 0 ? before * before : 1.0);
                            if (rel > worst) worst = rel;
                        }
                    }
                } else {
                    /* Angles of the round from the current A, then the disjoint
                     * rotations applied: first all row pairs, then all column
                     * pairs, then Q; the pivot entries are set as in the
                     * sequential form. */
                    double *cs = (double *)malloc(sizeof(double) * 6 * (size_t)np);
                    double *dpp = cs + 4 * (size_t)np, *dqq = dpp + np;
                    for (int k = 0; k < np; ++k) {
                        int p = pr[2 * k], q = pr[2 * k + 1];
                        double apq = A[IDX(p, q, n)];
                        dpp[k] = A[IDX(p, p, n)];
                        dqq[k] = A[IDX(q, q, n)];
                        if (!rotate_it(dpp[k], dqq[k], apq, tol, relative)) apq = 0.0;  /* not rotated */
                        cs[4 * k + 3] = apq;
                        if (apq == 0.0) { cs[4 * k] = 1.0; cs[4 * k + 1] = 0.0; cs[4 * k + 2] = 0.0; continue; }
                        schur2(A[IDX(p, p, n)], A[IDX(q, q, n)], apq, &cs[4 * k], &cs[4 * k + 1], &cs[4 * k + 2]);
                        ++nrot;
                    }
#pragma omp parallel for num_threads(nthreads) schedule(static)
                    for (int k = 0; k < np; ++k) { /* rows p, q: A <- J^T A */
                        int p = pr[2 * k], q = pr[2 * k + 1];
                        double c = cs[4 * k], s = cs[4 * k + 1];
                        if (cs[4 * k + 3] == 0.0) continue;
                        for (int j = 0; j < n; ++j) {
                            double ap = A[IDX(p, j, n)], aq = A[IDX(q, j, n)];
                            A[IDX(p, j, n)] = c * ap - s * aq;
                            A[IDX(q, j, n)] = s * ap + c * aq;
                        }
                    }
#pragma omp parallel for num_threads(nthreads) schedule(static)
                    for (int k = 0; k < np; ++k) { /* columns p, q: A <- A J, Q <- Q J */
                        int p = pr[2 * k], q = pr[2 * k + 1];
                        double c = cs[4 * k], s = cs[4 * k + 1];
                        if (cs[4 * k + 3] == 0.0) continue;
                        for (int i = 0; i < n; ++i) {
                            double ap = A[IDX(i, p, n)], aq = A[IDX(i, q, n)];
                            A[IDX(i, p, n)] = c * ap - s * aq;
                            A[IDX(i, q, n)] = s * ap + c * aq;
                        }
                        if (Qw)
                            for (int i = 0; i < n; ++i) {
                                double ap = Qw[IDX(i, p, n)], aq = Qw[IDX(i, q, n)];
                                Qw[IDX(i, p, n)] = c * ap - s * aq;
                                Qw[IDX(i, q, n)] = s * ap + c * aq;
                            }
                    }
                    /* pivot block as in the sequential form: exact zeros and
                     * the closed-form diagonal (no other rotation of the round
                     * touches a_pp, a_qq or a_pq) */
                    for (int k = 0; k < np; ++k) {
                        int p = pr[2 * k], q = pr[2 * k + 1];
                        double apq = cs[4 * k + 3], t = cs[4 * k + 2];
                        if (apq == 0.0) continue;
                        A[IDX(p, p, n)] = dpp[k] - t * apq;
                        A[IDX(q, q, n)] = dqq[k] + t * apq;
                        A[IDX(p, q, n)] = 0.0;
                        A[IDX(q, p, n)] = 0.0;
                    }
                    free(cs);
                }
            }
        }
        ++sweeps;
    }

    if (status != 2) {
        for (int i = 0; i < n; ++i) W[i] = A[IDX(i, i, n)];
        int *perm = (int *)malloc(sizeof(int) * (size_t)n);
        double *w2 = (double *)malloc(sizeof(double) * (size_t)n);
        sort_index(n, W, perm, +1);
        for (int i = 0; i < n; ++i) w2[i] = W[perm[i]];
        memcpy(W, w2, sizeof(double) * (size_t)n);
        if (Q)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i) Q[IDX(i, j, ldq)] = Qw[IDX(i, perm[j], n)];
        free(perm);
        free(w2);
    }
    if (sweeps_out) *sweeps_out = sweeps;
    if (rot_out) *rot_out = nrot;
    if (check_rot) *check_rot = worst;
    free(A);
    free(Qw);
    free(rr_pairs);
    free(rr_sizes);
    return status;
}

/* ------------------------------------------------------------------------ */
/* One-sided Jacobi SVD (Alg. 6 with b = 1)                                  */
/* ------------------------------------------------------------------------ */

/*
 *   m >= n, G (m x n, ldg)  input, read only
 *   S       out: n singular values, descending (stable by index)
 *   U, ldu  out: m x n, U = G_final Sigma^+ (a zero sigma gives a zero column)
 *   V, ldv  out: n x n right singular vectors
 *   tol     a pair (p, q) is rotated when |g_p^T g_q| > tol sqrt(|g_p|^2 |g_q|^2);
 *           the sweeps stop when a sweep rotates nothing
 *   order   0 = row-cyclic, 1 = round-robin
 *   nthreads > 1 with order 1: the pairs of a round are disjoint column pairs,
 *           each rotation touching only its own two columns of G and V, so
 *           they run in parallel with the same result as one after another
 */
/* One Hestenes step on columns p, q of G (m rows) and V (n rows); returns 1
 * when the pair was rotated. */
static int hestenes_pair(int m, int n, double *G, double *Vw, int p, int q, double tol)
{
    double al = 0.0, be = 0.0, ga = 0.0;
    for (int i = 0; i < m; ++i) {
        double gp = G[IDX(i, p, m)], gq = G[IDX(i, q, m)];
        al += gp * gp;
        be += gq * gq;
        ga += gp * gq;
    }
    if (!(fabs(ga) > tol * sqrt(al * be))) return 0;
    double c, s, t;
    schur2(al, be, ga, &c, &s, &t);
    for (int i = 0; i < m; ++i) {
        double gp = G[IDX(i, p, m)], gq = G[IDX(i, q, m)];
        G[IDX(i, p, m)] = c * gp - s * gq;
        G[IDX(i, q, m)] = s * gp + c * gq;
    }
    for (int i = 0; i < n; ++i) {
        double vp = Vw[IDX(i, p, n)], vq = Vw[IDX(i, q, n)];
        Vw[IDX(i, p, n)] = c * vp - s * vq;
        Vw[IDX(i, q, n)] = s * vp + c * vq;
    }
    return 1;
}

int ora_svd(int m, int n, const double *G_in, int ldg, double *S, double *U, int ldu,
            double *V, int ldv, double tol, int max_sweeps, int order, int nthreads,
            int *sweeps_out, long long *rot_out)
{
    if (n < 0) return -2;
    if (m < n) return -1;
    if (ldg < (m > 1 ? m : 1)) return -4;
    if (sweeps_out) *sweeps_out = 0;
    if (rot_out) *rot_out = 0;
    if (n == 0) return 0;
    if (!all_finite(m, n, G_in, ldg)) return 2;

    double *G = (double *)malloc(sizeof(double) * (size_t)m * n);
    double *Vw = (double *)calloc((size_t)n * n, sizeof(double));
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) G[IDX(i, j, m)] = G_in[IDX(i, j, ldg)];
    for (int i = 0; i < n; ++i) Vw[IDX(i, i, n)] = 1.0;

    int *rr_pairs = NULL, *rr_sizes = NULL, rounds = 0, npairs_total = n * (n - 1) / 2;
    int *plist = (int *)malloc(sizeof(int) * 2 * (size_t)(npairs_total > 0 ? npairs_total : 1));
    if (order == 1 && n >= 2) {
        rr_pairs = plist;
        rr_sizes = (int *)malloc(sizeof(int) * (size_t)(n + 1));
        rounds = ora_rr_list(n, rr_pairs, rr_sizes);
    } else {
        int k = 0;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) { plist[2 * k] = p; plist[2 * k + 1] = q; ++k; }
    }
    int status = 1, sweeps = 0;
    long long nrot = 0;
    while (sweeps < max_sweeps) {
        int rotated = 0;
        if (order == 1 && nthreads > 1 && n >= 2) {
            int base = 0;
            for (int K = 0; K < rounds; ++K) {
                const int np = rr_sizes[K];
                const int *pr = plist + 2 * base;
                base += np;
                int rk = 0;
#pragma omp parallel for num_threads(nthreads) reduction(+ : rk) schedule(dynamic, 1)
                for (int k = 0; k < np; ++k) rk += hestenes_pair(m, n, G, Vw, pr[2 * k], pr[2 * k + 1], tol);
                rotated += rk;
            }
        } else {
            for (int k = 0; k < npairs_total; ++k)
                rotated += hestenes_pair(m, n, G, Vw, plist[2 * k], plist[2 * k + 1], tol);
        }
        nrot += rotated;
        ++sweeps;
        if (!all_finite(m, n, G, m)) { status = 2; break; }
        if (rotated == 0) { status = 0; break; }
    }
    if (status != 2) {
        double *sig = (double *)malloc(sizeof(double) * (size_t)n);
        for (int j = 0; j < n; ++j) {
            double s = 0.0;
            for (int i = 0; i < m; ++i) s += G[IDX(i, j, m)] * G[IDX(i, j, m)];
            sig[j] = sqrt(s);
        }
        int *perm = (int *)malloc(sizeof(int) * (size_t)n);
        sort_index(n, sig, perm, -1);
        for (int j = 0; j < n; ++j) {
            int pj = perm[j];
            S[j] = sig[pj];
            if (U)
                for (int i = 0; i < m; ++i)
                    U[IDX(i, j, ldu)] = sig[pj] > 0.0 ? G[IDX(i, pj, m)] / sig[pj] : 0.0;
            if (V)
                for (int i = 0; i < n; ++i) V[IDX(i, j, ldv)] = Vw[IDX(i, pj, n)];
        }
        free(sig);
        free(perm);
    }
    if (sweeps_out) *sweeps_out = sweeps;
    if (rot_out) *rot_out = nrot;
    free(G);
    free(Vw);
    free(plist);
    free(rr_sizes);
    return status;
}

/* ------------------------------------------------------------------------ */
/* One parallel step of Alg. 2 in long double                                */
/* ------------------------------------------------------------------------ */

/*
 * A (n x n, full, column-major) and Q (n x n, may be NULL) are updated in
 * place for one group of `npairs` disjoint block pairs (I, J), 0-based block
 * indices, block size b.  Vhat: npairs matrices of order 2b, column-major,
 * each split into b x b blocks V11 V12 / V21 V22; Dhat likewise (may be NULL,
 * then A([I,J],[I,J]) is left to the formulas).  The formulas of Alg. 2 (§3):
 *   A_IK <- V11^T A_IK + V21^T A_JK,   A_JK <- V12^T A_IK + V22^T A_JK  (K != I, J)
 *   A_KI <- A_KI V11 + A_KJ V21,       A_KJ <- A_KI V12 + A_KJ V22      (K != I, J)
 *   Q_KI <- Q_KI V11 + Q_KJ V21,       Q_KJ <- Q_KI V12 + Q_KJ V22      (all K)
 *   A([I,J],[I,J]) <- D
 * A block touched by two transformations is multiplied by one on the left and
 * by the other on the right, in either order (§3); here every left update of
 * the group is applied first, then every right update.
 */
static long double vget(const double *Vh, int b, int r, int c) { return (long double)Vh[IDX(r, c, 2 * b)]; }

int ora_block_step(int n, int b, double *A, double *Q, int npairs, const int *pairs,
                   const double *Vhat, const double *Dhat)
{
    if (b <= 0 || n % b) return -2;
    size_t nn = (size_t)n * n;
    long double *L = (long double *)malloc(sizeof(long double) * nn);
    long double *R = (long double *)malloc(sizeof(long double) * nn);
    for (size_t i = 0; i < nn; ++i) L[i] = A[i];
    int N = n / b;
    char *inpair = (char *)calloc((size_t)N, 1);
    for (int k = 0; k < npairs; ++k) { inpair[pairs[2 * k]] = 1; inpair[pairs[2 * k + 1]] = 1; }
    /* left (row) updates: rows of blocks I and J, every block column K != I, J */
    for (int k = 0; k < npairs; ++k) {
        int I = pairs[2 * k], J = pairs[2 * k + 1];
        const double *Vh = Vhat + (size_t)k * 4 * b * b;
        for (int K = 0; K < N; ++K) {
            if (K == I || K == J) continue;
            for (int c = 0; c < b; ++c) {
                int col = K * b + c;
                for (int r = 0; r < b; ++r) {
                    long double sI = 0.0L, sJ = 0.0L;
                    for (int t = 0; t < b; ++t) {
                        long double aI = (long double)A[IDX(I * b + t, col, n)];
                        long double aJ = (long double)A[IDX(J * b + t, col, n)];
                        /* (V11^T)(r,t) = V11(t,r); V21 = rows b.. of column r */
                        sI += vget(Vh, b, t, r) * aI + vget(Vh, b, b + t, r) * aJ;
                        sJ += vget(Vh, b, t, b + r) * aI + vget(Vh, b, b + t, b + r) * aJ;
                    }
                    L[IDX(I * b + r, col, n)] = sI;
                    L[IDX(J * b + r, col, n)] = sJ;
                }
            }
        }
    }
    for (size_t i = 0; i < nn; ++i) R[i] = L[i];
    /* right (column) updates: columns of blocks I and J, every block row K != I, J */
    for (int k = 0; k < npairs; ++k) {
        int I = pairs[2 * k], J = pairs[2 * k + 1];
        const double *Vh = Vhat + (size_t)k * 4 * b * b;
        for (int K = 0; K < N; ++K) {
            if (K == I || K == J) continue;
            for (int r = 0; r < b; ++r) {
                int row = K * b + r;
                for (int c = 0; c < b; ++c) {
                    long double sI = 0.0L, sJ = 0.0L;
                    for (int t = 0; t < b; ++t) {
                        long double aI = L[IDX(row, I * b + t, n)];
                        long double aJ = L[IDX(row, J * b + t, n)];
                        sI += aI * vget(Vh, b, t, c) + aJ * vget(Vh, b, b + t, c);
                        sJ += aI * vget(Vh, b, t, b + c) + aJ * vget(Vh, b, b + t, b + c);
                    }
                    R[IDX(row, I * b + c, n)] = sI;
                    R[IDX(row, J * b + c, n)] = sJ;
                }
            }
        }
    }
    /* A([I,J],[I,J]) <- D */
    if (Dhat)
        for (int k = 0; k < npairs; ++k) {
            int I = pairs[2 * k], J = pairs[2 * k + 1];
            const double *D = Dhat + (size_t)k * 4 * b * b;
            int base[2] = {I * b, J * b};
            for (int c = 0; c < 2 * b; ++c)
                for (int r = 0; r < 2 * b; ++r)
                    R[IDX(base[r / b] + r % b, base[c / b] + c % b, n)] = D[IDX(r, c, 2 * b)];
        }
    for (size_t i = 0; i < nn; ++i) A[i] = (double)R[i];
    /* Q: right updates on every block row */
    if (Q) {
        for (size_t i = 0; i < nn; ++i) L[i] = Q[i];
        for (int k = 0; k < npairs; ++k) {
            int I = pairs[2 * k], J = pairs[2 * k + 1];
            const double *Vh = Vhat + (size_t)k * 4 * b * b;
            for (int row = 0; row < n; ++row)
                for (int c = 0; c < b; ++c) {
                    long double sI = 0.0L, sJ = 0.0L;
                    for (int t = 0; t < b; ++t) {
                        long double qI = (long double)Q[IDX(row, I * b + t, n)];
                        long double qJ = (long double)Q[IDX(row, J * b + t, n)];
                        sI += qI * vget(Vh, b, t, c) + qJ * vget(Vh, b, b + t, c);
                        sJ += qI * vget(Vh, b, t, b + c) + qJ * vget(Vh, b, b + t, b + c);
                    }
                    L[IDX(row, I * b + c, n)] = sI;
                    L[IDX(row, J * b + c, n)] = sJ;
                }
        }
        for (size_t i = 0; i < nn; ++i) Q[i] = (double)L[i];
    }
    free(L);
    free(R);
    free(inpair);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Pivoting step                                                             */
/* ------------------------------------------------------------------------ */

/*
 * Column selection by LU with partial pivoting (§2.1, the pivoting step of the
 * convergence conditions): M is rows x cols (rows <= cols), here the leading
 * b rows of the 2b x 2b rotation V_hat.  Gaussian elimination with partial
 * pivoting runs on X = M^T (cols x rows): at step k the row i >= k of X with
 * the largest |X(i, k)| (the first such i on ties) is swapped into place k,
 * then X(i, j) -= l_i X(k, j) for i > k, j > k, with l_i = X(i, k) / X(k, k)
 * (skipped when the whole column is zero).  The row swaps of X are column
 * swaps of M; perm receives them applied to the identity: column j of M P is
 * column perm[j] of M, the first `rows` entries being the selected columns.
 * The update is written as fma(-l, x_kj, x_ij) (one rounding), the form a
 * fused multiply-add unit evaluates.  Returns 0, or -1 on bad sizes.
 */
int ora_lupp_cols(int rows, int cols, const double *M, int ldm, int *perm)
{
    if (rows < 0 || cols < rows || ldm < (rows > 1 ? rows : 1)) return -1;
    double *X = (double *)malloc(sizeof(double) * ((size_t)cols * rows + 1));
    for (int i = 0; i < cols; ++i) {
        perm[i] = i;
        for (int k = 0; k < rows; ++k) X[IDX(i, k, cols)] = M[IDX(k, i, ldm)];
    }
    for (int k = 0; k < rows; ++k) {
        int piv = k;
        double best = fabs(X[IDX(k, k, cols)]);
        for (int i = k + 1; i < cols; ++i)
            if (fabs(X[IDX(i, k, cols)]) > best) { best = fabs(X[IDX(i, k, cols)]); piv = i; }
        if (piv != k) {
            for (int j = 0; j < rows; ++j) {
                double t = X[IDX(k, j, cols)];
                X[IDX(k, j, cols)] = X[IDX(piv, j, cols)];
                X[IDX(piv, j, cols)] = t;
            }
            int t = perm[k]; perm[k] = perm[piv]; perm[piv] = t;
        }
        double d = X[IDX(k, k, cols)];
        if (d == 0.0) continue;
        for (int i = k + 1; i < cols; ++i) {
            double l = X[IDX(i, k, cols)] / d;
            for (int j = k + 1; j < rows; ++j) X[IDX(i, j, cols)] = fma(-l, X[IDX(k, j, cols)], X[IDX(i, j, cols)]);
        }
    }
    free(X);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Long-double checkers                                                      */
/* ------------------------------------------------------------------------ */

/* Xi(A) in long double (eq. (Omega_A)). */
double ora_check_offnorm(int n, const double *A, int lda)
{
    long double s = 0.0L;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i)
            if (i != j) s += (long double)A[IDX(i, j, lda)] * A[IDX(i, j, lda)];
    return (double)sqrtl(s);
}

/*
 * out[0] = ||A - Q diag(W) Q^T||_F / ||A||_F, out[1] = ||Q^T Q - I||_F,
 * out[2] = trace(A) - sum(W), out[3] = ||A||_F^2 - sum(W^2) (relative to ||A||_F^2).
 * All sums in long double.  Column j of Q diag(W) Q^T is accumulated as
 * sum_k (Q(j,k) W(k)) Q(:,k), so every inner loop runs down a column
 * (contiguous), and the Gram entries q_i^T q_j as column dot products; the
 * columns are spread over OpenMP threads.
 */
void ora_check_eig(int n, const double *A, int lda, const double *W, const double *Q, int ldq,
                   double *out)
{
    long double res = 0.0L, nA = 0.0L, orth = 0.0L, tr = 0.0L, sw = 0.0L, sw2 = 0.0L;
    for (int i = 0; i < n; ++i) {
        tr += A[IDX(i, i, lda)];
        sw += W[i];
        sw2 += (long double)W[i] * W[i];
    }
#pragma omp parallel reduction(+ : res, nA, orth)
    {
        long double *acc = (long double *)malloc(sizeof(long double) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 4)
        for (int j = 0; j < n; ++j) {
            for (int i = 0; i < n; ++i) acc[i] = 0.0L;
            for (int k = 0; k < n; ++k) {
                long double f = (long double)Q[IDX(j, k, ldq)] * W[k];
                const double *qk = Q + IDX(0, k, ldq);
                for (int i = 0; i < n; ++i) acc[i] += f * qk[i];
            }
            for (int i = 0; i < n; ++i) {
                long double a = A[IDX(i, j, lda)];
                res += (a - acc[i]) * (a - acc[i]);
                nA += a * a;
            }
            /* Gram entries (i, j), i <= j: the off-diagonal ones count twice */
            const double *qj = Q + IDX(0, j, ldq);
            for (int i = 0; i <= j; ++i) {
                const double *qi = Q + IDX(0, i, ldq);
                long double o = 0.0L;
                for (int k = 0; k < n; ++k) o += (long double)qi[k] * qj[k];
                if (i == j) o -= 1.0L;
                orth += (i == j ? 1.0L : 2.0L) * o * o;
            }
        }
        free(acc);
    }
    out[0] = (double)(sqrtl(res) / (nA > 0 ? sqrtl(nA) : 1.0L));
    out[1] = (double)sqrtl(orth);
    out[2] = (double)(tr - sw);
    out[3] = (double)((nA - sw2) / (nA > 0 ? nA : 1.0L));
}

/*
 * Sampled form for orders where the full O(n^3) check is too slow: for each
 * listed column index c, res_c = ||A q_c - w_c q_c||_2 / ||A||_F and, for
 * every pair of listed columns, |q_c^T q_d - delta_cd|.  out[0] = max res_c,
 * out[1] = max orthogonality deviation.
 */
void ora_check_eig_sampled(int n, const double *A, int lda, const double *W, const double *Q,
                           int ldq, int ncols, const int *cols, double *out)
{
    long double nA = 0.0L;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) nA += (long double)A[IDX(i, j, lda)] * A[IDX(i, j, lda)];
    nA = sqrtl(nA);
    double worst_res = 0.0, worst_orth = 0.0;
#pragma omp parallel for reduction(max : worst_res) schedule(dynamic, 1)
    for (int t = 0; t < ncols; ++t) {
        int c = cols[t];
        long double r2 = 0.0L;
        for (int i = 0; i < n; ++i) {
            long double s = 0.0L;
            for (int k = 0; k < n; ++k) s += (long double)A[IDX(i, k, lda)] * Q[IDX(k, c, ldq)];
            s -= (long double)W[c] * Q[IDX(i, c, ldq)];
            r2 += s * s;
        }
        double r = (double)(sqrtl(r2) / nA);
        if (r > worst_res) worst_res = r;
    }
#pragma omp parallel for reduction(max : worst_orth) schedule(dynamic, 1)
    for (int t = 0; t < ncols; ++t)
        for (int u = 0; u < ncols; ++u) {
            long double s = 0.0L;
            for (int k = 0; k < n; ++k) s += (long double)Q[IDX(k, cols[t], ldq)] * Q[IDX(k, cols[u], ldq)];
            if (cols[t] == cols[u]) s -= 1.0L;
            double d = (double)fabsl(s);
            if (d > worst_orth) worst_orth = d;
        }
    out[0] = worst_res;
    out[1] = worst_orth;
}

/*
 * SVD invariants: out[0] = ||G - U diag(S) V^T||_F / ||G||_F,
 * out[1] = ||V^T V - I||_F, out[2] = ||U^T U - I||_F over the columns with
 * S > 0 (zero columns of U are left out), all in long double.  Column j of
 * U diag(S) V^T is accumulated as sum_k (V(j,k) S(k)) U(:,k) (contiguous
 * inner loops); Gram entries are column dot products; OpenMP over columns.
 */
void ora_check_svd(int m, int n, const double *G, int ldg, const double *S, const double *U,
                   int ldu, const double *V, int ldv, double *out)
{
    long double res = 0.0L, nG = 0.0L, ov = 0.0L, ou = 0.0L;
#pragma omp parallel reduction(+ : res, nG)
    {
        long double *acc = (long double *)malloc(sizeof(long double) * (size_t)(m > 0 ? m : 1));
#pragma omp for schedule(dynamic, 4)
        for (int j = 0; j < n; ++j) {
            for (int i = 0; i < m; ++i) acc[i] = 0.0L;
            for (int k = 0; k < n; ++k) {
                long double f = (long double)V[IDX(j, k, ldv)] * S[k];
                const double *uk = U + IDX(0, k, ldu);
                for (int i = 0; i < m; ++i) acc[i] += f * uk[i];
            }
            for (int i = 0; i < m; ++i) {
                long double g = G[IDX(i, j, ldg)];
                res += (g - acc[i]) * (g - acc[i]);
                nG += g * g;
            }
        }
        free(acc);
    }
#pragma omp parallel for reduction(+ : ov, ou) schedule(dynamic, 4)
    for (int j = 0; j < n; ++j)
        for (int i = 0; i <= j; ++i) {
            const long double w = (i == j) ? 1.0L : 2.0L; /* (i, j) and (j, i) */
            long double s = 0.0L;
            for (int k = 0; k < n; ++k) s += (long double)V[IDX(k, i, ldv)] * V[IDX(k, j, ldv)];
            if (i == j) s -= 1.0L;
            ov += w * s * s;
            if (S[i] > 0.0 && S[j] > 0.0) {
                long double u = 0.0L;
                for (int k = 0; k < m; ++k) u += (long double)U[IDX(k, i, ldu)] * U[IDX(k, j, ldu)];
                if (i == j) u -= 1.0L;
                ou += w * u * u;
            }
        }
    out[0] = (double)(sqrtl(res) / (nG > 0 ? sqrtl(nG) : 1.0L));
    out[1] = (double)sqrtl(ov);
    out[2] = (double)sqrtl(ou);
}

/*
 * Gram block of the one-sided method, eq. (SVD_subproblem) of §6: out =
 * G(:, ca)^T G(:, cb) for the column lists ca (na entries) and cb (nb), the
 * sum over all m rows taken in long double and rounded once.  out is na x nb,
 * column-major (ld = na).
 */
void ora_gram(int m, const double *G, int ldg, int na, const int *ca, int nb, const int *cb, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int j = 0; j < nb; ++j)
        for (int i = 0; i < na; ++i) {
            const double *gi = G + IDX(0, ca[i], ldg), *gj = G + IDX(0, cb[j], ldg);
            long double s = 0.0L;
            for (int k = 0; k < m; ++k) s += (long double)gi[k] * gj[k];
            out[IDX(i, j, na)] = (double)s;
        }
}

/* ------------------------------------------------------------------------ */
/* Reduced QR (the preprocessing of the one-sided SVD, §6)                   */
/* ------------------------------------------------------------------------ */

/*
 * G = Q R for m >= n: Householder reflections in long double (Golub & Van
 * Loan §5.2), then the signs chosen so that diag(R) >= 0, which makes the
 * factorization of a full-rank G unique.  G (m x n, ldg) is read only; Q
 * (m x n, ldq, may be NULL) and R (n x n, ldr, zero below the diagonal) are
 * written.  Returns 0, or -1 for m < n.
 */
int ora_qr(int m, int n, const double *G, int ldg, double *Q, int ldq, double *R, int ldr)
{
    if (m < n) return -1;
    long double *A = (long double *)malloc(sizeof(long double) * (size_t)m * (n > 0 ? n : 1));
    long double *V = (long double *)malloc(sizeof(long double) * (size_t)m * (n > 0 ? n : 1));
    long double *beta = (long double *)calloc((size_t)(n > 0 ? n : 1), sizeof(long double));
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) A[IDX(i, j, m)] = G[IDX(i, j, ldg)];
    for (int k = 0; k < n; ++k) {
        /* reflector H = I - beta v v^T with H A(k:m, k) = alpha e_1 */
        long double nx = 0.0L;
        for (int i = k; i < m; ++i) nx += A[IDX(i, k, m)] * A[IDX(i, k, m)];
        nx = sqrtl(nx);
        long double x0 = A[IDX(k, k, m)];
        long double alpha = x0 >= 0.0L ? -nx : nx;
        for (int i = 0; i < m; ++i) V[IDX(i, k, m)] = 0.0L;
        if (nx == 0.0L) { beta[k] = 0.0L; continue; }
        V[IDX(k, k, m)] = x0 - alpha;
        for (int i = k + 1; i < m; ++i) V[IDX(i, k, m)] = A[IDX(i, k, m)];
        long double vv = 0.0L;
        for (int i = k; i < m; ++i) vv += V[IDX(i, k, m)] * V[IDX(i, k, m)];
        beta[k] = vv > 0.0L ? 2.0L / vv : 0.0L;
        for (int j = k; j < n; ++j) {
            long double d = 0.0L;
            for (int i = k; i < m; ++i) d += V[IDX(i, k, m)] * A[IDX(i, j, m)];
            d *= beta[k];
            for (int i = k; i < m; ++i) A[IDX(i, j, m)] -= d * V[IDX(i, k, m)];
        }
    }
    /* signs: D = diag(sgn(r_kk)), R <- D R, Q <- Q D */
    long double *sg = (long double *)malloc(sizeof(long double) * (size_t)(n > 0 ? n : 1));
    for (int k = 0; k < n; ++k) sg[k] = A[IDX(k, k, m)] < 0.0L ? -1.0L : 1.0L;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) R[IDX(i, j, ldr)] = i <= j ? (double)(sg[i] * A[IDX(i, j, m)]) : 0.0;
    if (Q) {
        /* Q = H_0 H_1 ... H_{n-1} (first n columns of I), applied backwards */
        long double *W = (long double *)calloc((size_t)m * (n > 0 ? n : 1), sizeof(long double));
        for (int j = 0; j < n; ++j) W[IDX(j, j, m)] = 1.0L;
        for (int k = n - 1; k >= 0; --k)
            for (int j = 0; j < n; ++j) {
                long double d = 0.0L;
                for (int i = k; i < m; ++i) d += V[IDX(i, k, m)] * W[IDX(i, j, m)];
                d *= beta[k];
                for (int i = k; i < m; ++i) W[IDX(i, j, m)] -= d * V[IDX(i, k, m)];
            }
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < m; ++i) Q[IDX(i, j, ldq)] = (double)(W[IDX(i, j, m)] * sg[j]);
        free(W);
    }
    free(sg);
    free(A);
    free(V);
    free(beta);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Cayley map                                                                */
/* ------------------------------------------------------------------------ */

/* Solve M X = B (n x n, column-major, long double) by Gaussian elimination
 * with partial pivoting; M and B are overwritten, X returned in B. */
static int gauss_solve(int n, long double *M, long double *B, int nrhs)
{
    for (int k = 0; k < n; ++k) {
        int piv = k;
        for (int i = k + 1; i < n; ++i)
            if (fabsl(M[IDX(i, k, n)]) > fabsl(M[IDX(piv, k, n)])) piv = i;
        if (M[IDX(piv, k, n)] == 0.0L) return 1;
        if (piv != k) {
            for (int j = 0; j < n; ++j) { long double t = M[IDX(k, j, n)]; M[IDX(k, j, n)] = M[IDX(piv, j, n)]; M[IDX(piv, j, n)] = t; }
            for (int j = 0; j < nrhs; ++j) { long double t = B[IDX(k, j, n)]; B[IDX(k, j, n)] = B[IDX(piv, j, n)]; B[IDX(piv, j, n)] = t; }
        }
        for (int i = k + 1; i < n; ++i) {
            long double f = M[IDX(i, k, n)] / M[IDX(k, k, n)];
            for (int j = k; j < n; ++j) M[IDX(i, j, n)] -= f * M[IDX(k, j, n)];
            for (int j = 0; j < nrhs; ++j) B[IDX(i, j, n)] -= f * B[IDX(k, j, n)];
        }
    }
    for (int j = 0; j < nrhs; ++j)
        for (int i = n - 1; i >= 0; --i) {
            long double s = B[IDX(i, j, n)];
            for (int k = i + 1; k < n; ++k) s -= M[IDX(i, k, n)] * B[IDX(k, j, n)];
            B[IDX(i, j, n)] = s / M[IDX(i, i, n)];
        }
    return 0;
}

/* W = (I - S)^{-1} (I + S) for a skew-symmetric S (n x n, column-major). */
int ora_cayley(int n, const double *S, double *W)
{
    size_t nn = (size_t)n * n;
    long double *M = (long double *)malloc(sizeof(long double) * nn);
    long double *B = (long double *)malloc(sizeof(long double) * nn);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            long double s = S[IDX(i, j, n)];
            M[IDX(i, j, n)] = (i == j ? 1.0L : 0.0L) - s;
            B[IDX(i, j, n)] = (i == j ? 1.0L : 0.0L) + s;
        }
    int rc = gauss_solve(n, M, B, n);
    for (size_t i = 0; i < nn; ++i) W[i] = (double)B[i];
    free(M);
    free(B);
    return rc;
}

/* Inverse Cayley: S = (W - I)(W + I)^{-1}, computed as the transpose of the
 * solution of (W + I)^T X = (W - I)^T. */
int ora_cayley_inverse(int n, const double *W, double *S)
{
    size_t nn = (size_t)n * n;
    long double *M = (long double *)malloc(sizeof(long double) * nn);
    long double *B = (long double *)malloc(sizeof(long double) * nn);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            long double w = W[IDX(j, i, n)]; /* transpose */
            M[IDX(i, j, n)] = w + (i == j ? 1.0L : 0.0L);
            B[IDX(i, j, n)] = w - (i == j ? 1.0L : 0.0L);
        }
    int rc = gauss_solve(n, M, B, n);
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) S[IDX(i, j, n)] = (double)B[IDX(j, i, n)];
    free(M);
    free(B);
    return rc;
}

/*
 * Sampled SVD checks for orders where the full products are too slow: for
 * each listed column c, out[0] = max_c ||G v_c - s_c u_c||_2 / ||G||_F; for all
 * listed pairs, out[1] = max |v_c^T v_d - delta_cd| and out[2] = max
 * |u_c^T u_d - delta_cd| (columns with s > 0 only).  Long double.
 */
void ora_check_svd_sampled(int m, int n, const double *G, int ldg, const double *S, const double *U,
                           int ldu, const double *V, int ldv, int ncols, const int *cols, double *out)
{
    long double nG = 0.0L;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < m; ++i) nG += (long double)G[IDX(i, j, ldg)] * G[IDX(i, j, ldg)];
    nG = sqrtl(nG);
    double wr = 0.0, wv = 0.0, wu = 0.0;
#pragma omp parallel for reduction(max : wr) schedule(dynamic, 1)
    for (int t = 0; t < ncols; ++t) {
        int c = cols[t];
        long double r2 = 0.0L;
        for (int i = 0; i < m; ++i) {
            long double s = 0.0L;
            for (int k = 0; k < n; ++k) s += (long double)G[IDX(i, k, ldg)] * V[IDX(k, c, ldv)];
            s -= (long double)S[c] * U[IDX(i, c, ldu)];
            r2 += s * s;
        }
        double r = (double)(sqrtl(r2) / (nG > 0 ? nG : 1.0L));
        if (r > wr) wr = r;
    }
#pragma omp parallel for reduction(max : wv, wu) schedule(dynamic, 1)
    for (int t = 0; t < ncols; ++t)
        for (int q = 0; q < ncols; ++q) {
            int c = cols[t], d = cols[q];
            long double sv = 0.0L, su = 0.0L;
            for (int k = 0; k < n; ++k) sv += (long double)V[IDX(k, c, ldv)] * V[IDX(k, d, ldv)];
            for (int k = 0; k < m; ++k) su += (long double)U[IDX(k, c, ldu)] * U[IDX(k, d, ldu)];
            if (c == d) { sv -= 1.0L; su -= 1.0L; }
            double dv = (double)fabsl(sv), du = (double)fabsl(su);
            if (dv > wv) wv = dv;
            if (S[c] > 0.0 && S[d] > 0.0 && du > wu) wu = du;
        }
    out[0] = wr;
    out[1] = wv;
    out[2] = wu;
}
