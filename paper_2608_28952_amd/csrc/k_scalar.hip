// k_scalar.hip -- the b = 1 case of Alg. 1 (§2.1): scalar two-sided Jacobi in
// round-robin order, every sweep in one persistent workgroup.
//
// A round rotates n/2 disjoint index pairs (p_k, q_k) at once: the rotations
// are computed from the current A (the symmetric Schur 2 x 2 of each pair),
// then A <- J^T A J is applied as 2 x 2 pair blocks (rows of pair k1 with
// J_k1, columns of pair k2 with J_k2; a pair's own block gets the closed form
// a_pp - t a_pq, a_qq + t a_pq, 0), and Q <- Q J.  Disjoint rotations commute,
// so this equals applying them one after another.  A and Q stay in global
// memory (L2-resident at these orders); workgroup barriers order the rounds.
// After each sweep the off-norm Xi(A) of eq. (Omega_A) is summed directly;
// with the relative threshold the sweeps end once a sweep rotates nothing.
//
// Two forms: k_scalar_rr runs every sweep in one persistent workgroup (small
// orders); k_scalar_round runs one round over n/2 workgroups, workgroup k
// owning the two columns of pair k (larger orders, one launch per round).
#include "jx_common.hpp"
#include "jx_sweep.hpp"

namespace jx {

namespace {

constexpr int SNT = 1024;

__global__ void __launch_bounds__(SNT) k_scalar_rr(int n, int ne, const int *__restrict__ pairs, double *__restrict__ A,
                                                   double *__restrict__ Q, double tol, int max_sweeps, int relative,
                                                   double *__restrict__ out) {
    extern __shared__ double sm[];
    const int H = ne / 2;
    double *cs = sm, *sn = sm + H, *ta = sm + 2 * H, *red = sm + 3 * H;
    int *pq = reinterpret_cast<int *>(red + 32);  // the round's pairs
    const int tid = threadIdx.x;
    double fro2 = 0.0, off2 = 0.0;
    for (int e = tid; e < n * n; e += SNT) {
        const int i = e % n, j = e / n;
        const double v = A[e];
        fro2 += v * v;
        if (i != j) off2 += v * v;
    }
    fro2 = block_sum<SNT>(fro2, red);
    off2 = block_sum<SNT>(off2, red);
    const double thr = tol * sqrt(fro2);
    // absolute mode: a pair is rotated only when |a_pq| > tol ||A||_F /
    // sqrt(n (n - 1)), so a sweep that rotates none meets the stop test
    const double skip = thr / sqrt((double)n * (n - 1));
    int sweeps = 0;
    double rotated = 1.0;  // rotations of the last sweep (relative threshold)
    while (sweeps < max_sweeps && off2 == off2 && (relative ? rotated > 0.0 : sqrt(off2) > thr)) {
        double my_rot = 0.0;
        for (int r = 0; r < ne - 1; ++r) {
            const int *pr = pairs + (size_t)2 * r * H;
            for (int k = tid; k < H; k += SNT) {
                const int p = pr[2 * k], q = pr[2 * k + 1];
                pq[2 * k] = p;
                pq[2 * k + 1] = q;
                double c = 1.0, s = 0.0, t = 0.0;
                if (q < n) {  // index ne - 1 = n is a placeholder when n is odd
                    const double apq = A[(size_t)q * n + p], app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                    // relative threshold (Demmel & Veselic): only couplings
                    // above tol sqrt(|a_pp a_qq|) are rotated
                    if (relative ? fabs(apq) > tol * sqrt(fabs(app * aqq)) : fabs(apq) > skip) {
                        rot_cst(app, aqq, apq, c, s, t);
                        t *= apq;
                        my_rot += (s != 0.0) ? 1.0 : 0.0;
                    }
                }
                cs[k] = c;
                sn[k] = s;
                ta[k] = t;
            }
            __syncthreads();
            // A: pair block (k1, k2) = rows (p1, q1), columns (p2, q2)
            for (int e = tid; e < H * H; e += SNT) {
                const int k1 = e % H, k2 = e / H;
                const int p1 = pq[2 * k1], q1 = pq[2 * k1 + 1], p2 = pq[2 * k2], q2 = pq[2 * k2 + 1];
                if (k1 == k2) {
                    if (q1 < n && sn[k1] != 0.0) {
                        A[(size_t)p1 * n + p1] -= ta[k1];
                        A[(size_t)q1 * n + q1] += ta[k1];
                        A[(size_t)q1 * n + p1] = 0.0;
                        A[(size_t)p1 * n + q1] = 0.0;
                    }
                    continue;
                }
                const double c1 = cs[k1], s1 = sn[k1], c2 = cs[k2], s2 = sn[k2];
                const bool hq1 = q1 < n, hq2 = q2 < n;
                const double a11 = A[(size_t)p2 * n + p1];
                const double a12 = hq2 ? A[(size_t)q2 * n + p1] : 0.0;
                const double a21 = hq1 ? A[(size_t)p2 * n + q1] : 0.0;
                const double a22 = (hq1 && hq2) ? A[(size_t)q2 * n + q1] : 0.0;
                // rows: p' = c p - s q, q' = s p + c q; then columns alike
                const double b11 = c1 * a11 - s1 * a21, b21 = s1 * a11 + c1 * a21;
                const double b12 = c1 * a12 - s1 * a22, b22 = s1 * a12 + c1 * a22;
                A[(size_t)p2 * n + p1] = c2 * b11 - s2 * b12;
                if (hq2) A[(size_t)q2 * n + p1] = s2 * b11 + c2 * b12;
                if (hq1) A[(size_t)p2 * n + q1] = c2 * b21 - s2 * b22;
                if (hq1 && hq2) A[(size_t)q2 * n + q1] = s2 * b21 + c2 * b22;
            }
            if (Q)
                for (int e = tid; e < n * H; e += SNT) {
                    const int i = e % n, k = e / n;
                    const int p = pq[2 * k], q = pq[2 * k + 1];
                    if (q >= n || sn[k] == 0.0) continue;
                    const double qp = Q[(size_t)p * n + i], qq = Q[(size_t)q * n + i];
                    Q[(size_t)p * n + i] = cs[k] * qp - sn[k] * qq;
                    Q[(size_t)q * n + i] = sn[k] * qp + cs[k] * qq;
                }
            __syncthreads();
        }
        ++sweeps;
        rotated = block_sum<SNT>(my_rot, red);
        off2 = 0.0;
        for (int e = tid; e < n * n; e += SNT) {
            const int i = e % n, j = e / n;
            if (i != j) off2 += A[e] * A[e];
        }
        off2 = block_sum<SNT>(off2, red);
    }
    if (tid == 0) {
        out[0] = (double)sweeps;
        out[1] = sqrt(off2);
        out[2] = sqrt(fro2);
        out[3] = rotated;
    }
}

// dst (n x n, ld n) = the symmetric matrix whose `upper` (or lower) triangle
// src holds.
__global__ void k_sym_full(int n, const double *__restrict__ src, int lds_, int upper, double *__restrict__ dst) {
    const int j = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const bool own = upper ? (i <= j) : (i >= j);
        dst[(size_t)j * n + i] = own ? src[(size_t)j * lds_ + i] : src[(size_t)i * lds_ + j];
    }
}

// One round of the multi-workgroup form.  A is full, column-major (n x n);
// this round reads Acur only and writes Anext, so every workgroup sees the
// matrix as the round found it.  Workgroup k1 computes the rotations of all
// H pairs (each workgroup the same values), loads its columns p1, q1, and for
// every pair k2 writes the 2 x 2 block (rows p2, q2; columns p1, q1) of
// J^T A J: rows rotated by pair k2, columns by pair k1 (its own block by the
// closed form).  Q(:, [p1, q1]) <- Q(:, [p1, q1]) J_k1 in place (only this
// workgroup touches those columns).  rot (optional): workgroup 0 adds the
// number of rotations of the round.  Absolute mode rotates a pair only when
// |a_pq| > skip; relative mode when |a_pq| > tol sqrt(|a_pp a_qq|).
__global__ void __launch_bounds__(256) k_scalar_round(int n, int H, const int *__restrict__ pr,
                                                      const double *__restrict__ Acur, double *__restrict__ Anext,
                                                      double *__restrict__ Q, double tol, int relative,
                                                      double skip, int *__restrict__ rot) {
    extern __shared__ double sm[];
    double *cs = sm, *sn = sm + H, *ta = sm + 2 * H, *cp = sm + 3 * H, *cq = cp + n;
    const int tid = threadIdx.x, k1 = blockIdx.x;
    const int p1 = pr[2 * k1], q1 = pr[2 * k1 + 1];
    const bool hq1 = q1 < n;  // index n is the placeholder of an odd order
    int mine = 0;
    for (int k = tid; k < H; k += 256) {
        const int p = pr[2 * k], q = pr[2 * k + 1];
        double c = 1.0, s = 0.0, t = 0.0;
        if (q < n) {
            const double apq = Acur[(size_t)q * n + p], app = Acur[(size_t)p * n + p], aqq = Acur[(size_t)q * n + q];
            if (relative ? fabs(apq) > tol * sqrt(fabs(app * aqq)) : fabs(apq) > skip) {
                rot_cst(app, aqq, apq, c, s, t);
                t *= apq;
                mine += (s != 0.0) ? 1 : 0;
            }
        }
        cs[k] = c;
        sn[k] = s;
        ta[k] = t;
    }
    if (rot && k1 == 0 && mine) atomicAdd(rot, mine);
    for (int i = tid; i < n; i += 256) {
        cp[i] = Acur[(size_t)p1 * n + i];
        cq[i] = hq1 ? Acur[(size_t)q1 * n + i] : 0.0;
    }
    __syncthreads();
    const double c1 = cs[k1], s1 = sn[k1];
    double *op = Anext + (size_t)p1 * n, *oq = Anext + (size_t)q1 * n;
    for (int k2 = tid; k2 < H; k2 += 256) {
        const int p2 = pr[2 * k2], q2 = pr[2 * k2 + 1];
        if (k2 == k1) {  // the pair's own block: a_pp - t a_pq, a_qq + t a_pq, 0
            const bool r = hq1 && s1 != 0.0;
            op[p1] = r ? cp[p1] - ta[k1] : cp[p1];
            if (hq1) {
                oq[q1] = r ? cq[q1] + ta[k1] : cq[q1];
                op[q1] = r ? 0.0 : cp[q1];
                oq[p1] = r ? 0.0 : cq[p1];
            }
            continue;
        }
        const bool hq2 = q2 < n;
        const double c2 = cs[k2], s2 = sn[k2];
        const double a11 = cp[p2], a12 = cq[p2];
        const double a21 = hq2 ? cp[q2] : 0.0, a22 = hq2 ? cq[q2] : 0.0;
        // rows by pair k2: p' = c p - s q, q' = s p + c q; then columns by pair k1
        const double b11 = c2 * a11 - s2 * a21, b21 = s2 * a11 + c2 * a21;
        const double b12 = c2 * a12 - s2 * a22, b22 = s2 * a12 + c2 * a22;
        op[p2] = c1 * b11 - s1 * b12;
        if (hq1) oq[p2] = s1 * b11 + c1 * b12;
        if (hq2) {
            op[q2] = c1 * b21 - s1 * b22;
            if (hq1) oq[q2] = s1 * b21 + c1 * b22;
        }
    }
    if (Q && hq1 && s1 != 0.0)
        for (int i = tid; i < n; i += 256) {
            const double qp = Q[(size_t)p1 * n + i], qq = Q[(size_t)q1 * n + i];
            Q[(size_t)p1 * n + i] = c1 * qp - s1 * qq;
            Q[(size_t)q1 * n + i] = s1 * qp + c1 * qq;
        }
}

// out[0] = Xi(A)^2 (off-diagonal sum of squares), out[1] = ||A||_F^2 of the
// full n x n matrix, in one workgroup (a fixed order).
__global__ void __launch_bounds__(1024) k_scalar_norms(int n, const double *__restrict__ A, double *__restrict__ out) {
    __shared__ double red[32];
    double off2 = 0.0, fro2 = 0.0;
    for (size_t e = threadIdx.x; e < (size_t)n * n; e += 1024) {
        const int i = (int)(e % n), j = (int)(e / n);
        const double v = A[e];
        fro2 += v * v;
        if (i != j) off2 += v * v;
    }
    off2 = block_sum<1024>(off2, red);
    fro2 = block_sum<1024>(fro2, red);
    if (threadIdx.x == 0) {
        out[0] = off2;
        out[1] = fro2;
    }
}

}  // namespace

void launch_scalar_round(int n, int ne, const int *pairs_round, const double *Acur, double *Anext, double *Q,
                         double tol, int relative, double skip, int *rot, hipStream_t s) {
    const int H = ne / 2;
    const size_t lds = sizeof(double) * (3 * (size_t)H + 2 * (size_t)n);
    hipLaunchKernelGGL(k_scalar_round, dim3(H), dim3(256), lds, s, n, H, pairs_round, Acur, Anext, Q, tol, relative,
                       skip, rot);
    JX_LAUNCHED();
}

void launch_scalar_norms(int n, const double *A, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_scalar_norms, dim3(1), dim3(1024), 0, s, n, A, out);
    JX_LAUNCHED();
}

void launch_sym_full(int n, const double *src, int lds_, char uplo, double *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_sym_full, dim3((n + 255) / 256, n), dim3(256), 0, s, n, src, lds_,
                       (uplo == 'U' || uplo == 'u') ? 1 : 0, dst);
    JX_LAUNCHED();
}

void launch_scalar_rr(int n, int ne, const int *pairs, double *A, double *Q, double tol, int max_sweeps, int relative,
                      double *out, hipStream_t s) {
    const size_t lds = sizeof(double) * (3 * (size_t)(ne / 2) + 32) + sizeof(int) * (size_t)ne;
    hipLaunchKernelGGL(k_scalar_rr, dim3(1), dim3(SNT), lds, s, n, ne, pairs, A, Q, tol, max_sweeps, relative, out);
    JX_LAUNCHED();
}

}  // namespace jx
