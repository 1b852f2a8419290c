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
                    if (!relative || fabs(apq) > tol * sqrt(fabs(app * aqq))) {
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

}  // namespace

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
