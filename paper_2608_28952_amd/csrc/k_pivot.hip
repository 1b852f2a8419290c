// k_pivot.hip -- the pivoting step of block Jacobi (§2.1, the convergence
// conditions after eq. (sweep cost)): after a subproblem is diagonalised,
// LU with partial pivoting on the leading b rows of its rotation V_hat
// (2b x 2b) selects a column permutation P, and V_hat <- V_hat P together with
// D_hat <- P^T D_hat P (so that V_hat^T A_hat V_hat = D_hat still holds and
// the tile updates see the permuted rotation).
//
// One workgroup per pair.  The elimination runs on X = V_hat(0:b, :)^T
// (2b x b) in LDS: at step k the row i >= k with the largest |X(i, k)| (the
// first on ties) is swapped into place k, then X(i, j) <- fma(-l_i, X(k, j),
// X(i, j)) for i, j > k with l_i = X(i, k) / X(k, k).  The permuted V_hat and
// D_hat are then written back through an LDS copy of each.
#include "jx_common.hpp"
#include "jx_sweep.hpp"

namespace jx {

namespace {

constexpr int PNT = 256;

template <int M2>
struct PivLds {
    static constexpr int B = M2 / 2;
    static constexpr int LDX = B + 1;                                   // X row stride (doubles)
    static constexpr size_t STAGE = sizeof(double) * (size_t)M2 * M2;  // >= X (M2 x LDX)
    // stage | multipliers (M2) | next-pivot candidates (PNT / B values and
    // rows) | perm (M2)
    static constexpr size_t BYTES = STAGE + sizeof(double) * (M2 + PNT / B) + sizeof(int) * (PNT / B + M2);
};

// Element (r, c) of the pair's rotation and (r <= c) of its D_hat, and the
// matching stores, for the two storage modes: the solver's (V_hat in vperm
// order, D_hat in the upper block storage of A: blocks (I, I) and (J, J)
// whole, (I, J)) and plain column-major.
template <int M2>
struct PivData {
    static constexpr int B = M2 / 2;
    double *V;
    double *Dii = nullptr, *Dij = nullptr, *Djj = nullptr;  // block storage
    double *Dp = nullptr;                                   // plain
    bool blocks;
    __device__ double v(int r, int c) const { return blocks ? V[vperm(r, c, M2)] : V[(size_t)c * M2 + r]; }
    __device__ void set_v(int r, int c, double x) const {
        if (blocks) V[vperm(r, c, M2)] = x;
        else V[(size_t)c * M2 + r] = x;
    }
    __device__ bool has_d() const { return blocks || Dp != nullptr; }
    // r <= c
    __device__ double d(int r, int c) const {
        if (!blocks) return Dp[(size_t)c * M2 + r];
        if (c < B) return Dii[c * B + r];
        if (r < B) return Dij[(c - B) * B + r];
        return Djj[(c - B) * B + (r - B)];
    }
    __device__ void set_d(int r, int c, double x) const {
        if (!blocks) {
            Dp[(size_t)c * M2 + r] = x;
            Dp[(size_t)r * M2 + c] = x;
            return;
        }
        // the diagonal blocks are stored whole: both triangles
        if (c < B) {
            Dii[c * B + r] = x;
            Dii[r * B + c] = x;
        } else if (r < B) {
            Dij[(c - B) * B + r] = x;
        } else {
            Djj[(c - B) * B + (r - B)] = x;
            Djj[(r - B) * B + (c - B)] = x;
        }
    }
};

template <int M2>
__global__ void __launch_bounds__(PNT) k_pivot(PivotArgs a) {
    using L = PivLds<M2>;
    constexpr int B = M2 / 2, LDX = L::LDX;
    static_assert((M2 * B) % (8 * PNT) == 0 && PNT % B == 0, "pivot kernel geometry");
    extern __shared__ double smem[];
    double *X = smem;                                         // M2 x LDX, later the M2 x M2 stage
    double *lmul = smem + (size_t)M2 * M2;                    // multipliers l_i
    int *perm = reinterpret_cast<int *>(lmul + M2 + PNT / B) + PNT / B;  // M2 (after the candidates)
    const int tid = threadIdx.x, lane = tid & 63;
    const int pr = blockIdx.x;
    int *pout = a.perm_out ? a.perm_out + (size_t)pr * M2 : nullptr;
    if (a.flags && a.flags[pr]) {  // skipped pair: V_hat = I is not stored, nothing to permute
        if (pout)
            for (int i = tid; i < M2; i += PNT) pout[i] = i;
        return;
    }
    PivData<M2> dat;
    dat.blocks = a.ablk != nullptr;
    dat.V = a.V + (size_t)pr * M2 * M2;
    if (dat.blocks) {
        const int I = a.pairs[2 * pr], J = a.pairs[2 * pr + 1];
        dat.Dii = a.ablk + ublk(I, I) * (size_t)(B * B);
        dat.Djj = a.ablk + ublk(J, J) * (size_t)(B * B);
        dat.Dij = a.ablk + ublk(I, J) * (size_t)(B * B);
    } else if (a.D) {
        dat.Dp = a.D + (size_t)pr * M2 * M2;
    }

    // global loads eight at a time per thread before their LDS stores
    // (M2 B and M2^2 are multiples of 8 PNT)
    for (int e0 = 0; e0 < M2 * B; e0 += 8 * PNT) {  // X(i, k) = V_hat(k, i)
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * PNT + tid;
            v[u] = dat.v(e % B, e / B);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * PNT + tid;
            X[(e / B) * LDX + e % B] = v[u];
        }
    }
    for (int i = tid; i < M2; i += PNT) perm[i] = i;
    __syncthreads();

    // Step k: wave 0 takes the pivot (from the column maxima the previous
    // step's update left; step 0 searches itself), swaps the rows and forms
    // the multipliers, its lanes ordered among themselves by wave-level LDS
    // syncs; then every wave updates the trailing block, and the threads of
    // column k + 1 record that column's maxima for the next step.  Two
    // workgroup barriers per step.
    constexpr int RS = PNT / B;  // threads per column in the update
    double *candv = lmul + M2;   // RS candidates (|x|, row) for the next pivot
    int *candi = reinterpret_cast<int *>(candv + RS);
    if (tid < RS) {  // step 0's candidates: rows tid, tid + RS, ... of column 0
        double best = -1.0;
        int bi = M2;
        for (int i = tid; i < M2; i += RS) {
            const double m = fabs(X[i * LDX]);
            if (m > best) { best = m; bi = i; }
        }
        candv[tid] = best;
        candi[tid] = bi;
    }
    __syncthreads();
    for (int k = 0; k < B; ++k) {
        if (tid < 64) {
            // the first maximal row: largest |x|, the smaller row on ties
            double best = candv[0];
            int p = candi[0];
#pragma unroll
            for (int r = 1; r < RS; ++r) {
                const double v = candv[r];
                const int i = candi[r];
                if (v > best || (v == best && i < p)) { best = v; p = i; }
            }
            if (p != k) {  // swap rows k and p of X (lane j: column j), entries k and p of perm
                for (int j = lane; j < B; j += 64) {
                    const double t = X[k * LDX + j];
                    X[k * LDX + j] = X[p * LDX + j];
                    X[p * LDX + j] = t;
                }
                if (lane == 0) {
                    const int t = perm[k];
                    perm[k] = perm[p];
                    perm[p] = t;
                }
            }
            wave_lds_sync();
            const double dk = X[k * LDX + k];
            for (int i = k + 1 + lane; i < M2; i += 64) lmul[i] = dk != 0.0 ? X[i * LDX + k] / dk : 0.0;
        }
        __syncthreads();
        if (k + 1 < B) {
            // thread: column j = tid mod B, rows k + 1 + tid / B in steps of RS
            // (a zero pivot leaves zero multipliers: the column is all zero)
            const int j = tid % B, r = tid / B;
            if (j > k) {
                double *__restrict__ Xj = X + j;
                const double *__restrict__ lm = lmul;
                const double xkj = Xj[k * LDX];
                // four rows per iteration, their loads issued before any
                // store; every column tracks its maxima (only column k + 1's
                // are kept: a branch here would split the waves)
                double best = -1.0;
                int bi = M2;
                int i = k + 1 + r;
                for (; i + 3 * RS < M2; i += 4 * RS) {
                    const double l0 = lm[i], l1 = lm[i + RS], l2 = lm[i + 2 * RS], l3 = lm[i + 3 * RS];
                    const double x0 = Xj[i * LDX], x1 = Xj[(i + RS) * LDX], x2 = Xj[(i + 2 * RS) * LDX],
                                 x3 = Xj[(i + 3 * RS) * LDX];
                    const double v0 = fma(-l0, xkj, x0), v1 = fma(-l1, xkj, x1), v2 = fma(-l2, xkj, x2),
                                 v3 = fma(-l3, xkj, x3);
                    Xj[i * LDX] = v0;
                    Xj[(i + RS) * LDX] = v1;
                    Xj[(i + 2 * RS) * LDX] = v2;
                    Xj[(i + 3 * RS) * LDX] = v3;
                    // rows ascending: the first maximum is kept
                    if (fabs(v0) > best) { best = fabs(v0); bi = i; }
                    if (fabs(v1) > best) { best = fabs(v1); bi = i + RS; }
                    if (fabs(v2) > best) { best = fabs(v2); bi = i + 2 * RS; }
                    if (fabs(v3) > best) { best = fabs(v3); bi = i + 3 * RS; }
                }
                for (; i < M2; i += RS) {
                    const double v = fma(-lm[i], xkj, Xj[i * LDX]);
                    Xj[i * LDX] = v;
                    if (fabs(v) > best) { best = fabs(v); bi = i; }
                }
                if (j == k + 1) {
                    candv[r] = best;
                    candi[r] = bi;
                }
            }
        }
        __syncthreads();
    }
    if (pout)
        for (int i = tid; i < M2; i += PNT) pout[i] = perm[i];
    __syncthreads();  // every read of X done: the stage below overwrites it

    // V_hat <- V_hat P: column j of the result is column perm[j]
    double *S = smem;
    for (int e0 = 0; e0 < M2 * M2; e0 += 8 * PNT) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * PNT + tid;
            v[u] = dat.v(e % M2, e / M2);
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) S[e0 + u * PNT + tid] = v[u];
    }
    __syncthreads();
    for (int e = tid; e < M2 * M2; e += PNT) {
        const int r = e % M2, c = e / M2;
        dat.set_v(r, c, S[(size_t)perm[c] * M2 + r]);
    }
    if (!dat.has_d()) return;
    __syncthreads();
    // D_hat <- P^T D_hat P: entry (r, c) of the result is D_hat(perm[r], perm[c])
    for (int e0 = 0; e0 < M2 * M2; e0 += 8 * PNT) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * PNT + tid, r = e % M2, c = e / M2;
            v[u] = r <= c ? dat.d(r, c) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int e = e0 + u * PNT + tid, r = e % M2, c = e / M2;
            if (r <= c) {
                S[(size_t)c * M2 + r] = v[u];
                S[(size_t)r * M2 + c] = v[u];
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < M2 * M2; e += PNT) {
        const int r = e % M2, c = e / M2;
        if (r <= c) dat.set_d(r, c, S[(size_t)perm[c] * M2 + perm[r]]);
    }
}

template <int M2>
void launch_pivot_t(const PivotArgs &a, hipStream_t s) {
    ensure_lds_limit(reinterpret_cast<const void *>(&k_pivot<M2>), (int)PivLds<M2>::BYTES);
    hipLaunchKernelGGL(k_pivot<M2>, dim3(a.count), dim3(PNT), PivLds<M2>::BYTES, s, a);
    JX_LAUNCHED();
}

// col-major (k, i) <- vperm order: the inverse of k_vperm_from_colmajor
__global__ void k_colmajor_from_vperm(int m2, const double *__restrict__ src, double *__restrict__ dst) {
    const double *s = src + (size_t)blockIdx.x * m2 * m2;
    double *d = dst + (size_t)blockIdx.x * m2 * m2;
    for (int e = threadIdx.x; e < m2 * m2; e += blockDim.x) {
        const int k = e % m2, i = e / m2;
        d[e] = s[vperm(k, i, m2)];
    }
}

}  // namespace

void launch_pivot(const PivotArgs &a, hipStream_t s) {
    if (a.count <= 0) return;
    if (a.m2 == 64) launch_pivot_t<64>(a, s);
    else if (a.m2 == 128) launch_pivot_t<128>(a, s);
    else throw HipFail{hipErrorInvalidValue};
}

void launch_colmajor_from_vperm(int count, int m2, const double *src, double *dst, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_colmajor_from_vperm, dim3(count), dim3(256), 0, s, m2, src, dst);
    JX_LAUNCHED();
}

}  // namespace jx
