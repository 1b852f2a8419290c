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

namespace jx {

namespace {

constexpr int PNT = 256;

template <int M2>
struct PivLds {
    static constexpr int B = M2 / 2;
    static constexpr int LDX = B + 1;                                   // X row stride (doubles)
    static constexpr size_t STAGE = sizeof(double) * (size_t)M2 * M2;  // >= X (M2 x LDX)
    static constexpr size_t BYTES = STAGE + sizeof(double) * M2 + sizeof(int) * (M2 + 8);
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
    int *perm = reinterpret_cast<int *>(lmul + M2);           // M2
    int *piv = perm + M2;  // pivot row of step k in piv[k & 1] (a step's slot is
                           // rewritten two steps later, after every thread read it)
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

    for (int k = 0; k < B; ++k) {
        if (tid < 64) {  // pivot search by wave 0: (|x|, -i) maximal
            double best = -1.0;
            int bi = M2;
            for (int i = k + lane; i < M2; i += 64) {
                const double m = fabs(X[i * LDX + k]);
                if (m > best) { best = m; bi = i; }  // rows ascending per lane: first max kept
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double ob = __shfl_xor(best, o, 64);
                const int oi = __shfl_xor(bi, o, 64);
                if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
            }
            if (lane == 0) piv[k & 1] = bi;
        }
        __syncthreads();
        const int p = piv[k & 1];
        if (p != k) {  // swap rows k and p of X, entries k and p of perm
            for (int j = tid; j < B; j += PNT) {
                const double t = X[k * LDX + j];
                X[k * LDX + j] = X[p * LDX + j];
                X[p * LDX + j] = t;
            }
            if (tid == 0) {
                const int t = perm[k];
                perm[k] = perm[p];
                perm[p] = t;
            }
            __syncthreads();
        }
        const double dk = X[k * LDX + k];
        if (dk != 0.0 && k + 1 < B) {
            for (int i = k + 1 + tid; i < M2; i += PNT) lmul[i] = X[i * LDX + k] / dk;
            __syncthreads();
            // thread: column j = tid mod B, rows k + 1 + tid / B in steps of PNT / B
            constexpr int RS = PNT / B;
            const int j = tid % B;
            if (j > k) {
                const double xkj = X[k * LDX + j];
#pragma unroll 4
                for (int i = k + 1 + tid / B; i < M2; i += RS) X[i * LDX + j] = fma(-lmul[i], xkj, X[i * LDX + j]);
            }
            __syncthreads();
        }
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
    static bool attr = false;
    if (!attr) {
        JX_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_pivot<M2>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)PivLds<M2>::BYTES));
        attr = true;
    }
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
