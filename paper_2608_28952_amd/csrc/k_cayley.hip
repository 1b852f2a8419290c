// k_cayley.hip -- batched Cayley map of the learned warm start:
// Q0 = Qref (I - S)^{-1} (I + S) for skew-symmetric S (FP64), one workgroup per
// matrix, n <= 64.  I - S has symmetric part I (x^T (I - S) x = |x|^2), so its
// leading minors are nonzero and elimination needs no pivoting.  Order 64
// runs Gauss-Jordan on the augmented [I - S | I + S] in registers; other
// orders eliminate it in LDS and back-substitute the solution columns
// independently.  The solution is then multiplied by Qref.
#include "jx_common.hpp"
#include "jx_mlp.hpp"

namespace jx {

namespace {

constexpr int NMAX = 64, NT = 256;

__global__ void __launch_bounds__(NT) k_cayley(int n, const double *S, const double *Qref, double *Q0) {
    extern __shared__ double sm[];
    const int w = 2 * n;
    double *M = sm;              // n x 2n, row-major
    double *R = sm + n * w;      // Qref, column-major
    const double *Sb = S + (size_t)blockIdx.x * n * n;
    double *Qb = Q0 + (size_t)blockIdx.x * n * n;
    const int tid = threadIdx.x;
    for (int e = tid; e < n * n; e += NT) {
        const int i = e % n, j = e / n;  // column-major element (i, j)
        const double s = Sb[e], d = (i == j) ? 1.0 : 0.0;
        M[i * w + j] = d - s;
        M[i * w + n + j] = d + s;
        R[e] = Qref[e];
    }
    __syncthreads();
    for (int k = 0; k < n - 1; ++k) {
        const double pinv = 1.0 / M[k * w + k];
        const int rows = n - k - 1, cols = w - k - 1;
        for (int e = tid; e < rows * cols; e += NT) {
            const int i = k + 1 + e / cols, j = k + 1 + e % cols;
            M[i * w + j] -= M[i * w + k] * pinv * M[k * w + j];
        }
        __syncthreads();
    }
    // back substitution, one solution column per thread
    for (int c = tid; c < n; c += NT) {
        for (int k = n - 1; k >= 0; --k) {
            double x = M[k * w + n + c];
            for (int j = k + 1; j < n; ++j) x -= M[k * w + j] * M[j * w + n + c];
            M[k * w + n + c] = x / M[k * w + k];
        }
    }
    __syncthreads();
    // Q0 = Qref X, column-major
    for (int e = tid; e < n * n; e += NT) {
        const int i = e % n, j = e / n;
        double acc = 0.0;
        for (int k = 0; k < n; ++k) acc += R[k * n + i] * M[k * w + n + j];
        Qb[e] = acc;
    }
}

// Value of v in lane l of the wave (l < 64, every lane active).
__device__ __forceinline__ double readlane_f64(double v, int l) {
    const unsigned long long u = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffull), l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Order 64 (the warm start's family): Gauss-Jordan on [I - S | I + S] held
// in registers.  Thread (row i = lane, wave g) holds columns 32 g .. 32 g + 31
// of row i, so each wave holds the pivot row k of its own columns in lane k
// and reads it from there (no LDS); only column k (the multipliers, from the
// wave that holds it) passes through LDS, double-buffered by step parity: one
// barrier per step.  Every row is updated as m -= f p with p the pivot row:
// f = a_ik / a_kk eliminates column k from the other rows, f = 1 - 1 / a_kk
// scales the pivot row itself (m = p in its lane), so no lane takes another
// path.  The right half ends as X = (I - S)^{-1} (I + S).  Then Q0 = Qref X
// with a 4 x 4 register block per thread, both operands from LDS.
__global__ void __launch_bounds__(NT) k_cayley64(const double *S, const double *Qref, double *Q0) {
    constexpr int N = 64, W = 2 * N, NQ = W / 4;
    __shared__ double mcol[2][N];
    __shared__ double Qs[N * N];  // Qs[i N + r] = Qref(r, i)
    __shared__ double Xs[N * N];  // Xs[i N + c] = X(i, c)
    const int tid = threadIdx.x, i = tid & 63, g = tid >> 6;
    const double *Sb = S + (size_t)blockIdx.x * N * N;
    double m[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int j = NQ * g + q;  // S(i, c) at c N + i (column-major)
        m[q] = j < N ? (i == j ? 1.0 : 0.0) - Sb[j * N + i] : (i == j - N ? 1.0 : 0.0) + Sb[(j - N) * N + i];
    }
    for (int e = tid; e < N * N; e += NT) Qs[e] = Qref[e];  // column-major Qref: e = i N + r
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const int b = k & 1;
        if (g == k / NQ) mcol[b][i] = m[k % NQ];
        __syncthreads();
        const double pinv = 1.0 / mcol[b][k];
        const double f = i == k ? 1.0 - pinv : mcol[b][i] * pinv;
#pragma unroll
        for (int q = 0; q < NQ; ++q) m[q] -= f * readlane_f64(m[q], k);
    }
    if (g >= 2) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) Xs[i * N + NQ * (g - 2) + q] = m[q];
    }
    __syncthreads();
    const int r0 = 4 * (tid & 15), c0 = 4 * (tid >> 4);
    double acc[4][4] = {};
#pragma unroll 8
    for (int k = 0; k < N; ++k) {
        double a[4], x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] = Qs[k * N + r0 + u];
            x[u] = Xs[k * N + c0 + u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] += a[u] * x[v];
    }
    double *Qb = Q0 + (size_t)blockIdx.x * N * N;
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int u = 0; u < 4; ++u) Qb[(c0 + v) * N + r0 + u] = acc[u][v];
}

}  // namespace

void cayley_batched(int batch, int n, const double *S, const double *Qref, double *Q0, hipStream_t s) {
    if (batch <= 0 || n <= 0) return;
    if (n > NMAX) {
        set_error("cayley: order above 64");
        throw HipFail{hipErrorInvalidValue};
    }
    if (n == NMAX) {
        hipLaunchKernelGGL(k_cayley64, dim3(batch), dim3(NT), 0, s, S, Qref, Q0);
        JX_LAUNCHED();
        return;
    }
    const size_t lds = sizeof(double) * ((size_t)n * 2 * n + (size_t)n * n);
    ensure_lds_limit(reinterpret_cast<const void *>(&k_cayley), (int)(sizeof(double) * 3 * NMAX * NMAX));
    hipLaunchKernelGGL(k_cayley, dim3(batch), dim3(NT), lds, s, n, S, Qref, Q0);
    JX_LAUNCHED();
}

}  // namespace jx
