// k_cayley.hip -- batched Cayley map of the learned warm start:
// Q0 = Qref (I - S)^{-1} (I + S) for skew-symmetric S (FP64), one workgroup per
// matrix, n <= 64.  I - S has symmetric part I (x^T (I - S) x = |x|^2), so its
// leading minors are nonzero and Gaussian elimination needs no pivoting; the
// elimination runs on the augmented [I - S | I + S] in LDS, the solution
// columns are back-substituted independently, then multiplied by Qref.
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

}  // namespace

void cayley_batched(int batch, int n, const double *S, const double *Qref, double *Q0, hipStream_t s) {
    if (batch <= 0 || n <= 0) return;
    if (n > NMAX) {
        set_error("cayley: order above 64");
        throw HipFail{hipErrorInvalidValue};
    }
    const size_t lds = sizeof(double) * ((size_t)n * 2 * n + (size_t)n * n);
    static bool attr = false;
    if (!attr) {
        JX_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_cayley), hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)(sizeof(double) * 3 * NMAX * NMAX)));
        attr = true;
    }
    hipLaunchKernelGGL(k_cayley, dim3(batch), dim3(NT), lds, s, n, S, Qref, Q0);
    JX_LAUNCHED();
}

}  // namespace jx
