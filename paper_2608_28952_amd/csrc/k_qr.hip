// k_qr.hip -- pieces of the reduced QR G = Q R that precedes the one-sided
// Jacobi SVD (§6, "Preprocessing with QR"), computed as CholeskyQR: R from the
// Cholesky factor of the Gram matrix G^T G, Q = G R^{-1}, done twice (the
// second pass on Q restores orthogonality to working accuracy).  The GEMMs run
// on the FP64 MFMA kernel (k_gemm.hip); this file holds the small kernels
// between them.
#include "jx_common.hpp"

namespace jx {

namespace {

constexpr int QB = 128;        // diagonal block order (the GEMM tile)
constexpr int QLD = QB + 1;    // LDS stride

// Cholesky of the diagonal block W(k0:k0+QB, k0:k0+QB) (upper triangle read)
// of the SPD matrix W (column-major, ldw): W_kk = R_kk^T R_kk.  R_kk is
// written back over W's block (upper triangle; the strictly lower part set
// to zero), and its inverse (upper triangular) to Rinv (QB x QB,
// column-major).  A pivot that is not positive and finite sets *flag = 1
// and is replaced by 1 so that the kernel completes.
constexpr size_t CHOL_LDS = sizeof(double) * (QB * QLD + QB);

constexpr int CNT = 1024;  // threads of k_chol_diag

__global__ void __launch_bounds__(CNT) k_chol_diag(double *__restrict__ W, int ldw, int k0,
                                                   double *__restrict__ Rinv, int *__restrict__ flag) {
    extern __shared__ double lds[];
    double *T = lds;               // T[i * QLD + j] = element (i, j)
    double *rd = lds + QB * QLD;   // R's diagonal
    const int tid = threadIdx.x;
    for (int e = tid; e < QB * QB; e += CNT) {
        const int i = e % QB, j = e / QB;
        T[i * QLD + j] = i <= j ? W[(size_t)(k0 + j) * ldw + k0 + i] : 0.0;  // upper triangle
    }
    __syncthreads();
    // right-looking: step j takes row j's pivot, scales row j, updates the
    // trailing upper triangle
    int bad = 0;
    for (int j = 0; j < QB; ++j) {
        double d = T[j * QLD + j];
        if (!(d > 0.0) || !(d < HUGE_VAL)) {
            bad = 1;
            d = 1.0;
        }
        const double r = sqrt(d), ir = 1.0 / r;
        __syncthreads();  // every lane has read the pivot
        for (int c = j + 1 + tid; c < QB; c += CNT) T[j * QLD + c] *= ir;
        if (tid == 0) {
            T[j * QLD + j] = r;
            rd[j] = r;
        }
        __syncthreads();
        // trailing upper triangle: thread (rg, cc) takes column c = j + 1 + cc,
        // rows j + 1 + rg, + CNT / QB, ... up to c
        {
            constexpr int RG = CNT / QB;
            const int c = j + 1 + (tid % QB), rg = tid / QB;
            if (c < QB) {
                const double tjc = T[j * QLD + c];
                for (int i = j + 1 + rg; i <= c; i += RG) T[i * QLD + c] -= T[j * QLD + i] * tjc;
            }
        }
        __syncthreads();
    }
    if (bad && tid == 0) flag[0] = 1;  // one workgroup per launch: a plain store
    // R_kk back to W (upper), zero below
    for (int e = tid; e < QB * QB; e += CNT) {
        const int i = e % QB, j = e / QB;
        W[(size_t)(k0 + j) * ldw + k0 + i] = i <= j ? T[i * QLD + j] : 0.0;
    }
    // inverse: column c of X = R^{-1} by back substitution, one thread per
    // column; X(i, c) is kept in T's strictly lower part as T[c * QLD + i]
    // (i < c) -- row c, left of the diagonal, which R does not use -- and
    // X(c, c) = 1 / r_cc.
    if (tid < QB) {
        const int c = tid;
        const double xcc = 1.0 / rd[c];
        for (int i = c - 1; i >= 0; --i) {
            // four partial sums (independent FMA chains), added at the end
            double s0 = T[i * QLD + c] * xcc, s1 = 0.0, s2 = 0.0, s3 = 0.0;  // l = c
            int l = i + 1;
            for (; l + 3 < c; l += 4) {
                s0 += T[i * QLD + l] * T[c * QLD + l];
                s1 += T[i * QLD + l + 1] * T[c * QLD + l + 1];
                s2 += T[i * QLD + l + 2] * T[c * QLD + l + 2];
                s3 += T[i * QLD + l + 3] * T[c * QLD + l + 3];
            }
            for (; l < c; ++l) s0 += T[i * QLD + l] * T[c * QLD + l];
            T[c * QLD + i] = -((s0 + s1) + (s2 + s3)) / rd[i];
        }
        for (int i = 0; i < QB; ++i)
            Rinv[(size_t)c * QB + i] = i < c ? T[c * QLD + i] : (i == c ? xcc : 0.0);
    }
}

// Diagonal of W over the padding (indices n .. npad-1) set to 1: the padded
// columns of G are zero, so this keeps the Gram matrix positive definite
// with R = I there.
__global__ void k_unit_pad_diag(int n, int npad, double *W, int ldw) {
    const int i = n + blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npad) W[(size_t)i * ldw + i] = 1.0;
}

// W += shift * I on the first n indices.
__global__ void k_shift_diag(int n, double shift, double *W, int ldw) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) W[(size_t)i * ldw + i] += shift;
}

// Strictly lower part of W set to zero (W holds R in its upper triangle).
__global__ void k_zero_lower(int npad, double *W, int ldw) {
    const int j = blockIdx.y;
    for (int i = j + 1 + blockIdx.x * blockDim.x + threadIdx.x; i < npad; i += gridDim.x * blockDim.x)
        W[(size_t)j * ldw + i] = 0.0;
}

// ||X||_F^2 of the leading m x n part: column sums of squares into
// partial[j], then a fixed-order sum on one block.
__global__ void __launch_bounds__(256) k_col_sumsq(int m, int n, const double *__restrict__ X, int ldx,
                                                   double *__restrict__ partial) {
    __shared__ double red[4];
    const double *c = X + (size_t)blockIdx.x * ldx;
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) s += c[i] * c[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}
__global__ void __launch_bounds__(256) k_sum_fixed(int n, const double *__restrict__ partial, double *__restrict__ out) {
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

// partial[j] = sum over i < n of (X(i, j) - delta_ij)^2 for j < n.
__global__ void __launch_bounds__(256) k_dev_identity(int n, const double *__restrict__ X, int ldx,
                                                      double *__restrict__ partial) {
    __shared__ double red[4];
    const int j = blockIdx.x;
    const double *c = X + (size_t)j * ldx;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) {
        const double d = c[i] - (i == j ? 1.0 : 0.0);
        s += d * d;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[j] = red[0] + red[1] + red[2] + red[3];
}

// out[i] = X(i, i), i < n.
__global__ void k_diag_of(int n, const double *__restrict__ X, int ldx, double *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = X[(size_t)i * ldx + i];
}

// X(i, j) = a pseudo-random value in [-1, 1) for i < n, zero below (npad
// rows, `cols` columns, ld npad): a fixed counter-based hash of (i, j)
// (splitmix64 finaliser), so the probe is the same on every call.
__global__ void k_fill_probe(int n, int npad, int cols, double *X) {
    const int j = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npad; i += gridDim.x * blockDim.x) {
        unsigned long long z = 0x9e3779b97f4a7c15ull * (unsigned long long)(j * 65536 + i + 1);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
        z ^= z >> 31;
        X[(size_t)j * npad + i] = i < n ? (double)(z >> 11) * 0x1p-52 - 1.0 : 0.0;
    }
}

// partial[j] = ||Y(:, j) - Z(:, j)||^2 over m rows (fixed order).
__global__ void __launch_bounds__(256) k_diff_colsq(int m, const double *__restrict__ Y, const double *__restrict__ Z,
                                                    int ld, double *__restrict__ partial) {
    __shared__ double red[4];
    const double *y = Y + (size_t)blockIdx.x * ld, *z = Z + (size_t)blockIdx.x * ld;
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) {
        const double d = y[i] - z[i];
        s += d * d;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// partial[j] = number of entries of column j (m rows) that are not finite.
__global__ void __launch_bounds__(256) k_col_nonfinite(int m, const double *__restrict__ X, int ldx,
                                                       double *__restrict__ partial) {
    __shared__ double red[4];
    const double *x = X + (size_t)blockIdx.x * ldx;
    double c = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) c += (fabs(x[i]) <= 1.7976931348623157e308) ? 0.0 : 1.0;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

}  // namespace

void launch_count_nonfinite(int m, int n, const double *X, int ldx, double *partial, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_col_nonfinite, dim3(n), dim3(256), 0, s, m, X, ldx, partial);
    JX_LAUNCHED();
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, s, n, partial, out);
    JX_LAUNCHED();
}

void launch_fill_probe(int n, int npad, int cols, double *X, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_probe, dim3((npad + 255) / 256, cols), dim3(256), 0, s, n, npad, cols, X);
    JX_LAUNCHED();
}

void launch_diff_frob2(int m, int cols, const double *Y, const double *Z, int ld, double *partial, double *out,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_diff_colsq, dim3(cols), dim3(256), 0, s, m, Y, Z, ld, partial);
    JX_LAUNCHED();
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, s, cols, partial, out);
    JX_LAUNCHED();
}

void launch_diag_of(int n, const double *X, int ldx, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_of, dim3((n + 255) / 256), dim3(256), 0, s, n, X, ldx, out);
    JX_LAUNCHED();
}

void launch_dev_identity(int n, const double *X, int ldx, double *partial, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_dev_identity, dim3(n), dim3(256), 0, s, n, X, ldx, partial);
    JX_LAUNCHED();
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, s, n, partial, out);
    JX_LAUNCHED();
}

void launch_chol_diag(double *W, int ldw, int k0, double *Rinv, int *flag, hipStream_t s) {
    ensure_lds_limit(reinterpret_cast<const void *>(&k_chol_diag), (int)CHOL_LDS);
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(CNT), CHOL_LDS, s, W, ldw, k0, Rinv, flag);
    JX_LAUNCHED();
}

void launch_unit_pad_diag(int n, int npad, double *W, int ldw, hipStream_t s) {
    if (npad <= n) return;
    hipLaunchKernelGGL(k_unit_pad_diag, dim3((npad - n + 255) / 256), dim3(256), 0, s, n, npad, W, ldw);
    JX_LAUNCHED();
}

void launch_shift_diag(int n, double shift, double *W, int ldw, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_shift_diag, dim3((n + 255) / 256), dim3(256), 0, s, n, shift, W, ldw);
    JX_LAUNCHED();
}

void launch_zero_lower(int npad, double *W, int ldw, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_lower, dim3((npad + 255) / 256, npad), dim3(256), 0, s, npad, W, ldw);
    JX_LAUNCHED();
}

void launch_frob2(int m, int n, const double *X, int ldx, double *partial, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_col_sumsq, dim3(n), dim3(256), 0, s, m, n, X, ldx, partial);
    JX_LAUNCHED();
    hipLaunchKernelGGL(k_sum_fixed, dim3(1), dim3(256), 0, s, n, partial, out);
    JX_LAUNCHED();
}

}  // namespace jx
