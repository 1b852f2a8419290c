// k_gemm.hip -- general FP64 GEMM on gfx950 MFMA for the orthogonality
// refinement (Newton-Schulz step Q <- Q (3 I - Q^T Q) / 2) and the FP64
// recomputation of the iterate from the original matrix (A1 = Q^T A0 Q).
//
// C = alpha op(A) op(B) + beta C, column-major, M, N multiples of 128, K a
// multiple of 16.  Each workgroup computes a 128 x 128 tile of C as the tile
// of C^T = op(B)^T op(A)^T, so that in the MFMA result layout consecutive
// lanes hold consecutive rows of the column-major C (coalesced stores).
// Both operand tiles pass through LDS in k-major order (transposed on the way
// in when the source is stored the other way).  Waves in a 2 x 2 layout, each
// 64 x 64 of C^T.
#include "jx_common.hpp"

namespace jx {

namespace {

constexpr int GT = 128;       // tile
constexpr int GK = 16;        // k chunk
constexpr int GLD = GT + 1;   // LDS stride

__global__ void __launch_bounds__(256, 2)
k_gemm_f64(int ta, int tb, int K, double alpha, const double *__restrict__ A, int lda,
           const double *__restrict__ B, int ldb, double beta, double *__restrict__ C, int ldc) {
    extern __shared__ double lds[];
    double *As = lds;             // op(A)(j, k) at As[k * GLD + j]   (j: rows of C)
    double *Bs = lds + GK * GLD;  // op(B)(k, i) at Bs[k * GLD + i]   (i: cols of C)
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int g = lane >> 4, x = lane & 15;
    const int wi = w & 1, wj = w >> 1;
    const size_t rowC0 = (size_t)blockIdx.x * GT;  // rows of C (j)
    const size_t colC0 = (size_t)blockIdx.y * GT;  // cols of C (i)

    d4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};

    double ra[GT * GK / 256], rb[GT * GK / 256];
    auto fetch = [&](int k0) {
#pragma unroll
        for (int m = 0; m < GT * GK / 256; ++m) {
            const int e = tid + 256 * m;  // 0 .. GT*GK-1
            if (!ta) { const int j = e % GT, k = e / GT; ra[m] = A[(size_t)(k0 + k) * lda + rowC0 + j]; }
            else { const int k = e % GK, j = e / GK; ra[m] = A[(rowC0 + j) * lda + k0 + k]; }
            if (tb) { const int i = e % GT, k = e / GT; rb[m] = B[(size_t)(k0 + k) * ldb + colC0 + i]; }
            else { const int k = e % GK, i = e / GK; rb[m] = B[(colC0 + i) * ldb + k0 + k]; }
        }
    };
    auto stage = [&]() {
#pragma unroll
        for (int m = 0; m < GT * GK / 256; ++m) {
            const int e = tid + 256 * m;
            if (!ta) { const int j = e % GT, k = e / GT; As[k * GLD + j] = ra[m]; }
            else { const int k = e % GK, j = e / GK; As[k * GLD + j] = ra[m]; }
            if (tb) { const int i = e % GT, k = e / GT; Bs[k * GLD + i] = rb[m]; }
            else { const int k = e % GK, i = e / GK; Bs[k * GLD + i] = rb[m]; }
        }
    };

    fetch(0);
    for (int k0 = 0; k0 < K; k0 += GK) {
        __syncthreads();
        stage();
        __syncthreads();
        if (k0 + GK < K) fetch(k0 + GK);
#pragma unroll 1
        for (int kk = 0; kk < GK; kk += 4) {
            const int k = kk + g;
            double af[4], bf[4];
            // MFMA A operand: op(B)^T (i, k); B operand: op(A)^T (k, j)
#pragma unroll
            for (int a = 0; a < 4; ++a) af[a] = Bs[k * GLD + 64 * wi + 16 * a + x];
#pragma unroll
            for (int b = 0; b < 4; ++b) bf[b] = As[k * GLD + 64 * wj + 16 * b + x];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) acc[a][b] = mfma_f64(af[a], bf[b], acc[a][b]);
        }
    }
    // acc[a][b] lane (g, x), component v = C^T(64 wi + 16 a + g + 4 v, 64 wj + 16 b + x)
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            double *cc = C + (colC0 + 64 * wi + 16 * a + g + 4 * v) * ldc + rowC0 + 64 * wj;
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                double val = alpha * acc[a][b][v];
                if (beta != 0.0) val += beta * cc[16 * b + x];
                cc[16 * b + x] = val;
            }
        }
}

}  // namespace

void launch_gemm_f64(char ta, char tb, int M, int N, int K, double alpha, const double *A, int lda,
                     const double *B, int ldb, double beta, double *C, int ldc, hipStream_t s) {
    if (M % GT || N % GT || K % GK) {
        set_error("gemm: M, N must be multiples of 128 and K of 16");
        throw HipFail{hipErrorInvalidValue};
    }
    const int ita = (ta == 'T' || ta == 't'), itb = (tb == 'T' || tb == 't');
    constexpr size_t lds_bytes = sizeof(double) * 2 * GK * GLD;
    ensure_lds_limit(reinterpret_cast<const void *>(&k_gemm_f64), (int)lds_bytes);
    hipLaunchKernelGGL(k_gemm_f64, dim3(M / GT, N / GT), dim3(256), lds_bytes, s, ita, itb, K, alpha, A, lda, B,
                       ldb, beta, C, ldc);
    JX_LAUNCHED();
}

}  // namespace jx
