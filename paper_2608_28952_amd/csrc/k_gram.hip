// k_gram.hip -- Gram blocks of the one-sided Jacobi SVD on gfx950 FP64 MFMA,
// and the SVD's final column norms / U = G Sigma^+.
//
// Alg. 6 (§6) forms each 2b x 2b subproblem A_hat = G(:,[I,J])^T G(:,[I,J])
// on the fly; eq. (SVD_subproblem) writes it as the sum over row tiles K of
// G_KI^T G_KJ.  Here a workgroup computes the partial sum over one chunk of
// rows for one pair (MFMA, both operands from one LDS tile of the chunk), and
// a second kernel adds the partials of a pair in a fixed order (no atomics,
// the result does not depend on scheduling).
#include "jx_common.hpp"

namespace jx {

namespace {

constexpr int GKR = 16;  // rows per LDS stage

template <int B, class T>
__global__ void __launch_bounds__(256, 2)
k_gram_partial(const T *__restrict__ G, int ldg, const int *__restrict__ pairs, int rows_per_chunk,
               T *__restrict__ partial) {
    using MT = MfmaTraits<T>;
    typedef typename MT::acc_t acc_t;
    constexpr int M2 = 2 * B;
    constexpr int LDX = M2 + 1;
    constexpr int HALF = M2 / 2;           // output rows/cols per wave
    constexpr int TI = HALF / 16;          // 16-tiles per wave and dimension
    constexpr int PER = GKR * M2 / 256;    // staged values per thread
    __shared__ T xs[2][GKR * LDX];
    const int p = blockIdx.y, ch = blockIdx.x;
    const int I = pairs[2 * p], J = pairs[2 * p + 1];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int g = lane >> 4, x = lane & 15;
    const int wi = w & 1, wj = w >> 1;
    const size_t r0 = (size_t)ch * rows_per_chunk;

    acc_t acc[TI][TI];
#pragma unroll
    for (int a = 0; a < TI; ++a)
#pragma unroll
        for (int b = 0; b < TI; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

    auto colof = [&](int c) { return c < B ? I * B + c : J * B + (c - B); };
    T reg[PER];
    auto fetch = [&](size_t rr) {
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int e = tid + 256 * m;
            const int r = e % GKR, c = e / GKR;
            reg[m] = G[(size_t)colof(c) * ldg + rr + r];
        }
    };
    auto stage = [&](T *dst) {
#pragma unroll
        for (int m = 0; m < PER; ++m) {
            const int e = tid + 256 * m;
            const int r = e % GKR, c = e / GKR;
            dst[r * LDX + c] = reg[m];
        }
    };
    const int nst = rows_per_chunk / GKR;
    fetch(r0);
    stage(xs[0]);
    __syncthreads();
    for (int st = 0; st < nst; ++st) {
        if (st + 1 < nst) fetch(r0 + (size_t)(st + 1) * GKR);
        const T *X = xs[st & 1];
#pragma unroll
        for (int kk = 0; kk < GKR; kk += 4) {
            const int k = kk + g;  // rows of the chunk: any order, the same for both operands
            T af[TI], bf[TI];
#pragma unroll
            for (int a = 0; a < TI; ++a) af[a] = X[k * LDX + HALF * wi + 16 * a + x];  // X^T(i, k)
#pragma unroll
            for (int b = 0; b < TI; ++b) bf[b] = X[k * LDX + HALF * wj + 16 * b + x];  // X(k, j)
#pragma unroll
            for (int a = 0; a < TI; ++a)
#pragma unroll
                for (int b = 0; b < TI; ++b) acc[a][b] = MT::mma(af[a], bf[b], acc[a][b]);
        }
        if (st + 1 < nst) stage(xs[(st + 1) & 1]);
        __syncthreads();
    }
    // acc[a][b] lane (g, x) comp v = C(i, j), i = HALF wi + 16 a + rrow(g, v),
    // j = HALF wj + 16 b + x; stored at [i * M2 + j] (the transpose, equal by
    // symmetry; consecutive lanes write consecutive addresses)
    T *out = partial + ((size_t)p * gridDim.x + ch) * M2 * M2;
#pragma unroll
    for (int a = 0; a < TI; ++a)
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
            for (int b = 0; b < TI; ++b)
                out[(size_t)(HALF * wi + 16 * a + MT::rrow(g, v)) * M2 + HALF * wj + 16 * b + x] = acc[a][b][v];
}

// ahat[p] = sum over chunks c = 0 .. nch-1 of partial[p][c], in that order (FP64).
template <class T>
__global__ void k_gram_reduce(int m2sq, int nch, const T *__restrict__ partial, double *__restrict__ ahat) {
    const int p = blockIdx.y;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m2sq) return;
    const T *src = partial + (size_t)p * nch * m2sq + e;
    double s = 0.0;
    for (int c = 0; c < nch; ++c) s += (double)src[(size_t)c * m2sq];
    ahat[(size_t)p * m2sq + e] = s;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// sigma[j] = ||G(:, j)||_2 over the first m rows (fixed-order reduction, in
// FP64 for either storage type).
template <class T>
__global__ void __launch_bounds__(256) k_col_norms(int m, const T *__restrict__ G, int ldg,
                                                   double *__restrict__ sigma) {
    __shared__ double red[4];
    const T *c = G + (size_t)blockIdx.x * ldg;
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) s += (double)c[i] * (double)c[i];
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) sigma[blockIdx.x] = sqrt(red[0] + red[1] + red[2] + red[3]);
}

// U(:, rank[j]) = G(:, j) / sigma[j] (zero column for sigma = 0), rows 0..m-1.
__global__ void __launch_bounds__(256) k_scale_scatter(int m, const double *__restrict__ G, int ldg,
                                                       const double *__restrict__ sigma, const int *__restrict__ rank,
                                                       double *__restrict__ U, int ldu) {
    const int j = blockIdx.x;
    const double sj = sigma[j];
    const double inv = sj > 0.0 ? 1.0 / sj : 0.0;
    const double *src = G + (size_t)j * ldg;
    double *dst = U + (size_t)rank[j] * ldu;
    for (int i = threadIdx.x; i < m; i += 256) dst[i] = sj > 0.0 ? src[i] * inv : 0.0;
}

}  // namespace

template <class T>
static void launch_gram_t(int b, int npairs, const int *pairs, const T *G, int ldg, int m_rows, int nchunks,
                          T *partial, double *ahat, hipStream_t s) {
    if (npairs <= 0) return;
    const int rows_per_chunk = m_rows / nchunks;
    if (rows_per_chunk % GKR || rows_per_chunk * nchunks != m_rows) {
        set_error("gram: row chunks must be equal multiples of 16");
        throw HipFail{hipErrorInvalidValue};
    }
    dim3 grid(nchunks, npairs);
    if (b == 64) hipLaunchKernelGGL((k_gram_partial<64, T>), grid, dim3(256), 0, s, G, ldg, pairs, rows_per_chunk, partial);
    else if (b == 32) hipLaunchKernelGGL((k_gram_partial<32, T>), grid, dim3(256), 0, s, G, ldg, pairs, rows_per_chunk, partial);
    else { set_error("gram: block size must be 32 or 64"); throw HipFail{hipErrorInvalidValue}; }
    JX_LAUNCHED();
    const int m2sq = 4 * b * b;
    hipLaunchKernelGGL((k_gram_reduce<T>), dim3((m2sq + 255) / 256, npairs), dim3(256), 0, s, m2sq, nchunks, partial, ahat);
    JX_LAUNCHED();
}

void launch_gram(int b, int npairs, const int *pairs, const double *G, int ldg, int m_rows, int nchunks,
                 double *partial, double *ahat, hipStream_t s) {
    launch_gram_t<double>(b, npairs, pairs, G, ldg, m_rows, nchunks, partial, ahat, s);
}
void launch_gram32(int b, int npairs, const int *pairs, const float *G, int ldg, int m_rows, int nchunks,
                   float *partial, double *ahat, hipStream_t s) {
    launch_gram_t<float>(b, npairs, pairs, G, ldg, m_rows, nchunks, partial, ahat, s);
}

void launch_col_norms(int m, int n, const double *G, int ldg, double *sigma, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_col_norms<double>, dim3(n), dim3(256), 0, s, m, G, ldg, sigma);
    JX_LAUNCHED();
}
void launch_col_norms32(int m, int n, const float *G, int ldg, double *sigma, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_col_norms<float>, dim3(n), dim3(256), 0, s, m, G, ldg, sigma);
    JX_LAUNCHED();
}

void launch_scale_scatter(int m, int n, const double *G, int ldg, const double *sigma, const int *rank,
                          double *U, int ldu, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scale_scatter, dim3(n), dim3(256), 0, s, m, G, ldg, sigma, rank, U, ldu);
    JX_LAUNCHED();
}

}  // namespace jx
