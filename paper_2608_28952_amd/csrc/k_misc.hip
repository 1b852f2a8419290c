// k_misc.hip -- layout conversion, reductions and the final sort of the
// eigensolver (gfx950).
//
// The symmetric iterate is kept as its upper block triangle (block (I, J),
// I <= J, of order b, column-major, slot J (J + 1) / 2 + I); the input is
// column-major with only one triangle valid.  The off-norm Xi(A) of
// eq. (Omega_A), §2.1, is summed directly over the off-diagonal entries
// (never as ||A||_F^2 minus the diagonal, which cancels): per-block partial
// sums, then one workgroup adds them in a fixed order, so the result does not
// depend on scheduling.
#include "jx_common.hpp"

namespace jx {

namespace {

__device__ __forceinline__ void slot_to_block(int s, int &I, int &J) {
    int j = (int)((sqrt(8.0 * s + 1.0) - 1.0) * 0.5);
    while ((j + 1) * (j + 2) / 2 <= s) ++j;
    while (j * (j + 1) / 2 > s) --j;
    J = j;
    I = s - j * (j + 1) / 2;
}

// One workgroup per stored block (I, J).  The b x b source region holding
// the valid triangle's copy of that block is staged in LDS (S[c * (b+1) + r]).
__global__ void __launch_bounds__(256) k_pack_sym(int n, int b, const double *__restrict__ A, int lda,
                                                  int upper, double *__restrict__ ablk) {
    extern __shared__ double S[];
    int I, J;
    slot_to_block(blockIdx.x, I, J);
    const int R0 = upper ? I : J, C0 = upper ? J : I;  // source region (block rows R0, cols C0)
    const int ld = b + 1;
    for (int e = threadIdx.x; e < b * b; e += 256) {
        const int r = e % b, c = e / b;
        const int gi = R0 * b + r, gj = C0 * b + c;
        S[c * ld + r] = (gi < n && gj < n) ? A[(size_t)gj * lda + gi] : 0.0;
    }
    __syncthreads();
    double *dst = ablk + ublk(I, J) * (size_t)(b * b);
    for (int e = threadIdx.x; e < b * b; e += 256) {
        const int r = e % b, c = e / b;  // element (r, c) of block (I, J)
        const int gi = I * b + r, gj = J * b + c;
        double v;
        if (upper) v = (gi <= gj) ? S[c * ld + r] : S[r * ld + c];
        else v = (gi <= gj) ? S[r * ld + c] : S[c * ld + r];
        dst[e] = v;
    }
}

__global__ void __launch_bounds__(256) k_unpack_sym(int b, const double *__restrict__ ablk,
                                                    double *__restrict__ F, int ldf) {
    int I, J;
    slot_to_block(blockIdx.x, I, J);
    const double *src = ablk + ublk(I, J) * (size_t)(b * b);
    for (int e = threadIdx.x; e < b * b; e += 256) {
        const int r = e % b, c = e / b;
        const double v = src[e];
        F[(size_t)(J * b + c) * ldf + I * b + r] = v;
        F[(size_t)(I * b + r) * ldf + J * b + c] = v;
    }
}

// F (npad x npad) = symmetric completion of the `uplo` triangle of A, zero pad.
// One workgroup per 64 x 64 tile of F.
__global__ void __launch_bounds__(256) k_full_from_tri(int n, const double *__restrict__ A, int lda,
                                                       int upper, double *__restrict__ F, int ldf) {
    __shared__ double S[64 * 65];
    const int ti = blockIdx.x, tj = blockIdx.y;  // tile rows ti*64, cols tj*64
    const bool mirror = upper ? (ti > tj) : (ti < tj);
    const int R0 = mirror ? tj : ti, C0 = mirror ? ti : tj;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e & 63, c = e >> 6;
        const int gi = R0 * 64 + r, gj = C0 * 64 + c;
        S[c * 65 + r] = (gi < n && gj < n) ? A[(size_t)gj * lda + gi] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e & 63, c = e >> 6;
        const int gi = ti * 64 + r, gj = tj * 64 + c;
        double v;
        if (!mirror && ti != tj) v = S[c * 65 + r];
        else if (mirror) v = S[r * 65 + c];
        else {  // diagonal tile: take the valid triangle
            const bool valid = upper ? (gi <= gj) : (gi >= gj);
            v = valid ? S[c * 65 + r] : S[r * 65 + c];
        }
        F[(size_t)gj * ldf + gi] = v;
    }
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void __launch_bounds__(256) k_block_norms(int b, const double *__restrict__ ablk,
                                                     double *__restrict__ partial) {
    __shared__ double red[8];
    int I, J;
    slot_to_block(blockIdx.x, I, J);
    const double *src = ablk + ublk(I, J) * (size_t)(b * b);
    double off = 0.0, dia = 0.0;
    for (int e = threadIdx.x; e < b * b; e += 256) {
        const double v = src[e];
        if (I != J) off += 2.0 * v * v;
        else if (e % b == e / b) dia += v * v;
        else off += v * v;
    }
    off = wave_sum(off);
    dia = wave_sum(dia);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[w] = off; red[4 + w] = dia; }
    __syncthreads();
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = red[0] + red[1] + red[2] + red[3];
        partial[2 * blockIdx.x + 1] = red[4] + red[5] + red[6] + red[7];
    }
}

// out[0] = sum of partial[2 i], out[1] = sum of partial[2 i + 1]; fixed order.
__global__ void __launch_bounds__(256) k_reduce_pairs(int count, const double *__restrict__ partial,
                                                      double *__restrict__ out) {
    __shared__ double red[8];
    double a = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < count; i += 256) {
        a += partial[2 * i];
        c += partial[2 * i + 1];
    }
    a = wave_sum(a);
    c = wave_sum(c);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[w] = a; red[4 + w] = c; }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = red[0] + red[1] + red[2] + red[3];
        out[1] = red[4] + red[5] + red[6] + red[7];
    }
}

__global__ void k_set_identity(int npad, double *Q, int ldq) {
    const size_t j = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npad; i += gridDim.x * blockDim.x)
        Q[j * ldq + i] = (i == (int)j) ? 1.0 : 0.0;
}

// dst (npad x npad) = src (n x n) with the pad part set to the identity.
__global__ void k_copy_pad(int n, const double *__restrict__ src, int lds_, double *__restrict__ dst,
                           int ldd, int npad) {
    const int j = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npad; i += gridDim.x * blockDim.x) {
        double v;
        if (i < n && j < n) v = src[(size_t)j * lds_ + i];
        else v = (i == j) ? 1.0 : 0.0;
        dst[(size_t)j * ldd + i] = v;
    }
}

__global__ void k_extract_diag(int npad, int b, const double *__restrict__ ablk, double *__restrict__ w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    const int I = i / b, r = i % b;
    w[i] = ablk[ublk(I, I) * (size_t)(b * b) + (size_t)r * b + r];
}

// rank[i] = #{ j : w_j strictly before w_i, or equal with j < i } (stable).
// A workgroup ranks 64 values (one per lane); its 16 waves split the j range
// and their counts are added at the end.
__global__ void __launch_bounds__(1024) k_rank(int n, const double *__restrict__ w, int dir,
                                               int *__restrict__ rank) {
    __shared__ int part[16][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const double wi = (i < n) ? w[i] : 0.0;
    const int chunk = (n + 15) / 16, j0 = wv * chunk, j1 = min(n, j0 + chunk);
    int cnt = 0;
    for (int j = j0; j < j1; ++j) {
        const double wj = w[j];
        const bool before = dir > 0 ? (wj < wi || (wj == wi && j < i)) : (wj > wi || (wj == wi && j < i));
        cnt += before ? 1 : 0;
    }
    part[wv][lane] = cnt;
    __syncthreads();
    if (wv == 0 && i < n) {
        int s = 0;
        for (int k = 0; k < 16; ++k) s += part[k][lane];
        rank[i] = s;
    }
}

__global__ void k_scatter_values(int n, const double *__restrict__ w, const int *__restrict__ rank,
                                 double *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[rank[i]] = w[i];
}

__global__ void __launch_bounds__(256) k_scatter_columns(int rows, const double *__restrict__ src, int lds_,
                                                         const int *__restrict__ rank, double *__restrict__ out,
                                                         int ldo) {
    const int j = blockIdx.x;
    const double *s = src + (size_t)j * lds_;
    double *d = out + (size_t)rank[j] * ldo;
    for (int i = threadIdx.x; i < rows; i += 256) d[i] = s[i];
}

}  // namespace

void launch_pack_sym(int n, int npad, int b, const double *A, int lda, char uplo, double *ablk,
                     hipStream_t s) {
    const int N = npad / b;
    const int nb = N * (N + 1) / 2;
    const int upper = (uplo == 'U' || uplo == 'u') ? 1 : 0;
    hipLaunchKernelGGL(k_pack_sym, dim3(nb), dim3(256), sizeof(double) * b * (b + 1), s, n, b, A, lda, upper, ablk);
    JX_LAUNCHED();
}

void launch_unpack_sym(int npad, int b, const double *ablk, double *A, int lda, hipStream_t s) {
    const int N = npad / b;
    hipLaunchKernelGGL(k_unpack_sym, dim3(N * (N + 1) / 2), dim3(256), 0, s, b, ablk, A, lda);
    JX_LAUNCHED();
}

void launch_full_from_triangle(int n, int npad, const double *A, int lda, char uplo, double *F,
                               hipStream_t s) {
    const int T = npad / 64;
    const int upper = (uplo == 'U' || uplo == 'u') ? 1 : 0;
    hipLaunchKernelGGL(k_full_from_tri, dim3(T, T), dim3(256), 0, s, n, A, lda, upper, F, npad);
    JX_LAUNCHED();
}

void launch_block_norms(int npad, int b, const double *ablk, double *partial, double *out,
                        hipStream_t s) {
    const int N = npad / b;
    const int nb = N * (N + 1) / 2;
    hipLaunchKernelGGL(k_block_norms, dim3(nb), dim3(256), 0, s, b, ablk, partial);
    JX_LAUNCHED();
    hipLaunchKernelGGL(k_reduce_pairs, dim3(1), dim3(256), 0, s, nb, partial, out);
    JX_LAUNCHED();
}

void launch_set_identity(int n, int npad, double *Q, int ldq, hipStream_t s) {
    (void)n;
    hipLaunchKernelGGL(k_set_identity, dim3((npad + 255) / 256, npad), dim3(256), 0, s, npad, Q, ldq);
    JX_LAUNCHED();
}

void launch_copy_pad(int n, int npad, const double *src, int lds_, double *dst, int ldd,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_copy_pad, dim3((npad + 255) / 256, npad), dim3(256), 0, s, n, src, lds_, dst, ldd, npad);
    JX_LAUNCHED();
}

void launch_extract_diag(int npad, int b, const double *ablk, double *w, hipStream_t s) {
    hipLaunchKernelGGL(k_extract_diag, dim3((npad + 255) / 256), dim3(256), 0, s, npad, b, ablk, w);
    JX_LAUNCHED();
}

void launch_rank(int n, const double *w, int dir, int *rank, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_rank, dim3((n + 63) / 64), dim3(1024), 0, s, n, w, dir, rank);
    JX_LAUNCHED();
}

void launch_scatter_values(int n, const double *w, const int *rank, double *out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scatter_values, dim3((n + 255) / 256), dim3(256), 0, s, n, w, rank, out);
    JX_LAUNCHED();
}

void launch_scatter_columns(int rows, int n, const double *src, int lds_, const int *rank,
                            double *out, int ldo, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_scatter_columns, dim3(n), dim3(256), 0, s, rows, src, lds_, rank, out, ldo);
    JX_LAUNCHED();
}

}  // namespace jx

namespace jx {
namespace {

__global__ void k_vperm_from_colmajor(int m2, const double *__restrict__ src, double *__restrict__ dst) {
    const double *s = src + (size_t)blockIdx.x * m2 * m2;
    double *d = dst + (size_t)blockIdx.x * m2 * m2;
    for (int e = threadIdx.x; e < m2 * m2; e += blockDim.x) {
        const int k = e % m2, i = e / m2;  // element (k, i), column-major
        d[vperm(k, i, m2)] = s[e];
    }
}

// The same in FP32, in the vperm32 order of the FP32 MFMA kernels.
__global__ void k_vperm32_from_colmajor(int m2, const double *__restrict__ src, float *__restrict__ dst) {
    const double *s = src + (size_t)blockIdx.x * m2 * m2;
    float *d = dst + (size_t)blockIdx.x * m2 * m2;
    for (int e = threadIdx.x; e < m2 * m2; e += blockDim.x) {
        const int k = e % m2, i = e / m2;  // element (k, i), column-major
        d[vperm32(k, i, m2)] = (float)s[e];
    }
}

// A([I,J],[I,J]) <- D for each pair (upper block storage).
__global__ void k_write_pair_blocks(int b, const int *__restrict__ pairs, const double *__restrict__ D,
                                    double *__restrict__ ablk) {
    const int p = blockIdx.x, m2 = 2 * b;
    const int I = pairs[2 * p], J = pairs[2 * p + 1];
    const double *d = D + (size_t)p * m2 * m2;
    for (int e = threadIdx.x; e < m2 * m2; e += blockDim.x) {
        const int r = e % m2, c = e / m2;
        const double v = d[e];
        if (c < b && r < b) ablk[ublk(I, I) * (size_t)(b * b) + c * b + r] = v;
        else if (r < b && c >= b) ablk[ublk(I, J) * (size_t)(b * b) + (c - b) * b + r] = v;
        else if (r >= b && c >= b) ablk[ublk(J, J) * (size_t)(b * b) + (c - b) * b + (r - b)] = v;
    }
}

}  // namespace

void launch_vperm_from_colmajor(int count, int m2, const double *src, double *dst, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_vperm_from_colmajor, dim3(count), dim3(256), 0, s, m2, src, dst);
    JX_LAUNCHED();
}

void launch_vperm32_from_colmajor(int count, int m2, const double *src, float *dst, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_vperm32_from_colmajor, dim3(count), dim3(256), 0, s, m2, src, dst);
    JX_LAUNCHED();
}

void launch_write_pair_blocks(int count, int b, const int *pairs, const double *D, double *ablk,
                              hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_write_pair_blocks, dim3(count), dim3(256), 0, s, b, pairs, D, ablk);
    JX_LAUNCHED();
}

}  // namespace jx

namespace jx {
namespace {
// dst (mpad x npad) = src (m x n) with zero padding.
__global__ void k_copy_rect(int m, int n, const double *__restrict__ src, int lds_, double *__restrict__ dst,
                            int ldd, int mpad) {
    const int j = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < mpad; i += gridDim.x * blockDim.x)
        dst[(size_t)j * ldd + i] = (i < m && j < n) ? src[(size_t)j * lds_ + i] : 0.0;
}
}  // namespace
void launch_copy_rect(int m, int n, const double *src, int lds_, double *dst, int ldd, int mpad, int npad,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_copy_rect, dim3((mpad + 255) / 256, npad), dim3(256), 0, s, m, n, src, lds_, dst, ldd, mpad);
    JX_LAUNCHED();
}
}  // namespace jx

namespace jx {
namespace {
template <class S, class D>
__global__ void k_cast(size_t count, const S *__restrict__ src, D *__restrict__ dst) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = (D)src[i];
}
__global__ void k_set_identity32(int npad, float *Q, int ldq) {
    const size_t j = blockIdx.y;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < npad; i += gridDim.x * blockDim.x)
        Q[j * ldq + i] = (i == (int)j) ? 1.0f : 0.0f;
}
__global__ void __launch_bounds__(256) k_block_norms32(int b, const float *__restrict__ ablk, double *__restrict__ partial) {
    __shared__ double red[8];
    const int s = blockIdx.x;
    int j = (int)((sqrt(8.0 * s + 1.0) - 1.0) * 0.5);
    while ((j + 1) * (j + 2) / 2 <= s) ++j;
    while (j * (j + 1) / 2 > s) --j;
    const int J = j, I = s - j * (j + 1) / 2;
    const float *src = ablk + ublk(I, J) * (size_t)(b * b);
    double off = 0.0, dia = 0.0;
    for (int e = threadIdx.x; e < b * b; e += 256) {
        const double v = src[e];
        if (I != J) off += 2.0 * v * v;
        else if (e % b == e / b) dia += v * v;
        else off += v * v;
    }
    for (int o = 32; o > 0; o >>= 1) { off += __shfl_xor(off, o, 64); dia += __shfl_xor(dia, o, 64); }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[w] = off; red[4 + w] = dia; }
    __syncthreads();
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = red[0] + red[1] + red[2] + red[3];
        partial[2 * blockIdx.x + 1] = red[4] + red[5] + red[6] + red[7];
    }
}
__global__ void __launch_bounds__(256) k_reduce_pairs2(int count, const double *__restrict__ partial, double *__restrict__ out) {
    __shared__ double red[8];
    double a = 0.0, c = 0.0;
    for (int i = threadIdx.x; i < count; i += 256) { a += partial[2 * i]; c += partial[2 * i + 1]; }
    for (int o = 32; o > 0; o >>= 1) { a += __shfl_xor(a, o, 64); c += __shfl_xor(c, o, 64); }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[w] = a; red[4 + w] = c; }
    __syncthreads();
    if (threadIdx.x == 0) { out[0] = red[0] + red[1] + red[2] + red[3]; out[1] = red[4] + red[5] + red[6] + red[7]; }
}
}  // namespace

void launch_cast_to_f32(size_t count, const double *src, float *dst, hipStream_t s) {
    if (!count) return;
    hipLaunchKernelGGL((k_cast<double, float>), dim3(2048), dim3(256), 0, s, count, src, dst);
    JX_LAUNCHED();
}
void launch_cast_to_f64(size_t count, const float *src, double *dst, hipStream_t s) {
    if (!count) return;
    hipLaunchKernelGGL((k_cast<float, double>), dim3(2048), dim3(256), 0, s, count, src, dst);
    JX_LAUNCHED();
}
void launch_set_identity32(int npad, float *Q, int ldq, hipStream_t s) {
    hipLaunchKernelGGL(k_set_identity32, dim3((npad + 255) / 256, npad), dim3(256), 0, s, npad, Q, ldq);
    JX_LAUNCHED();
}
void launch_block_norms32(int npad, int b, const float *ablk, double *partial, double *out, hipStream_t s) {
    const int N = npad / b, nb = N * (N + 1) / 2;
    hipLaunchKernelGGL(k_block_norms32, dim3(nb), dim3(256), 0, s, b, ablk, partial);
    JX_LAUNCHED();
    hipLaunchKernelGGL(k_reduce_pairs2, dim3(1), dim3(256), 0, s, nb, partial, out);
    JX_LAUNCHED();
}
}  // namespace jx

// ---------------------------------------------------------------------------
// Re-sorting the indices by the current diagonal (between sweeps)
// ---------------------------------------------------------------------------
namespace jx {
namespace {

// inv[rank[i]] = i for i < n (rank: a permutation of 0 .. n-1); inv[i] = i
// on the padding n .. npad-1.
__global__ void k_inverse_perm(int n, int npad, const int *__restrict__ rank, int *__restrict__ inv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) inv[rank[i]] = i;
    else if (i < npad) inv[i] = i;
}

// dst(i', j') = src(inv[i'], inv[j']) in the upper block storage (block
// order b, diagonal blocks held whole); one workgroup per stored block of dst.
template <class T>
__global__ void __launch_bounds__(256) k_permute_sym(int b, const int *__restrict__ inv, const T *__restrict__ src,
                                                     T *__restrict__ dst) {
    int I, J;
    slot_to_block(blockIdx.x, I, J);
    T *out = dst + ublk(I, J) * (size_t)(b * b);
    for (int e = threadIdx.x; e < b * b; e += 256) {
        const int r = e % b, c = e / b;
        const int i = inv[I * b + r], j = inv[J * b + c];
        const int bi = i / b, bj = j / b;
        T v;
        if (bi <= bj) v = src[ublk(bi, bj) * (size_t)(b * b) + (size_t)(j % b) * b + i % b];
        else v = src[ublk(bj, bi) * (size_t)(b * b) + (size_t)(i % b) * b + j % b];
        out[e] = v;
    }
}

// dst(:, j') = src(:, inv[j']) for `rows` rows of `cols` columns.
template <class T>
__global__ void k_permute_cols(int rows, const int *__restrict__ inv, const T *__restrict__ src, int lds_,
                               T *__restrict__ dst, int ldd) {
    const int j = blockIdx.y;
    const T *s = src + (size_t)inv[j] * lds_;
    T *d = dst + (size_t)j * ldd;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += gridDim.x * blockDim.x) d[i] = s[i];
}

}  // namespace

void launch_inverse_perm(int n, int npad, const int *rank, int *inv, hipStream_t s) {
    hipLaunchKernelGGL(k_inverse_perm, dim3((npad + 255) / 256), dim3(256), 0, s, n, npad, rank, inv);
    JX_LAUNCHED();
}

template <class T>
static void permute_sym_t(int npad, int b, const int *inv, const T *src, T *dst, hipStream_t s) {
    const int N = npad / b;
    hipLaunchKernelGGL((k_permute_sym<T>), dim3(N * (N + 1) / 2), dim3(256), 0, s, b, inv, src, dst);
    JX_LAUNCHED();
}
void launch_permute_sym(int npad, int b, const int *inv, const double *src, double *dst, hipStream_t s) {
    permute_sym_t<double>(npad, b, inv, src, dst, s);
}
void launch_permute_sym32(int npad, int b, const int *inv, const float *src, float *dst, hipStream_t s) {
    permute_sym_t<float>(npad, b, inv, src, dst, s);
}

template <class T>
static void permute_cols_t(int rows, int cols, const int *inv, const T *src, int lds_, T *dst, int ldd,
                           hipStream_t s) {
    hipLaunchKernelGGL((k_permute_cols<T>), dim3((rows + 255) / 256, cols), dim3(256), 0, s, rows, inv, src, lds_,
                       dst, ldd);
    JX_LAUNCHED();
}
void launch_permute_cols(int rows, int cols, const int *inv, const double *src, int lds_, double *dst, int ldd,
                         hipStream_t s) {
    permute_cols_t<double>(rows, cols, inv, src, lds_, dst, ldd, s);
}
void launch_permute_cols32(int rows, int cols, const int *inv, const float *src, int lds_, float *dst, int ldd,
                           hipStream_t s) {
    permute_cols_t<float>(rows, cols, inv, src, lds_, dst, ldd, s);
}

}  // namespace jx

namespace jx {
namespace {
__global__ void k_extract_diag32(int npad, int b, const float *__restrict__ ablk, double *__restrict__ w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    const int I = i / b, r = i % b;
    w[i] = (double)ablk[ublk(I, I) * (size_t)(b * b) + (size_t)r * b + r];
}
}  // namespace
void launch_extract_diag32(int npad, int b, const float *ablk, double *w, hipStream_t s) {
    hipLaunchKernelGGL(k_extract_diag32, dim3((npad + 255) / 256), dim3(256), 0, s, npad, b, ablk, w);
    JX_LAUNCHED();
}
}  // namespace jx
