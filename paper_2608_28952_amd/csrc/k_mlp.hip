// k_mlp.hip -- the learned warm start's network on gfx950: forward, backward,
// MSE gradient and Adam for the MLP theta (8) -> 256 -> 256 -> 2016 (the
// strictly upper coordinates of a 64 x 64 skew generator).  GEMMs run on BF16
// MFMA (v_mfma_f32_16x16x16_bf16) with FP32 accumulation; master weights are
// FP32 with a BF16 copy refreshed by the optimiser step.
//
// Parameter vector (FP32 master, gradients and the BF16 copy share it),
// row-major K x N weights:
//   W1 16 x 256 (rows 8..15 are zero: the input is padded to 16 features),
//   W2 256 x 256, W3 256 x 2016, then b1 (256), b2 (256), b3 (2016).
// Activation buffer (BF16), per batch of B samples, row-major B x features:
//   X0 (16) | Z1 (256) | H1 (256) | Z2 (256) | H2 (256) | dZ2 (256) | dZ1 (256)
//   | dY (2016)
#include "jx_common.hpp"
#include "jx_mlp.hpp"

namespace jx {

namespace {

typedef short s4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

constexpr float C_GELU = 0.7978845608028654f;  // sqrt(2 / pi)
__device__ __forceinline__ float gelu(float z) {
    return 0.5f * z * (1.0f + tanhf(C_GELU * (z + 0.044715f * z * z * z)));
}
__device__ __forceinline__ float gelu_grad(float z) {
    const float t = tanhf(C_GELU * (z + 0.044715f * z * z * z));
    return 0.5f * (1.0f + t) + 0.5f * z * (1.0f - t * t) * C_GELU * (1.0f + 3.0f * 0.044715f * z * z);
}

enum Epi { EPI_HIDDEN = 0, EPI_OUT = 1, EPI_DGELU = 2, EPI_STORE = 3 };

struct GemmArgs {
    int M, N, K;
    const uint16_t *A;  // op(A) = TA ? A^T : A, leading dimension lda
    int lda;
    const uint16_t *B;  // op(B) = TB ? B^T : B, leading dimension ldb
    int ldb;
    const float *bias;  // EPI_HIDDEN / EPI_OUT: per column
    uint16_t *Zout;     // EPI_HIDDEN: pre-activation (BF16); EPI_DGELU: dZ (BF16)
    uint16_t *Hout;     // EPI_HIDDEN: activation (BF16)
    const uint16_t *Zin;  // EPI_DGELU: saved pre-activation
    float *Fout;        // EPI_OUT / EPI_STORE: FP32 result
    int ldc;
};

// C = op(A) op(B) (+ epilogue), 64 x 64 tile per 256-thread workgroup, each
// wave a 32 x 32 quarter (2 x 2 MFMA tiles), K staged through LDS in chunks of
// 16 (one MFMA step).  Out-of-range rows, columns and k read as zero.
template <bool TA, bool TB, int EPI>
__global__ void __launch_bounds__(256) k_gemm_bf16(GemmArgs g) {
    constexpr int LDA_S = 16 + 4, LDB_S = 64 + 4;
    __shared__ uint16_t As[64 * LDA_S];  // As[m][k]
    __shared__ uint16_t Bs[16 * LDB_S];  // Bs[k][n]
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int x = lane & 15, q = lane >> 4;
    const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
    const int wm = (wv & 1) * 32, wn = (wv >> 1) * 32;
    f4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < g.K; k0 += 16) {
        // stage op(A)(m0..m0+63, k0..k0+15) and op(B)(k0..k0+15, n0..n0+63)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = tid + 256 * r;
            int m, k;
            if (TA) { m = e % 64; k = e / 64; }   // consecutive threads along m = contiguous in A^T
            else { k = e % 16; m = e / 16; }
            const int gm = m0 + m, gk = k0 + k;
            uint16_t v = 0;
            if (gm < g.M && gk < g.K) v = TA ? g.A[(size_t)gk * g.lda + gm] : g.A[(size_t)gm * g.lda + gk];
            As[m * LDA_S + k] = v;
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int e = tid + 256 * r;
            int n, k;
            if (TB) { k = e % 16; n = e / 16; }
            else { n = e % 64; k = e / 64; }
            const int gn = n0 + n, gk = k0 + k;
            uint16_t v = 0;
            if (gn < g.N && gk < g.K) v = TB ? g.B[(size_t)gn * g.ldb + gk] : g.B[(size_t)gk * g.ldb + gn];
            Bs[k * LDB_S + n] = v;
        }
        __syncthreads();
        // lane (q, x): A rows x of the 16-row tile with k = 4q .. 4q+3, B the
        // same k for column x
        s4 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int t = 0; t < 4; ++t) a[i][t] = (short)As[(wm + 16 * i + x) * LDA_S + 4 * q + t];
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int t = 0; t < 4; ++t) b[j][t] = (short)Bs[(4 * q + t) * LDB_S + wn + 16 * j + x];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
    // component v of lane (q, x) holds C(4 q + v, x) of the 16 x 16 tile
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int m = m0 + wm + 16 * i + 4 * q + v, n = n0 + wn + 16 * j + x;
                if (m >= g.M || n >= g.N) continue;
                const float c = acc[i][j][v];
                const size_t e = (size_t)m * g.ldc + n;
                if (EPI == EPI_HIDDEN) {
                    const float z = c + g.bias[n];
                    g.Zout[e] = to_bf16(z);
                    g.Hout[e] = to_bf16(gelu(z));
                } else if (EPI == EPI_OUT) {
                    g.Fout[e] = c + g.bias[n];
                } else if (EPI == EPI_DGELU) {
                    g.Zout[e] = to_bf16(c * gelu_grad(from_bf16(g.Zin[e])));
                } else {
                    g.Fout[e] = c;
                }
            }
}

template <bool TA, bool TB, int EPI>
void gemm(const GemmArgs &a, hipStream_t s) {
    if (a.M <= 0 || a.N <= 0) return;
    dim3 grid((a.N + 63) / 64, (a.M + 63) / 64);
    hipLaunchKernelGGL((k_gemm_bf16<TA, TB, EPI>), grid, dim3(256), 0, s, a);
    JX_LAUNCHED();
}

// X0 (B x 16 BF16) from theta (B x 8 FP32), features 8..15 zero.
__global__ void k_pack_input(int B, const float *theta, uint16_t *X0) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= B * 16) return;
    const int r = e / 16, c = e % 16;
    X0[e] = c < 8 ? to_bf16(theta[(size_t)r * 8 + c]) : (uint16_t)0;
}

__global__ void k_to_bf16(size_t count, const float *src, uint16_t *dst) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) dst[e] = to_bf16(src[e]);
}

// out[n] = sum over rows r of X[r][n] (BF16), FP32 in row order.
__global__ void k_colsum(int rows, int cols, const uint16_t *X, float *out) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= cols) return;
    float s = 0.f;
    for (int r = 0; r < rows; ++r) s += from_bf16(X[(size_t)r * cols + n]);
    out[n] = s;
}

// grad = 2 (Y - T) / count; loss[0] = mean((Y - T)^2) in FP64 (fixed order).
__global__ void __launch_bounds__(1024) k_mse(size_t count, const float *Y, const float *T, float *grad, double *loss) {
    __shared__ double red[16];
    double s = 0.0;
    const float sc = 2.0f / (float)count;
    for (size_t e = threadIdx.x; e < count; e += 1024) {
        const float d = Y[e] - T[e];
        if (grad) grad[e] = sc * d;
        s += (double)d * d;
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < 16; ++i) t += red[i];
        loss[0] = t / (double)count;
    }
}

__global__ void k_adam(int count, float *p, uint16_t *pb, const float *g, float *m, float *v, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= count) return;
    const float gi = g[e];
    const float mi = b1 * m[e] + (1.0f - b1) * gi;
    const float vi = b2 * v[e] + (1.0f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    const float pi = p[e] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[e] = pi;
    pb[e] = to_bf16(pi);
}

// S (column-major n x n, batch of them) = skew matrix with strictly upper
// entries c * std + mean (row-major order of (i, j), i < j).
__global__ void k_skew(int batch, int n, const float *coords, const float *mean, const float *stdv, double *S) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t per = (size_t)n * n;
    if (e >= per * batch) return;
    const int b = (int)(e / per), r = (int)(e % per);
    const int i = r % n, j = r / n;  // column-major element (i, j)
    double v = 0.0;
    if (i != j) {
        const int lo = min(i, j), hi = max(i, j);
        const int idx = lo * n - lo * (lo + 1) / 2 + (hi - lo - 1);
        const int nc = n * (n - 1) / 2;
        const float c = coords[(size_t)b * nc + idx] * (stdv ? stdv[idx] : 1.0f) + (mean ? mean[idx] : 0.0f);
        v = i < j ? (double)c : -(double)c;
    }
    S[e] = v;
}

// The same, one workgroup per matrix for n(n-1)/2 <= MAXNC: the matrix's
// coordinates are read once, coalesced, into LDS, and S is written column by
// column (the lower triangle's gather would otherwise stride by about n).
template <int MAXNC>
__global__ void __launch_bounds__(256) k_skew_blk(int n, const float *coords, const float *mean, const float *stdv,
                                                  double *S) {
    __shared__ float cs[MAXNC];
    const int nc = n * (n - 1) / 2, b = blockIdx.x;
    const float *cb = coords + (size_t)b * nc;
    for (int k = threadIdx.x; k < nc; k += 256) cs[k] = cb[k] * (stdv ? stdv[k] : 1.0f) + (mean ? mean[k] : 0.0f);
    __syncthreads();
    double *Sb = S + (size_t)b * n * n;
    for (int e = threadIdx.x; e < n * n; e += 256) {
        const int i = e % n, j = e / n;  // column-major element (i, j)
        double v = 0.0;
        if (i != j) {
            const int lo = min(i, j), hi = max(i, j);
            const float c = cs[lo * n - lo * (lo + 1) / 2 + (hi - lo - 1)];
            v = i < j ? (double)c : -(double)c;
        }
        Sb[e] = v;
    }
}

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

void mlp_forward(int B, const float *theta, const uint16_t *Wb, const float *bias, float *out, uint16_t *acts,
                 hipStream_t s) {
    using namespace mlp;
    uint16_t *X0 = acts + act_off(B, ACT_X0), *Z1 = acts + act_off(B, ACT_Z1), *H1 = acts + act_off(B, ACT_H1),
             *Z2 = acts + act_off(B, ACT_Z2), *H2 = acts + act_off(B, ACT_H2);
    hipLaunchKernelGGL(k_pack_input, dim3((B * 16 + 255) / 256), dim3(256), 0, s, B, theta, X0);
    JX_LAUNCHED();
    GemmArgs a{};
    a.M = B; a.N = H; a.K = K1; a.A = X0; a.lda = K1; a.B = Wb + OFF_W1; a.ldb = H;
    a.bias = bias + (OFF_B1 - OFF_B1); a.Zout = Z1; a.Hout = H1; a.ldc = H;
    gemm<false, false, EPI_HIDDEN>(a, s);
    a = GemmArgs{};
    a.M = B; a.N = H; a.K = H; a.A = H1; a.lda = H; a.B = Wb + OFF_W2; a.ldb = H;
    a.bias = bias + (OFF_B2 - OFF_B1); a.Zout = Z2; a.Hout = H2; a.ldc = H;
    gemm<false, false, EPI_HIDDEN>(a, s);
    a = GemmArgs{};
    a.M = B; a.N = NOUT; a.K = H; a.A = H2; a.lda = H; a.B = Wb + OFF_W3; a.ldb = NOUT;
    a.bias = bias + (OFF_B3 - OFF_B1); a.Fout = out; a.ldc = NOUT;
    gemm<false, false, EPI_OUT>(a, s);
}

void mlp_backward(int B, const uint16_t *acts_c, const float *dY, const uint16_t *Wb, float *gW, float *gB,
                  hipStream_t s) {
    using namespace mlp;
    uint16_t *acts = const_cast<uint16_t *>(acts_c);
    const uint16_t *X0 = acts + act_off(B, ACT_X0), *Z1 = acts + act_off(B, ACT_Z1), *H1 = acts + act_off(B, ACT_H1),
                   *Z2 = acts + act_off(B, ACT_Z2), *H2 = acts + act_off(B, ACT_H2);
    uint16_t *dZ2 = acts + act_off(B, ACT_DZ2), *dZ1 = acts + act_off(B, ACT_DZ1), *dYb = acts + act_off(B, ACT_DY);
    const size_t ny = (size_t)B * NOUT;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((ny + 255) / 256)), dim3(256), 0, s, ny, dY, dYb);
    JX_LAUNCHED();
    // layer 3: dW3 = H2^T dY, db3 = colsum dY, dZ2 = (dY W3^T) * gelu'(Z2)
    GemmArgs a{};
    a.M = H; a.N = NOUT; a.K = B; a.A = H2; a.lda = H; a.B = dYb; a.ldb = NOUT; a.Fout = gW + OFF_W3; a.ldc = NOUT;
    gemm<true, false, EPI_STORE>(a, s);
    hipLaunchKernelGGL(k_colsum, dim3((NOUT + 255) / 256), dim3(256), 0, s, B, NOUT, dYb, gB + (OFF_B3 - OFF_B1));
    JX_LAUNCHED();
    a = GemmArgs{};
    a.M = B; a.N = H; a.K = NOUT; a.A = dYb; a.lda = NOUT; a.B = Wb + OFF_W3; a.ldb = NOUT;
    a.Zin = Z2; a.Zout = dZ2; a.ldc = H;
    gemm<false, true, EPI_DGELU>(a, s);
    // layer 2
    a = GemmArgs{};
    a.M = H; a.N = H; a.K = B; a.A = H1; a.lda = H; a.B = dZ2; a.ldb = H; a.Fout = gW + OFF_W2; a.ldc = H;
    gemm<true, false, EPI_STORE>(a, s);
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, s, B, H, dZ2, gB + (OFF_B2 - OFF_B1));
    JX_LAUNCHED();
    a = GemmArgs{};
    a.M = B; a.N = H; a.K = H; a.A = dZ2; a.lda = H; a.B = Wb + OFF_W2; a.ldb = H; a.Zin = Z1; a.Zout = dZ1; a.ldc = H;
    gemm<false, true, EPI_DGELU>(a, s);
    // layer 1
    a = GemmArgs{};
    a.M = K1; a.N = H; a.K = B; a.A = X0; a.lda = K1; a.B = dZ1; a.ldb = H; a.Fout = gW + OFF_W1; a.ldc = H;
    gemm<true, false, EPI_STORE>(a, s);
    hipLaunchKernelGGL(k_colsum, dim3(1), dim3(256), 0, s, B, H, dZ1, gB);
    JX_LAUNCHED();
}

void mlp_mse(size_t count, const float *Y, const float *T, float *grad, double *loss, hipStream_t s) {
    hipLaunchKernelGGL(k_mse, dim3(1), dim3(1024), 0, s, count, Y, T, grad, loss);
    JX_LAUNCHED();
}

void mlp_adam(int count, float *p, uint16_t *pb, const float *g, float *m, float *v, float lr, float b1, float b2,
              float eps, float c1, float c2, hipStream_t s) {
    hipLaunchKernelGGL(k_adam, dim3((count + 255) / 256), dim3(256), 0, s, count, p, pb, g, m, v, lr, b1, b2, eps, c1,
                       c2);
    JX_LAUNCHED();
}

void mlp_to_bf16(size_t count, const float *src, uint16_t *dst, hipStream_t s) {
    if (count == 0) return;
    hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, count, src, dst);
    JX_LAUNCHED();
}

void skew_from_coords(int batch, int n, const float *coords, const float *mean, const float *stdv, double *S,
                      hipStream_t s) {
    const size_t total = (size_t)batch * n * n;
    if (total == 0) return;
    constexpr int MAXNC = 128 * 127 / 2;
    if (n * (n - 1) / 2 <= MAXNC) {
        hipLaunchKernelGGL(k_skew_blk<MAXNC>, dim3(batch), dim3(256), 0, s, n, coords, mean, stdv, S);
        JX_LAUNCHED();
        return;
    }
    hipLaunchKernelGGL(k_skew, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, batch, n, coords, mean, stdv, S);
    JX_LAUNCHED();
}

}  // namespace jx
