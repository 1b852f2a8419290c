// k_canon.hip -- training data of the learned warm start (an addition to the
// method; the paper has no learned part):
//   * the family A(theta) = A0 + sum_k theta_k B_k, batched;
//   * the canonical skew generator of each solved matrix: W = Qref^T Q with
//     its columns matched to Qref's by overlap (greedy, largest remaining
//     |W_ij| first), column signs with diag(W) >= 0, the column of smallest
//     |W_jj| negated when det W < 0, then S = (W - I)(W + I)^{-1} made
//     exactly skew; its strictly upper entries (row-major) are the target;
//   * column statistics of the kept targets and their standardised copy.
// One workgroup per matrix for the generator (order <= 64, FP64 in LDS).
#include "jx_common.hpp"

namespace jx {

namespace {

constexpr int CN = 64, CNT = 256;

// A[c] = A0 + sum_k theta[c][k] B[k], every matrix n x n (any storage order,
// the same for all).
__global__ void k_family(int count, int nn, int k, const double *__restrict__ theta,
                         const double *__restrict__ A0, const double *__restrict__ B, double *__restrict__ A) {
    const size_t total = (size_t)count * nn;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const size_t c = e / nn, i = e % nn;
        double v = A0[i];
        for (int t = 0; t < k; ++t) v += theta[c * k + t] * B[(size_t)t * nn + i];
        A[e] = v;
    }
}

// (value, flat index) max with ties to the lower index, across a wave.
__device__ __forceinline__ void wave_argmax(double &v, int &f) {
    for (int o = 32; o > 0; o >>= 1) {
        const double v2 = __shfl_xor(v, o, 64);
        const int f2 = __shfl_xor(f, o, 64);
        if (v2 > v || (v2 == v && f2 < f)) {
            v = v2;
            f = f2;
        }
    }
}

constexpr int WLD = CN + 1;        // stride of W in LDS
constexpr int ALD = 2 * CN + 1;    // stride of the augmented system
constexpr size_t CANON_LDS = sizeof(double) * (CN * WLD + CN * ALD) + sizeof(int) * (4 * CN + 16) +
                             sizeof(double) * 16;

__global__ void __launch_bounds__(CNT) k_canon(int n, const double *__restrict__ Q, const double *__restrict__ Qref,
                                               float *__restrict__ coords, int *__restrict__ keep, double maxabs) {
    extern __shared__ double lds[];
    double *Wm = lds;                    // W(i, j) at Wm[i * WLD + j]
    double *Ag = lds + CN * WLD;         // scratch, then the augmented system (row-major, ALD)
    int *rowfree = reinterpret_cast<int *>(Ag + CN * ALD);
    int *colfree = rowfree + CN, *cmatch = colfree + CN, *perm = cmatch + CN;
    int *ired = perm + CN;               // 16 ints
    double *dred = reinterpret_cast<double *>(ired + 16);  // 16 doubles
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const double *Qb = Q + (size_t)blockIdx.x * n * n;
    // Q (column-major) to Ag[k * WLD + j] = Q(k, j); Qref to Ag + CN * WLD as [k * CN + i] = Qref(k, i)
    double *QS = Ag, *QR = Ag + CN * WLD;
    for (int e = tid; e < CN * CN; e += CNT) {
        const int r = e % CN, c = e / CN;
        QS[r * WLD + c] = (r < n && c < n) ? Qb[(size_t)c * n + r] : 0.0;
        QR[r * CN + c] = (r < n && c < n) ? Qref[(size_t)c * n + r] : 0.0;
    }
    if (tid < CN) {
        rowfree[tid] = tid < n;
        colfree[tid] = tid < n;
        cmatch[tid] = 0;
    }
    __syncthreads();
    // W = Qref^T Q: thread (i = lane, wave wv) computes columns j = wv + 4 r
    {
        double acc[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[r] = 0.0;
        for (int k = 0; k < n; ++k) {
            const double a = QR[k * CN + lane];
#pragma unroll
            for (int r = 0; r < 16; ++r) acc[r] += a * QS[k * WLD + wv + 4 * r];
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) Wm[lane * WLD + wv + 4 * r] = acc[r];
    }
    __syncthreads();
    // greedy matching: n times the largest remaining |W_ij| (ties: lowest i n + j)
    for (int it = 0; it < n; ++it) {
        double bv = -1.0;
        int bf = 0x7fffffff;
        if (lane < n && rowfree[lane]) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int j = wv + 4 * r;
                if (j < n && colfree[j]) {
                    const double v = fabs(Wm[lane * WLD + j]);
                    const int f = lane * n + j;
                    if (v > bv || (v == bv && f < bf)) {
                        bv = v;
                        bf = f;
                    }
                }
            }
        }
        wave_argmax(bv, bf);
        if (lane == 0) {
            dred[wv] = bv;
            ired[wv] = bf;
        }
        __syncthreads();
        if (tid == 0) {
            double v = dred[0];
            int f = ired[0];
            for (int w = 1; w < 4; ++w)
                if (dred[w] > v || (dred[w] == v && ired[w] < f)) {
                    v = dred[w];
                    f = ired[w];
                }
            const int i = f / n, j = f % n;
            rowfree[i] = 0;
            colfree[j] = 0;
            cmatch[i] = j;
        }
        __syncthreads();
    }
    // W' (:, i) = s_i W(:, c_i) with s_i making W'(i, i) >= 0: into Ag as a copy for the determinant
    double *Wp = Ag;  // W'(r, i) at Wp[r * WLD + i]
    for (int e = tid; e < CN * CN; e += CNT) {
        const int r = e / CN, i = e % CN;
        double v = 0.0;
        if (r < n && i < n) {
            const int c = cmatch[i];
            const double d = Wm[i * WLD + c];
            v = (d < 0.0 ? -1.0 : 1.0) * Wm[r * WLD + c];
        }
        Wp[r * WLD + i] = v;
    }
    __syncthreads();
    for (int e = tid; e < CN * CN; e += CNT) Wm[(e / CN) * WLD + e % CN] = Wp[(e / CN) * WLD + e % CN];
    __syncthreads();
    // sign of det W' by LU with partial pivoting on the copy in Wp (rows swapped
    // through perm[]), one wave; negative pivots and swaps counted
    if (wv == 0) {
        int negs = 0, singular = 0;
        if (lane < CN) perm[lane] = lane;
        for (int k = 0; k < n; ++k) {
            // pivot: largest |a_ik| over i >= k (ties: lowest i)
            double bv = -1.0;
            int bf = 0x7fffffff;
            if (lane >= k && lane < n) {
                bv = fabs(Wp[perm[lane] * WLD + k]);
                bf = lane;
            }
            wave_argmax(bv, bf);
            const int p = bf;
            if (lane == 0 && p != k) {
                const int t = perm[k];
                perm[k] = perm[p];
                perm[p] = t;
            }
            negs += (p != k);
            __builtin_amdgcn_wave_barrier();
            const double piv = Wp[perm[k] * WLD + k];
            if (piv == 0.0) {  // det 0: not negative
                singular = 1;
                break;
            }
            negs += piv < 0.0;
            if (lane > k && lane < n) {
                const int ri = perm[lane];
                const double f = Wp[ri * WLD + k] / piv;
                for (int j = k + 1; j < n; ++j) Wp[ri * WLD + j] -= f * Wp[perm[k] * WLD + j];
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (lane == 0) ired[8] = singular ? 0 : (negs & 1);
    }
    __syncthreads();
    if (ired[8]) {  // det < 0: negate the column of smallest |W'_jj| (lowest j on ties)
        if (wv == 0) {
            double bv = -1.0;
            int bf = 0x7fffffff;
            if (lane < n) {
                bv = -fabs(Wm[lane * WLD + lane]);
                bf = lane;
            }
            wave_argmax(bv, bf);
            if (lane < n) Wm[lane * WLD + bf] = -Wm[lane * WLD + bf];
        }
        __syncthreads();
    }
    // S (W' + I) = W' - I, i.e. (W' + I)^T S^T = (W' - I)^T: Gauss-Jordan with
    // partial pivoting on [M | B], M = (W' + I)^T, B = (W' - I)^T; S^T = X
    for (int e = tid; e < CN * CN; e += CNT) {
        const int r = e / CN, c = e % CN;  // M(r, c) = W'(c, r) + delta
        const double w = (r < n && c < n) ? Wm[c * WLD + r] : 0.0, d = (r == c) ? 1.0 : 0.0;
        Ag[r * ALD + c] = w + d;
        Ag[r * ALD + CN + c] = w - d;
    }
    __syncthreads();
    int bad = 0;
    for (int k = 0; k < n; ++k) {
        if (wv == 0) {  // pivot row: largest |M(i, k)|, i >= k
            double bv = -1.0;
            int bf = 0x7fffffff;
            if (lane >= k && lane < n) {
                bv = fabs(Ag[lane * ALD + k]);
                bf = lane;
            }
            wave_argmax(bv, bf);
            if (lane == 0) ired[9] = bf;
        }
        __syncthreads();
        const int p = ired[9];
        if (p != k)  // swap rows k and p (both halves)
            for (int j = tid; j < 2 * CN; j += CNT) {
                const double t = Ag[k * ALD + j];
                Ag[k * ALD + j] = Ag[p * ALD + j];
                Ag[p * ALD + j] = t;
            }
        __syncthreads();
        const double piv = Ag[k * ALD + k];
        if (!(fabs(piv) > 0.0)) {
            bad = 1;
            break;
        }
        // eliminate column k from every other row, then scale row k
        for (int e = tid; e < n * 2 * CN; e += CNT) {
            const int i = e / (2 * CN), j = e % (2 * CN);
            if (i != k && j > k) Ag[i * ALD + j] -= Ag[i * ALD + k] / piv * Ag[k * ALD + j];
        }
        __syncthreads();
        for (int j = tid; j < 2 * CN; j += CNT)
            if (j > k) Ag[k * ALD + j] /= piv;
        if (tid < CN && tid != k) Ag[tid * ALD + k] = 0.0;
        __syncthreads();
        if (tid == 0) Ag[k * ALD + k] = 1.0;
        __syncthreads();
    }
    // S(i, j) = X(j, i); the skew part (S - S^T) / 2; coordinates (i < j, row-major)
    const int nc = n * (n - 1) / 2;
    float *out = coords + (size_t)blockIdx.x * nc;
    double mx = 0.0;
    int fin = 1;
    for (int e = tid; e < nc; e += CNT) {
        // row i of the strictly upper triangle: e = i n - i (i + 1) / 2 + (j - i - 1)
        int i = 0, base = 0;
        while (base + (n - 1 - i) <= e) {
            base += n - 1 - i;
            ++i;
        }
        const int j = i + 1 + (e - base);
        const double sij = Ag[j * ALD + CN + i], sji = Ag[i * ALD + CN + j];
        const double v = 0.5 * (sij - sji);
        if (!(fabs(v) < HUGE_VAL)) fin = 0;
        mx = fmax(mx, fabs(v));
        out[e] = (float)v;
    }
    // block-wide: finite and max |S_ij| <= maxabs, else the sample is dropped
    for (int o = 32; o > 0; o >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, o, 64));
        fin &= __shfl_xor(fin, o, 64);
    }
    if (lane == 0) {
        dred[wv] = mx;
        ired[wv] = fin;
    }
    __syncthreads();
    const bool ok = !bad && ired[0] && ired[1] && ired[2] && ired[3] && fmax(fmax(dred[0], dred[1]), fmax(dred[2], dred[3])) <= maxabs;
    if (!ok)
        for (int e = tid; e < nc; e += CNT) out[e] = 0.0f;
    if (tid == 0) keep[blockIdx.x] = ok ? 1 : 0;
}

// Column sums (FP64) of the kept rows of X (rows x cols FP32, row-major), per
// chunk of `chunk` rows: part[ch][0][c] = sum x, part[ch][1][c] = sum x^2.
__global__ void k_col_partials(int rows, int cols, int chunk, const float *__restrict__ X,
                               const int *__restrict__ keep, double *__restrict__ part) {
    const int ch = blockIdx.y;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    double s = 0.0, s2 = 0.0;
    const int r1 = min(rows, (ch + 1) * chunk);
    for (int r = ch * chunk; r < r1; ++r)
        if (keep[r]) {
            const double v = X[(size_t)r * cols + c];
            s += v;
            s2 += v * v;
        }
    part[((size_t)ch * 2) * cols + c] = s;
    part[((size_t)ch * 2 + 1) * cols + c] = s2;
}

// mean and standard deviation (population, + eps) of each column over the kept
// rows, the chunk partials summed in order.
__global__ void k_col_finish(int cols, int nch, const double *__restrict__ part, int nkeep,
                             float eps, float *__restrict__ mean, float *__restrict__ stdv) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    double s = 0.0, s2 = 0.0;
    for (int ch = 0; ch < nch; ++ch) {
        s += part[((size_t)ch * 2) * cols + c];
        s2 += part[((size_t)ch * 2 + 1) * cols + c];
    }
    const double k = (double)max(nkeep, 1);
    const double mu = s / k;
    const double var = fmax(s2 / k - mu * mu, 0.0);
    mean[c] = (float)mu;
    stdv[c] = (float)(sqrt(var) + (double)eps);
}

// Kept rows gathered in order: Xo[r] = X[idx[r]], To[r] = (T[idx[r]] - mean) / std.
__global__ void k_gather_std(int kept, int xcols, int tcols, const int *__restrict__ idx, const float *__restrict__ X,
                             const float *__restrict__ T, const float *__restrict__ mean,
                             const float *__restrict__ stdv, float *__restrict__ Xo, float *__restrict__ To) {
    const int r = blockIdx.x;
    if (r >= kept) return;
    const size_t src = (size_t)idx[r];
    for (int c = threadIdx.x; c < xcols; c += blockDim.x) Xo[(size_t)r * xcols + c] = X[src * xcols + c];
    for (int c = threadIdx.x; c < tcols; c += blockDim.x)
        To[(size_t)r * tcols + c] = (T[src * tcols + c] - mean[c]) / stdv[c];
}

}  // namespace

void family_matrices(int count, int n, int k, const double *theta, const double *A0, const double *B, double *A,
                     hipStream_t s) {
    const size_t total = (size_t)count * n * n;
    if (total == 0) return;
    const unsigned grid = (unsigned)std::min<size_t>((total + 255) / 256, 65535);
    hipLaunchKernelGGL(k_family, dim3(grid), dim3(256), 0, s, count, n * n, k, theta, A0, B, A);
    JX_LAUNCHED();
}

void canonical_targets(int count, int n, const double *Q, const double *Qref, float *coords, int *keep,
                       double maxabs, hipStream_t s) {
    if (count <= 0) return;
    ensure_lds_limit(reinterpret_cast<const void *>(&k_canon), (int)CANON_LDS);
    hipLaunchKernelGGL(k_canon, dim3(count), dim3(CNT), CANON_LDS, s, n, Q, Qref, coords, keep, maxabs);
    JX_LAUNCHED();
}

void column_stats(int rows, int cols, const float *X, const int *keep, int nkeep, float eps, float *mean,
                  float *stdv, double *part, int chunk, hipStream_t s) {
    const int nch = (rows + chunk - 1) / chunk;
    if (rows <= 0 || cols <= 0) return;
    hipLaunchKernelGGL(k_col_partials, dim3((cols + 255) / 256, nch), dim3(256), 0, s, rows, cols, chunk, X, keep,
                       part);
    JX_LAUNCHED();
    hipLaunchKernelGGL(k_col_finish, dim3((cols + 255) / 256), dim3(256), 0, s, cols, nch, part, nkeep, eps, mean,
                       stdv);
    JX_LAUNCHED();
}

void gather_standardize(int kept, int xcols, int tcols, const int *idx, const float *X, const float *T,
                        const float *mean, const float *stdv, float *Xo, float *To, hipStream_t s) {
    if (kept <= 0) return;
    hipLaunchKernelGGL(k_gather_std, dim3(kept), dim3(256), 0, s, kept, xcols, tcols, idx, X, T, mean, stdv, Xo, To);
    JX_LAUNCHED();
}

}  // namespace jx
