// jx_common.hpp -- shared definitions of the gfx950 kernels and their host
// drivers (libjacobi.so).  Nothing here is exported; the public surface is
// include/jacobi.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/jacobi.h"

namespace jx {

// ---------------------------------------------------------------------------
// Errors
// ---------------------------------------------------------------------------
void set_error(const std::string &msg);
const char *last_error();

struct HipFail {
    hipError_t err;
};

#define JX_HIP(call)                                                                      \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess) {                                                           \
            ::jx::set_error(std::string(#call) + ": " + hipGetErrorString(e_) + " at " +  \
                            __FILE__ + ":" + std::to_string(__LINE__));                   \
            throw ::jx::HipFail{e_};                                                      \
        }                                                                                 \
    } while (0)

#define JX_LAUNCHED() JX_HIP(hipGetLastError())

// ---------------------------------------------------------------------------
// MFMA operand vectors
// ---------------------------------------------------------------------------
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

// v_mfma_f64_16x16x4_f64 (lane layout measured on gfx950): lane l = 16 g + x
// (g = l / 16, x = l % 16) supplies A(x, g) and B(g, x); component v of the
// lane's d4 result holds D(g + 4 v, x) -- rows interleaved by 4.
// v_mfma_f32_16x16x4_f32: same operands; component v holds D(4 g + v, x).
// The contraction index g may be mapped to any column of A / row of B as long
// as both operands use the same map.  With the f64 layout, component s of the
// result tile of rows 16 a .. 16 a + 15 is exactly the B operand of the k-step
// k = 16 a + 4 s + g, so a product can feed the next one from registers.
__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// ---------------------------------------------------------------------------
// Rotation storage ("V_hat") in the MFMA-operand order.
//
// V_hat of order m2 (multiple of 16) is consumed as an MFMA operand with the
// contraction index k = k0 + g (k0 a multiple of 4, g the lane group) and the
// free index i.  vperm(k, i) places the 64 values of one MFMA step (4 lane
// groups x 16 consecutive i) in 64 consecutive doubles.
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ int vperm(int k, int i, int m2) {
    return (((k >> 2) * (m2 >> 4) + (i >> 4)) << 6) + ((k & 3) << 4) + (i & 15);
}

// FP32 counterpart for v_mfma_f32_16x16x4_f32, whose result rows are 4 g + v:
// the contraction index of a step is k = 16 A + 4 g + s (A: 16-block, g: lane
// group, s: step 0..3), and the 64 values of step (A, s) are contiguous.
__host__ __device__ __forceinline__ int vperm32(int k, int i, int m2) {
    return ((((k >> 4) << 2) + (k & 3)) * (m2 >> 4) + (i >> 4)) * 64 + ((k >> 2) & 3) * 16 + (i & 15);
}

// Per-type MFMA conventions of the rotation-apply kernels.
template <class T>
struct MfmaTraits;
template <>
struct MfmaTraits<double> {
    typedef d4 acc_t;
    static __device__ __forceinline__ d4 mma(double a, double b, d4 c) { return mfma_f64(a, b, c); }
    // contraction index of step st (0..3 within a 16-block) for lane group g
    static __host__ __device__ __forceinline__ int kstep(int st, int g) { return 4 * st + g; }
    // result row of component v in lane group g (within a 16-row tile)
    static __host__ __device__ __forceinline__ int rrow(int g, int v) { return g + 4 * v; }
    static __host__ __device__ __forceinline__ int vidx(int k, int i, int m2) { return vperm(k, i, m2); }
};
template <>
struct MfmaTraits<float> {
    typedef f4 acc_t;
    static __device__ __forceinline__ f4 mma(float a, float b, f4 c) { return mfma_f32(a, b, c); }
    static __host__ __device__ __forceinline__ int kstep(int st, int g) { return 4 * g + st; }
    static __host__ __device__ __forceinline__ int rrow(int g, int v) { return 4 * g + v; }
    static __host__ __device__ __forceinline__ int vidx(int k, int i, int m2) { return vperm32(k, i, m2); }
};

// Upper block-triangle storage of the symmetric iterate: block (I, J), I <= J,
// of order b, column-major, at block slot J (J + 1) / 2 + I.
__host__ __device__ __forceinline__ size_t ublk(int I, int J) {
    return (size_t)J * (J + 1) / 2 + I;
}

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files)
// ---------------------------------------------------------------------------

// Where the subproblem solver reads A_hat and writes its results.
enum SubMode {
    SUB_EIG = 0,     // A_hat from the upper block storage, D_hat written back there
    SUB_PLAIN = 1,   // A_hat contiguous (count x m2 x m2), V and D col-major out
    SUB_GRAM = 2     // A_hat contiguous (Gram blocks), only V_hat (vperm) out
};

struct SubArgs {
    int mode;
    int m2;                 // 2b
    int count;              // subproblems (pairs) in this launch
    const int *pairs;       // device, 2 ints per pair (SUB_EIG)
    double *ablk;           // SUB_EIG: upper block storage of A (b = m2 / 2)
    const double *ahat;     // SUB_PLAIN / SUB_GRAM input
    double *vout;           // V_hat per pair: vperm (SUB_EIG/GRAM) or col-major (PLAIN)
    double *dout;           // SUB_PLAIN: D_hat col-major
    int *flags;             // per pair: 1 = skipped (V_hat = I), may be NULL
    double skip_thr;        // skip a pair whose off(A_hat) <= skip_thr (SUB_EIG/GRAM)
    int inner_sweeps;       // 0 = to inner convergence (cap 30)
    double *inner_off;      // optional per-pair |off(A_hat)| before the solve
    const int *force_skip;  // optional per pair: 1 = placeholder pair, never rotated
    int *rot_count;         // optional: +1 per pair that is rotated (not skipped)
    float *ablk32;          // SUB_EIG with FP32 storage of A (instead of ablk)
    float *vout32;          // V_hat written in FP32, vperm32 order (instead of vout)
    int spin_limit;         // bound of the in-kernel hand-off waits (0: the default)
};
// Raises kernel `func`'s dynamic LDS limit to `bytes` on the current device,
// once per (device, kernel); thread-safe (host code, ctx.cpp).
void ensure_lds_limit(const void *func, int bytes);

void launch_subproblem(const SubArgs &a, hipStream_t s);

// Pivoting step (k_pivot.hip): per pair, LU with partial pivoting on the
// leading m2/2 rows of V_hat gives P; V_hat <- V_hat P, D_hat <- P^T D_hat P.
// Solver storage (ablk != nullptr: V in vperm order, D_hat in the pair's
// blocks of the upper block storage, pairs I < J) or plain column-major
// (V and, if non-null, D per pair).  m2 = 64 or 128.
struct PivotArgs {
    int count;          // pairs
    int m2;
    const int *pairs;   // solver storage: 2 ints per pair
    double *ablk;       // solver storage: upper block storage of A (else nullptr)
    double *V;          // per pair m2 x m2
    double *D;          // plain storage: per pair m2 x m2 symmetric (may be nullptr)
    const int *flags;   // optional: 1 = skipped pair (left alone)
    int *perm_out;      // optional: per pair m2 ints, column j of V P = column perm[j] of V
};
void launch_pivot(const PivotArgs &a, hipStream_t s);
void launch_colmajor_from_vperm(int count, int m2, const double *src, double *dst, hipStream_t s);

// Batched solver (k_batched.hip): one persistent launch per size class.  A
// class holds the matrices whose order pads to M2 = 2 * bs * npp (npp pair
// problems of order 2 bs per middle round); every matrix has its own padded
// M2 x M2 column-major workspace (A and Q in the phase's type, two FP64
// temporaries for the refinement GEMMs).
struct BatchArgs {
    int count;               // matrices of this class
    int m2;                  // padded order
    const int *ids;          // class-local order (LPT: n descending) -> matrix id
    const int *n;            // per matrix id: order
    const int64_t *offA;     // per matrix id: element offset in A_in / Q_out (ld = n)
    const int64_t *offW;     // per matrix id: offset in W_out
    const int64_t *offWs;    // per matrix id: element offset of its M2 x M2 workspace slots
    int dtype;               // JACOBI_F32 / JACOBI_F64 (A_in)
    const void *A_in;
    const double *Q0;        // optional warm starts (layout of Q_out)
    float *A32, *Q32;        // FP32 phase
    double *A64, *Q64, *T64, *U64;  // FP64 phase
    double *W_out, *Q_out;
    int *queue;              // [0]: next class-local slot (zeroed before the launch)
    int *stat;               // per matrix id: sweeps32, sweeps64, status, fallback
    double *offrel;          // per matrix id: final off(A) / ||A||_F
    double tol;              // FP64 stop: off(A) <= tol ||A||_F
    int max_sweeps;          // FP64 sweeps
    int lp_max_sweeps;       // FP32 sweeps (0: no FP32 phase)
    double lp_switch;        // FP32 phase ends at off(A) <= lp_switch ||A||_F
    int want_vectors, sort;
};
void launch_batched_lp(const BatchArgs &a, int bs, int grid, hipStream_t s);
void launch_batched_hp(const BatchArgs &a, int bs, int grid, hipStream_t s);
void launch_fill_int(int *p, int count, int value, hipStream_t s);
int batched_threads(int bs, int m2);      // threads of the class kernel
int batched_blocks_per_cu(int bs, int m2, bool lp);  // resident workgroups per CU
size_t batched_lds_bytes(int bs, int m2); // dynamic LDS of the class kernel

// Fused two-sided update of the off-diagonal pair tiles of one round:
// A[p,q] <- V_p^T A[p,q] V_q for p < q (pair indices of the round).
// reserve > 0: on at most (CUs - reserve) CUs.  UA_QUAD: only the blocks
// qmask[i] of tile i (bit 2 h + c: row block h of pair p, column block c of
// pair q), read from copies of their originals at side + (4 i + 2 h + c) b^2
// (made beforehand, e.g. by launch_copy_blocks) and written in place.  A
// bounded launch with nq > 0 then does the rest of its first nq tiles (same
// qmask and side) and the other tiles whole.  snext / smap (bounded launch):
// quadrant quad of tile i, once written, is also copied to snext + slot b^2,
// slot = smap[4 i + quad] (negative: none).
constexpr int UA_QUAD = -2;
void launch_update_a(int b, int npairs, const int *pairs, double *ablk, const double *vhat,
                     const int *flags, const int *tiles, int ntiles, hipStream_t s, int reserve = 0,
                     const int *qmask = nullptr, int nq = 0, void *side = nullptr, void *snext = nullptr,
                     const int *smap = nullptr);
// Block copies: block lst[2 j] (slot of the upper block storage) of ablk to
// side + lst[2 j + 1] b^2, j < n.
void launch_copy_blocks(int b, const double *ablk, const int *lst, int n, void *side, hipStream_t s);
void launch_copy_blocks32(int b, const float *ablk, const int *lst, int n, void *side, hipStream_t s);
// Gram blocks of the one-sided SVD: ahat[p] = G(:, [I,J])^T G(:, [I,J]) over the
// first m_rows rows (nchunks equal row chunks, partial sums added in order).
void launch_gram(int b, int npairs, const int *pairs, const double *G, int ldg, int m_rows, int nchunks,
                 double *partial, double *ahat, hipStream_t s);
void launch_gram32(int b, int npairs, const int *pairs, const float *G, int ldg, int m_rows, int nchunks,
                   float *partial, double *ahat, hipStream_t s);
void launch_col_norms(int m, int n, const double *G, int ldg, double *sigma, hipStream_t s);
void launch_col_norms32(int m, int n, const float *G, int ldg, double *sigma, hipStream_t s);
void launch_scale_scatter(int m, int n, const double *G, int ldg, const double *sigma, const int *rank,
                          double *U, int ldu, hipStream_t s);

// One-sided update Q(:, [I,J]) <- Q(:, [I,J]) V_p for every pair p and every
// 128-row chunk of Q (n_rows multiple of 128).  reserve > 0: run on at most
// (CUs - reserve) CUs, leaving `reserve` CUs free for a kernel running beside it.
void launch_update_q(int b, int npairs, const int *pairs, double *Q, int ldq, int n_rows,
                     const double *vhat, const int *flags, hipStream_t s, int reserve = 0);
// The rest-of-tile update (as a bounded launch_update_a with nq critical
// tiles) and the Q update (Q may be NULL) of one round in one persistent
// launch on at most (CUs - reserve) CUs; b = 64 only.
void launch_update_aq(int b, int npairs, const int *pairs, double *ablk, const double *vhat, const int *flags,
                      const int *tiles, int ntiles, const int *qmask, int nq, void *side, void *snext,
                      const int *smap, double *Q, int ldq, int n_rows, int reserve, hipStream_t s);
void launch_update_aq32(int b, int npairs, const int *pairs, float *ablk, const float *vhat, const int *flags,
                        const int *tiles, int ntiles, const int *qmask, int nq, void *side, void *snext,
                        const int *smap, float *Q, int ldq, int n_rows, int reserve, hipStream_t s);
// FP32 versions (FP32 storage, FP32 MFMA with FP32 accumulation, V_hat in vperm32 order).
void launch_update_a32(int b, int npairs, const int *pairs, float *ablk, const float *vhat, const int *flags,
                       const int *tiles, int ntiles, hipStream_t s, int reserve = 0, const int *qmask = nullptr,
                       int nq = 0, void *side = nullptr, void *snext = nullptr, const int *smap = nullptr);
void launch_update_q32(int b, int npairs, const int *pairs, float *Q, int ldq, int n_rows, const float *vhat,
                       const int *flags, hipStream_t s, int reserve = 0);

// Layout conversion and reductions.
void launch_pack_sym(int n, int npad, int b, const double *A, int lda, char uplo, double *ablk,
                     hipStream_t s);
void launch_unpack_sym(int npad, int b, const double *ablk, double *A, int lda, hipStream_t s);
void launch_full_from_triangle(int n, int npad, const double *A, int lda, char uplo, double *F,
                               hipStream_t s);
// partial[blk] = {off-diagonal sum of squares counted for both triangles,
// sum of squares of the diagonal}; then reduce to out[0..1] in a fixed order.
void launch_block_norms(int npad, int b, const double *ablk, double *partial, double *out,
                        hipStream_t s);
void launch_set_identity(int n, int npad, double *Q, int ldq, hipStream_t s);
void launch_copy_pad(int n, int npad, const double *src, int lds_, double *dst, int ldd,
                     hipStream_t s);
void launch_extract_diag(int npad, int b, const double *ablk, double *w, hipStream_t s);
// Stable rank sort of w[0..n) (ascending if dir > 0, descending otherwise):
// rank[i] = number of j with w_j before w_i.
void launch_rank(int n, const double *w, int dir, int *rank, hipStream_t s);
void launch_scatter_values(int n, const double *w, const int *rank, double *out, hipStream_t s);
// out(:, rank[i]) = src(:, i) for the first `rows` rows of n columns.
void launch_scatter_columns(int rows, int n, const double *src, int lds_, const int *rank,
                            double *out, int ldo, hipStream_t s);

// Scalar round-robin Jacobi (b = 1) in one persistent workgroup (k_scalar.hip):
// A (n x n full, ld n) and Q (may be NULL) in place, ne = n rounded up to even
// (index n a placeholder), pairs: (ne - 1) rounds of ne / 2.  relative: rotate
// only when |a_pq| > tol sqrt(|a_pp a_qq|), stop after a sweep without
// rotations.  out[0] = sweeps, out[1] = Xi(A), out[2] = ||A||_F, out[3] =
// rotations of the last sweep.
void launch_scalar_rr(int n, int ne, const int *pairs, double *A, double *Q, double tol, int max_sweeps, int relative,
                      double *out, hipStream_t s);
void launch_sym_full(int n, const double *src, int lds_, char uplo, double *dst, hipStream_t s);
// one round of scalar Jacobi over n/2 workgroups (reads Acur, writes Anext,
// updates Q's columns in place); rot (optional) += rotations of the round;
// absolute mode rotates pairs with |a_pq| > skip, relative mode pairs with
// |a_pq| > tol sqrt(|a_pp a_qq|)
void launch_scalar_round(int n, int ne, const int *pairs_round, const double *Acur, double *Anext, double *Q,
                         double tol, int relative, double skip, int *rot, hipStream_t s);
// out[0] = Xi(A)^2, out[1] = ||A||_F^2 (full n x n A, fixed order)
void launch_scalar_norms(int n, const double *A, double *out, hipStream_t s);

// Re-sorting between sweeps: inv from the ranks of the diagonal (identity on
// the padding), then dst(i', j') = src(inv[i'], inv[j']) (upper block storage)
// and dst(:, j') = src(:, inv[j']).
void launch_inverse_perm(int n, int npad, const int *rank, int *inv, hipStream_t s);
void launch_permute_sym(int npad, int b, const int *inv, const double *src, double *dst, hipStream_t s);
void launch_permute_sym32(int npad, int b, const int *inv, const float *src, float *dst, hipStream_t s);
void launch_permute_cols(int rows, int cols, const int *inv, const double *src, int lds_, double *dst, int ldd,
                         hipStream_t s);
void launch_permute_cols32(int rows, int cols, const int *inv, const float *src, int lds_, float *dst, int ldd,
                           hipStream_t s);
void launch_extract_diag32(int npad, int b, const float *ablk, double *w, hipStream_t s);

// Precision ladder helpers.
void launch_cast_to_f32(size_t count, const double *src, float *dst, hipStream_t s);
void launch_cast_to_f64(size_t count, const float *src, double *dst, hipStream_t s);
void launch_set_identity32(int npad, float *Q, int ldq, hipStream_t s);
void launch_block_norms32(int npad, int b, const float *ablk, double *partial, double *out, hipStream_t s);

// Test helpers: column-major V_hat -> vperm order; D_hat -> pair blocks.
void launch_vperm_from_colmajor(int count, int m2, const double *src, double *dst, hipStream_t s);
void launch_vperm32_from_colmajor(int count, int m2, const double *src, float *dst, hipStream_t s);
void launch_write_pair_blocks(int count, int b, const int *pairs, const double *D, double *ablk,
                              hipStream_t s);

// Reduced QR of the one-sided SVD's preprocessing (k_qr.hip).  Diagonal block
// k0 .. k0+127 of the SPD matrix W: Cholesky W_kk = R_kk^T R_kk in place (upper
// triangle, zero below) and R_kk^{-1} (128 x 128) to Rinv; a pivot that is not
// positive and finite sets *flag = 1.
void launch_chol_diag(double *W, int ldw, int k0, double *Rinv, int *flag, hipStream_t s);
void launch_unit_pad_diag(int n, int npad, double *W, int ldw, hipStream_t s);
void launch_shift_diag(int n, double shift, double *W, int ldw, hipStream_t s);
void launch_zero_lower(int npad, double *W, int ldw, hipStream_t s);
void launch_diag_of(int n, const double *X, int ldx, double *out, hipStream_t s);
// out[0] = number of non-finite entries of X (m x n, ldx); partial: n doubles
void launch_count_nonfinite(int m, int n, const double *X, int ldx, double *partial, double *out, hipStream_t s);
// X (npad x cols, ld npad): fixed pseudo-random values in [-1, 1) on the first n rows, zero below
void launch_fill_probe(int n, int npad, int cols, double *X, hipStream_t s);
// out[0] = ||Y - Z||_F^2 over m rows and `cols` columns (ld); partial: cols doubles
void launch_diff_frob2(int m, int cols, const double *Y, const double *Z, int ld, double *partial, double *out,
                       hipStream_t s);
// out[0] = ||X(0:m, 0:n)||_F^2; partial: n doubles
void launch_frob2(int m, int n, const double *X, int ldx, double *partial, double *out, hipStream_t s);
// out[0] = ||X(0:n, 0:n) - I||_F^2; partial: n doubles
void launch_dev_identity(int n, const double *X, int ldx, double *partial, double *out, hipStream_t s);
// copy of the leading m x n part (destination padded with zeros to mpad x npad)
void launch_copy_rect(int m, int n, const double *src, int lds_, double *dst, int ldd, int mpad, int npad,
                      hipStream_t s);

// General FP64 GEMM on column-major operands: C = alpha op(A) op(B) + beta C,
// M x N result, K contraction, every dimension a multiple of 128 (16 for K).
void launch_gemm_f64(char ta, char tb, int M, int N, int K, double alpha, const double *A, int lda,
                     const double *B, int ldb, double beta, double *C, int ldc, hipStream_t s);

}  // namespace jx
