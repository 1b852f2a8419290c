// k_subproblem.hip -- the subproblem solver of block Jacobi on gfx950.
//
// One workgroup diagonalises one 2b x 2b symmetric subproblem
// A_hat = A([I,J],[I,J]) (Alg. 1 and the diagonalisation step of Alg. 2, §3).
// The paper leaves open whether the subproblem is diagonalised exactly or
// approximately (§3, after Alg. 3); `inner_sweeps` caps the inner sweeps
// (0 = until off(A_hat) <= eps ||A_hat||_F, at most 30).
//
// Two solvers:
//   * m2 = 32, 64: round-robin scalar Jacobi on the whole subproblem
//     (scalar_sweeps below, one workgroup);
//   * m2 = 128: two-level.  The 128 indices form 8 blocks of 16; a sweep of
//     the subproblem is 7 rounds over disjoint block pairs (the same
//     round-robin, at the block level).  Each round solves its four 32 x 32
//     pair problems by one scalar sweep on two waves each, then applies
//     the four rotations to A_hat (two-sided, per 32 x 32 tile) and to V_hat
//     with FP64 MFMA.  This is the recursive use of block Jacobi (§4: a
//     subproblem diagonalised by block Jacobi again) inside one subproblem.
//
// The scalar sweeps, their data placement and the rotation formulas are in
// jx_sweep.hpp.
#include "jx_common.hpp"
#include "jx_sweep.hpp"

namespace jx {

// ---------------------------------------------------------------------------
// Shared prologue and epilogue pieces
// ---------------------------------------------------------------------------

// Entry (r, c), r <= c, of this workgroup's A_hat in global memory.
template <int M2, int MODE>
struct HatSource {
    static constexpr int B = M2 / 2;
    const double *Wii = nullptr, *Wjj = nullptr, *Wij = nullptr, *src = nullptr;
    const float *Fii = nullptr, *Fjj = nullptr, *Fij = nullptr;
    __device__ HatSource(const SubArgs &a, int pr) {
        if (MODE == SUB_EIG) {
            const int I = a.pairs[2 * pr], J = a.pairs[2 * pr + 1];
            if (a.ablk32) {
                Fii = a.ablk32 + ublk(I, I) * (size_t)(B * B);
                Fjj = a.ablk32 + ublk(J, J) * (size_t)(B * B);
                Fij = a.ablk32 + ublk(I, J) * (size_t)(B * B);
            } else {
                Wii = a.ablk + ublk(I, I) * (size_t)(B * B);
                Wjj = a.ablk + ublk(J, J) * (size_t)(B * B);
                Wij = a.ablk + ublk(I, J) * (size_t)(B * B);
            }
        } else {
            src = a.ahat + (size_t)pr * M2 * M2;
        }
    }
    __device__ double operator()(int r, int c) const {
        if (MODE == SUB_EIG) {
            if (Fii) {  // FP32 storage: the subproblem is still solved in FP64
                if (c < B) return (double)Fii[c * B + r];
                if (r < B) return (double)Fij[(c - B) * B + r];
                return (double)Fjj[(c - B) * B + (r - B)];
            }
            if (c < B) return Wii[c * B + r];
            if (r < B) return Wij[(c - B) * B + r];
            return Wjj[(c - B) * B + (r - B)];
        }
        return src[(size_t)c * M2 + r];
    }
};

// Skip test of a loaded subproblem; get(r, c) reads entry (r, c) from LDS.
// Eigenproblem: skip when off(A_hat) <= skip_thr; Gram block of the SVD: skip
// when max |a_ij| / sqrt(a_ii a_jj) <= skip_thr (zero columns count as
// orthogonal).  Plain solves never skip.  Returns true when skipped.
template <int M2, int NT, int MODE, class Get>
__device__ bool skip_test(const SubArgs &a, int pr, double off2, double *red, Get get) {
    if (MODE == SUB_PLAIN) return false;
    const int tid = threadIdx.x;
    double meas = sqrt(off2);
    if (MODE == SUB_GRAM) {
        __syncthreads();
        double mx = 0.0;
        for (int e = tid; e < M2 * M2; e += NT) {
            const int rr = e % M2, cc = e / M2;
            if (rr >= cc) continue;
            const double dd = get(rr, rr) * get(cc, cc);
            const double v = get(rr, cc);
            if (dd > 0.0) mx = fmax(mx, fabs(v) / sqrt(dd));
        }
        for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
        __syncthreads();
        if ((tid & 63) == 0) red[tid >> 6] = mx;
        __syncthreads();
        mx = 0.0;
        for (int i = 0; i < NT / 64; ++i) mx = fmax(mx, red[i]);
        meas = mx;
    }
    if (tid == 0 && a.inner_off) a.inner_off[pr] = meas;
    const bool skip = !(meas > a.skip_thr);
    if (tid == 0 && a.flags) a.flags[pr] = skip ? 1 : 0;
    if (tid == 0 && a.rot_count && !skip) atomicAdd(a.rot_count, 1);
    return skip;
}

// Writes D_hat entry (rr, cc) to its place in the upper block storage
// (entries of the lower triangle of the diagonal blocks are not stored).
template <int M2>
__device__ __forceinline__ void store_dhat(const SubArgs &a, size_t oii, size_t ojj, size_t oij, int rr, int cc,
                                           double v) {
    constexpr int B = M2 / 2;
    size_t off;
    if (cc < B) {
        if (rr >= B) return;
        off = oii + cc * B + rr;
    } else if (rr < B) {
        off = oij + (cc - B) * B + rr;
    } else {
        off = ojj + (cc - B) * B + (rr - B);
    }
    if (a.ablk32) a.ablk32[off] = (float)v;
    else a.ablk[off] = v;
}

// ---------------------------------------------------------------------------
// m2 = 32, 64: one workgroup runs the scalar sweeps on the whole subproblem
// ---------------------------------------------------------------------------

template <int M2>
struct SubCfg {
    static constexpr int H = M2 / 2, G = M2 / 16, NT = M2 * G, LD = M2;
    static constexpr size_t LDS_BYTES = sizeof(double) * ((size_t)M2 * LD + 8 * H + NT / 64 + 2);
};

template <int M2, int MODE>
__global__ void __launch_bounds__(SubCfg<M2>::NT) k_subproblem(SubArgs a) {
    using C = SubCfg<M2>;
    constexpr int H = C::H, G = C::G, NT = C::NT, LD = C::LD, B = M2 / 2;
    extern __shared__ double smem[];
    double *As = smem;                    // M2 x LD slots
    double *prm0 = As + (size_t)M2 * LD;  // rotation parameters, two rounds
    double *red = prm0 + 8 * H;           // reduction scratch
    const int tid = threadIdx.x, pr = blockIdx.x;

    if (MODE != SUB_PLAIN && a.force_skip && a.force_skip[pr]) {  // placeholder pair
        if (tid == 0 && a.flags) a.flags[pr] = 1;
        return;
    }
    double off2 = 0.0, fro2 = 0.0;
    {
        const HatSource<M2, MODE> load(a, pr);
        for (int e = tid; e < M2 * M2; e += NT) {
            const int r = e % M2, c = e / M2;
            if (r > c) continue;
            const double v = load(r, c);
            const int u = slot_of(r, M2), w = slot_of(c, M2);
            As[min(u, w) * LD + max(u, w)] = v;
            if (r == c) fro2 += v * v;
            else { off2 += 2.0 * v * v; fro2 += 2.0 * v * v; }
        }
    }
    off2 = block_sum<NT>(off2, red);
    fro2 = block_sum<NT>(fro2, red);
    auto get = [&](int r, int c) {
        const int u = slot_of(r, M2), w = slot_of(c, M2);
        return As[min(u, w) * LD + max(u, w)];
    };
    if (skip_test<M2, NT, MODE>(a, pr, off2, red, get)) return;  // V_hat = I, A_hat unchanged

    double V[16];
    scalar_sweeps<M2, NT, false>(As, prm0, red, tid, a.inner_sweeps > 0 ? a.inner_sweeps : 30,
                                 a.inner_sweeps <= 0, fro2, V);

    const int r = tid / G, g = tid - (tid / G) * G;
    if (MODE == SUB_PLAIN) {
        double *vo = a.vout + (size_t)pr * M2 * M2;
#pragma unroll
        for (int x = 0; x < 16; ++x) vo[(size_t)(16 * g + x) * M2 + r] = V[x];
        double *dd = a.dout + (size_t)pr * M2 * M2;
        for (int e = tid; e < M2 * M2; e += NT) dd[e] = get(e % M2, e / M2);
    } else {
        if (a.vout32) {
            float *vo = a.vout32 + (size_t)pr * M2 * M2;
#pragma unroll
            for (int x = 0; x < 16; ++x) vo[vperm32(r, 16 * g + x, M2)] = (float)V[x];
        } else {
            double *vo = a.vout + (size_t)pr * M2 * M2;
#pragma unroll
            for (int x = 0; x < 16; ++x) vo[vperm(r, 16 * g + x, M2)] = V[x];
        }
        if (MODE == SUB_EIG) {  // A([I,J],[I,J]) <- D_hat
            const int I = a.pairs[2 * pr], J = a.pairs[2 * pr + 1];
            const size_t oii = ublk(I, I) * (size_t)(B * B), ojj = ublk(J, J) * (size_t)(B * B),
                         oij = ublk(I, J) * (size_t)(B * B);
            for (int e = tid; e < M2 * M2; e += NT) {
                const int rr = e % M2, cc = e / M2;
                store_dhat<M2>(a, oii, ojj, oij, rr, cc, get(rr, cc));
            }
        }
    }
}

// ---------------------------------------------------------------------------
// m2 = 128: two-level solver
// ---------------------------------------------------------------------------
// 512 threads (8 waves).  LDS: the upper triangle of A_hat packed row by row
// (Ap), and per 32 x 32 pair problem a slot array, its rotation parameters
// and its rotation W (row-major, stride 33).
// V_hat is kept transposed in registers, Vt = V_hat^T: wave w owns columns
// 16 w .. 16 w + 15 of Vt (rows of V_hat) as 8 MFMA result tiles of 16 rows.
// Tile p holds the rows of the block at ring position p of the current round,
// so block pair k (positions 2k, 2k+1) is always the tiles 2k, 2k+1; after
// each round the tiles move one step along the block ring (7 steps: back to
// block order).
namespace tl {
constexpr int M2 = 128, NB = 8, BS = 16, NT = 512;
constexpr int AP = M2 * (M2 + 1) / 2;           // packed upper triangle
constexpr int SW = 32 * 32 + 8 * 16 + 32 * 33;  // per pair problem: slots, parameters, W
constexpr int WOFF = 32 * 32 + 8 * 16;          // offset of W in a solver region
constexpr size_t LDS_BYTES = sizeof(double) * ((size_t)AP + 4 * SW + 16);
__device__ __forceinline__ int pk(int i, int j) {  // i <= j
    return i * (2 * M2 - 1 - i) / 2 + j;
}
__device__ __forceinline__ int pkm(int i, int j) { return i <= j ? pk(i, j) : pk(j, i); }
}  // namespace tl

template <int MODE>
__global__ void __launch_bounds__(512) k_subproblem2(SubArgs a) {
    using namespace tl;
    constexpr int B = M2 / 2;
    extern __shared__ double smem[];
    double *Ap = smem;
    double *red = Ap + AP + 4 * SW;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int g = lane >> 4, x = lane & 15;
    const int pr = blockIdx.x;

    if (MODE != SUB_PLAIN && a.force_skip && a.force_skip[pr]) {  // placeholder pair
        if (tid == 0 && a.flags) a.flags[pr] = 1;
        return;
    }
    double off2 = 0.0, fro2 = 0.0;
    {
        const HatSource<M2, MODE> load(a, pr);
        for (int e = tid; e < M2 * M2; e += NT) {
            const int r = e % M2, c = e / M2;
            if (r > c) continue;
            const double v = load(r, c);
            Ap[pk(r, c)] = v;
            if (r == c) fro2 += v * v;
            else { off2 += 2.0 * v * v; fro2 += 2.0 * v * v; }
        }
    }
    off2 = block_sum<NT>(off2, red);
    fro2 = block_sum<NT>(fro2, red);
    auto get = [&](int r, int c) { return Ap[pkm(r, c)]; };
    if (skip_test<M2, NT, MODE>(a, pr, off2, red, get)) return;

    // Vt = I: tile tt, lane (g, x), component v holds Vt(16 tt + g + 4 v, 16 wv + x)
    d4 vt[NB];
#pragma unroll
    for (int tt = 0; tt < NB; ++tt)
#pragma unroll
        for (int v = 0; v < 4; ++v) vt[tt][v] = (16 * tt + g + 4 * v == 16 * wv + x) ? 1.0 : 0.0;

    const double eps = 2.220446049250313e-16;
    const bool conv = a.inner_sweeps <= 0;
    const int cap = conv ? 30 : a.inner_sweeps;
    for (int swp = 0; swp < cap; ++swp) {
        if (conv && swp > 0) {
            double o = 0.0;
            for (int e = tid; e < M2 * M2; e += NT) {
                const int rr = e % M2, cc = e / M2;
                if (rr < cc) { const double v = Ap[pk(rr, cc)]; o += 2.0 * v * v; }
            }
            o = block_sum<NT>(o, red);
            if (sqrt(o) <= eps * sqrt(fro2)) break;
        }
        for (int t = 0; t < NB - 1; ++t) {
            // ---- phase 1: waves k, k+4 diagonalise (one sweep) the 32 x 32
            //      problem of block pair k (waves k and k+4 run on different
            //      SIMDs, and so do the four waves holding the rotation
            //      producers); local index l < 16 is row l of block ba,
            //      l >= 16 row l - 16 of block bb
            {
                const int k = wv & 3, lt = ((wv >> 2) << 6) | lane;
                double *S = Ap + AP + k * SW;  // slots
                double *prm = S + 32 * 32;     // parameters
                double *W = S + WOFF;          // rotation, row-major stride 33
                const int ba = index_at(2 * k, t, NB), bb = index_at(2 * k + 1, t, NB);
                for (int e = lt; e < 32 * 32; e += 128) {
                    const int r = e & 31, c = e >> 5;
                    if (r > c) continue;
                    const int gr = r < BS ? BS * ba + r : BS * bb + (r - BS);
                    const int gc = c < BS ? BS * ba + c : BS * bb + (c - BS);
                    const int u = slot_of(r, 32), w = slot_of(c, 32);
                    S[min(u, w) * 32 + max(u, w)] = Ap[pkm(gr, gc)];
                }
                __syncthreads();
                double Vl[8];
                scalar_sweeps<32, 128, false>(S, prm, nullptr, lt, 1, false, 0.0, Vl);
                // W(r, 8 h + xx) = Vl[xx], r = lt / 4, h = lt mod 4; D back into A_hat
                const int r = lt >> 2, h = lt & 3;
#pragma unroll
                for (int xx = 0; xx < 8; ++xx) W[r * 33 + 8 * h + xx] = Vl[xx];
                for (int e = lt; e < 32 * 32; e += 128) {
                    const int rr = e & 31, cc = e >> 5;
                    if (rr > cc) continue;
                    const int gr = rr < BS ? BS * ba + rr : BS * bb + (rr - BS);
                    const int gc = cc < BS ? BS * ba + cc : BS * bb + (cc - BS);
                    const int u = slot_of(rr, 32), w = slot_of(cc, 32);
                    Ap[pkm(gr, gc)] = S[min(u, w) * 32 + max(u, w)];
                }
            }
            __syncthreads();

            // ---- phase 2a: waves 0..5, tile (p, q), p < q:
            //      A_hat(p, q) <- W_p^T A_hat(p, q) W_q
            if (wv < 6) {
                const int p = wv < 3 ? 0 : (wv < 5 ? 1 : 2);
                const int q = wv < 3 ? wv + 1 : (wv < 5 ? wv - 1 : 3);
                const double *Wp = Ap + AP + p * SW + WOFF;
                const double *Wq = Ap + AP + q * SW + WOFF;
                const int pa = index_at(2 * p, t, NB), pb = index_at(2 * p + 1, t, NB);
                const int qa = index_at(2 * q, t, NB), qb = index_at(2 * q + 1, t, NB);
                auto gp = [&](int l) { return l < BS ? BS * pa + l : BS * pb + (l - BS); };
                auto gq = [&](int l) { return l < BS ? BS * qa + l : BS * qb + (l - BS); };
                // T = X W_q, X(i, k) = A_hat(gp(i), gq(k)); T[i][j] lane (g, x)
                // component v = T(16 i + g + 4 v, 16 j + x)
                d4 T[2][2];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) T[i][j] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int k0 = 0; k0 < 32; k0 += 4) {
                    const int k = k0 + g;
                    const double b0 = Wq[k * 33 + x], b1 = Wq[k * 33 + 16 + x];
                    const double a0 = Ap[pkm(gp(x), gq(k))], a1 = Ap[pkm(gp(16 + x), gq(k))];
                    T[0][0] = mfma_f64(a0, b0, T[0][0]);
                    T[0][1] = mfma_f64(a0, b1, T[0][1]);
                    T[1][0] = mfma_f64(a1, b0, T[1][0]);
                    T[1][1] = mfma_f64(a1, b1, T[1][1]);
                }
                // out = W_p^T T; step (ti, s) contracts over row 16 ti + g + 4 s of T
                d4 O[2][2];
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j) O[i][j] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const int k = 16 * ti + g + 4 * s;
                        const double a0 = Wp[k * 33 + x], a1 = Wp[k * 33 + 16 + x];
                        O[0][0] = mfma_f64(a0, T[ti][0][s], O[0][0]);
                        O[0][1] = mfma_f64(a0, T[ti][1][s], O[0][1]);
                        O[1][0] = mfma_f64(a1, T[ti][0][s], O[1][0]);
                        O[1][1] = mfma_f64(a1, T[ti][1][s], O[1][1]);
                    }
                // every read of this tile fed T, so it can be overwritten in place
#pragma unroll
                for (int i = 0; i < 2; ++i)
#pragma unroll
                    for (int j = 0; j < 2; ++j)
#pragma unroll
                        for (int v = 0; v < 4; ++v) Ap[pkm(gp(16 * i + g + 4 * v), gq(16 * j + x))] = O[i][j][v];
            }

            // ---- phase 2b: all waves, Vt rows of block pair k <- W_k^T (those rows)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double *Wk = Ap + AP + k * SW + WOFF;
                d4 n0 = d4{0.0, 0.0, 0.0, 0.0}, n1 = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        const int rr = 16 * ti + g + 4 * s;
                        const double a0 = Wk[rr * 33 + x], a1 = Wk[rr * 33 + 16 + x];
                        const double bv = vt[2 * k + ti][s];
                        n0 = mfma_f64(a0, bv, n0);
                        n1 = mfma_f64(a1, bv, n1);
                    }
                vt[2 * k] = n0;
                vt[2 * k + 1] = n1;
            }
            __syncthreads();
            // ---- tiles follow the block ring: 1 <- 2 <- 4 <- 6 <- 7 <- 5 <- 3 <- 1
            {
                const d4 o1 = vt[1];
                vt[1] = vt[2];
                vt[2] = vt[4];
                vt[4] = vt[6];
                vt[6] = vt[7];
                vt[7] = vt[5];
                vt[5] = vt[3];
                vt[3] = o1;
            }
        }
    }

    // ---- results: V_hat(16 wv + x, 16 tt + g + 4 v) = vt[tt][v]
    if (MODE == SUB_PLAIN) {
        double *vo = a.vout + (size_t)pr * M2 * M2;
#pragma unroll
        for (int tt = 0; tt < NB; ++tt)
#pragma unroll
            for (int v = 0; v < 4; ++v) vo[(size_t)(16 * tt + g + 4 * v) * M2 + 16 * wv + x] = vt[tt][v];
        double *dd = a.dout + (size_t)pr * M2 * M2;
        for (int e = tid; e < M2 * M2; e += NT) dd[e] = Ap[pkm(e % M2, e / M2)];
    } else {
        if (a.vout32) {
            float *vo = a.vout32 + (size_t)pr * M2 * M2;
#pragma unroll
            for (int tt = 0; tt < NB; ++tt)
#pragma unroll
                for (int v = 0; v < 4; ++v) vo[vperm32(16 * wv + x, 16 * tt + g + 4 * v, M2)] = (float)vt[tt][v];
        } else {
            double *vo = a.vout + (size_t)pr * M2 * M2;
#pragma unroll
            for (int tt = 0; tt < NB; ++tt)
#pragma unroll
                for (int v = 0; v < 4; ++v) vo[vperm(16 * wv + x, 16 * tt + g + 4 * v, M2)] = vt[tt][v];
        }
        if (MODE == SUB_EIG) {  // A([I,J],[I,J]) <- D_hat
            const int I = a.pairs[2 * pr], J = a.pairs[2 * pr + 1];
            const size_t oii = ublk(I, I) * (size_t)(B * B), ojj = ublk(J, J) * (size_t)(B * B),
                         oij = ublk(I, J) * (size_t)(B * B);
            for (int e = tid; e < M2 * M2; e += NT) {
                const int rr = e % M2, cc = e / M2;
                store_dhat<M2>(a, oii, ojj, oij, rr, cc, Ap[pkm(rr, cc)]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

template <int M2, int MODE>
static void launch_sub_t(const SubArgs &a, hipStream_t s) {
    using C = SubCfg<M2>;
    static bool attr_set = false;
    if (!attr_set) {
        JX_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_subproblem<M2, MODE>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)C::LDS_BYTES));
        attr_set = true;
    }
    hipLaunchKernelGGL((k_subproblem<M2, MODE>), dim3(a.count), dim3(C::NT), C::LDS_BYTES, s, a);
    JX_LAUNCHED();
}

template <int MODE>
static void launch_sub2_t(const SubArgs &a, hipStream_t s) {
    static bool attr_set = false;
    if (!attr_set) {
        JX_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_subproblem2<MODE>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)tl::LDS_BYTES));
        attr_set = true;
    }
    hipLaunchKernelGGL((k_subproblem2<MODE>), dim3(a.count), dim3(tl::NT), tl::LDS_BYTES, s, a);
    JX_LAUNCHED();
}

template <int MODE>
static void launch_sub_m(const SubArgs &a, hipStream_t s) {
    switch (a.m2) {
        case 32: launch_sub_t<32, MODE>(a, s); break;
        case 64: launch_sub_t<64, MODE>(a, s); break;
        case 128: launch_sub2_t<MODE>(a, s); break;
        default: set_error("subproblem order must be 32, 64 or 128"); throw HipFail{hipErrorInvalidValue};
    }
}

void launch_subproblem(const SubArgs &a, hipStream_t s) {
    if (a.count <= 0) return;
    switch (a.mode) {
        case SUB_EIG: launch_sub_m<SUB_EIG>(a, s); break;
        case SUB_PLAIN: launch_sub_m<SUB_PLAIN>(a, s); break;
        case SUB_GRAM: launch_sub_m<SUB_GRAM>(a, s); break;
        default: set_error("bad subproblem mode"); throw HipFail{hipErrorInvalidValue};
    }
}

}  // namespace jx
