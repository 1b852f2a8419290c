// k_batched.hip -- many independent symmetric eigenproblems (orders up to 256)
// in one persistent launch per size class.
//
// Method: the two-level block Jacobi used by the subproblem solver, applied
// to a whole small matrix.  The padded order M2 is split into NB = M2 / bs
// blocks of bs = 8 or 16 indices; a sweep is NB - 1 rounds of the
// round-robin ordering over block pairs (§3, Alg. 2 with workgroup waves as
// the processors); in each round the NB / 2 disjoint pair problems of order
// 2 bs are diagonalised (one scalar round-robin sweep each, in LDS, FP64) and
// their rotations W_k are applied to the matrix, A(p, q) <- W_p^T A(p, q) W_q,
// and to Q, Q(:, pair k) <- Q(:, pair k) W_k, with MFMA.
//
// Two persistent kernels per class:
//   * low precision: A and Q stored in FP32, tile products in FP32 MFMA with
//     FP32 accumulation, pair problems and rotation angles in FP64; sweeps
//     until off(A) <= lp_switch ||A||_F or the decrease stalls;
//   * FP64 refinement: two Newton-Schulz steps Q <- Q (3 I - Q^T Q) / 2 (one
//     from a warm start Q0), the
//     recomputed A_1 = Q^T A Q from the input (FP64 MFMA), then FP64 sweeps
//     until off(A_1) <= tol ||A||_F; eigenvalues sorted ascending with their
//     vectors.  With a warm start Q0 the refinement starts from Q0 and falls
//     back to the cold start when off(Q0^T A Q0) >= off(A).
// Each workgroup takes the next matrix of its class from an atomic counter;
// the class list is ordered by decreasing n (longest processing time first).
#include "jx_common.hpp"
#include "jx_sweep.hpp"

namespace jx {

namespace {

// Pair-problem geometry for block size BS.
template <int BS>
struct PCfg {
    static constexpr int PP = 2 * BS;                // pair problem order
    static constexpr int PW = PP == 32 ? 128 : 64;   // threads per pair problem
    static constexpr int PV = PP * PP / PW;          // V positions per thread
    static constexpr int G = PP / PV;                // threads per V row
    static constexpr int LDW = PP + 1;               // row stride of W in LDS
    static constexpr int SW = PP * PP + 4 * PP + PP * LDW;  // LDS doubles per pair problem
};

template <int BS, int NPP>
struct KCfg {
    static constexpr int NT = PCfg<BS>::PW * NPP;
    static constexpr int M2 = 2 * BS * NPP;
    static constexpr int NB = 2 * NPP;
    static constexpr int NW = NT / 64;
    static constexpr size_t LDS = sizeof(double) * ((size_t)NPP * PCfg<BS>::SW + 16 + 256) + 64;
};

__device__ __forceinline__ double finite_or_flag(double v, int &bad) {
    if (!(fabs(v) <= 1.7976931348623157e308)) bad = 1;
    return v;
}

// Element (r, c) of the input, upper triangle mirrored.
__device__ __forceinline__ double input_at(const BatchArgs &a, int64_t off, int n, int r, int c) {
    const int lo = min(r, c), hi = max(r, c);
    const int64_t e = off + (int64_t)hi * n + lo;
    return a.dtype == JACOBI_F32 ? (double)((const float *)a.A_in)[e] : ((const double *)a.A_in)[e];
}

// off(A) of an M2 x M2 column-major matrix, summed directly in FP64.
template <int NT, int M2, class T>
__device__ double offnorm(const T *A, double *red) {
    double s = 0.0;
    for (int e = threadIdx.x; e < M2 * M2; e += NT) {
        const int r = e % M2, c = e / M2;
        const double v = (double)A[e];
        if (r != c) s += v * v;
    }
    return sqrt(block_sum<NT>(s, red));
}

// One sweep of the two-level scheme on A (M2 x M2, column-major, both
// triangles kept) and Q, type T; pair problems in FP64.
template <int BS, int NPP, class T>
__device__ void sweep_two_level(T *A, T *Q, double *smem) {
    using PC = PCfg<BS>;
    using KC = KCfg<BS, NPP>;
    using MT = MfmaTraits<T>;
    typedef typename MT::acc_t acc_t;
    constexpr int PP = PC::PP, PW = PC::PW, PV = PC::PV, G = PC::G, LDW = PC::LDW, SW = PC::SW;
    constexpr int M2 = KC::M2, NB = KC::NB, NW = KC::NW, TI = PP / 16;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int g = lane >> 4, x = lane & 15;

    for (int t = 0; t < NB - 1; ++t) {
        // ---- pair problems: problem k on waves k (+ k + NPP when PW = 128)
        {
            const int k = wv % NPP;
            const int lt = (PW == 128) ? (((wv / NPP) << 6) | lane) : lane;
            double *S = smem + k * SW;
            double *prm = S + PP * PP;
            double *W = prm + 4 * PP;
            const int ba = index_at(2 * k, t, NB), bb = index_at(2 * k + 1, t, NB);
            for (int e = lt; e < PP * PP; e += PW) {
                const int r = e % PP, c = e / PP;
                if (r > c) continue;
                const int gr = r < BS ? BS * ba + r : BS * bb + (r - BS);
                const int gc = c < BS ? BS * ba + c : BS * bb + (c - BS);
                const int u = slot_of(r, PP), w = slot_of(c, PP);
                S[min(u, w) * PP + max(u, w)] = (double)A[(size_t)gc * M2 + gr];
            }
            __syncthreads();
            double Vl[PV];
            scalar_sweeps<PP, PW, false>(S, prm, nullptr, lt, 1, false, 0.0, Vl);
            const int r = lt / G, h = lt % G;
#pragma unroll
            for (int xx = 0; xx < PV; ++xx) W[r * LDW + PV * h + xx] = Vl[xx];
            for (int e = lt; e < PP * PP; e += PW) {
                const int rr = e % PP, cc = e / PP;
                const int gr = rr < BS ? BS * ba + rr : BS * bb + (rr - BS);
                const int gc = cc < BS ? BS * ba + cc : BS * bb + (cc - BS);
                const int u = slot_of(rr, PP), w = slot_of(cc, PP);
                A[(size_t)gc * M2 + gr] = (T)S[min(u, w) * PP + max(u, w)];
            }
        }
        __syncthreads();

        // ---- A(p, q) <- W_p^T A(p, q) W_q for p < q, and the mirror (q, p)
        constexpr int NTILE = NPP * (NPP - 1) / 2;
        for (int u = wv; u < NTILE; u += NW) {
            int p = 0, rem = u;
            while (rem >= NPP - 1 - p) { rem -= NPP - 1 - p; ++p; }
            const int q = p + 1 + rem;
            const double *Wp = smem + p * SW + PP * PP + 4 * PP;
            const double *Wq = smem + q * SW + PP * PP + 4 * PP;
            const int pa = index_at(2 * p, t, NB), pb = index_at(2 * p + 1, t, NB);
            const int qa = index_at(2 * q, t, NB), qb = index_at(2 * q + 1, t, NB);
            auto gp = [&](int l) { return l < BS ? BS * pa + l : BS * pb + (l - BS); };
            auto gq = [&](int l) { return l < BS ? BS * qa + l : BS * qb + (l - BS); };
            acc_t Tt[TI][TI];
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TI; ++j) Tt[i][j] = acc_t{0, 0, 0, 0};
            // T = X W_q, X(i, l) = A(gp(i), gq(l))
#pragma unroll 2
            for (int k0 = 0; k0 < PP; k0 += 4) {
                const int l = k0 + g;
                T av[TI], bv[TI];
#pragma unroll
                for (int j = 0; j < TI; ++j) bv[j] = (T)Wq[l * LDW + 16 * j + x];
#pragma unroll
                for (int i = 0; i < TI; ++i) av[i] = A[(size_t)gq(l) * M2 + gp(16 * i + x)];
#pragma unroll
                for (int i = 0; i < TI; ++i)
#pragma unroll
                    for (int j = 0; j < TI; ++j) Tt[i][j] = MT::mma(av[i], bv[j], Tt[i][j]);
            }
            // O = W_p^T T: step (ti, s) contracts over row 16 ti + rrow(g, s) of T
            acc_t O[TI][TI];
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TI; ++j) O[i][j] = acc_t{0, 0, 0, 0};
#pragma unroll
            for (int ti = 0; ti < TI; ++ti)
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int l = 16 * ti + MT::rrow(g, s);
#pragma unroll
                    for (int i = 0; i < TI; ++i) {
                        const T av = (T)Wp[l * LDW + 16 * i + x];
#pragma unroll
                        for (int j = 0; j < TI; ++j) O[i][j] = MT::mma(av, Tt[ti][j][s], O[i][j]);
                    }
                }
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TI; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int rp = gp(16 * i + MT::rrow(g, v)), cq = gq(16 * j + x);
                        A[(size_t)cq * M2 + rp] = O[i][j][v];
                        A[(size_t)rp * M2 + cq] = O[i][j][v];
                    }
        }

        // ---- Q(rows, pair k) <- Q(rows, pair k) W_k, computed as the transpose
        //      W_k^T Q(rows, pair k)^T so that loads and stores run along rows
        constexpr int NUNIT = (M2 / 16) * NPP;
        for (int u = wv; u < NUNIT; u += NW) {
            const int k = u % NPP, jr = u / NPP;
            const double *Wk = smem + k * SW + PP * PP + 4 * PP;
            const int ka = index_at(2 * k, t, NB), kb = index_at(2 * k + 1, t, NB);
            auto cq = [&](int l) { return l < BS ? BS * ka + l : BS * kb + (l - BS); };
            acc_t D[TI];
#pragma unroll
            for (int i = 0; i < TI; ++i) D[i] = acc_t{0, 0, 0, 0};
#pragma unroll 2
            for (int k0 = 0; k0 < PP; k0 += 4) {
                const int l = k0 + g;
                const T bv = Q[(size_t)cq(l) * M2 + 16 * jr + x];
#pragma unroll
                for (int i = 0; i < TI; ++i) D[i] = MT::mma((T)Wk[l * LDW + 16 * i + x], bv, D[i]);
            }
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int v = 0; v < 4; ++v) Q[(size_t)cq(16 * i + MT::rrow(g, v)) * M2 + 16 * jr + x] = D[i][v];
        }
        __syncthreads();
    }
}

// C = alpha op(X) Y + beta D for M2 x M2 column-major FP64 matrices (the whole
// workgroup; C must not alias X or Y, D may alias C).  Computed as tiles of
// C^T = Y^T op(X)^T so that the stores run along columns.
template <int NT, int M2>
__device__ void gemm_wg(double *C, double alpha, bool transX, const double *X, const double *Y, double beta,
                        const double *D) {
    constexpr int TT = (M2 % 32 == 0) ? 2 : 1;  // 16 x 16 MFMA tiles per tile edge
    constexpr int TE = 16 * TT, NTL = M2 / TE, NW = NT / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int g = lane >> 4, x = lane & 15;
    for (int u = wv; u < NTL * NTL; u += NW) {
        const int c0 = (u % NTL) * TE, r0 = (u / NTL) * TE;
        d4 acc[TT][TT];
#pragma unroll
        for (int i = 0; i < TT; ++i)
#pragma unroll
            for (int j = 0; j < TT; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
        for (int k0 = 0; k0 < M2; k0 += 4) {
            const int k = k0 + g;
            double av[TT], bv[TT];
#pragma unroll
            for (int i = 0; i < TT; ++i) av[i] = Y[(size_t)(c0 + 16 * i + x) * M2 + k];  // Y(k, col)
#pragma unroll
            for (int j = 0; j < TT; ++j) {
                const int row = r0 + 16 * j + x;
                bv[j] = transX ? X[(size_t)row * M2 + k] : X[(size_t)k * M2 + row];  // op(X)(row, k)
            }
#pragma unroll
            for (int i = 0; i < TT; ++i)
#pragma unroll
                for (int j = 0; j < TT; ++j) acc[i][j] = mfma_f64(av[i], bv[j], acc[i][j]);
        }
#pragma unroll
        for (int i = 0; i < TT; ++i)
#pragma unroll
            for (int j = 0; j < TT; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const size_t e = (size_t)(c0 + 16 * i + g + 4 * v) * M2 + r0 + 16 * j + x;
                    const double d = beta != 0.0 ? beta * D[e] : 0.0;
                    C[e] = alpha * acc[i][j][v] + d;
                }
    }
    __syncthreads();
}

// Next class-local slot from the queue (the same value in every thread); a
// value outside [0, count) ends the workgroup's loop.
template <int NT>
__device__ int next_slot(const BatchArgs &a, int *bcast) {
    if (threadIdx.x == 0) bcast[0] = atomicAdd(a.queue, 1);
    __syncthreads();
    const int slot = bcast[0];
    __syncthreads();
    return slot;
}

// ---------------------------------------------------------------------------
// Low-precision phase
// ---------------------------------------------------------------------------
template <int BS, int NPP>
__global__ void __launch_bounds__((KCfg<BS, NPP>::NT)) k_batched_lp(BatchArgs a) {
    using KC = KCfg<BS, NPP>;
    constexpr int NT = KC::NT, M2 = KC::M2;
    extern __shared__ double smem[];
    double *red = smem + NPP * PCfg<BS>::SW;
    int *bcast = (int *)(red + 16 + 256);
    for (;;) {
        const int slot = next_slot<NT>(a, bcast);
        if (slot < 0 || slot >= a.count) break;
        const int id = a.ids[slot];
        const int n = a.n[id];
        float *A = a.A32 + a.offWs[id];
        float *Q = a.Q32 + a.offWs[id];
        double fro2 = 0.0;
        int bad = 0;
        for (int e = threadIdx.x; e < M2 * M2; e += NT) {
            const int r = e % M2, c = e / M2;
            const double v = (r < n && c < n) ? finite_or_flag(input_at(a, a.offA[id], n, r, c), bad) : 0.0;
            A[e] = (float)v;
            Q[e] = r == c ? 1.0f : 0.0f;
            fro2 += v * v;
        }
        fro2 = block_sum<NT>(fro2, red);
        const double nbad = block_sum<NT>((double)bad, red);
        int sw = 0;
        if (nbad == 0.0 && a.lp_max_sweeps > 0) {
            const double fro = sqrt(fro2);
            double off = offnorm<NT, M2>(A, red);
            while (sw < a.lp_max_sweeps && off > a.lp_switch * fro) {
                sweep_two_level<BS, NPP, float>(A, Q, smem);
                ++sw;
                const double o = offnorm<NT, M2>(A, red);
                const bool stalled = sw >= 2 && o > 0.5 * off && o < 1e-3 * fro;
                off = o;
                if (stalled || !(off == off)) break;
            }
        }
        if (threadIdx.x == 0) a.stat[4 * id + 0] = sw;
        // every iteration ends at a barrier: otherwise the compiler may join
        // this lane-0 store with the lane-0 queue fetch of the next iteration
        // and run lane 0 and the other lanes in different iterations
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// FP64 refinement phase
// ---------------------------------------------------------------------------
template <int BS, int NPP>
__global__ void __launch_bounds__((KCfg<BS, NPP>::NT)) k_batched_hp(BatchArgs a) {
    using KC = KCfg<BS, NPP>;
    constexpr int NT = KC::NT, M2 = KC::M2;
    extern __shared__ double smem[];
    double *red = smem + NPP * PCfg<BS>::SW;
    int *rank = (int *)(red + 16);
    int *bcast = (int *)(red + 16 + 256);
    for (;;) {
        const int slot = next_slot<NT>(a, bcast);
        if (slot < 0 || slot >= a.count) break;
        const int id = a.ids[slot];
        const int n = a.n[id];
        const int64_t offA = a.offA[id], ws = a.offWs[id];
        double *A0 = a.A64 + ws, *Q = a.Q64 + ws, *T = a.T64 + ws, *U = a.U64 + ws;
        const int sw32 = a.lp_max_sweeps > 0 ? a.stat[4 * id + 0] : 0;
        const bool warm = a.Q0 != nullptr;
        double fro2 = 0.0;
        int bad = 0;
        for (int e = threadIdx.x; e < M2 * M2; e += NT) {
            const int r = e % M2, c = e / M2;
            const double v = (r < n && c < n) ? finite_or_flag(input_at(a, offA, n, r, c), bad) : 0.0;
            A0[e] = v;
            fro2 += v * v;
            double q = r == c ? 1.0 : 0.0;
            if (warm) {
                if (r < n && c < n) q = a.Q0[offA + (int64_t)c * n + r];
            } else if (sw32 > 0) {
                q = (double)a.Q32[ws + e];
            }
            Q[e] = q;
        }
        fro2 = block_sum<NT>(fro2, red);
        const double nbad = block_sum<NT>((double)bad, red);
        if (nbad != 0.0) {
            for (int i = threadIdx.x; i < n; i += NT) a.W_out[a.offW[id] + i] = __builtin_nan("");
            if (threadIdx.x == 0) {
                a.stat[4 * id + 1] = 0;
                a.stat[4 * id + 2] = 2;
                a.stat[4 * id + 3] = 0;
                a.offrel[id] = __builtin_nan("");
            }
            __syncthreads();  // see the FP32 phase: no lane-0 code across the back-edge
            continue;
        }
        const double fro = sqrt(fro2);
        double *Acur = A0;
        int fallback = 0;
        if (warm || sw32 > 0) {
            // Newton-Schulz steps Q <- Q (3 I - Q^T Q) / 2, then A_1 = Q^T A Q
            // from the input.  A step from ||Q^T Q - I||_F = e leaves about
            // e^2, so the steps stop after the first one that starts from
            // e <= 1e-8 (at most four: Q from the FP32 phase, e ~ 1e-6, takes
            // two; an FP64 warm start usually one).
            for (int it = 0; it < 4; ++it) {
                gemm_wg<NT, M2>(T, 1.0, true, Q, Q, 0.0, nullptr);
                double dev2 = 0.0;
                for (int e = threadIdx.x; e < M2 * M2; e += NT) {
                    const double d = T[e] - (e % M2 == e / M2 ? 1.0 : 0.0);
                    dev2 += d * d;
                }
                dev2 = block_sum<NT>(dev2, red);
                gemm_wg<NT, M2>(U, -0.5, false, Q, T, 1.5, Q);
                double *tmp = Q;
                Q = U;
                U = tmp;
                if (dev2 <= 1e-16) break;
            }
            gemm_wg<NT, M2>(T, 1.0, false, A0, Q, 0.0, nullptr);
            gemm_wg<NT, M2>(U, 1.0, true, Q, T, 0.0, nullptr);
            Acur = U;
            if (warm) {  // keep the warm start only if it lowers the off-norm
                const double off1 = offnorm<NT, M2>(U, red), off0 = offnorm<NT, M2>(A0, red);
                if (!(off1 < off0)) {
                    fallback = 1;
                    Acur = A0;
                    for (int e = threadIdx.x; e < M2 * M2; e += NT) Q[e] = (e % M2 == e / M2) ? 1.0 : 0.0;
                    __syncthreads();
                }
            }
        }
        double off = offnorm<NT, M2>(Acur, red);
        int sw = 0;
        while (sw < a.max_sweeps && off > a.tol * fro) {
            sweep_two_level<BS, NPP, double>(Acur, Q, smem);
            ++sw;
            off = offnorm<NT, M2>(Acur, red);
            if (!(off == off)) break;
        }
        if (a.want_vectors && sw >= 3 && off <= a.tol * fro) {
            // many FP64 sweeps let Q drift from orthogonality: one Newton-Schulz
            // step, A_1 = Q^T A Q recomputed from the input, and sweeps to tol
            double *buf[4] = {A0, Q, T, U};
            int iq = 1, ia = (Acur == A0) ? 0 : 3;
            const int it = 2, inew = ia;  // the iterate's buffer receives the new Q
            gemm_wg<NT, M2>(buf[it], 1.0, true, buf[iq], buf[iq], 0.0, nullptr);
            gemm_wg<NT, M2>(buf[inew], -0.5, false, buf[iq], buf[it], 1.5, buf[iq]);
            const int iin = iq;  // the old Q buffer receives the input
            iq = inew;
            for (int e = threadIdx.x; e < M2 * M2; e += NT) {
                const int r = e % M2, c = e / M2;
                buf[iin][e] = (r < n && c < n) ? input_at(a, offA, n, r, c) : 0.0;
            }
            __syncthreads();
            const int ires = 6 - iq - iin - it;  // the remaining buffer
            gemm_wg<NT, M2>(buf[it], 1.0, false, buf[iin], buf[iq], 0.0, nullptr);
            gemm_wg<NT, M2>(buf[ires], 1.0, true, buf[iq], buf[it], 0.0, nullptr);
            Q = buf[iq];
            Acur = buf[ires];
            off = offnorm<NT, M2>(Acur, red);
            int sw2 = 0;
            while (sw2 < a.max_sweeps && off > a.tol * fro) {
                sweep_two_level<BS, NPP, double>(Acur, Q, smem);
                ++sw2;
                off = offnorm<NT, M2>(Acur, red);
                if (!(off == off)) break;
            }
            sw += sw2;
        }
        // eigenvalues diag(A) of the n leading indices; ascending ranks (stable)
        for (int i = threadIdx.x; i < n; i += NT) {
            const double li = Acur[(size_t)i * M2 + i];
            int rk = i;
            if (a.sort) {
                rk = 0;
                for (int j = 0; j < n; ++j) {
                    const double lj = Acur[(size_t)j * M2 + j];
                    rk += (lj < li) || (lj == li && j < i);
                }
            }
            rank[i] = rk;
            a.W_out[a.offW[id] + rk] = li;
        }
        __syncthreads();
        if (a.want_vectors)
            for (int e = threadIdx.x; e < n * n; e += NT) {
                const int r = e % n, c = e / n;
                a.Q_out[offA + (int64_t)rank[c] * n + r] = Q[(size_t)c * M2 + r];
            }
        if (threadIdx.x == 0) {
            a.stat[4 * id + 1] = sw;
            a.stat[4 * id + 2] = (off <= a.tol * fro) ? 0 : ((off == off) ? 1 : 2);
            a.stat[4 * id + 3] = fallback;
            a.offrel[id] = fro > 0.0 ? off / fro : 0.0;
        }
        __syncthreads();
    }
}

__global__ void k_fill_int(int *p, int count, int value) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = value;
}

template <int BS, int NPP>
const void *class_kernel(bool lp) {
    return lp ? reinterpret_cast<const void *>(&k_batched_lp<BS, NPP>)
              : reinterpret_cast<const void *>(&k_batched_hp<BS, NPP>);
}

// Dynamic LDS above the default limit, set once per kernel and device (before
// any capture: the occupancy query of the driver runs first).
template <int BS, int NPP>
void ensure_attr(bool lp) {
    ensure_lds_limit(class_kernel<BS, NPP>(lp), (int)KCfg<BS, NPP>::LDS);
}

template <int BS, int NPP>
void launch_class(const BatchArgs &a, bool lp, int grid, hipStream_t s) {
    using KC = KCfg<BS, NPP>;
    ensure_attr<BS, NPP>(lp);
    if (lp) hipLaunchKernelGGL((k_batched_lp<BS, NPP>), dim3(grid), dim3(KC::NT), KC::LDS, s, a);
    else hipLaunchKernelGGL((k_batched_hp<BS, NPP>), dim3(grid), dim3(KC::NT), KC::LDS, s, a);
    JX_LAUNCHED();
}

template <int BS, int NPP>
int occupancy_class(bool lp) {
    using KC = KCfg<BS, NPP>;
    ensure_attr<BS, NPP>(lp);
    int nb = 0;
    JX_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, class_kernel<BS, NPP>(lp), KC::NT, KC::LDS));
    return nb;
}

// Launch (grid > 0) or occupancy query (grid == 0, result in *occ).
template <int BS, int NPP>
bool dispatch(int npp, const BatchArgs *a, bool lp, int grid, int *occ, hipStream_t s) {
    if constexpr (NPP == 0) {
        return false;
    } else {
        if (npp == NPP) {
            if (grid > 0) launch_class<BS, NPP>(*a, lp, grid, s);
            else *occ = occupancy_class<BS, NPP>(lp);
            return true;
        }
        return dispatch<BS, NPP - 1>(npp, a, lp, grid, occ, s);
    }
}

bool dispatch_bs(int bs, int m2, const BatchArgs *a, bool lp, int grid, int *occ, hipStream_t s) {
    if (bs == 16 && m2 % 32 == 0) return dispatch<16, 8>(m2 / 32, a, lp, grid, occ, s);
    if (bs == 8 && m2 % 16 == 0) return dispatch<8, 16>(m2 / 16, a, lp, grid, occ, s);
    return false;
}

void launch_batched(const BatchArgs &a, int bs, int grid, bool lp, hipStream_t s) {
    if (a.count <= 0 || grid <= 0) return;
    if (!dispatch_bs(bs, a.m2, &a, lp, grid, nullptr, s)) {
        set_error("batched: unsupported block size / padded order");
        throw HipFail{hipErrorInvalidValue};
    }
}

}  // namespace

void launch_batched_lp(const BatchArgs &a, int bs, int grid, hipStream_t s) { launch_batched(a, bs, grid, true, s); }
void launch_batched_hp(const BatchArgs &a, int bs, int grid, hipStream_t s) { launch_batched(a, bs, grid, false, s); }

void launch_fill_int(int *p, int count, int value, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_fill_int, dim3((count + 255) / 256), dim3(256), 0, s, p, count, value);
    JX_LAUNCHED();
}

int batched_blocks_per_cu(int bs, int m2, bool lp) {
    int occ = 0;
    if (!dispatch_bs(bs, m2, nullptr, lp, 0, &occ, nullptr)) {
        set_error("batched: unsupported block size / padded order");
        throw HipFail{hipErrorInvalidValue};
    }
    return occ;
}

int batched_threads(int bs, int m2) { return (bs == 16 ? 128 : 64) * (m2 / (2 * bs)); }

size_t batched_lds_bytes(int bs, int m2) {
    const int pp = 2 * bs, npp = m2 / pp;
    return sizeof(double) * ((size_t)npp * (pp * pp + 4 * pp + pp * (pp + 1)) + 16 + 256) + 64;
}

}  // namespace jx
