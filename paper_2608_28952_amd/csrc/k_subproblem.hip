// k_subproblem.hip -- the subproblem solver of block Jacobi on gfx950.
//
// One workgroup diagonalises one 2b x 2b symmetric subproblem
// A_hat = A([I,J],[I,J]) (Alg. 1 and the diagonalisation step of Alg. 2, §3)
// by inner scalar Jacobi: sweeps of m2 - 1 rounds, each round rotating m2/2
// disjoint index pairs at once (disjoint rotations commute, §3).  The exact
// or approximate diagonalisation of the subproblem is left open by the paper
// (§3, after Alg. 3); `inner_sweeps` caps the inner sweeps.
//
// Data placement
//   * A_hat: LDS, upper triangle only, row-major with stride LD = m2.  Index
//     x is stored at slot pi(x) = ring order (pi(0) = 0, pi(x) = 1 + ring
//     index of x): in round t the pair members p_k, q_k of consecutive k sit
//     at consecutive slots (p: slot 1 + (k + t) mod (m2-1), q: slot
//     1 + (t - k) mod (m2-1)), so the lanes of a wave touch addresses with odd
//     strides (m2 + 1, m2 - 1) and the LDS banks are not in conflict.
//   * V_hat: registers.  Thread (r, g) holds row r of V_hat at the 16
//     "positions" 16 g .. 16 g + 15.  Positions are paired (2k, 2k+1) in every
//     round; after a round the column content moves one step along the
//     round-robin ring 1 <- 2 <- 4 <- ... <- m2-2 <- m2-1 <- m2-3 <- ... <- 3 <- 1
//     (position 0 stays), so that every index pair meets once per sweep.  Two
//     values per thread cross to the neighbouring lane (lane shuffles).  After
//     m2 - 1 rounds the ring has turned once and positions equal indices.
//   * Rotation parameters: computed by m2/2 threads per round into LDS, one
//     array per quantity (c, s, t, a_pq, slot of p, slot of q).
//
// The 2x2 rotation of a pair (p, q) is the symmetric Schur form: with
// theta = (a_qq - a_pp) / (2 a_pq), t = sgn(theta) / (|theta| + hypot(1, theta)),
// c = 1 / sqrt(1 + t^2), s = t c, the plane rotation J = [[c, s], [-s, c]] on
// (p, q) gives J^T A J a zero (p, q) entry and diagonal a_pp - t a_pq,
// a_qq + t a_pq (Golub & Van Loan §8.5.2).
#include "jx_common.hpp"

namespace jx {

template <int M2>
struct SubCfg {
    static constexpr int H = M2 / 2;             // pairs per inner round
    static constexpr int G = M2 / 16;            // position groups per row
    static constexpr int NT = M2 * G;            // threads
    static constexpr int NW = NT / 64;           // waves
    static constexpr int LD = M2;                // LDS row stride of A_hat (slots)
    static constexpr int NOFF = H * (H - 1) / 2; // off-diagonal pair-blocks per round
    static constexpr size_t LDS_BYTES = sizeof(double) * ((size_t)M2 * LD + 2 * 4 * H + NW + 2);
};

// Ring of positions 1 .. m2-1 in the order their content moves.
__device__ __forceinline__ int ring_at(int i, int m2) {
    if (i == 0) return 1;
    if (i < m2 / 2) return 2 * i;
    return 2 * m2 - 1 - 2 * i;
}
__device__ __forceinline__ int ring_index(int x, int m2) {
    if (x == 1) return 0;
    if ((x & 1) == 0) return x >> 1;
    return (2 * m2 - 1 - x) >> 1;
}

// LDS slot of index x (its place along the ring; 0 stays 0).
__device__ __forceinline__ int slot_of(int x, int m2) { return x == 0 ? 0 : 1 + ring_index(x, m2); }

// Slots of the two members of pair k in round t of a sweep (t < m2 - 1):
// position 2k holds slot 1 + (k + t) mod (m2-1) (k >= 1; position 0 is slot 0),
// position 2k+1 holds slot 1 + (t - k) mod (m2-1) (k >= 1; position 1 is
// slot 1 + t).
__device__ __forceinline__ int slot_p(int k, int t, int m2) {
    if (k == 0) return 0;
    int i = k + t;
    if (i >= m2 - 1) i -= m2 - 1;
    return 1 + i;
}
__device__ __forceinline__ int slot_q(int k, int t, int m2) {
    int i = (k == 0) ? t : t - k;
    if (i < 0) i += m2 - 1;
    return 1 + i;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum x over the workgroup (fixed order); every thread gets the result.
template <int NT>
__device__ __forceinline__ double block_sum(double x, double *red) {
    x = wave_sum(x);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = x;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < NT / 64; ++i) s += red[i];
    return s;
}

// Rotation parameters of pair k (c, s, t, a_pq) from its diagonal and pivot.
// t = sgn(theta) / (|theta| + sqrt(1 + theta^2)), theta = (a_qq - a_pp) / (2 a_pq);
// for huge |theta| the square would overflow and t = 1 / (2 theta).
__device__ __forceinline__ void rot_params(double app, double aqq, double apq, double *prm, int k, int H) {
    double c = 1.0, s = 0.0, tt = 0.0;
    if (apq != 0.0) {
        const double th = (aqq - app) / (2.0 * apq);
        const double ath = fabs(th);
        tt = ath > 1e150 ? 0.5 / ath : 1.0 / (ath + sqrt(1.0 + th * th));
        if (th < 0.0) tt = -tt;
        c = 1.0 / sqrt(1.0 + tt * tt);
        s = tt * c;
    }
    prm[k] = c;
    prm[H + k] = s;
    prm[2 * H + k] = tt;
    prm[3 * H + k] = apq;
}

// Round structure (one workgroup barrier per round).  The rotation
// parameters of round t sit in an LDS buffer (c, s, t, a_pq per pair); every
// thread applies its share of the 2x2 pair-block updates A_hat <- J^T A_hat J
// (pair-blocks between different pairs) and of the V_hat rows.  The pivot
// a_pq of a round becomes zero and is not written: in the next round it lies
// in a known pair-block, which reads it as zero (cleared explicitly at the
// end of a sweep).  The pair-blocks that compute the next round's pivots --
// {k-1, k+1} for pair k, {0, 1} for pair 0, {H-2, H-1} for pair H-1 -- also
// bring the two diagonal entries of that pair up to date (a_pp - t a_pq,
// a_qq + t a_pq of their current rotation) and write the next round's
// parameters, so no separate angle phase is needed.
template <int M2, int MODE>
__global__ void __launch_bounds__(SubCfg<M2>::NT) k_subproblem(SubArgs a) {
    using C = SubCfg<M2>;
    constexpr int H = C::H, G = C::G, NT = C::NT, LD = C::LD, B = M2 / 2, R = M2 - 1;
    extern __shared__ double smem[];
    double *As = smem;                                   // M2 x LD slots
    double *prm0 = As + (size_t)M2 * LD;                 // parameters, two rounds
    double *red = prm0 + 8 * H;                          // reduction scratch

    const int tid = threadIdx.x;
    const int pr = blockIdx.x;
    double *Wii = nullptr, *Wjj = nullptr, *Wij = nullptr;

    if (MODE != SUB_PLAIN && a.force_skip && a.force_skip[pr]) {  // placeholder pair
        if (tid == 0 && a.flags) a.flags[pr] = 1;
        return;
    }

    // ---- load the upper triangle of A_hat into LDS (slot order) -----------
    double off2 = 0.0, fro2 = 0.0;
    const double *srcp = nullptr;
    const float *Fii = nullptr, *Fjj = nullptr, *Fij = nullptr;
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
        srcp = a.ahat + (size_t)pr * M2 * M2;
    }
    auto load = [&](int r, int c) -> double {
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
        return srcp[(size_t)c * M2 + r];
    };
    for (int e = tid; e < M2 * M2; e += NT) {
        const int r = e % M2, c = e / M2;
        if (r > c) continue;
        const double v = load(r, c);
        const int u = slot_of(r, M2), w = slot_of(c, M2);
        As[min(u, w) * LD + max(u, w)] = v;
        if (r == c) fro2 += v * v;
        else { off2 += 2.0 * v * v; fro2 += 2.0 * v * v; }
    }
    off2 = block_sum<NT>(off2, red);
    fro2 = block_sum<NT>(fro2, red);

    if (MODE != SUB_PLAIN) {
        // eigenproblem: skip when off(A_hat) is small; Gram block of the SVD:
        // skip when every column pair is nearly orthogonal,
        // max |a_ij| / sqrt(a_ii a_jj) <= skip_thr (zero columns count as orthogonal)
        double meas = sqrt(off2);
        if (MODE == SUB_GRAM) {
            __syncthreads();
            double mx = 0.0;
            for (int e = tid; e < M2 * M2; e += NT) {
                const int rr = e % M2, cc = e / M2;
                if (rr >= cc) continue;
                const int u = slot_of(rr, M2), w = slot_of(cc, M2);
                const double dd = As[u * (LD + 1)] * As[w * (LD + 1)];
                const double v = As[min(u, w) * LD + max(u, w)];
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
        if (skip) return;  // V_hat = I, A_hat unchanged
    }

    // ---- V_hat rows in position space -----------------------------------------
    const int r = tid / G, g = tid - (tid / G) * G;
    double V[16];
#pragma unroll
    for (int x = 0; x < 16; ++x) V[x] = (r == 16 * g + x) ? 1.0 : 0.0;

    // parameters of the first round
    if (tid < H) {
        const int up = slot_p(tid, 0, M2), uq = slot_q(tid, 0, M2);
        rot_params(As[up * (LD + 1)], As[uq * (LD + 1)], As[min(up, uq) * LD + max(up, uq)], prm0, tid, H);
    }
    __syncthreads();

    // ---- this thread's pair-blocks (fixed for all rounds) ------------------------
    // Slots of pair k advance by one per round along 1 .. m2-1 (slot 0 stays),
    // so they are kept in registers.  sel codes: entry 0 = (p1,p2), 1 = (p1,q2),
    // 2 = (q1,p2), 3 = (q1,q2); member codes: 0 = p1, 1 = q1, 2 = p2, 3 = q2.
    constexpr int MAXI = (C::NOFF + NT - 1) / NT;
    static_assert(2 * H <= NT, "pivot pair-blocks must be first items");
    // packed per item: ikk = k1 | k2 << 8; icode = (stale + 1) | (kn + 1) << 3 |
    // pivot entry << 10 | p' member << 12 | q' member << 14
    int ikk[MAXI], isl[MAXI][4], icode[MAXI];
#pragma unroll
    for (int ii = 0; ii < MAXI; ++ii) {
        const int it = tid + ii * NT;
        int k1 = 0, d = 1;
        if (it < H * (H / 2 - 1)) { d = it / H + 1; k1 = it - (d - 1) * H; }
        else { d = H / 2; k1 = it - H * (H / 2 - 1); }
        int k2 = k1 + d;
        if (k2 >= H) k2 -= H;
        const bool valid = it < C::NOFF;
        if (!valid) { k1 = 0; k2 = 1; }
        ikk[ii] = k1 | (k2 << 8);
        isl[ii][0] = slot_p(k1, 0, M2);
        isl[ii][1] = slot_q(k1, 0, M2);
        isl[ii][2] = slot_p(k2, 0, M2);
        isl[ii][3] = slot_q(k2, 0, M2);
        const int lo = min(k1, k2), hi = max(k1, k2);
        const bool fw = (k1 == lo);
        // previous round's pivot lying in this pair-block
        int st = -1;
        if (hi - lo == 2 && lo >= 1) st = fw ? 1 : 2;          // (p_lo, q_hi)
        else if (lo == 0 && hi == 2) st = 3;                    // (q0, q2)
        else if (lo == 0 && hi == 1) st = fw ? 1 : 2;           // (p0, q1)
        else if (lo == H - 2 && hi == H - 1) st = 0;            // (p(H-2), p(H-1))

        // next round's pivot computed by this pair-block: pair kn, pivot entry,
        // members p' (imp) and q' (imq)
        int kn = -1, pv = 0, mp = 0, mq = 0;
        if (hi - lo == 2) {                       // (q_lo, p_hi) -> pair lo + 1
            kn = lo + 1;
            pv = fw ? 2 : 1;
            mp = fw ? 2 : 0;                      // p_hi
            mq = fw ? 1 : 3;                      // q_lo
        } else if (lo == 0 && hi == 1) {          // (p0, p1) -> pair 0
            kn = 0; pv = 0;
            mp = fw ? 0 : 2;                      // p0
            mq = fw ? 2 : 0;                      // p1
        } else if (lo == H - 2 && hi == H - 1) {  // (q(H-2), q(H-1)) -> pair H-1
            kn = H - 1; pv = 3;
            mp = fw ? 3 : 1;                      // q(H-1)
            mq = fw ? 1 : 3;                      // q(H-2)
        }
        if (!valid) { st = -1; kn = -1; }
        icode[ii] = (st + 1) | ((kn + 1) << 3) | (pv << 10) | (mp << 12) | (mq << 14);
    }

    const int nsw = a.inner_sweeps > 0 ? a.inner_sweeps : 30;
    const double eps = 2.220446049250313e-16;
    int gr = 0;  // rounds done (parameter buffer parity)
    for (int swp = 0; swp < nsw; ++swp) {
        if (a.inner_sweeps <= 0 && swp > 0) {
            double o = 0.0;
            for (int e = tid; e < M2 * M2; e += NT) {
                const int rr = e % M2, cc = e / M2;
                if (rr < cc) { const double v = As[rr * LD + cc]; o += 2.0 * v * v; }
            }
            o = block_sum<NT>(o, red);
            if (sqrt(o) <= eps * sqrt(fro2)) break;
        }
        for (int t = 0; t < R; ++t, ++gr) {
            const double *pc = prm0 + (gr & 1) * 4 * H;        // this round
            double *pn = prm0 + ((gr + 1) & 1) * 4 * H;        // next round
#pragma unroll
            for (int ii = 0; ii < MAXI; ++ii) {
                if (ii * NT + tid < C::NOFF) {
                    const int k1 = ikk[ii] & 255, k2 = ikk[ii] >> 8;
                    const int code = icode[ii];
                    const int sp1 = isl[ii][0], sq1 = isl[ii][1], sp2 = isl[ii][2], sq2 = isl[ii][3];
                    const double c1 = pc[k1], s1 = pc[H + k1], c2 = pc[k2], s2 = pc[H + k2];
                    const int i11 = min(sp1, sp2) * LD + max(sp1, sp2);
                    const int i12 = min(sp1, sq2) * LD + max(sp1, sq2);
                    const int i21 = min(sq1, sp2) * LD + max(sq1, sp2);
                    const int i22 = min(sq1, sq2) * LD + max(sq1, sq2);
                    double x11 = As[i11], x12 = As[i12], x21 = As[i21], x22 = As[i22];
                    // (pair-blocks holding a previous or next pivot all have
                    // d <= 2, i.e. it < 2H <= NT: only the first item)
                    if (ii == 0 && t > 0) {
                        const int st = (code & 7) - 1;
                        x11 = st == 0 ? 0.0 : x11;
                        x12 = st == 1 ? 0.0 : x12;
                        x21 = st == 2 ? 0.0 : x21;
                        x22 = st == 3 ? 0.0 : x22;
                    }
                    // left: rows p1, q1; right: columns p2, q2
                    const double y11 = c1 * x11 - s1 * x21, y21 = s1 * x11 + c1 * x21;
                    const double y12 = c1 * x12 - s1 * x22, y22 = s1 * x12 + c1 * x22;
                    const double z11 = c2 * y11 - s2 * y12, z12 = s2 * y11 + c2 * y12;
                    const double z21 = c2 * y21 - s2 * y22, z22 = s2 * y21 + c2 * y22;
                    As[i11] = z11;
                    As[i12] = z12;
                    As[i21] = z21;
                    As[i22] = z22;
                    const int kn = ((code >> 3) & 127) - 1;
                    if (ii == 0 && kn >= 0) {
                        // diagonal of the members of next round's pair kn after this
                        // round's rotation (p-member: a_pp - t a_pq, q-member: a_qq + t a_pq)
                        // and next round's parameters of pair kn
                        const int pv = (code >> 10) & 3, mp = (code >> 12) & 3, mq = (code >> 14) & 3;
                        const double piv = pv == 0 ? z11 : (pv == 1 ? z12 : (pv == 2 ? z21 : z22));
                        const int sp_ = isl[ii][0] * (mp == 0) + isl[ii][1] * (mp == 1) + isl[ii][2] * (mp == 2) +
                                        isl[ii][3] * (mp == 3);
                        const int sq_ = isl[ii][0] * (mq == 0) + isl[ii][1] * (mq == 1) + isl[ii][2] * (mq == 2) +
                                        isl[ii][3] * (mq == 3);
                        const int pp = mp < 2 ? k1 : k2, pq_ = mq < 2 ? k1 : k2;
                        const double tp = pc[2 * H + pp] * pc[3 * H + pp];
                        const double tq = pc[2 * H + pq_] * pc[3 * H + pq_];
                        const double dp = As[sp_ * (LD + 1)] + ((mp & 1) ? tp : -tp);
                        const double dq = As[sq_ * (LD + 1)] + ((mq & 1) ? tq : -tq);
                        As[sp_ * (LD + 1)] = dp;
                        As[sq_ * (LD + 1)] = dq;
                        rot_params(dp, dq, piv, pn, kn, H);
                    }
                }
                // slots advance one step along the ring (slot 0 stays)
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int sl = isl[ii][m];
                    isl[ii][m] = sl == 0 ? 0 : (sl == R ? 1 : sl + 1);
                }
            }

            // -- V_hat <- V_hat J on this thread's 8 position pairs
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = 8 * g + j;
                const double cc = pc[k], ss = pc[H + k];
                const double e = V[2 * j], o = V[2 * j + 1];
                V[2 * j] = cc * e - ss * o;
                V[2 * j + 1] = ss * e + cc * o;
            }
            // -- one ring step of the column content
            {
                const double from_right = __shfl_down(V[0], 1, G);
                const double from_left = __shfl_up(V[15], 1, G);
                const double e0 = V[0], e1 = V[2], o7 = V[15];
#pragma unroll
                for (int j = 0; j < 7; ++j) V[2 * j] = V[2 * j + 2];
                V[14] = (g < G - 1) ? from_right : o7;
#pragma unroll
                for (int j = 7; j > 0; --j) V[2 * j + 1] = V[2 * j - 1];
                V[1] = (g > 0) ? from_left : e1;
                if (g == 0) V[0] = e0;
            }
            __syncthreads();
        }
        // end of sweep: clear the last round's pivots (the diagonal is current;
        // positions equal indices again after m2 - 1 ring steps)
        if (tid < H) {
            const int up = slot_p(tid, R - 1, M2), uq = slot_q(tid, R - 1, M2);
            As[min(up, uq) * LD + max(up, uq)] = 0.0;
        }
        __syncthreads();
    }

    // ---- results ------------------------------------------------------------
    if (MODE == SUB_PLAIN) {
        double *vo = a.vout + (size_t)pr * M2 * M2;
#pragma unroll
        for (int x = 0; x < 16; ++x) vo[(size_t)(16 * g + x) * M2 + r] = V[x];
        double *dd = a.dout + (size_t)pr * M2 * M2;
        for (int e = tid; e < M2 * M2; e += NT) {
            const int u = slot_of(e % M2, M2), w = slot_of(e / M2, M2);
            dd[e] = As[min(u, w) * LD + max(u, w)];
        }
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
        if (MODE == SUB_EIG) {
            // A([I,J],[I,J]) <- D_hat (pointers recomputed: not kept live through the sweeps)
            const int I = a.pairs[2 * pr], J = a.pairs[2 * pr + 1];
            const size_t oii = ublk(I, I) * (size_t)(B * B), ojj = ublk(J, J) * (size_t)(B * B),
                         oij = ublk(I, J) * (size_t)(B * B);
            for (int e = tid; e < M2 * M2; e += NT) {
                const int rr = e % M2, cc = e / M2;
                const int u = slot_of(rr, M2), w = slot_of(cc, M2);
                const double v = As[min(u, w) * LD + max(u, w)];
                size_t off;
                if (cc < B) {
                    if (rr >= B) continue;
                    off = oii + cc * B + rr;
                } else if (rr < B) {
                    off = oij + (cc - B) * B + rr;
                } else {
                    off = ojj + (cc - B) * B + (rr - B);
                }
                if (a.ablk32) a.ablk32[off] = (float)v;
                else a.ablk[off] = v;
            }
        }
    }
}

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
static void launch_sub_m(const SubArgs &a, hipStream_t s) {
    switch (a.m2) {
        case 32: launch_sub_t<32, MODE>(a, s); break;
        case 64: launch_sub_t<64, MODE>(a, s); break;
        case 128: launch_sub_t<128, MODE>(a, s); break;
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
