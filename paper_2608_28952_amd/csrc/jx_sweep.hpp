// jx_sweep.hpp -- round-robin scalar Jacobi held in LDS, shared by the
// subproblem solver (k_subproblem.hip) and the batched solver (k_batched.hip).
//
// Scalar rotation (symmetric Schur form): with theta = (a_qq - a_pp) / (2 a_pq),
// t = sgn(theta) / (|theta| + sqrt(1 + theta^2)), c = 1 / sqrt(1 + t^2), s = t c,
// the plane rotation J = [[c, s], [-s, c]] on (p, q) gives J^T A J a zero
// (p, q) entry and diagonal a_pp - t a_pq, a_qq + t a_pq (Golub & Van Loan
// §8.5.2).
//
// Data placement of the scalar sweeps
//   * A: LDS, upper triangle, row stride m2.  Index x sits at slot pi(x) =
//     ring order (pi(0) = 0, pi(x) = 1 + ring index of x): in round t the
//     members of consecutive pairs sit at consecutive slots, so the lanes of a
//     wave touch addresses with odd strides (m2 + 1, m2 - 1): no bank conflicts.
//   * V: registers; thread (r, g) holds row r of V at P consecutive
//     positions P g .. P g + P - 1.  Positions are paired (2k, 2k+1) every round; after a
//     round the column content moves one step along the ring
//     1 <- 2 <- 4 <- ... <- m2-2 <- m2-1 <- m2-3 <- ... <- 3 <- 1 (0 stays), so
//     that every index pair meets once per sweep; two values per thread cross
//     to the neighbouring lane.  After m2 - 1 rounds positions equal indices.
//   * Rotation parameters (c, s and the diagonal shift t a_pq per pair): LDS,
//     two rounds.  The pivot a_pq of a round becomes zero and is not written:
//     in the next round it lies in a known pair-block, which reads it as zero.
//     The pair-blocks that compute the next round's pivots also update the two
//     diagonal entries of that pair and write the next round's parameters, so
//     a round needs one barrier.
//   * A round is bound by VALU issue (every lane of a wave executes every
//     instruction): the next round's parameters are computed only in the
//     waves that hold producers (a wave-uniform branch).
#pragma once

#include "jx_common.hpp"

namespace jx {

// ---------------------------------------------------------------------------
// Ring bookkeeping
// ---------------------------------------------------------------------------

// Ring of positions 1 .. m2-1 in the order their content moves.
__host__ __device__ constexpr __forceinline__ int ring_at(int i, int m2) {
    if (i == 0) return 1;
    if (i < m2 / 2) return 2 * i;
    return 2 * m2 - 1 - 2 * i;
}
__host__ __device__ constexpr __forceinline__ int ring_index(int x, int m2) {
    if (x == 1) return 0;
    if ((x & 1) == 0) return x >> 1;
    return (2 * m2 - 1 - x) >> 1;
}
// LDS slot of index x (its place along the ring; 0 stays 0).
__host__ __device__ constexpr __forceinline__ int slot_of(int x, int m2) { return x == 0 ? 0 : 1 + ring_index(x, m2); }
// Slots of the members of pair k in round t of a sweep (t < m2 - 1):
// position 2k holds slot 1 + (k + t) mod (m2-1) (position 0: slot 0),
// position 2k+1 holds slot 1 + (t - k) mod (m2-1).
__host__ __device__ constexpr __forceinline__ int slot_p(int k, int t, int m2) {
    if (k == 0) return 0;
    int i = k + t;
    if (i >= m2 - 1) i -= m2 - 1;
    return 1 + i;
}
__host__ __device__ constexpr __forceinline__ int slot_q(int k, int t, int m2) {
    int i = (k == 0) ? t : t - k;
    if (i < 0) i += m2 - 1;
    return 1 + i;
}
// Index found at position x in round t.
__host__ __device__ constexpr __forceinline__ int index_at(int x, int t, int m2) {
    if (x == 0) return 0;
    int i = ring_index(x, m2) + t;
    if (i >= m2 - 1) i -= m2 - 1;
    return ring_at(i, m2);
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

// Orders the LDS accesses of one wave (stores of some lanes, loads of others):
// nothing moves across.  Wavefront-scope fences: a wave's LDS operations are
// performed in issue order, so no wait for outstanding operations is needed
// (the compiler emits none at this scope).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool WAVE>
__device__ __forceinline__ void group_sync() {
    if constexpr (WAVE) wave_lds_sync();
    else __syncthreads();
}

// 1/x and 1/sqrt(x) from the hardware seeds (v_rcp_f64, v_rsq_f64) and two
// Newton steps each: y <- y + y (1 - x y) and y <- y + y (1 - x y^2) / 2 (the
// error squares every step), a few ulp for normal positive x.
__device__ __forceinline__ double rcp_nr(double x) {
    double y = __builtin_amdgcn_rcp(x);
    double e = fma(-x, y, 1.0);
    y = fma(y, e, y);
    e = fma(-x, y, 1.0);
    return fma(y, e, y);
}
__device__ __forceinline__ double rsq_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double r = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, r, y);
    r = fma(-x * y, y, 1.0);
    return fma(0.5 * y, r, y);
}

// Rotation (c, s, t) that zeroes a_pq, without branches.  With d = a_qq - a_pp,
// e = 2 a_pq, theta = d / e and r = sqrt(d^2 + e^2), the smaller root of
// t^2 + 2 theta t = 1 is t = sgn(theta) / (|theta| + sqrt(1 + theta^2)) =
// sgn(theta) |e| / (|d| + r) (sgn(0) = +1), c = 1 / sqrt(1 + t^2), s = t c.
// d and e are first scaled by one power of two (t depends only on their
// ratio) so that the larger magnitude lies in [1/2, 1): d^2 + e^2 then lies in
// [1/4, 2), with no overflow or harmful underflow at any input magnitude.  One
// reciprocal and two reciprocal square roots.
__device__ __forceinline__ void rot_cst(double app, double aqq, double apq, double &c, double &s, double &t) {
    const double d0 = aqq - app, e0 = 2.0 * apq;
    int k;
    (void)frexp(fmax(fabs(d0), fabs(e0)), &k);
    const double d = ldexp(d0, -k), e = ldexp(e0, -k);
    const double x = fma(d, d, e * e);
    const double r = x * rsq_nr(x);
    double tt = fabs(e) * rcp_nr(fabs(d) + r);
    tt = (d != 0.0 && ((d < 0.0) != (e < 0.0))) ? -tt : tt;
    const double cc = rsq_nr(fma(tt, tt, 1.0));
    const bool none = apq == 0.0;
    c = none ? 1.0 : cc;
    s = none ? 0.0 : tt * cc;
    t = none ? 0.0 : tt;
}

// Rotation parameters of pair k into the parameter arrays: c, s and the
// diagonal shift t a_pq (a_pp -= t a_pq, a_qq += t a_pq).
__device__ __forceinline__ void rot_params(double app, double aqq, double apq, double *prm, int k, int H) {
    double c, s, t;
    rot_cst(app, aqq, apq, c, s, t);
    prm[k] = c;
    prm[H + k] = s;
    prm[2 * H + k] = t * apq;
}

// Value of the next / previous lane within groups of G consecutive lanes (the
// group's last / first lane gets an unspecified value).  G = 2, 4: DPP quad
// permutes, which stay in the VALU (no LDS round trip); otherwise shuffles.
template <int CTRL>
__device__ __forceinline__ double dpp_quad_t(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <int G>
__device__ __forceinline__ double lane_next(double v) {
    if constexpr (G == 2) return dpp_quad_t<(1 | 1 << 2 | 3 << 4 | 3 << 6)>(v);  // quad_perm [1,1,3,3]
    else if constexpr (G == 4) return dpp_quad_t<(1 | 2 << 2 | 3 << 4 | 3 << 6)>(v);  // [1,2,3,3]
    else return __shfl_down(v, 1, G);
}
template <int G>
__device__ __forceinline__ double lane_prev(double v) {
    if constexpr (G == 2) return dpp_quad_t<(0 | 0 << 2 | 2 << 4 | 2 << 6)>(v);  // quad_perm [0,0,2,2]
    else if constexpr (G == 4) return dpp_quad_t<(0 | 0 << 2 | 1 << 4 | 2 << 6)>(v);  // [0,0,1,2]
    else return __shfl_up(v, 1, G);
}

// Item it of a sweep (a pair-block between pairs k1 and k2, or padding when
// it >= H (H - 1) / 2): pairs packed k1 | k2 << 8, the four slots in round 0
// and the code of its stale and next-round pivot roles (see scalar_sweeps).
__host__ __device__ constexpr void sweep_item(int it, int M2, int &ikk, int *isl, int &icode) {
    const int H = M2 / 2, NOFF = H * (H - 1) / 2;
    int k1 = 0, d = 1;
    if (it < H * (H / 2 - 1)) { d = it / H + 1; k1 = it - (d - 1) * H; }
    else { d = H / 2; k1 = it - H * (H / 2 - 1); }
    int k2 = k1 + d;
    if (k2 >= H) k2 -= H;
    const bool valid = it < NOFF;
    if (!valid) { k1 = 0; k2 = 1; }
    ikk = k1 | (k2 << 8);
    isl[0] = slot_p(k1, 0, M2);
    isl[1] = slot_q(k1, 0, M2);
    isl[2] = slot_p(k2, 0, M2);
    isl[3] = slot_q(k2, 0, M2);
    const int lo = k1 < k2 ? k1 : k2, hi = k1 < k2 ? k2 : k1;
    const bool fw = (k1 == lo);
    // the previous round's pivot of pair k lies at (p of k-1, q of k+1) for
    // 2 <= k <= H-2; pair 0: (p0, q1); pair 1: (q0, q2); pair H-1:
    // (p(H-2), p(H-1))
    int st = -1;
    if (hi - lo == 2 && lo >= 1) st = fw ? 1 : 2;
    else if (lo == 0 && hi == 2) st = 3;
    else if (lo == 0 && hi == 1) st = fw ? 1 : 2;
    else if (lo == H - 2 && hi == H - 1) st = 0;
    // the next round's pivot of pair lo + 1 is (q_lo, p_hi); of pair 0,
    // (p0, p1); of pair H-1, (q(H-2), q(H-1))
    int kn = -1, pv = 0, mp = 0, mq = 0;
    if (hi - lo == 2) {
        kn = lo + 1; pv = fw ? 2 : 1; mp = fw ? 2 : 0; mq = fw ? 1 : 3;
    } else if (lo == 0 && hi == 1) {
        kn = 0; pv = 0; mp = fw ? 0 : 2; mq = fw ? 2 : 0;
    } else if (lo == H - 2 && hi == H - 1) {
        kn = H - 1; pv = 3; mp = fw ? 3 : 1; mq = fw ? 1 : 3;
    }
    if (!valid) { st = -1; kn = -1; }
    icode = (st + 1) | ((kn + 1) << 3) | (pv << 10) | (mp << 12) | (mq << 14);
}

// Next slot along the ring (slot 0 stays).
__host__ __device__ constexpr __forceinline__ int slot_next(int sl, int R) { return sl == 0 ? 0 : (sl == R ? 1 : sl + 1); }

// LDS addresses of a whole sweep, per round and thread, for one wave per
// problem: the four entries of each item (upper-triangle index min * m2 + max
// of its slots) and the producer's two diagonal entries, as 16-bit halves.
// Computed at compile time; a round then reads its addresses with one vector
// load (prefetched a round ahead) instead of advancing slots and recomputing
// addresses in the VALU.
template <int M2, int NT>
struct SweepTable {
    static constexpr int H = M2 / 2, R = M2 - 1, NOFF = H * (H - 1) / 2, MAXI = (NOFF + NT - 1) / NT;
    static_assert(MAXI == 2, "layout: two items per thread");
    unsigned int item[R][NT][4];  // item ii entry m: half (2 ii + m / 2), bits 16 (m & 1)
    unsigned int prod[R][NT];     // diagonal of the next-round pair's p and q member
};
template <int M2, int NT>
constexpr SweepTable<M2, NT> make_sweep_table() {
    using T = SweepTable<M2, NT>;
    T tb{};
    for (int tid = 0; tid < NT; ++tid) {
        int ikk[T::MAXI] = {}, isl[T::MAXI][4] = {}, icode[T::MAXI] = {};
        for (int ii = 0; ii < T::MAXI; ++ii) sweep_item(tid + ii * NT, M2, ikk[ii], isl[ii], icode[ii]);
        const int mp = (icode[0] >> 12) & 3, mq = (icode[0] >> 14) & 3;
        for (int t = 0; t < T::R; ++t) {
            for (int ii = 0; ii < T::MAXI; ++ii) {
                const int a = isl[ii][0], b = isl[ii][1], c = isl[ii][2], d = isl[ii][3];
                const int e[4] = {(a < c ? a : c) * M2 + (a < c ? c : a), (a < d ? a : d) * M2 + (a < d ? d : a),
                                  (b < c ? b : c) * M2 + (b < c ? c : b), (b < d ? b : d) * M2 + (b < d ? d : b)};
                tb.item[t][tid][2 * ii] = (unsigned)e[0] | ((unsigned)e[1] << 16);
                tb.item[t][tid][2 * ii + 1] = (unsigned)e[2] | ((unsigned)e[3] << 16);
            }
            const int spn = isl[0][mp], sqn = isl[0][mq];
            tb.prod[t][tid] = (unsigned)(spn * (M2 + 1)) | ((unsigned)(sqn * (M2 + 1)) << 16);
            for (int ii = 0; ii < T::MAXI; ++ii)
                for (int m = 0; m < 4; ++m) isl[ii][m] = slot_next(isl[ii][m], T::R);
        }
    }
    return tb;
}

// Hand-off of a sweep's rotations to another wave of the workgroup, which
// accumulates V while the sweep runs on.  The (c, s) of global round n sit in
// ring slot n mod VR_DEPTH; sdone counts the rounds whose parameters are in
// the ring, vdone the rounds the follower has applied.  Both counters only
// grow.  Waits are bounded (VR_SPIN polls, thousands of times the longest
// legitimate wait): a wait that runs out gives up rather than hang and sets
// *fail, and the kernel then poisons its output with NaN (reported as a
// non-finite iterate) instead of returning wrong numbers.
constexpr int VR_DEPTH = 8;
constexpr int VR_SPIN = 1 << 16;
struct VRing {
    double *ring;  // VR_DEPTH x (c[H], s[H])
    int *sdone;
    int *vdone;
    int base;      // global round number of this sweep's round 0
    int *fail;     // set when a wait runs out
    int spin;      // polls per wait
};
__device__ __forceinline__ int lds_load_acquire(int *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_store_release(int *p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// Wait until *p >= v (at most `spin` polls; *fail = 1 when they run out).
__device__ __forceinline__ void lds_wait_geq(int *p, int v, int *fail, int spin) {
    for (int it = 0; it < spin; ++it) {
        if (lds_load_acquire(p) >= v) return;
        __builtin_amdgcn_s_sleep(1);
    }
    lds_store_release(fail, 1);
}
// The same wait with the last value read kept in `seen`: no load while that
// value already satisfies it (the counter only grows, and the acquire that
// read it orders everything after it).
__device__ __forceinline__ void lds_wait_geq_seen(int *p, int v, int &seen, int *fail, int spin) {
    if (seen >= v) return;
    for (int it = 0; it < spin; ++it) {
        seen = lds_load_acquire(p);
        if (seen >= v) return;
        __builtin_amdgcn_s_sleep(1);
    }
    lds_store_release(fail, 1);
}

// ---------------------------------------------------------------------------
// Round-robin scalar Jacobi on an m2 x m2 matrix held in LDS (slot order)
// ---------------------------------------------------------------------------
// NT threads (tid 0 .. NT-1) cooperate, each holding P = m2^2 / NT positions
// of one row of V; WAVE: the group is one wave (wave-level ordering instead
// of workgroup barriers).  Runs `nsw` sweeps, or (conv) up to 30 sweeps until
// off <= eps sqrt(fro2).  V receives this thread's part of the accumulated
// rotation (row r = tid / G, columns P g .. P g + P - 1, g = tid mod G,
// G = m2 / P); position space equals index space at the end of a sweep.
template <int M2, int NT, bool WAVE, bool TBL = false, bool VOUT = false>
__device__ void scalar_sweeps(double *As, double *prm0, double *red, int tid, int nsw, bool conv, double fro2,
                              double *V, const SweepTable<M2, NT> *tbl = nullptr, VRing vr = VRing{}) {
    // VOUT: V is not accumulated here; every round's (c, s) goes to the ring
    // for a follower wave (follow_sweep) instead.
    static_assert(!VOUT || (WAVE && TBL), "hand-off: one wave per problem, table addressing");
    constexpr int H = M2 / 2, P = M2 * M2 / NT, G = M2 / P, LD = M2, R = M2 - 1;
    constexpr int NOFF = H * (H - 1) / 2;  // pair-blocks between different pairs
    static_assert(P >= 4 && P % 2 == 0 && M2 % P == 0, "whole position pairs per thread");
    const int r = tid / G, g = tid - (tid / G) * G;
    if constexpr (!VOUT) {
#pragma unroll
        for (int x = 0; x < P; ++x) V[x] = (r == P * g + x) ? 1.0 : 0.0;
    }

    int vseen = -(1 << 30);  // last follower count read (VOUT)
    // parameters of the first round
    if (tid < H) {
        const int up = slot_p(tid, 0, M2), uq = slot_q(tid, 0, M2);
        rot_params(As[up * (LD + 1)], As[uq * (LD + 1)], As[min(up, uq) * LD + max(up, uq)], prm0, tid, H);
        if constexpr (VOUT) {
            double *rb = vr.ring + (vr.base & (VR_DEPTH - 1)) * 2 * H;
            lds_wait_geq_seen(vr.vdone, vr.base + 1 - VR_DEPTH, vseen, vr.fail, vr.spin);
            rb[tid] = prm0[tid];
            rb[H + tid] = prm0[H + tid];
        }
    }
    group_sync<WAVE>();
    if constexpr (VOUT) lds_store_release(vr.sdone, vr.base + 1);

    // This thread's pair-blocks (fixed for all rounds); their slots advance by
    // one per round along 1 .. m2-1 (slot 0 stays), kept in registers.  Entry
    // codes: 0 = (p1,p2), 1 = (p1,q2), 2 = (q1,p2), 3 = (q1,q2); member codes:
    // 0 = p1, 1 = q1, 2 = p2, 3 = q2.  Packed: ikk = k1 | k2 << 8; icode =
    // (stale + 1) | (kn + 1) << 3 | pivot entry << 10 | p' member << 12 |
    // q' member << 14.
    constexpr int MAXI = (NOFF + NT - 1) / NT;
    static_assert(2 * H <= NT, "pivot pair-blocks must be first items");
    int ikk[MAXI], isl[MAXI][4], icode[MAXI];
#pragma unroll
    for (int ii = 0; ii < MAXI; ++ii) sweep_item(tid + ii * NT, M2, ikk[ii], isl[ii], icode[ii]);

    // The producer items (distance <= 2, the first item of threads < 2H) fill
    // whole waves: a wave-uniform branch keeps the parameter work out of the others.
    const bool prod_wave = WAVE || __builtin_amdgcn_readfirstlane(tid) < 2 * H;
    // One wave per problem: the round is kept free of branches (lanes without
    // a store target write a never-read lower-triangle entry of their own), so
    // the scheduler can fill the parameter chain's latency with the rest of
    // the round.
    const int dum = (M2 - 1 - (tid & 63) / H) * LD + (tid & 63) % H;
    const double eps = 2.220446049250313e-16;
    const int cap = conv ? 30 : nsw;
    int gr = 0;  // rounds done (parameter buffer parity)
    uint4 cur = {0, 0, 0, 0};  // table: this round's item addresses and producer diagonal
    unsigned int curp = 0;
    if constexpr (TBL) {
        cur = *reinterpret_cast<const uint4 *>(tbl->item[0][tid]);
        curp = tbl->prod[0][tid];
    }
    for (int swp = 0; swp < cap; ++swp) {
        if (conv && swp > 0) {
            double o = 0.0;
            for (int e = tid; e < M2 * M2; e += NT) {
                const int rr = e % M2, cc = e / M2;
                if (rr < cc) { const double v = As[rr * LD + cc]; o += 2.0 * v * v; }
            }
            if constexpr (WAVE) o = wave_sum(o);
            else o = block_sum<NT>(o, red);
            if (sqrt(o) <= eps * sqrt(fro2)) break;
        }
        for (int t = 0; t < R; ++t, ++gr) {
            const double *pc = prm0 + (gr & 1) * 4 * H;  // this round
            double *pn = prm0 + ((gr + 1) & 1) * 4 * H;  // next round
            // ---- every load of the round first: the compiler keeps LDS loads
            //      behind earlier stores that might alias, so loads issued after
            //      a store would cost one LDS round trip each
            double cs[MAXI][4], xv[MAXI][4];
            int ia[MAXI][4];
            int dpa = 0, dqa = 0;  // producer's diagonal entries
            if constexpr (TBL) {   // this round's addresses; fetch the next round's
                const uint4 ta = cur;
                dpa = (int)(curp & 0xffff);
                dqa = (int)(curp >> 16);
                const int tn = t + 1 < R ? t + 1 : 0;
                cur = *reinterpret_cast<const uint4 *>(tbl->item[tn][tid]);
                curp = tbl->prod[tn][tid];
                const unsigned int w[4] = {ta.x, ta.y, ta.z, ta.w};
#pragma unroll
                for (int ii = 0; ii < MAXI; ++ii)
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const unsigned int h = w[2 * ii + m / 2];
                        ia[ii][m] = (int)((m & 1) ? (h >> 16) : (h & 0xffff));
                    }
            }
#pragma unroll
            for (int ii = 0; ii < MAXI; ++ii) {
                const int k1 = ikk[ii] & 255, k2 = ikk[ii] >> 8;
                cs[ii][0] = pc[k1];
                cs[ii][1] = pc[H + k1];
                cs[ii][2] = pc[k2];
                cs[ii][3] = pc[H + k2];
                if constexpr (!TBL) {
                    const int sp1 = isl[ii][0], sq1 = isl[ii][1], sp2 = isl[ii][2], sq2 = isl[ii][3];
                    ia[ii][0] = min(sp1, sp2) * LD + max(sp1, sp2);
                    ia[ii][1] = min(sp1, sq2) * LD + max(sp1, sq2);
                    ia[ii][2] = min(sq1, sp2) * LD + max(sq1, sp2);
                    ia[ii][3] = min(sq1, sq2) * LD + max(sq1, sq2);
                }
#pragma unroll
                for (int m = 0; m < 4; ++m) xv[ii][m] = As[ia[ii][m]];
            }
            // producer operands (first item of the producer waves; diagonal
            // entries are written by their producer alone, never by an item)
            const int code = icode[0];
            const int kn = ((code >> 3) & 127) - 1;
            const int pv = (code >> 10) & 3, mp = (code >> 12) & 3, mq = (code >> 14) & 3;
            double dpo = 0.0, dqo = 0.0, tp = 0.0, tq = 0.0;
            if (prod_wave) {
                const int k1 = ikk[0] & 255, k2 = ikk[0] >> 8;
                if constexpr (!TBL) {
                    const int sp1 = isl[0][0], sq1 = isl[0][1], sp2 = isl[0][2], sq2 = isl[0][3];
                    // two-level selects on single bits stay selects
                    dpa = ((mp & 2) ? ((mp & 1) ? sq2 : sp2) : ((mp & 1) ? sq1 : sp1)) * (LD + 1);
                    dqa = ((mq & 2) ? ((mq & 1) ? sq2 : sp2) : ((mq & 1) ? sq1 : sp1)) * (LD + 1);
                }
                dpo = As[dpa];
                dqo = As[dqa];
                tp = pc[2 * H + (mp < 2 ? k1 : k2)];
                tq = pc[2 * H + (mq < 2 ? k1 : k2)];
                // the previous round's pivot lies in this block: read as zero
                const int st0 = t > 0 ? (code & 7) - 1 : -1;
#pragma unroll
                for (int m = 0; m < 4; ++m) xv[0][m] = st0 == m ? 0.0 : xv[0][m];
            }
            double vc[P / 2], vs[P / 2];  // this thread's position pairs
#pragma unroll
            for (int j = 0; j < P / 2; ++j) {
                vc[j] = VOUT ? 0.0 : pc[(P / 2) * g + j];
                vs[j] = VOUT ? 0.0 : pc[H + (P / 2) * g + j];
            }
            // rounds <= t are in the ring (the previous round's stores are
            // complete once this round's loads are: the release waits for
            // nothing the rotation below would not wait for)
            if constexpr (VOUT) {
                if (t > 0) lds_store_release(vr.sdone, vr.base + t + 1);
            }

            // ---- rotate the pair-blocks: left rows p1, q1; right columns p2, q2
            double piv = 0.0;
#pragma unroll
            for (int ii = 0; ii < MAXI; ++ii) {
                const double c1 = cs[ii][0], s1 = cs[ii][1], c2 = cs[ii][2], s2 = cs[ii][3];
                const double x11 = xv[ii][0], x12 = xv[ii][1], x21 = xv[ii][2], x22 = xv[ii][3];
                const double y11 = c1 * x11 - s1 * x21, y21 = s1 * x11 + c1 * x21;
                const double y12 = c1 * x12 - s1 * x22, y22 = s1 * x12 + c1 * x22;
                const double z11 = c2 * y11 - s2 * y12, z12 = s2 * y11 + c2 * y12;
                const double z21 = c2 * y21 - s2 * y22, z22 = s2 * y21 + c2 * y22;
                if constexpr (WAVE) {
                    const bool ok = ii * NT + tid < NOFF;
                    As[ok ? ia[ii][0] : dum] = z11;
                    As[ok ? ia[ii][1] : dum] = z12;
                    As[ok ? ia[ii][2] : dum] = z21;
                    As[ok ? ia[ii][3] : dum] = z22;
                } else if (ii * NT + tid < NOFF) {
                    As[ia[ii][0]] = z11;
                    As[ia[ii][1]] = z12;
                    As[ia[ii][2]] = z21;
                    As[ia[ii][3]] = z22;
                }
                if (ii == 0) piv = (pv & 2) ? ((pv & 1) ? z22 : z21) : ((pv & 1) ? z12 : z11);
            }

            // ---- next round's parameters: diagonal of pair kn after this
            //      round's rotation (p-member a_pp - t a_pq, q-member
            //      a_qq + t a_pq), then (c, s, t a_pq); computed by the whole
            //      wave, stored by the producers
            if (prod_wave) {
                const double dp = dpo + ((mp & 1) ? tp : -tp);
                const double dq = dqo + ((mq & 1) ? tq : -tq);
                double cn, sn, tn;
                rot_cst(dp, dq, piv, cn, sn, tn);
                if constexpr (WAVE) {
                    const bool ok = kn >= 0;
                    As[ok ? dpa : dum] = dp;
                    As[ok ? dqa : dum] = dq;
                    double *const pd = ok ? pn + kn : As + dum;
                    pd[0] = cn;
                    pd[ok ? H : 0] = sn;
                    pd[ok ? 2 * H : 0] = tn * piv;
                    if constexpr (VOUT) {  // next round's slot, once the follower is done with it
                        const int nr = vr.base + t + 1;
                        double *const rd = ok ? vr.ring + (nr & (VR_DEPTH - 1)) * 2 * H + kn : As + dum;
                        lds_wait_geq_seen(vr.vdone, nr + 1 - VR_DEPTH, vseen, vr.fail, vr.spin);
                        rd[0] = cn;
                        rd[ok ? H : 0] = sn;
                    }
                } else if (kn >= 0) {
                    As[dpa] = dp;
                    As[dqa] = dq;
                    pn[kn] = cn;
                    pn[H + kn] = sn;
                    pn[2 * H + kn] = tn * piv;
                }
            }
            if constexpr (!TBL) {
#pragma unroll
                for (int ii = 0; ii < MAXI; ++ii)
#pragma unroll
                    for (int m = 0; m < 4; ++m) isl[ii][m] = slot_next(isl[ii][m], R);
            }

            // ---- V <- V J on this thread's P/2 position pairs, then one ring step
            if constexpr (!VOUT) {
#pragma unroll
                for (int j = 0; j < P / 2; ++j) {
                    const double e = V[2 * j], o = V[2 * j + 1];
                    V[2 * j] = vc[j] * e - vs[j] * o;
                    V[2 * j + 1] = vs[j] * e + vc[j] * o;
                }
                const double from_right = lane_next<G>(V[0]);
                const double from_left = lane_prev<G>(V[P - 1]);
                const double e0 = V[0], e1 = V[2], olast = V[P - 1];
#pragma unroll
                for (int j = 0; j < P / 2 - 1; ++j) V[2 * j] = V[2 * j + 2];
                V[P - 2] = (g < G - 1) ? from_right : olast;
#pragma unroll
                for (int j = P / 2 - 1; j > 0; --j) V[2 * j + 1] = V[2 * j - 1];
                V[1] = (g > 0) ? from_left : e1;
                if (g == 0) V[0] = e0;
            }
            group_sync<WAVE>();
            // (the next round publishes this round's ring slot; the last
            // round's "next" parameters are not published: the next sweep
            // writes its round 0 itself)
        }
        // end of sweep: clear the last round's pivots (the diagonal is current)
        if (tid < H) {
            const int up = slot_p(tid, R - 1, M2), uq = slot_q(tid, R - 1, M2);
            As[min(up, uq) * LD + max(up, uq)] = 0.0;
        }
        group_sync<WAVE>();
    }
}

// The follower of a sweep run with VOUT: applies each round's rotations to
// V (same layout and ring steps as scalar_sweeps with one wave, P = m2^2 / 64
// positions of one row per thread) as soon as the ring holds them.  V starts
// as the identity; after the m2 - 1 rounds positions equal indices.
template <int M2>
__device__ void follow_sweep(const VRing &vr, int lane, double *V) {
    constexpr int NT = 64, H = M2 / 2, P = M2 * M2 / NT, G = M2 / P, R = M2 - 1;
    const int r = lane / G, g = lane - (lane / G) * G;
#pragma unroll
    for (int x = 0; x < P; ++x) V[x] = (r == P * g + x) ? 1.0 : 0.0;
    for (int t = 0; t < R; ++t) {
        const int n = vr.base + t;
        lds_wait_geq(vr.sdone, n + 1, vr.fail, vr.spin);
        const double *rb = vr.ring + (n & (VR_DEPTH - 1)) * 2 * H + (P / 2) * g;
        double vc[P / 2], vs[P / 2];
#pragma unroll
        for (int j = 0; j < P / 2; ++j) {
            vc[j] = rb[j];
            vs[j] = rb[H + j];
        }
#pragma unroll
        for (int j = 0; j < P / 2; ++j) {
            const double e = V[2 * j], o = V[2 * j + 1];
            V[2 * j] = vc[j] * e - vs[j] * o;
            V[2 * j + 1] = vs[j] * e + vc[j] * o;
        }
        // this round's slot is read (the values are in registers): free it
        lds_store_release(vr.vdone, n + 1);
        const double from_right = lane_next<G>(V[0]);
        const double from_left = lane_prev<G>(V[P - 1]);
        const double e0 = V[0], e1 = V[2], olast = V[P - 1];
#pragma unroll
        for (int j = 0; j < P / 2 - 1; ++j) V[2 * j] = V[2 * j + 2];
        V[P - 2] = (g < G - 1) ? from_right : olast;
#pragma unroll
        for (int j = P / 2 - 1; j > 0; --j) V[2 * j + 1] = V[2 * j - 1];
        V[1] = (g > 0) ? from_left : e1;
        if (g == 0) V[0] = e0;
    }
}

}  // namespace jx
