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
#include <algorithm>
#include <cstdlib>

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
constexpr int RING = VR_DEPTH * 32;                // per pair problem: rotations handed to the V role
constexpr size_t LDS_BYTES = sizeof(double) * ((size_t)AP + 4 * SW + 16 + 4 * RING) + 9 * sizeof(int);
__device__ __forceinline__ int pk(int i, int j) {  // i <= j
    return i * (2 * M2 - 1 - i) / 2 + j;
}
__device__ __forceinline__ int pkm(int i, int j) { return i <= j ? pk(i, j) : pk(j, i); }
}  // namespace tl

// Addresses of the 32 x 32 pair problems' sweeps (compile-time table).
__device__ const SweepTable<32, 64> kSweep32 = make_sweep_table<32, 64>();

// Cross rotations of a 32 x 32 pair problem of blocks ba (local indices
// 0..15) and bb (16..31) whose within-block pairs were rotated in an earlier
// block round of the same inner sweep: 16 rounds, round sh pairs k with
// q(k, sh) = 16 + (k + sh) mod 16, so that each (ba, bb) index pair is
// rotated once.  One wave.  S: upper triangle, entry (a, b), a <= b, at
// S[32 a + (a + b) mod 32] (rows rotated by their index, so that the lanes
// of a round spread over the LDS banks).  prm: two rounds of (c[16], s[16], shift[16]), shift = t a_pq
// (a_pp -= shift, a_qq += shift).  Every round's (c, s) go to the ring for
// the follower (follow_cross); the round's 120 pair-blocks (k1 < k2: entries
// (p1, p2), (p1, q2), (q1, p2), (q1, q2)) are disjoint, two per lane.  Lanes
// 0..15 own the pair-blocks that hold the next round's pivots ((k, k + 1):
// entry (p1, q2); (0, 15): entry (q1, p2)), update the two diagonal entries
// of that pivot and write the next round's parameters, so a round needs one
// wave-level ordering.
__device__ __forceinline__ int cross_q(int k, int sh) { return 16 + ((k + sh) & 15); }
__device__ __forceinline__ int cross_at(int a, int b) { return 32 * (a < b ? a : b) + ((a + b) & 31); }
__device__ void cross_sweep(double *S, double *prm, int lane, const VRing &vr) {
    constexpr int H = 16, NI = 120;
    int vseen = -(1 << 30);  // last follower count read
    // parameters of round 0: pivots (k, 16 + k); the ring gets (c, s) from
    // registers (a load after the acquiring wait could not be forwarded)
    if (lane < H) {
        const int p = lane, q = cross_q(lane, 0);
        const double apq = S[cross_at(p, q)];
        double c, s, t;
        rot_cst(S[cross_at(p, p)], S[cross_at(q, q)], apq, c, s, t);
        prm[lane] = c;
        prm[H + lane] = s;
        prm[2 * H + lane] = t * apq;
        double *rb = vr.ring + (vr.base & (VR_DEPTH - 1)) * 2 * H;
        lds_wait_geq_seen(vr.vdone, vr.base + 1 - VR_DEPTH, vseen, vr.fail, vr.spin);
        rb[lane] = c;
        rb[H + lane] = s;
    }
    wave_lds_sync();
    lds_store_release(vr.sdone, vr.base + 1);

    // this lane's pair-blocks it = lane, lane + 64: 0..14 (k, k+1), 15 (0, 15),
    // then distance d = 2 .. 14 in order of d and k1
    int k1[2], k2[2];
    bool ok[2];
#pragma unroll
    for (int ii = 0; ii < 2; ++ii) {
        const int it = lane + 64 * ii;
        ok[ii] = it < NI;
        int a = 0, b = 1;
        if (it < 15) { a = it; b = it + 1; }
        else if (it == 15) { a = 0; b = 15; }
        else if (it < NI) {
            int r = it - 16, d = 2;
            while (r >= H - d) { r -= H - d; ++d; }
            a = r; b = r + d;
        }
        k1[ii] = a;
        k2[ii] = b;
    }
    const bool prod = lane < H;  // item 0 holds the pivot of pair `lane` for the next round
    const int kn = (lane + 1) & 15, lp = lane & 15;
    // LDS addresses: entry (a, b) of each item and the producer's (p, p)
    // stay; the others move with the round and are computed a round ahead,
    // while that round's loads are in flight, so that each round's loads
    // issue at its start
    int a00[2];
#pragma unroll
    for (int ii = 0; ii < 2; ++ii) a00[ii] = cross_at(k1[ii], k2[ii]);
    const int adp = cross_at(lp, lp);
    auto round_ad = [&](int sh, int (&ad)[2][3], int &adq, int &adz) {
#pragma unroll
        for (int ii = 0; ii < 2; ++ii) {
            const int a = k1[ii], b = k2[ii], qa = cross_q(a, sh), qb = cross_q(b, sh);
            ad[ii][0] = cross_at(a, qb);
            ad[ii][1] = cross_at(qa, b);
            ad[ii][2] = cross_at(qa, qb);
        }
        const int qk = cross_q(kn, sh);
        adq = cross_at(qk, qk);                // q of the next pair
        adz = cross_at(lp, cross_q(lp, sh));   // this round's pivot of pair lp
    };
    int ad[2][3], adq, adz;
    round_ad(0, ad, adq, adz);
    for (int sh = 0; sh < H; ++sh) {
        const double *cur = prm + (sh & 1) * 3 * H;
        double *nxt = prm + ((sh + 1) & 1) * 3 * H;
        // producer: the two diagonal entries of pair `lane`'s next pivot
        // (p of this pair, q of the next pair), read before the round's stores
        double dp = 0.0, dq = 0.0, shp = 0.0, shq = 0.0;
        if (prod) {
            dp = S[adp];
            dq = S[adq];
            shp = cur[2 * H + lane];
            shq = cur[2 * H + kn];
        }
        double c1[2], s1[2], c2[2], s2[2], b00[2], b01[2], b10[2], b11[2];
#pragma unroll
        for (int ii = 0; ii < 2; ++ii) {
            const int a = k1[ii], b = k2[ii];
            c1[ii] = cur[a];
            s1[ii] = cur[H + a];
            c2[ii] = cur[b];
            s2[ii] = cur[H + b];
            b00[ii] = S[a00[ii]];
            b01[ii] = S[ad[ii][0]];
            b10[ii] = S[ad[ii][1]];
            b11[ii] = S[ad[ii][2]];
        }
        int nad[2][3], nadq, nadz;
        round_ad(sh + 1, nad, nadq, nadz);
        double nv[2][4];
#pragma unroll
        for (int ii = 0; ii < 2; ++ii) {
            // rows: J1^T, then columns: J2 (J = [[c, s], [-s, c]] on (p, q))
            const double r00 = c1[ii] * b00[ii] - s1[ii] * b10[ii], r01 = c1[ii] * b01[ii] - s1[ii] * b11[ii];
            const double r10 = s1[ii] * b00[ii] + c1[ii] * b10[ii], r11 = s1[ii] * b01[ii] + c1[ii] * b11[ii];
            nv[ii][0] = c2[ii] * r00 - s2[ii] * r01;
            nv[ii][1] = s2[ii] * r00 + c2[ii] * r01;
            nv[ii][2] = c2[ii] * r10 - s2[ii] * r11;
            nv[ii][3] = s2[ii] * r10 + c2[ii] * r11;
        }
        // the previous round's parameters are in the ring (its stores are
        // complete once this round's loads are)
        if (sh > 0) lds_store_release(vr.sdone, vr.base + sh + 1);
#pragma unroll
        for (int ii = 0; ii < 2; ++ii) {
            if (!ok[ii]) continue;
            S[a00[ii]] = nv[ii][0];
            S[ad[ii][0]] = nv[ii][1];
            S[ad[ii][1]] = nv[ii][2];
            S[ad[ii][2]] = nv[ii][3];
        }
        if (prod) {
            const double app = dp - shp, aqq = dq + shq;
            S[adp] = app;
            S[adq] = aqq;
            S[adz] = 0.0;  // this round's pivot (no item holds it)
            if (sh + 1 < H) {
                const double apq = lane < 15 ? nv[0][1] : nv[0][2];
                double c, s, t;
                rot_cst(app, aqq, apq, c, s, t);
                nxt[lane] = c;
                nxt[H + lane] = s;
                nxt[2 * H + lane] = t * apq;
                const int n = vr.base + sh + 1;
                double *rb = vr.ring + (n & (VR_DEPTH - 1)) * 2 * H;
                lds_wait_geq_seen(vr.vdone, n + 1 - VR_DEPTH, vseen, vr.fail, vr.spin);
                rb[lane] = c;
                rb[H + lane] = s;
            }
        }
        wave_lds_sync();
        // (the next round publishes this round's ring slot)
#pragma unroll
        for (int ii = 0; ii < 2; ++ii)
#pragma unroll
            for (int m = 0; m < 3; ++m) ad[ii][m] = nad[ii][m];
        adq = nadq;
        adz = nadz;
    }
}

// The follower of cross_sweep: W (32 x 32) <- W J for every round, lane
// 2 r + h holding row r at 16 positions.  h = 0: columns 0..15 (block ba)
// in order; h = 1: block bb, rotated so that in round sh position j holds
// column 16 + (j + sh) mod 16, the partner of column j.  After 16 rounds
// positions equal columns again.
__device__ void follow_cross(const VRing &vr, int lane, double *V) {
    constexpr int H = 16;
    const int r = lane >> 1, h = lane & 1;
#pragma unroll
    for (int j = 0; j < H; ++j) V[j] = (r == 16 * h + j) ? 1.0 : 0.0;
    for (int sh = 0; sh < H; ++sh) {
        const int n = vr.base + sh;
        lds_wait_geq(vr.sdone, n + 1, vr.fail, vr.spin);
        const double *rb = vr.ring + (n & (VR_DEPTH - 1)) * 2 * H;
        // four positions at a time (the V role keeps V_hat^T in half of its
        // registers); the partner lane's positions (same row, other block)
        // come from DPP quad permutation [1, 0, 3, 2], which swaps the lanes
        // of each pair; column p = c p - s q, column q = s p + c q
#pragma unroll
        for (int j0 = 0; j0 < H; j0 += 4) {
            double vc[4], vs[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                vc[j] = rb[j0 + j];
                vs[j] = rb[H + j0 + j];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double pt = dpp_quad_t<(1 | 0 << 2 | 3 << 4 | 2 << 6)>(V[j0 + j]);
                V[j0 + j] = h ? vs[j] * pt + vc[j] * V[j0 + j] : vc[j] * V[j0 + j] - vs[j] * pt;
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        // this round's slot is read: free it
        lds_store_release(vr.vdone, n + 1);
        if (h) {
            const double v0 = V[0];
#pragma unroll
            for (int j = 0; j < H - 1; ++j) V[j] = V[j + 1];
            V[H - 1] = v0;
        }
    }
}

template <int MODE>
__global__ void __launch_bounds__(512) k_subproblem2(SubArgs a) {
    using namespace tl;
    constexpr int B = M2 / 2;
    extern __shared__ double smem[];
    double *Ap = smem;
    double *red = Ap + AP + 4 * SW;
    double *rings = red + 16;                                // 4 x RING
    int *ctr = reinterpret_cast<int *>(rings + 4 * RING);  // sdone[4], vdone[4], fail
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int g = lane >> 4, x = lane & 15;
    const int pr = blockIdx.x;
    if (tid < 9) ctr[tid] = 0;  // ordered before use by the prologue's barriers
    const int spin = a.spin_limit > 0 ? a.spin_limit : VR_SPIN;

    if (MODE != SUB_PLAIN && a.force_skip && a.force_skip[pr]) {  // placeholder pair
        if (tid == 0 && a.flags) a.flags[pr] = 1;
        return;
    }
    double off2 = 0.0, fro2 = 0.0;
    {
        // the upper triangle of A_hat, column-major positions e = c M2 + r (a
        // wave's 64 positions share a column half: one source block per
        // wave), all 32 of a thread's loads in flight before their LDS
        // stores (the three source blocks come from other CUs' writes: 8 at a
        // time cost about 0.5 % of the n = 4096 solve)
        const HatSource<M2, MODE> load(a, pr);
        constexpr int PER = M2 * M2 / NT;
        {
            double v[PER];
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int e = u * NT + tid, r = e % M2, c = e / M2;
                v[u] = r <= c ? load(r, c) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < PER; ++u) {
                const int e = u * NT + tid, r = e % M2, c = e / M2;
                if (r <= c) {
                    Ap[pk(r, c)] = v[u];
                    const double w2 = v[u] * v[u];
                    if (r == c) fro2 += w2;
                    else { off2 += 2.0 * w2; fro2 += 2.0 * w2; }
                }
            }
        }
    }
    off2 = block_sum<NT>(off2, red);
    fro2 = block_sum<NT>(fro2, red);
    auto get = [&](int r, int c) { return Ap[pkm(r, c)]; };
    if (skip_test<M2, NT, MODE>(a, pr, off2, red, get)) return;

    // Number of inner sweeps: both roles evaluate this identically (the same
    // workgroup barriers, the same decision).
    const double eps = 2.220446049250313e-16;
    const bool conv = a.inner_sweeps <= 0;
    const int cap = conv ? 30 : a.inner_sweeps;
    auto more = [&](int swp) -> bool {
        if (swp >= cap) return false;
        if (!conv || swp == 0) return true;
        double o = 0.0;
        for (int e = tid; e < M2 * M2; e += NT) {
            const int rr = e % M2, cc = e / M2;
            if (rr < cc) { const double v = Ap[pk(rr, cc)]; o += 2.0 * v * v; }
        }
        o = block_sum<NT>(o, red);
        return !(sqrt(o) <= eps * sqrt(fro2));
    };

    if (wv < 4) {
        // ================= solver role: wave k owns pair problem k =================
        const int k = wv;
        double *S = Ap + AP + k * SW;  // slots
        double *prm = S + 32 * 32;     // parameters
        const double *Wl = Ap + AP + WOFF + g * 33 + x;  // W reads: lane base + constant
        int rnd = 0;  // global round number of the next sweep's round 0
        // This lane's entries of the 528-entry upper triangle (diagonal
        // included) of a 32 x 32 pair problem: the triangle is read as a 16 x 33
        // rectangle (rows a and 31 - a together hold 33 entries); entry i is
        // e = lane + 64 i.  lr: local (row, col) packed; si: slot-array index.
        constexpr int NG = (528 + 63) / 64;
        int lr[NG], si[NG];
#pragma unroll
        for (int i = 0; i < NG; ++i) {
            const int e = min(lane + 64 * i, 527), ra = e / 33, cb = e - 33 * ra;
            const int r = cb < 32 - ra ? ra : 31 - ra, c = cb < 32 - ra ? ra + cb : cb - 1;
            const int u = slot_of(r, 32), w = slot_of(c, 32);
            lr[i] = r | (c << 8);
            si[i] = min(u, w) * 32 + max(u, w);
        }
        for (int swp = 0; more(swp); ++swp) {
            for (int t = 0; t < NB - 1; ++t) {
                // ---- phase 1: one sweep on the 32 x 32 problem of block pair k;
                //      local index l < 16 is row l of block ba, l >= 16 row
                //      l - 16 of block bb
                //      (block round 0: a full sweep; later block rounds: the
                //      16 rounds of cross pairs only, the within-block pairs
                //      having been rotated in block round 0)
                const int ba = index_at(2 * k, t, NB), bb = index_at(2 * k + 1, t, NB);
                auto glob = [&](int l) { return l < BS ? BS * ba + l : BS * bb + (l - BS); };
                const bool cross = t > 0;
                int ai[NG];  // A_hat (packed) index of each entry
#pragma unroll
                for (int i = 0; i < NG; ++i) ai[i] = pkm(glob(lr[i] & 255), glob(lr[i] >> 8));
                // S index of entry i: slot order for the full sweep, plain for the cross rounds
                auto sx = [&](int i) { return cross ? cross_at(lr[i] & 255, lr[i] >> 8) : si[i]; };
                {
                    double v[NG];
#pragma unroll
                    for (int i = 0; i < NG; ++i) v[i] = Ap[ai[i]];
#pragma unroll
                    for (int i = 0; i < NG; ++i)
                        if (lane + 64 * i < 528) S[sx(i)] = v[i];
                }
                wave_lds_sync();
                const VRing vr{rings + k * RING, ctr + k, ctr + 4 + k, rnd, ctr + 8, spin};
                if (cross) {
                    cross_sweep(S, prm, lane, vr);
                    rnd += 16;
                } else {
                    scalar_sweeps<32, 64, true, true, true>(S, prm, nullptr, lane, 1, false, 0.0, nullptr, &kSweep32,
                                                            vr);
                    rnd += 31;
                }
                __syncthreads();  // X: W of this round written by the V role; D back into A_hat
                {
                    double v[NG];
#pragma unroll
                    for (int i = 0; i < NG; ++i) v[i] = S[sx(i)];
#pragma unroll
                    for (int i = 0; i < NG; ++i)
                        if (lane + 64 * i < 528) Ap[ai[i]] = v[i];
                }
                __syncthreads();  // Y: all four W and diagonal blocks in place

                // ---- phase 2: A_hat(p, q) <- W_p^T A_hat(p, q) W_q for the six
                //      tiles p < q, as twelve column halves j (three per wave);
                //      computed into registers, written after a barrier (a
                //      half reads the whole tile)
                d4 O[3][2];
#pragma unroll
                for (int hh = 0; hh < 3; ++hh) {
                    const int h = k + 4 * hh, u = h >> 1, j = h & 1;
                    const int p = u < 3 ? 0 : (u < 5 ? 1 : 2);
                    const int q = u < 3 ? u + 1 : (u < 5 ? u - 1 : 3);
                    const double *Wp = Wl + p * SW;  // W_p(kk, i) = Wp[(kk - g) * 33 + i - x]
                    const double *Wq = Wl + q * SW;
                    const int pa = index_at(2 * p, t, NB), pb = index_at(2 * p + 1, t, NB);
                    const int qa = index_at(2 * q, t, NB), qb = index_at(2 * q + 1, t, NB);
                    auto gp = [&](int l) { return l < BS ? BS * pa + l : BS * pb + (l - BS); };
                    auto gq = [&](int l) { return l < BS ? BS * qa + l : BS * qb + (l - BS); };
                    // T = X W_q (column half j), X(i, kk) = A_hat(gp(i), gq(kk));
                    // T[i] lane (g, x) component v = T(16 i + g + 4 v, 16 j + x)
                    d4 T[2] = {d4{0.0, 0.0, 0.0, 0.0}, d4{0.0, 0.0, 0.0, 0.0}};
#pragma unroll
                    for (int k0 = 0; k0 < 32; k0 += 4) {
                        const int kk = k0 + g;
                        const double bq = Wq[k0 * 33 + 16 * j];
                        const double a0 = Ap[pkm(gp(x), gq(kk))], a1 = Ap[pkm(gp(16 + x), gq(kk))];
                        T[0] = mfma_f64(a0, bq, T[0]);
                        T[1] = mfma_f64(a1, bq, T[1]);
                    }
                    // O = W_p^T T; step (ti, s) contracts over row 16 ti + g + 4 s of T
                    O[hh][0] = d4{0.0, 0.0, 0.0, 0.0};
                    O[hh][1] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int ti = 0; ti < 2; ++ti)
#pragma unroll
                        for (int s4 = 0; s4 < 4; ++s4) {
                            const int kk = 16 * ti + 4 * s4;  // + g (in Wl)
                            const double a0 = Wp[kk * 33], a1 = Wp[kk * 33 + 16];
                            O[hh][0] = mfma_f64(a0, T[ti][s4], O[hh][0]);
                            O[hh][1] = mfma_f64(a1, T[ti][s4], O[hh][1]);
                        }
                }
                __syncthreads();  // every read of the six tiles is done
#pragma unroll
                for (int hh = 0; hh < 3; ++hh) {
                    const int h = k + 4 * hh, u = h >> 1, j = h & 1;
                    const int p = u < 3 ? 0 : (u < 5 ? 1 : 2);
                    const int q = u < 3 ? u + 1 : (u < 5 ? u - 1 : 3);
                    const int pa = index_at(2 * p, t, NB), pb = index_at(2 * p + 1, t, NB);
                    const int qa = index_at(2 * q, t, NB), qb = index_at(2 * q + 1, t, NB);
                    auto gp = [&](int l) { return l < BS ? BS * pa + l : BS * pb + (l - BS); };
                    auto gq = [&](int l) { return l < BS ? BS * qa + l : BS * qb + (l - BS); };
#pragma unroll
                    for (int i = 0; i < 2; ++i)
#pragma unroll
                        for (int v = 0; v < 4; ++v) Ap[pkm(gp(16 * i + g + 4 * v), gq(16 * j + x))] = O[hh][i][v];
                }
                __syncthreads();  // Z: A_hat complete for the next round
            }
        }
    } else {
        // ================= V role: Vt = V_hat^T in registers =================
        // wave 4 + c owns column tiles 2c, 2c + 1 of Vt (rows of V_hat);
        // vt[tt][j] lane (g, x) component v = Vt(16 tt + g + 4 v, 16 (2c + j) + x).
        // It applies round t's rotations while the solver role runs round t + 1.
        const int c = wv - 4;
        d4 vt[NB][2];
#pragma unroll
        for (int tt = 0; tt < NB; ++tt)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int v = 0; v < 4; ++v) vt[tt][j][v] = (16 * tt + g + 4 * v == 16 * (2 * c + j) + x) ? 1.0 : 0.0;
        // Vt rows of block pair k <- W_k^T (those rows), then the tiles follow
        // the block ring: 1 <- 2 <- 4 <- 6 <- 7 <- 5 <- 3 <- 1.  Every W read is
        // one lane base plus a constant (no per-address registers).
        // nz: bit 2 tt + j is set when tile vt[tt][j] may be nonzero (wave-
        // uniform).  Vt starts as the identity (tiles (2c, 0) and (2c + 1, 1))
        // and fills in over the first block rounds: the products with tiles
        // known to be zero are skipped (a third of the MFMAs of one inner
        // sweep, all in its first four block rounds).
        const double *Wl = Ap + AP + WOFF + g * 33 + x;
        const int cu = __builtin_amdgcn_readfirstlane(c);
        int nz = (1 << (4 * cu)) | (1 << (4 * cu + 3));
        auto apply = [&]() {
            int nzn = 0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const double *Wk = Wl + k * SW;
                d4 n0[2] = {d4{0.0, 0.0, 0.0, 0.0}, d4{0.0, 0.0, 0.0, 0.0}};
                d4 n1[2] = {d4{0.0, 0.0, 0.0, 0.0}, d4{0.0, 0.0, 0.0, 0.0}};
#pragma unroll
                for (int ti = 0; ti < 2; ++ti) {
                    const int tb = (nz >> (2 * (2 * k + ti))) & 3;  // column tiles j of vt[2k + ti] in use
                    if (tb == 0) continue;
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) {
                        const int rr = 16 * ti + 4 * s4;  // + g (in Wl)
                        const double a0 = Wk[rr * 33], a1 = Wk[rr * 33 + 16];
#pragma unroll
                        for (int j = 0; j < 2; ++j) {
                            if (!((tb >> j) & 1)) continue;
                            n0[j] = mfma_f64(a0, vt[2 * k + ti][j][s4], n0[j]);
                            n1[j] = mfma_f64(a1, vt[2 * k + ti][j][s4], n1[j]);
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    vt[2 * k][j] = n0[j];
                    vt[2 * k + 1][j] = n1[j];
                }
                const int pb = ((nz >> (4 * k)) | (nz >> (4 * k + 2))) & 3;
                nzn |= (pb | pb << 2) << (4 * k);
                // keep the next pair's W loads from being hoisted over this
                // one (Vt already holds half the register file)
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const d4 o1 = vt[1][j];
                vt[1][j] = vt[2][j];
                vt[2][j] = vt[4][j];
                vt[4][j] = vt[6][j];
                vt[6][j] = vt[7][j];
                vt[7][j] = vt[5][j];
                vt[5][j] = vt[3][j];
                vt[3][j] = o1;
            }
            auto tb = [&](int tt) { return (nzn >> (2 * tt)) & 3; };
            nz = tb(0) | tb(2) << 2 | tb(4) << 4 | tb(1) << 6 | tb(6) << 8 | tb(3) << 10 | tb(7) << 12 | tb(5) << 14;
        };
        // The same barriers and sweep decisions as the solver role; apply()
        // appears once (two inlined copies cost the register allocator its Vt).
        bool pend = false, run = more(0);
        int rnd = 0;
        for (int swp = 0, t = 0;;) {
            if (pend) apply();  // the previous round's W
            if (!run) break;
            {
                // this round's rotations of pair problem c, as the solver role
                // produces them; then W_c(r, 16 h + xx) = Vl[xx], r = lane / 2,
                // h = lane mod 2
                const VRing vr{rings + c * RING, ctr + c, ctr + 4 + c, rnd, ctr + 8, spin};
                double Vl[16];
                if (t > 0) {  // cross rounds (as the solver role)
                    follow_cross(vr, lane, Vl);
                    rnd += 16;
                } else {
                    follow_sweep<32>(vr, lane, Vl);
                    rnd += 31;
                }
                double *W = Ap + AP + c * SW + WOFF;
                const int r = lane >> 1, h = lane & 1;
#pragma unroll
                for (int xx = 0; xx < 16; ++xx) W[r * 33 + 16 * h + xx] = Vl[xx];
            }
            __syncthreads();  // X
            __syncthreads();  // Y
            __syncthreads();  // tile reads done
            __syncthreads();  // Z
            pend = true;
            if (++t == NB - 1) {
                t = 0;
                run = more(++swp);
            }
        }

        // ---- results: V_hat(16 (2c + j) + x, 16 tt + g + 4 v) = vt[tt][j][v].
        //      Each layout is a lane base plus (tt, j, v) constants; one tile row
        //      at a time keeps the store addresses out of the Vt registers.
        // (NaN if a hand-off wait ran out; every wait is behind the last barrier)
        const double bad = ctr[8] ? __builtin_nan("") : 0.0;
        auto put = [&](auto *base, int stt, int sj, int sv) {
#pragma unroll
            for (int tt = 0; tt < NB; ++tt) {
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v) base[tt * stt + j * sj + v * sv] = vt[tt][j][v] + bad;
                __builtin_amdgcn_sched_barrier(0);
            }
        };
        const size_t vofs = (size_t)pr * M2 * M2;
        if (MODE == SUB_PLAIN) {  // V_hat(r, col) at col * M2 + r
            put(a.vout + vofs + g * M2 + 32 * c + x, 16 * M2, 16, 4 * M2);
        } else if (a.vout32) {  // vperm32(16 (2c + j) + x, 16 tt + g + 4 v)
            put(a.vout32 + vofs + (8 * c + (x & 3)) * 512 + (x >> 2) * 16 + g, 64, 2048, 4);
        } else {  // vperm(16 (2c + j) + x, 16 tt + g + 4 v)
            put(a.vout + vofs + (8 * c + (x >> 2)) * 512 + (x & 3) * 16 + g, 64, 2048, 4);
        }
    }

    // ---- D_hat: A_hat is final after the last block round's barrier Z, and
    //      every hand-off wait ended before it, so the solver waves write it
    //      while the V role applies the last W and stores V_hat; NaN if a
    //      hand-off wait ran out (the caller sees a non-finite iterate)
    if (wv < 4) {
        constexpr int NS = NT / 2;  // solver threads
        const bool bad = ctr[8] != 0;
        auto dval = [&](int rr, int cc) { return bad ? __builtin_nan("") : Ap[pkm(rr, cc)]; };
        if (MODE == SUB_PLAIN) {
            double *dd = a.dout + (size_t)pr * M2 * M2;
            for (int e = tid; e < M2 * M2; e += NS) dd[e] = dval(e % M2, e / M2);
        } else if (MODE == SUB_EIG) {  // A([I,J],[I,J]) <- D_hat
            const int I = a.pairs[2 * pr], J = a.pairs[2 * pr + 1];
            const size_t oii = ublk(I, I) * (size_t)(B * B), ojj = ublk(J, J) * (size_t)(B * B),
                         oij = ublk(I, J) * (size_t)(B * B);
            for (int e = tid; e < M2 * M2; e += NS) {
                const int rr = e % M2, cc = e / M2;
                store_dhat<M2>(a, oii, ojj, oij, rr, cc, dval(rr, cc));
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
    ensure_lds_limit(reinterpret_cast<const void *>(&k_subproblem<M2, MODE>), (int)C::LDS_BYTES);
    hipLaunchKernelGGL((k_subproblem<M2, MODE>), dim3(a.count), dim3(C::NT), C::LDS_BYTES, s, a);
    JX_LAUNCHED();
}

// JACOBI_HANDOFF_SPIN (environment): bound of the hand-off waits, for tests
// of the failure path (a tiny bound makes them run out).
static int handoff_spin() {
    static const int v = [] {
        const char *e = std::getenv("JACOBI_HANDOFF_SPIN");
        return e ? std::max(0, std::atoi(e)) : 0;
    }();
    return v;
}

template <int MODE>
static void launch_sub2_t(const SubArgs &a0, hipStream_t s) {
    SubArgs a = a0;
    if (a.spin_limit <= 0) a.spin_limit = handoff_spin();
    ensure_lds_limit(reinterpret_cast<const void *>(&k_subproblem2<MODE>), (int)tl::LDS_BYTES);
    hipLaunchKernelGGL((k_subproblem2<MODE>), dim3(a.count), dim3(tl::NT), tl::LDS_BYTES, s, a);
    JX_LAUNCHED();
}

template <int MODE>
static void launch_sub_m(const SubArgs &a, hipStream_t s) {
    switch (a.m2) {
        case 32: launch_sub_t<32, MODE>(a, s); break;
        case 64: launch_sub_t<64, MODE>(a, s); break;
#ifdef JX_K1_ONE_LEVEL
        case 128: launch_sub_t<128, MODE>(a, s); break;
#else
        case 128: launch_sub2_t<MODE>(a, s); break;
#endif
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
