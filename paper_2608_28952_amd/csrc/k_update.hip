// k_update.hip -- rotation-apply kernels of one parallel step of block Jacobi
// on gfx950 FP64 MFMA (v_mfma_f64_16x16x4_f64), and on FP32 MFMA
// (v_mfma_f32_16x16x4_f32) for the FP32 phase of the precision ladder.
//
// Alg. 2 (§3) updates, for every pair (I, J) of a group, block rows I, J of A
// on the left by V^T, block columns I, J of A on the right by V, and block
// columns of Q on the right by V.  A block lying in the rows of pair p and the
// columns of pair q is multiplied by V_p^T on the left and by V_q on the right,
// in either order (§3).  On one GPU the two sides are fused: workgroup (p, q),
// p < q, computes the 2b x 2b pair tile
//     A[p, q] <- V_p^T (A[p, q] V_q)
// once, reading and writing only the upper block triangle (the iterate is
// symmetric, §3 notes the full matrix is kept only for bookkeeping).  The
// diagonal tiles A[p, p] are replaced by D_hat in the subproblem kernel.
//
// GEMM 1 (T = X V_q): X staged through LDS in 16-column chunks (transposed on
// the fly when the stored block is the mirror), V_q read from global memory in
// the MFMA-operand order of vperm().  Each wave owns 16 or 32 columns of T.
// GEMM 2 (out = V_p^T T): the contraction index of T is its row; the FP64
// MFMA result layout holds row 16 a + g + 4 v in lane group g, component v,
// so step (a, v) of GEMM 2 (k = 16 a + 4 v + g) takes its B operand straight
// from component v of the GEMM 1 accumulators: T stays in registers (the
// critical-block path, whose waves split T's rows, hands it over through LDS
// in that operand order).
//
// Per round: k_update_a_crit computes, on the solve's stream, only the
// blocks the next round's subproblems read; k_update_aq_bounded (b = 64;
// k_update_a_bounded and k_update_q_bounded for b = 32) the rest of every
// tile and the Q update on a bounded set of CUs beside the next round's
// subproblems.
#include "jx_common.hpp"

#include <type_traits>

namespace jx {

namespace {

constexpr int KC = 16;  // X chunk width (columns)

// 0 and 1 of each type.  The operand of a skipped rotation (V = I) is loaded
// from here: the address is chosen, not the value, so that operand loads
// never sit behind a branch and stay in flight together.
__device__ double kEye64[2] = {0.0, 1.0};
__device__ float kEye32[2] = {0.0f, 1.0f};
template <class T>
__device__ __forceinline__ const T *eye_ptr(bool diag);
template <>
__device__ __forceinline__ const double *eye_ptr<double>(bool diag) { return kEye64 + (diag ? 1 : 0); }
template <>
__device__ __forceinline__ const float *eye_ptr<float>(bool diag) { return kEye32 + (diag ? 1 : 0); }
// *p, or entry (diag) of the identity when the rotation is skipped
template <class T>
__device__ __forceinline__ T op_or_eye(const T *p, bool id, bool diag) {
    return *(id ? eye_ptr<T>(diag) : p);
}

// HALF: T is computed for one column half of the tile only (the columns of
// one block), which is all that one output block needs.
template <int B, int NTH = 256, bool HALF = false>
struct UaCfg {
    static constexpr int M2 = 2 * B;      // tile order
    static constexpr int RT = M2 / 16;    // 16-row tiles
    static constexpr int WW = (HALF ? B : M2) / (NTH / 64);  // columns per wave
    static constexpr int CT = WW / 16;    // 16-column tiles per wave
    static constexpr int XLD = M2 + 1;    // LDS stride of an X chunk [k][row]
    static constexpr int OLD = B + 1;     // LDS stride of an output half [col][row]
    static constexpr int NCH = M2 / KC;   // chunks
    static constexpr int PER = 2 * B * KC / NTH;  // X chunk values per thread
    static constexpr size_t XS_DOUBLES = 2 * (size_t)KC * XLD;
    static constexpr size_t OS_DOUBLES = (size_t)M2 * OLD;
    static constexpr size_t LDS_BYTES = sizeof(double) * (XS_DOUBLES > OS_DOUBLES ? XS_DOUBLES : OS_DOUBLES);
    static_assert(WW % 16 == 0, "a wave owns whole 16-column tiles");
};

// Which blocks of a tile are read from and written to where.  Quadrant
// (h, c) = block (row block h of pair p, column block c of pair q) has bit
// 2 h + c.  A tile's blocks that the next round's subproblems read (its
// "critical" quadrants) are computed first and alone, from copies of their
// originals made beforehand (the critical kernel writes them in place); the
// rest of the tile later, from the same copies:
//   wmask  quadrants written back (the others are computed or not, but left)
//   rmask  quadrants whose input block comes from side + quad B^2, not ablk
//   snext, smap  quadrant quad written back also goes to snext + slot B^2,
//          slot = smap[quad] (negative: none): the copies the next round's
//          critical kernel reads
// (side blocks are B x B, each stored as its block is in ablk).
template <class T>
struct TileIO {
    int wmask = 15, rmask = 0;
    T *side = nullptr;
    T *snext = nullptr;
    const int *smap = nullptr;  // 4 slots
};

// Fetch the PER values of X chunk `ch` (columns c0 .. c0+KC-1 of one block
// column) that this thread stages.  Rows h B .. h B + B-1 come from the block
// at src[h], stored column-major as block (row, column) when tr[h] is false
// and as its mirror (column, row) when tr[h] is true.
template <int B, class T, int NTH>
__device__ __forceinline__ void fetch_chunk(const T *const src[2], const bool tr[2], int c0, T *reg, int tid) {
    using U = UaCfg<B, NTH>;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int m = 0; m < U::PER / 2; ++m) {
            const int e = tid + NTH * m;  // 0 .. B*KC-1
            T v;
            if (!tr[h]) {
                const int rl = e % B, cl = e / B;
                v = src[h][(c0 + cl) * B + rl];
            } else {
                const int cl = e % KC, rl = e / KC;
                v = src[h][rl * B + c0 + cl];
            }
            reg[h * (U::PER / 2) + m] = v;
        }
    }
}

template <int B, class T, int NTH>
__device__ __forceinline__ void stage_chunk(T *xs, const bool tr[2], const T *reg, int tid) {
    using U = UaCfg<B, NTH>;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int m = 0; m < U::PER / 2; ++m) {
            const int e = tid + NTH * m;
            int rl, cl;
            if (!tr[h]) { rl = e % B; cl = e / B; }
            else { cl = e % KC; rl = e / KC; }
            xs[cl * U::XLD + h * B + rl] = reg[h * (U::PER / 2) + m];
        }
    }
}

// Tile (p, q) by NTH threads t = 0 .. NTH-1 (NTH / 64 waves, each owning
// WW columns of T) with `lds` (U::LDS_BYTES) of their own.  HALF: T only for
// column half `cb` (then io.wmask names quadrants of that half only).
// active false (no tile, or both rotations skipped): no work, but every
// barrier is still taken, so two halves of one workgroup stay in step.
template <int B, class T, int NTH = 256, bool HALF = false>
__device__ __forceinline__ void ua_tile(const int *__restrict__ pairs, T *__restrict__ ablk,
                                        const T *__restrict__ vhat, int p, int q, bool idp, bool idq, int tid,
                                        T *lds, bool active, const TileIO<T> &io, int cb = 0) {
    using U = UaCfg<B, NTH, HALF>;
    using MT = MfmaTraits<T>;
    typedef typename MT::acc_t acc_t;
    constexpr int M2 = U::M2, RT = U::RT, CT = U::CT, WW = U::WW;
    const int Rr[2] = {active ? pairs[2 * p] : 0, active ? pairs[2 * p + 1] : 1};
    const int Cq[2] = {active ? pairs[2 * q] : 0, active ? pairs[2 * q + 1] : 1};
    const T *vp = vhat + (size_t)p * M2 * M2;
    const T *vq = vhat + (size_t)q * M2 * M2;

    const int lane = tid & 63, w = tid >> 6;
    const int g = lane >> 4, x = lane & 15;
    const int wc0 = (HALF ? cb * B : 0) + w * WW;

    // input block of quadrant (h, c): ablk, or its saved original
    auto src_of = [&](int h, int c) -> const T * {
        if ((io.rmask >> (2 * h + c)) & 1) return io.side + (size_t)(2 * h + c) * B * B;
        const int R = Rr[h], C = Cq[c];
        return ablk + ublk(R < C ? R : C, R < C ? C : R) * (size_t)(B * B);
    };
    // chunk k0's column block c: its two row blocks (pointers formed at each
    // fetch, not kept: the bounded kernel has no registers to spare)
    auto fetch = [&](int k0, T *reg) {
        const int c = k0 / B;
        const T *src[2] = {src_of(0, c), src_of(1, c)};
        const bool tr[2] = {Rr[0] > Cq[c], Rr[1] > Cq[c]};
        fetch_chunk<B, T, NTH>(src, tr, k0 % B, reg, tid);
    };
    auto stage = [&](int k0, T *xs, const T *reg) {
        const int c = k0 / B;
        const bool tr[2] = {Rr[0] > Cq[c], Rr[1] > Cq[c]};
        stage_chunk<B, T, NTH>(xs, tr, reg, tid);
    };

    acc_t acc[RT][CT];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    // ---------------- GEMM 1: T(:, wc0 .. wc0+WW-1) = X V_q ----------------
    T reg[U::PER];
    // V_q operand of k-step st, column tile ct (V_q = I is applied as an exact
    // identity operand: products with 1.0 and sums of exact zeros reproduce X
    // bit for bit)
    auto vqk = [&](int ch, int st, int ct) {
        const int kg = ch * KC + MT::kstep(st, g), col = wc0 + 16 * ct + x;
        return op_or_eye(vq + MT::vidx(kg, col, M2), idq, kg == col);
    };
    // X chunks (and, with one column tile per wave, their V_q operands) are
    // fetched two chunks ahead, so that global-memory latency hides behind
    // two chunks' MFMAs; chunk ch is staged in LDS buffer ch mod 2 after chunk
    // ch - 1's products (with two column tiles the registers for V_q are not
    // there: those are loaded per k-step)
    constexpr bool PF = CT == 1;
    T reg2[U::PER];
    T bnext[KC / 4], bnext2[KC / 4];
    if (active) {
        fetch(0, reg);
        if constexpr (PF) {
#pragma unroll
            for (int st = 0; st < KC / 4; ++st) bnext[st] = vqk(0, st, 0);
        }
        stage(0, lds, reg);
        if (U::NCH > 1) {
            fetch(KC, reg);  // reg: chunk 1 until it is staged
            if constexpr (PF) {
#pragma unroll
                for (int st = 0; st < KC / 4; ++st) bnext2[st] = vqk(1, st, 0);
            }
        }
    }
    __syncthreads();
    for (int ch = 0; ch < U::NCH; ++ch) {
        T *xs = lds + (size_t)(ch & 1) * KC * U::XLD;
        T bcur[KC / 4];
#pragma unroll
        for (int st = 0; st < KC / 4; ++st) {
            bcur[st] = bnext[st];
            bnext[st] = bnext2[st];
        }
        if (active && ch + 2 < U::NCH) {
            fetch((ch + 2) * KC, reg2);
            if constexpr (PF) {
#pragma unroll
                for (int st = 0; st < KC / 4; ++st) bnext2[st] = vqk(ch + 2, st, 0);
            }
        }
        if constexpr (PF) {
            if (active) {
#pragma unroll
                for (int st = 0; st < KC / 4; ++st) {
                    const int kl = MT::kstep(st, g);
#pragma unroll
                    for (int rt = 0; rt < RT; ++rt)
                        acc[rt][0] = MT::mma(xs[kl * U::XLD + 16 * rt + x], bcur[st], acc[rt][0]);
                }
            }
        } else {
#pragma unroll 1
            for (int st = 0; st < (active ? KC / 4 : 0); ++st) {
                const int kl = MT::kstep(st, g);
                T bf[CT];
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) bf[ct] = vqk(ch, st, ct);
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    const T af = xs[kl * U::XLD + 16 * rt + x];
#pragma unroll
                    for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = MT::mma(af, bf[ct], acc[rt][ct]);
                }
            }
        }
        if (active && ch + 1 < U::NCH) {
            stage((ch + 1) * KC, lds + (size_t)((ch + 1) & 1) * KC * U::XLD, reg);
#pragma unroll
            for (int m = 0; m < U::PER; ++m) reg[m] = reg2[m];
        }
        __syncthreads();
    }

    // ---------------- GEMM 2: out = V_p^T T, one block row at a time ------------
    // Output row tiles run in a loop (one 16-row tile at a time, two
    // accumulator chains); the contraction over the rows of T is fully
    // unrolled so that the accumulator arrays are indexed with constants only.
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        T *os = lds;
        const bool hact = active && ((io.wmask >> (2 * h)) & 3) != 0;  // a block of this row half is written
#pragma unroll 1
        for (int ot = 0; ot < (hact ? RT / 2 : 0); ++ot) {
            acc_t o[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct) o[ct] = acc_t{0, 0, 0, 0};
            // (V_p = I is applied as an exact identity operand, as for V_q)
            const int orow = h * B + 16 * ot + x;
            const T *vrow = vp + MT::vidx(0, orow, M2);
            // V_p operand of step (rt, s): row 16 rt + rrow(g, s) of T sits in
            // component s of lane group g; vidx(k, i) - vidx(0, i) depends on k only
            auto vpk = [&](int rt, int s) {
                const int k = 16 * rt + MT::rrow(g, s);
                return op_or_eye(vrow + (MT::vidx(k, 0, M2) - MT::vidx(0, 0, M2)), idp, k == orow);
            };
            if constexpr (CT == 1) {
                // one output column tile per wave: every V_p operand of the
                // row tile is loaded at once (one global-memory latency, not RT)
                T af[RT][4];
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int s = 0; s < 4; ++s) af[rt][s] = vpk(rt, s);
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
#pragma unroll
                    for (int s = 0; s < 4; ++s) o[0] = MT::mma(af[rt][s], acc[rt][0][s], o[0]);
            } else {
#pragma unroll
                for (int rt = 0; rt < RT; ++rt) {
                    T af[4];
#pragma unroll
                    for (int s = 0; s < 4; ++s) af[s] = vpk(rt, s);
#pragma unroll
                    for (int s = 0; s < 4; ++s)
#pragma unroll
                        for (int ct = 0; ct < CT; ++ct) o[ct] = MT::mma(af[s], acc[rt][ct][s], o[ct]);
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    os[(wc0 + 16 * ct + x) * U::OLD + 16 * ot + MT::rrow(g, v)] = o[ct][v];
        }
        __syncthreads();
        const int R = h ? Rr[1] : Rr[0];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const int Cc = c ? Cq[1] : Cq[0];
            const int quad = 2 * h + c;
            if (!hact || !((io.wmask >> quad) & 1)) continue;
            T *dst = ablk + ublk(R < Cc ? R : Cc, R < Cc ? Cc : R) * (size_t)(B * B);
            const int slot = io.smap ? io.smap[quad] : -1;
            T *nx = io.snext && slot >= 0 ? io.snext + (size_t)slot * B * B : nullptr;
            // every read of the tile's inputs ended at GEMM 1's last barrier
            for (int e = tid; e < B * B; e += NTH) {
                int rl, cl;
                if (R < Cc) { rl = e % B; cl = e / B; }
                else { cl = e % B; rl = e / B; }  // stored (Cc, R): element (cl, rl)
                const T v = os[(c * B + cl) * U::OLD + rl];
                dst[e] = v;
                if (nx) nx[e] = v;
            }
        }
        __syncthreads();
    }
}

// Workgroups per critical block (b = 64): each owns 64 / CRIT_SPLIT of the
// block's columns.  The critical blocks run while the rest of the GPU
// waits for them, so their products are spread over more CUs.
constexpr int CRIT_SPLIT = 4;

// Columns part * 64 / NS .. of one block of tile (p, q) for b = 64 (FP64 or
// FP32, the MFMA conventions of MfmaTraits<T>): row half h, column half c, by
// 512 threads, latency first.  One round of
// global loads brings the whole input tile (to LDS; the block itself from
// its copy `orig`, which no workgroup writes), the V_q operands of the
// part's columns and the half of V_p that GEMM 2 reads (each value once, to
// LDS after GEMM 1).  Wave w = CTW rg + ctl (CTW = 4 / NS column tiles of 16)
// computes T's column tile ctl for row tiles RTW rg .. (GEMM 1) and hands it
// over through LDS in GEMM 2's operand order; GEMM 2 gives the waves the
// output tiles (row tile ot of half h, column tile ctl).  Two waves per SIMD:
// one wave's LDS waits are the other's MFMA time.  The part's columns of the
// new block are written in place.  `lds` holds 128 x 129 values of T.
template <int NS, class T>
__device__ __forceinline__ void ua_block64(const int *__restrict__ pairs, T *__restrict__ ablk,
                                           const T *__restrict__ vhat, int p, int q, bool idp, bool idq, int h,
                                           int c, int part, const T *__restrict__ orig, T *lds) {
    using MT = MfmaTraits<T>;
    typedef typename MT::acc_t acc_t;
    constexpr int B = 64, M2 = 128, XLD = M2 + 1, NTH = 512, PB = B * B / NTH;
    constexpr int VH = M2 * B;           // V_p(:, half h): 128 x 64
    constexpr int CTW = 4 / NS;          // column tiles of this part
    constexpr int RW = 8 / CTW;          // row groups of GEMM 1
    constexpr int RTW = 8 / RW;          // row tiles per wave in GEMM 1
    constexpr int NOT = 4 * CTW;         // output tiles of GEMM 2
    constexpr int OTW = NOT >= 8 ? NOT / 8 : 1;  // output tiles per working wave
    static_assert(NS == 1 || NS == 2 || NS == 4, "split of a critical block");
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int g = lane >> 4, x = lane & 15;
    const int ctl = w % CTW, rg = w / CTW;
    const int Rr[2] = {pairs[2 * p], pairs[2 * p + 1]};
    const int Cq[2] = {pairs[2 * q], pairs[2 * q + 1]};
    const T *vp = vhat + (size_t)p * M2 * M2;
    const T *vq = vhat + (size_t)q * M2 * M2;
    auto blk = [&](int hh, int cc) {
        const int R = Rr[hh], C = Cq[cc];
        return ablk + ublk(R < C ? R : C, R < C ? C : R) * (size_t)(B * B);
    };

    // every load at once: the four blocks (contiguous per thread), V_q, V_p's half
    T xr[4][PB];
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
        const T *src = bb == 2 * h + c ? orig : blk(bb >> 1, bb & 1);
#pragma unroll
        for (int m = 0; m < PB; ++m) xr[bb][m] = src[tid + NTH * m];
    }
    const int c0 = 16 * CTW * part;              // first column of this part within the block
    const int col = 64 * c + c0 + 16 * ctl + x;  // this lane's column of T
    T bq[M2 / 4];
#pragma unroll
    for (int s = 0; s < M2 / 4; ++s) {
        const int kg = 16 * (s >> 2) + MT::kstep(s & 3, g);
        bq[s] = op_or_eye(vq + MT::vidx(kg, col, M2), idq, kg == col);
    }
    // V_p(k, 64 h + il) sits at vidx(k, il, 64) of the half's copy: its 32
    // runs of 256 values are contiguous in V_hat too.  Position j of the copy
    // holds il = 16 ((j >> 6) & 3) + (j & 15) and, in run jr = j >> 8, k =
    // 4 jr + ((j >> 4) & 3) (FP64) or 16 (jr >> 2) + 4 ((j >> 4) & 3) + (jr & 3)
    // (FP32).
    T vr[VH / NTH];
#pragma unroll
    for (int m = 0; m < VH / NTH; ++m) {
        const int j = tid + NTH * m, jr = j >> 8;
        const int il = ((j >> 6) & 3) * 16 + (j & 15);
        const int k = std::is_same<T, double>::value ? 4 * jr + ((j >> 4) & 3)
                                                     : 16 * (jr >> 2) + 4 * ((j >> 4) & 3) + (jr & 3);
        vr[m] = op_or_eye(vp + MT::vidx(k, 64 * h + il, M2), idp, k == 64 * h + il);
    }
    // X(row, k) at lds[k XLD + row]: block (hh, cc) holds rows 64 hh .., k 64 cc ..
#pragma unroll
    for (int bb = 0; bb < 4; ++bb) {
        const int hh = bb >> 1, cc = bb & 1;
        const bool tr = Rr[hh] > Cq[cc];  // stored as the mirror (column block, row block)
#pragma unroll
        for (int m = 0; m < PB; ++m) {
            const int e = tid + NTH * m;
            const int rl = tr ? e / B : e % B, kl = tr ? e % B : e / B;
            lds[(64 * cc + kl) * XLD + 64 * hh + rl] = xr[bb][m];
        }
    }
    __syncthreads();

    // GEMM 1: T(row tiles RTW rg .., col tile ctl) = X(those rows, :) V_q(:, col tile)
    acc_t acc[RTW];
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt) acc[rt] = acc_t{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < M2 / 4; ++s) {
        const int kl = 16 * (s >> 2) + MT::kstep(s & 3, g);
#pragma unroll
        for (int rt = 0; rt < RTW; ++rt)
            acc[rt] = MT::mma(lds[kl * XLD + 16 * (RTW * rg + rt) + x], bq[s], acc[rt]);
    }
    __syncthreads();  // X no longer read: V_p's half and T take its place
    // T in GEMM 2's B-operand order: step (rt, s4) of column tile ctl at
    // tops[((4 rt + s4) CTW + ctl) 64 + lane] = T(16 rt + rrow(g, s4), ..),
    // which is component s4 of this wave's acc[rt - RTW rg]
    T *vps = lds;       // V_p(:, half h), vperm order of a 128 x 64 matrix
    T *tops = lds + VH; // 8 x 4 x CTW x 64 values
#pragma unroll
    for (int m = 0; m < VH / NTH; ++m) vps[tid + NTH * m] = vr[m];
#pragma unroll
    for (int rt = 0; rt < RTW; ++rt)
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
            tops[((4 * (RTW * rg + rt) + s4) * CTW + ctl) * 64 + lane] = acc[rt][s4];
    __syncthreads();

    // GEMM 2: output tile n = OTW w + j (row tile ot = n / CTW of half h,
    // column tile n mod CTW) = V_p(:, ..)^T T.  Row tile ot's operand for step
    // (rt, s4) is vperm(16 rt + rrow(g, s4), 16 ot + x, 64) = 256 (4 rt + s4) + 64 ot + lane
    const bool g2 = OTW * w < NOT;  // waves with output tiles
    acc_t o[OTW];
#pragma unroll
    for (int j = 0; j < OTW; ++j) o[j] = acc_t{0, 0, 0, 0};
    if (g2) {
#pragma unroll
        for (int rt = 0; rt < M2 / 16; ++rt)
#pragma unroll
            for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
                for (int j = 0; j < OTW; ++j) {
                    const int n = OTW * w + j, ot = n / CTW, cn = n % CTW;
                    o[j] = MT::mma(vps[256 * (4 * rt + s4) + 64 * ot + lane],
                                   tops[((4 * rt + s4) * CTW + cn) * 64 + lane], o[j]);
                }
    }
    __syncthreads();  // V_p's half and T no longer read
    T *os = lds;  // [part column 0 .. 16 CTW - 1][row 0 .. 63], stride B + 1
    if (g2) {
#pragma unroll
        for (int j = 0; j < OTW; ++j) {
            const int n = OTW * w + j, ot = n / CTW, cn = n % CTW;
#pragma unroll
            for (int v = 0; v < 4; ++v) os[(16 * cn + x) * (B + 1) + 16 * ot + MT::rrow(g, v)] = o[j][v];
        }
    }
    __syncthreads();

    // columns c0 .. c0 + 16 CTW - 1 of block (Rr[h], Cq[c]), in place
    const int R = Rr[h], C = Cq[c];
    T *dst = blk(h, c);
    constexpr int PW = 16 * CTW;  // columns of the part
#pragma unroll
    for (int m = 0; m < B * PW / NTH; ++m) {
        const int e = tid + NTH * m;  // element (rl, c0 + cl) of block (R, C)
        const int rl = R < C ? e % B : e / PW, cl = R < C ? e / B : e % PW;
        const int at = R < C ? (c0 + cl) * B + rl : rl * B + c0 + cl;
        dst[at] = os[cl * (B + 1) + rl];
    }
}

// A tile whose two rotations are both skipped does not change; the copies
// its blocks owe the next round (smap: 4 slots, as in TileIO) are made from
// ablk.
template <int B, class T, int NTH>
__device__ __forceinline__ void copy_skipped(const int *__restrict__ pairs, const T *__restrict__ ablk, int p,
                                             int q, T *__restrict__ snext, const int *smap, int tid) {
#pragma unroll
    for (int quad = 0; quad < 4; ++quad) {
        const int slot = smap[quad];
        if (slot < 0) continue;
        const int R = pairs[2 * p + (quad >> 1)], C = pairs[2 * q + (quad & 1)];
        const T *src = ablk + ublk(R < C ? R : C, R < C ? C : R) * (size_t)(B * B);
        T *dst = snext + (size_t)slot * B * B;
        for (int e = tid; e < B * B; e += NTH) dst[e] = src[e];
    }
}

// Only the critical quadrants qmask[i] of tile i, one tile per workgroup
// (CRIT_SPLIT workgroups for the one-block case of b = 64), from copies
// of their originals at side + 4 i B^2 (+ quad B^2), made beforehand; the
// new blocks are written in place.  Blocks within one column half (b = 64)
// take T for that half only, and V_p^T T for the row halves written: 3/8 of
// a tile's products for one block (the whole tile staged in LDS at once).
// Two opposite blocks, and b = 32, take all of T.
template <int B, class T>
__global__ void __launch_bounds__(512, 1)
k_update_a_crit(const int *__restrict__ pairs, T *__restrict__ ablk, const T *__restrict__ vhat,
                const int *__restrict__ flags, const int *__restrict__ tiles, const int *__restrict__ qmask,
                const T *__restrict__ side) {
    extern __shared__ double lds_raw[];
    constexpr int NS = B == 64 ? CRIT_SPLIT : 1;
    // Workgroups are dispatched round-robin over the 8 XCDs (each with its
    // own L2): workgroup w runs on XCD w mod 8.  Numbering the (tile, part)
    // units XCD by XCD puts the NS parts of a tile on one XCD, so the tile is
    // fetched from HBM into one L2 instead of NS of them (a bijection on the
    // first 8 floor(G / 8) workgroups, identity on the rest).
    const int per = gridDim.x / 8;
    int u = blockIdx.x;
    if (u < 8 * per) u = (u % 8) * per + u / 8;
    const int i = u / NS, part = u % NS;
    const int p = tiles[2 * i], q = tiles[2 * i + 1];
    const bool idp = flags[p] != 0, idq = flags[q] != 0;
    if (idp && idq) return;  // the tile does not change (and its rest is skipped the same way)
    TileIO<T> io;
    io.wmask = qmask[i] & 15;
    io.rmask = io.wmask;
    io.side = const_cast<T *>(side) + (size_t)4 * i * B * B;
    T *lds = reinterpret_cast<T *>(lds_raw);
    const int m = io.wmask;
    if constexpr (B == 64) {
        if (m == 1 || m == 2 || m == 4 || m == 8) {  // one block: bit 2 h + c
            const int quad = m == 1 ? 0 : m == 2 ? 1 : m == 4 ? 2 : 3;
            ua_block64<NS, T>(pairs, ablk, vhat, p, q, idp, idq, quad >> 1, quad & 1, part,
                           io.side + (size_t)quad * B * B, lds);
            return;
        }
    }
    if (part != 0) return;  // the other masks take one workgroup per tile
    // four waves work, the other four take the same barriers
    const int t = threadIdx.x & 255;
    const bool act = threadIdx.x < 256;
    if constexpr (B == 64) {
        if ((m & 10) == 0 || (m & 5) == 0) {  // one column half (bits 1, 4: column 0; 2, 8: column 1)
            ua_tile<B, T, 256, true>(pairs, ablk, vhat, p, q, idp, idq, t, lds, act, io, (m & 5) ? 0 : 1);
            return;
        }
    }
    ua_tile<B, T>(pairs, ablk, vhat, p, q, idp, idq, t, lds, act, io);
}

// Copies of n blocks of ablk: block lst[2 j] (a slot of the upper block
// storage) to side + lst[2 j + 1] B^2, one block per workgroup.
template <int B, class T>
__global__ void k_copy_blocks(const T *__restrict__ ablk, const int *__restrict__ lst, T *__restrict__ side) {
    const T *src = ablk + (size_t)lst[2 * blockIdx.x] * B * B;
    T *dst = side + (size_t)lst[2 * blockIdx.x + 1] * B * B;
    for (int e = threadIdx.x; e < B * B; e += blockDim.x) dst[e] = src[e];
}

// The same tiles on a bounded set of CUs (as k_update_q_bounded): 512 threads
// and an LDS request that keeps one workgroup per CU, so a grid of
// CUs - reserve leaves `reserve` CUs free.  b = 64: one tile at a time on all
// eight waves (one 16-column tile of T each), tile k gridDim + blockIdx;
// b = 32: two 256-thread halves with their own LDS, each one tile at a time
// (tile 2 (k gridDim + blockIdx) + half).  The first nq tiles are critical
// tiles whose quadrants qmask[i] were done by k_update_a_crit: those are read
// from their saved originals and not written.
template <int B, class T>
__global__ void __launch_bounds__(512, 1)
k_update_a_bounded(const int *__restrict__ pairs, T *__restrict__ ablk, const T *__restrict__ vhat,
                   const int *__restrict__ flags, const int *__restrict__ tiles, int ntiles,
                   const int *__restrict__ qmask, int nq, T *__restrict__ side, T *__restrict__ snext,
                   const int *__restrict__ smap) {
    extern __shared__ double lds_raw[];
    auto tile_io = [&](int i) {
        TileIO<T> io;
        if (i < nq) {
            io.rmask = qmask[i] & 15;
            io.wmask = 15 & ~io.rmask;
            io.side = side + (size_t)4 * i * B * B;
        }
        if (snext && i < ntiles) {
            io.snext = snext;
            io.smap = smap + 4 * i;
        }
        return io;
    };
    if constexpr (B == 64) {
        T *lds = reinterpret_cast<T *>(lds_raw);
        for (int i = blockIdx.x; i < ntiles; i += gridDim.x) {
            const int p = tiles[2 * i], q = tiles[2 * i + 1];
            const bool idp = flags[p] != 0, idq = flags[q] != 0;
            if (idp && idq) {  // uniform over the workgroup
                if (snext) copy_skipped<B, T, 512>(pairs, ablk, p, q, snext, smap + 4 * i, threadIdx.x);
                continue;
            }
            ua_tile<B, T, 512>(pairs, ablk, vhat, p, q, idp, idq, threadIdx.x, lds, true, tile_io(i));
        }
    } else {
        using U = UaCfg<B>;
        const int half = threadIdx.x >> 8, t = threadIdx.x & 255;
        T *lds = reinterpret_cast<T *>(reinterpret_cast<char *>(lds_raw) + half * U::LDS_BYTES);
        for (int i0 = 2 * blockIdx.x; i0 < ntiles; i0 += 2 * gridDim.x) {
            const int i = i0 + half;
            const int p = i < ntiles ? tiles[2 * i] : 0, q = i < ntiles ? tiles[2 * i + 1] : 1;
            const bool idp = flags[p] != 0, idq = flags[q] != 0;
            const bool active = i < ntiles && !(idp && idq);
            ua_tile<B, T>(pairs, ablk, vhat, p, q, idp, idq, t, lds, active, tile_io(i));
            if (i < ntiles && idp && idq && snext) copy_skipped<B, T, 256>(pairs, ablk, p, q, snext, smap + 4 * i, t);
        }
    }
}

// Q(r0 .. r0+127, [I,J]) <- Q(r0 .. r0+127, [I,J]) V_p, computed as
// out^T = V_p^T X^T so that lanes hold consecutive rows of the column-major Q.
// NW waves (t = 0 .. 64 NW - 1) in a 2 x NW/2 layout: wave (wi, wj) owns out
// columns b wi .. b wi + b-1 (of the 2b pair columns) and 128 / (NW / 2) Q
// rows from r0 + wj 128 / (NW / 2).  `active` false: no work, but the
// barrier before the in-place store is still taken (the caller's barrier
// count).
template <int B, class T, int NW = 4>
__device__ __forceinline__ void uq_item(const int *__restrict__ pairs, T *__restrict__ Q, int ldq,
                                        const T *__restrict__ vhat, int p, int rb, int t, bool active) {
    using MT = MfmaTraits<T>;
    typedef typename MT::acc_t acc_t;
    constexpr int M2 = 2 * B;
    constexpr int HALF = M2 / 2;     // out columns per wave
    constexpr int IT = HALF / 16;    // 16-tiles of out columns per wave
    constexpr int RW = 128 / (NW / 2);  // rows per wave
    constexpr int JT = RW / 16;      // 16-tiles of rows per wave
    const int I = active ? pairs[2 * p] : 0, J = active ? pairs[2 * p + 1] : 0;
    const T *vp = vhat + (size_t)p * M2 * M2;
    const int lane = t & 63, w = t >> 6;
    const int g = lane >> 4, x = lane & 15;
    const int wi = w & 1, wj = w >> 1;
    const size_t r0 = (size_t)rb * 128 + RW * wj;

    acc_t acc[IT][JT];
#pragma unroll
    for (int i = 0; i < IT; ++i)
#pragma unroll
        for (int j = 0; j < JT; ++j) acc[i][j] = acc_t{0, 0, 0, 0};

    auto colof = [&](int k) { return k < B ? I * B + k : J * B + (k - B); };

    if (active) {
        // operands of step st: V_p rows and Q columns (contraction index k),
        // fetched a step ahead
        auto fetch = [&](int st, T *a, T *b) {
            const int k = 16 * (st >> 2) + MT::kstep(st & 3, g);
            const T *qc = Q + (size_t)colof(k) * ldq + r0;
#pragma unroll
            for (int i = 0; i < IT; ++i) a[i] = vp[MT::vidx(k, HALF * wi + 16 * i + x, M2)];
#pragma unroll
            for (int j = 0; j < JT; ++j) b[j] = qc[16 * j + x];
        };
        T an[IT], bn[JT];
        fetch(0, an, bn);
#pragma unroll 4
        for (int st = 0; st < M2 / 4; ++st) {
            T a_[IT], b_[JT];
#pragma unroll
            for (int i = 0; i < IT; ++i) a_[i] = an[i];
#pragma unroll
            for (int j = 0; j < JT; ++j) b_[j] = bn[j];
            if (st + 1 < M2 / 4) fetch(st + 1, an, bn);
#pragma unroll
            for (int i = 0; i < IT; ++i)
#pragma unroll
                for (int j = 0; j < JT; ++j) acc[i][j] = MT::mma(a_[i], b_[j], acc[i][j]);
        }
    }
    // the two waves sharing these rows read every pair column: wait for both
    // before the in-place store
    __syncthreads();
    if (active) {
#pragma unroll
        for (int i = 0; i < IT; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                T *qc = Q + (size_t)colof(HALF * wi + 16 * i + MT::rrow(g, v)) * ldq + r0;
#pragma unroll
                for (int j = 0; j < JT; ++j) qc[16 * j + x] = acc[i][j][v];
            }
    }
}

// One 128-row block of one pair per workgroup: grid (n_rows / 128, npairs).
template <int B, class T>
__global__ void __launch_bounds__(256, 2)
k_update_q(const int *__restrict__ pairs, T *__restrict__ Q, int ldq,
           const T *__restrict__ vhat, const int *__restrict__ flags) {
    const int p = blockIdx.y;
    if (flags[p]) return;
    uq_item<B, T>(pairs, Q, ldq, vhat, p, blockIdx.x, threadIdx.x, true);
}

// The same work on a bounded set of CUs: 512 threads, one row block of one
// pair at a time on all eight waves (item k gridDim + blockIdx: row block
// i mod nrb of pair i / nrb), and a dynamic LDS request larger than half a
// CU's, so each workgroup holds a CU of its own and a grid of CUs - reserve
// workgroups leaves `reserve` CUs free for the subproblem kernel that runs
// beside it.
template <int B, class T>
__global__ void __launch_bounds__(512, 1)
k_update_q_bounded(const int *__restrict__ pairs, T *__restrict__ Q, int ldq,
                   const T *__restrict__ vhat, const int *__restrict__ flags, int nrb, int nwork) {
    for (int i = blockIdx.x; i < nwork; i += gridDim.x) {
        const int p = i / nrb, rb = i - p * nrb;
        if (flags[p]) continue;  // V_p = I (uniform over the workgroup)
        uq_item<B, T, 8>(pairs, Q, ldq, vhat, p, rb, threadIdx.x, true);
    }
}
constexpr size_t UQ_BOUNDED_LDS = 81 * 1024;  // > half of the 160 KB LDS: one workgroup per CU

// The rest of every tile (as k_update_a_bounded, b = 64) and the Q update (as
// k_update_q_bounded) of one round in one persistent kernel on a bounded set
// of CUs, all eight waves on one item at a time.  Items 0 .. ntiles-1 are
// tiles, ntiles .. ntiles + nqw - 1 row blocks of Q (item ntiles + j: row
// block j mod nrb of pair j / nrb).  Workgroup b takes items b + k G (G =
// gridDim) while they fill whole rounds; the last, partial round goes to the
// workgroups that took one tile fewer (from ntiles mod G on), since a tile
// costs about two row blocks.
template <class T>
__global__ void __launch_bounds__(512, 1)
k_update_aq_bounded(const int *__restrict__ pairs, T *__restrict__ ablk, const T *__restrict__ vhat,
                    const int *__restrict__ flags, const int *__restrict__ tiles, int ntiles,
                    const int *__restrict__ qmask, int nq, T *__restrict__ side, T *__restrict__ snext,
                    const int *__restrict__ smap, T *__restrict__ Q, int ldq, int nrb, int nqw) {
    constexpr int B = 64;
    extern __shared__ double lds_raw[];
    T *lds = reinterpret_cast<T *>(lds_raw);
    const int G = gridDim.x, b = blockIdx.x;
    const int nwork = ntiles + nqw, nfull = nwork / G * G, nh = ntiles % G;
    for (int v = b; v < nfull + G; v += G) {  // every workgroup visits the partial round's slot
        int i = v;
        if (v >= nfull) {  // the partial round: workgroup b takes item nfull + (b - nh) mod G
            const int pos = (b - nh + G) % G;
            if (pos >= nwork - nfull) break;
            i = nfull + pos;
        }
        if (i < ntiles) {
            const int p = tiles[2 * i], q = tiles[2 * i + 1];
            const bool idp = flags[p] != 0, idq = flags[q] != 0;
            if (idp && idq) {  // uniform over the workgroup
                if (snext) copy_skipped<B, T, 512>(pairs, ablk, p, q, snext, smap + 4 * i, threadIdx.x);
                continue;
            }
            TileIO<T> io;
            if (i < nq) {
                io.rmask = qmask[i] & 15;
                io.wmask = 15 & ~io.rmask;
                io.side = side + (size_t)4 * i * B * B;
            }
            if (snext) {
                io.snext = snext;
                io.smap = smap + 4 * i;
            }
            ua_tile<B, T, 512>(pairs, ablk, vhat, p, q, idp, idq, threadIdx.x, lds, true, io);
        } else {
            const int j = i - ntiles, p = j / nrb, rb = j - p * nrb;
            if (flags[p]) continue;  // V_p = I
            uq_item<B, T, 8>(pairs, Q, ldq, vhat, p, rb, threadIdx.x, true);
        }
    }
}

int device_cus();

template <class T>
void launch_uaq(int b, int npairs, const int *pairs, T *ablk, const T *vhat, const int *flags, const int *tiles,
                int ntiles, const int *qmask, int nq, T *side, T *snext, const int *smap, T *Q, int ldq, int n_rows,
                int reserve, hipStream_t s) {
    if (b != 64 || reserve <= 0 || n_rows % 128 != 0 || (nq > 0 && (!qmask || !side)) || nq > ntiles ||
        (snext && !smap)) {
        set_error("fused update kernel: b = 64, a positive reserve, 128-row blocks of Q");
        throw HipFail{hipErrorInvalidValue};
    }
    const size_t lds = std::max<size_t>(UaCfg<64, 512>::LDS_BYTES, 81 * 1024);
    ensure_lds_limit(reinterpret_cast<const void *>(&k_update_aq_bounded<T>), (int)lds);
    const int nrb = n_rows / 128, nqw = Q ? nrb * npairs : 0;
    const int nwork = std::max(ntiles, 0) + nqw;
    if (nwork <= 0) return;
    const int grid = std::max(1, std::min(device_cus() - reserve, nwork));
    hipLaunchKernelGGL((k_update_aq_bounded<T>), dim3(grid), dim3(512), lds, s, pairs, ablk, vhat, flags, tiles,
                       std::max(ntiles, 0), qmask, nq, side, snext, smap, Q, ldq, nrb, nqw);
    JX_LAUNCHED();
}

int device_cus();

template <int B, class T>
void launch_ua_bounded(const int *pairs, T *ablk, const T *vhat, const int *flags, const int *tiles, int ntiles,
                       int reserve, const int *qmask, int nq, T *side, T *snext, const int *smap, hipStream_t s) {
    // one tile's LDS (b = 64) or two halves' (b = 32), and more than half a
    // CU's in any case: one workgroup per CU
    size_t need = 2 * UaCfg<B>::LDS_BYTES;
    if constexpr (B == 64) need = UaCfg<B, 512>::LDS_BYTES;
    const size_t lds = std::max<size_t>(need, 81 * 1024);
    ensure_lds_limit(reinterpret_cast<const void *>(&k_update_a_bounded<B, T>), (int)lds);
    const int grid = std::max(1, std::min(device_cus() - reserve, B == 64 ? ntiles : (ntiles + 1) / 2));
    hipLaunchKernelGGL((k_update_a_bounded<B, T>), dim3(grid), dim3(512), lds, s, pairs, ablk, vhat, flags, tiles,
                       ntiles, qmask, nq, side, snext, smap);
    JX_LAUNCHED();
}

template <int B, class T>
void launch_ua_crit(const int *pairs, T *ablk, const T *vhat, const int *flags, const int *tiles, int ntiles,
                    const int *qmask, const T *side, hipStream_t s) {
    using U = UaCfg<B>;
    // more than half a CU's LDS: no CU shared with the bounded kernels on the
    // other stream, nor with a second critical tile (b = 64: a whole tile)
    size_t need = U::LDS_BYTES;
    if constexpr (B == 64) need = std::max(need, sizeof(T) * 128 * 129);
    const size_t lds = std::max<size_t>(need, 81 * 1024);
    ensure_lds_limit(reinterpret_cast<const void *>(&k_update_a_crit<B, T>), (int)lds);
    const int ns = B == 64 ? CRIT_SPLIT : 1;
    hipLaunchKernelGGL((k_update_a_crit<B, T>), dim3(ntiles * ns), dim3(512), lds, s, pairs, ablk, vhat, flags,
                       tiles, qmask, side);
    JX_LAUNCHED();
}

template <class T>
void launch_ua(int b, int npairs, const int *pairs, T *ablk, const T *vhat, const int *flags, const int *tiles,
               int ntiles, int reserve, const int *qmask, int nq, T *side, T *snext, const int *smap,
               hipStream_t s) {
    if (ntiles <= 0) return;
    if (b != 64 && b != 32) { set_error("update kernel: block size must be 32 or 64"); throw HipFail{hipErrorInvalidValue}; }
    if ((reserve == UA_QUAD || nq > 0) && (!qmask || !side || nq > ntiles)) {
        set_error("update kernel: quadrant split without masks or side blocks");
        throw HipFail{hipErrorInvalidValue};
    }
    if (snext && !smap) {
        set_error("update kernel: next-round copies without their slot map");
        throw HipFail{hipErrorInvalidValue};
    }
    if (reserve == UA_QUAD) {
        if (b == 64) launch_ua_crit<64, T>(pairs, ablk, vhat, flags, tiles, ntiles, qmask, side, s);
        else launch_ua_crit<32, T>(pairs, ablk, vhat, flags, tiles, ntiles, qmask, side, s);
        return;
    }
    if (reserve <= 0) {
        set_error("update kernel: reserve must be positive (bounded kernel) or UA_QUAD");
        throw HipFail{hipErrorInvalidValue};
    }
    if (b == 64) launch_ua_bounded<64, T>(pairs, ablk, vhat, flags, tiles, ntiles, reserve, qmask, nq, side, snext,
                                          smap, s);
    else launch_ua_bounded<32, T>(pairs, ablk, vhat, flags, tiles, ntiles, reserve, qmask, nq, side, snext, smap, s);
}

// CUs of the current device (cached per device).
int device_cus() {
    static int cus[64] = {0};
    int dev = 0;
    JX_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return 256;
    if (!cus[dev]) {
        hipDeviceProp_t pr;
        JX_HIP(hipGetDeviceProperties(&pr, dev));
        cus[dev] = pr.multiProcessorCount;
    }
    return cus[dev];
}

template <int B, class T>
void launch_uq_bounded(int npairs, const int *pairs, T *Q, int ldq, int n_rows, const T *vhat, const int *flags,
                       int reserve, hipStream_t s) {
    ensure_lds_limit(reinterpret_cast<const void *>(&k_update_q_bounded<B, T>), (int)UQ_BOUNDED_LDS);
    const int nrb = n_rows / 128, nwork = nrb * npairs;
    const int grid = std::max(1, std::min(device_cus() - reserve, nwork));
    hipLaunchKernelGGL((k_update_q_bounded<B, T>), dim3(grid), dim3(512), UQ_BOUNDED_LDS, s, pairs, Q, ldq, vhat,
                       flags, nrb, nwork);
    JX_LAUNCHED();
}

template <class T>
void launch_uq(int b, int npairs, const int *pairs, T *Q, int ldq, int n_rows, const T *vhat, const int *flags,
               int reserve, hipStream_t s) {
    if (npairs <= 0 || n_rows <= 0) return;
    if (b != 64 && b != 32) { set_error("update kernel: block size must be 32 or 64"); throw HipFail{hipErrorInvalidValue}; }
    if (reserve > 0) {
        if (b == 64) launch_uq_bounded<64, T>(npairs, pairs, Q, ldq, n_rows, vhat, flags, reserve, s);
        else launch_uq_bounded<32, T>(npairs, pairs, Q, ldq, n_rows, vhat, flags, reserve, s);
        return;
    }
    dim3 grid(n_rows / 128, npairs);
    if (b == 64) hipLaunchKernelGGL((k_update_q<64, T>), grid, dim3(256), 0, s, pairs, Q, ldq, vhat, flags);
    else hipLaunchKernelGGL((k_update_q<32, T>), grid, dim3(256), 0, s, pairs, Q, ldq, vhat, flags);
    JX_LAUNCHED();
}

}  // namespace

void launch_update_a(int b, int npairs, const int *pairs, double *ablk, const double *vhat,
                     const int *flags, const int *tiles, int ntiles, hipStream_t s, int reserve,
                     const int *qmask, int nq, void *side, void *snext, const int *smap) {
    launch_ua<double>(b, npairs, pairs, ablk, vhat, flags, tiles, ntiles, reserve, qmask, nq,
                      static_cast<double *>(side), static_cast<double *>(snext), smap, s);
}
void launch_update_a32(int b, int npairs, const int *pairs, float *ablk, const float *vhat, const int *flags,
                       const int *tiles, int ntiles, hipStream_t s, int reserve, const int *qmask, int nq,
                       void *side, void *snext, const int *smap) {
    launch_ua<float>(b, npairs, pairs, ablk, vhat, flags, tiles, ntiles, reserve, qmask, nq,
                     static_cast<float *>(side), static_cast<float *>(snext), smap, s);
}
void launch_update_aq(int b, int npairs, const int *pairs, double *ablk, const double *vhat, const int *flags,
                      const int *tiles, int ntiles, const int *qmask, int nq, void *side, void *snext,
                      const int *smap, double *Q, int ldq, int n_rows, int reserve, hipStream_t s) {
    launch_uaq<double>(b, npairs, pairs, ablk, vhat, flags, tiles, ntiles, qmask, nq, static_cast<double *>(side),
                       static_cast<double *>(snext), smap, Q, ldq, n_rows, reserve, s);
}
void launch_update_aq32(int b, int npairs, const int *pairs, float *ablk, const float *vhat, const int *flags,
                        const int *tiles, int ntiles, const int *qmask, int nq, void *side, void *snext,
                        const int *smap, float *Q, int ldq, int n_rows, int reserve, hipStream_t s) {
    launch_uaq<float>(b, npairs, pairs, ablk, vhat, flags, tiles, ntiles, qmask, nq, static_cast<float *>(side),
                      static_cast<float *>(snext), smap, Q, ldq, n_rows, reserve, s);
}
void launch_copy_blocks(int b, const double *ablk, const int *lst, int n, void *side, hipStream_t s) {
    if (n <= 0) return;
    if (b == 64)
        hipLaunchKernelGGL((k_copy_blocks<64, double>), dim3(n), dim3(256), 0, s, ablk, lst, static_cast<double *>(side));
    else
        hipLaunchKernelGGL((k_copy_blocks<32, double>), dim3(n), dim3(256), 0, s, ablk, lst, static_cast<double *>(side));
    JX_LAUNCHED();
}
void launch_copy_blocks32(int b, const float *ablk, const int *lst, int n, void *side, hipStream_t s) {
    if (n <= 0) return;
    if (b == 64)
        hipLaunchKernelGGL((k_copy_blocks<64, float>), dim3(n), dim3(256), 0, s, ablk, lst, static_cast<float *>(side));
    else
        hipLaunchKernelGGL((k_copy_blocks<32, float>), dim3(n), dim3(256), 0, s, ablk, lst, static_cast<float *>(side));
    JX_LAUNCHED();
}
void launch_update_q(int b, int npairs, const int *pairs, double *Q, int ldq, int n_rows,
                     const double *vhat, const int *flags, hipStream_t s, int reserve) {
    launch_uq<double>(b, npairs, pairs, Q, ldq, n_rows, vhat, flags, reserve, s);
}
void launch_update_q32(int b, int npairs, const int *pairs, float *Q, int ldq, int n_rows, const float *vhat,
                       const int *flags, hipStream_t s, int reserve) {
    launch_uq<float>(b, npairs, pairs, Q, ldq, n_rows, vhat, flags, reserve, s);
}

}  // namespace jx
