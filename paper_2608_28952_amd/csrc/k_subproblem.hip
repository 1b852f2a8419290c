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
//   * A_hat: LDS, upper triangle only (row-major, element (i, j), i <= j, at
//     i * LD + j).  Index space: rows/columns keep their natural order.
//   * V_hat: registers.  Thread (r, g) holds row r of V_hat at the 16
//     "positions" 16 g .. 16 g + 15.  Positions are paired (2k, 2k+1) in every
//     round; after a round the column content moves one step along the
//     round-robin ring 1 <- 2 <- 4 <- ... <- m2-2 <- m2-1 <- m2-3 <- ... <- 3 <- 1
//     (position 0 stays), so that every index pair meets once per sweep.  Two
//     values per thread cross to the neighbouring lane (lane shuffles).  After
//     m2 - 1 rounds the ring has turned once and positions equal indices.
//   * Rotation angles: computed by m2/2 threads per round into LDS.
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
    static constexpr int LD = M2 + 1;            // LDS row stride of A_hat
    static constexpr int NITEMS = H * (H + 1) / 2;
    static constexpr size_t LDS_BYTES =
        sizeof(double) * ((size_t)M2 * LD + 4 * H + 2 * (NT / 64) + 2) + sizeof(int) * 2 * H;
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
// Index held by position x in round t of a sweep (t < m2 - 1).
__device__ __forceinline__ int index_at(int x, int t, int m2) {
    if (x == 0) return 0;
    int i = ring_index(x, m2) + t;
    if (i >= m2 - 1) i -= m2 - 1;
    return ring_at(i, m2);
}

// Unordered pair-block (k1, k2) of item `it`: distance classes d = 0 .. H/2.
template <int H>
__device__ __forceinline__ void item_pairs(int it, int &k1, int &k2) {
    if (it < H * (H / 2)) {
        int d = it / H;
        k1 = it - d * H;
        k2 = k1 + d;
        if (k2 >= H) k2 -= H;
    } else {
        k1 = it - H * (H / 2);
        k2 = k1 + H / 2;
    }
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

template <int M2, int MODE>
__global__ void __launch_bounds__(SubCfg<M2>::NT) k_subproblem(SubArgs a) {
    using C = SubCfg<M2>;
    constexpr int H = C::H, G = C::G, NT = C::NT, LD = C::LD, B = M2 / 2;
    extern __shared__ double smem[];
    double *As = smem;                       // M2 x LD
    double *cs = As + (size_t)M2 * LD;       // per pair: c, s, t, a_pq
    double *red = cs + 4 * H;                // reduction scratch
    int *pq = reinterpret_cast<int *>(red + 2 * (NT / 64) + 2);  // per pair: p, q

    const int tid = threadIdx.x;
    const int pr = blockIdx.x;
    const double *Bii = nullptr, *Bjj = nullptr, *Bij = nullptr;
    double *Wii = nullptr, *Wjj = nullptr, *Wij = nullptr;

    if (MODE != SUB_PLAIN && a.force_skip && a.force_skip[pr]) {  // placeholder pair
        if (tid == 0 && a.flags) a.flags[pr] = 1;
        return;
    }

    // ---- load the upper triangle of A_hat into LDS ------------------------
    double off2 = 0.0, fro2 = 0.0;
    if (MODE == SUB_EIG) {
        const int I = a.pairs[2 * pr], J = a.pairs[2 * pr + 1];
        Wii = a.ablk + ublk(I, I) * (size_t)(B * B);
        Wjj = a.ablk + ublk(J, J) * (size_t)(B * B);
        Wij = a.ablk + ublk(I, J) * (size_t)(B * B);
        Bii = Wii;
        Bjj = Wjj;
        Bij = Wij;
        for (int e = tid; e < M2 * M2; e += NT) {
            const int r = e % M2, c = e / M2;
            if (r > c) continue;
            double v;
            if (c < B) v = Bii[c * B + r];
            else if (r < B) v = Bij[(c - B) * B + r];
            else v = Bjj[(c - B) * B + (r - B)];
            As[r * LD + c] = v;
            if (r == c) fro2 += v * v;
            else { off2 += 2.0 * v * v; fro2 += 2.0 * v * v; }
        }
    } else {
        const double *src = a.ahat + (size_t)pr * M2 * M2;
        for (int e = tid; e < M2 * M2; e += NT) {
            const int r = e % M2, c = e / M2;
            if (r > c) continue;
            const double v = src[(size_t)c * M2 + r];
            As[r * LD + c] = v;
            if (r == c) fro2 += v * v;
            else { off2 += 2.0 * v * v; fro2 += 2.0 * v * v; }
        }
    }
    off2 = block_sum<NT>(off2, red);
    fro2 = block_sum<NT>(fro2, red);

    if (MODE != SUB_PLAIN) {
        const double off = sqrt(off2);
        if (tid == 0 && a.inner_off) a.inner_off[pr] = off;
        const bool skip = !(off > a.skip_thr);
        if (tid == 0 && a.flags) a.flags[pr] = skip ? 1 : 0;
        if (skip) return;  // V_hat = I, A_hat unchanged
    }

    // ---- V_hat = I in position space ---------------------------------------
    const int r = tid / G, g = tid - (tid / G) * G;
    double V[16];
#pragma unroll
    for (int x = 0; x < 16; ++x) V[x] = (r == 16 * g + x) ? 1.0 : 0.0;

    const int nsw = a.inner_sweeps > 0 ? a.inner_sweeps : 30;
    const double eps = 2.220446049250313e-16;
    for (int sw = 0; sw < nsw; ++sw) {
        if (a.inner_sweeps <= 0 && sw > 0) {
            double o = 0.0;
            for (int e = tid; e < M2 * M2; e += NT) {
                const int rr = e % M2, cc = e / M2;
                if (rr < cc) { const double v = As[rr * LD + cc]; o += 2.0 * v * v; }
            }
            o = block_sum<NT>(o, red);
            if (sqrt(o) <= eps * sqrt(fro2)) break;
        }
        for (int t = 0; t < M2 - 1; ++t) {
            // angles of this round
            if (tid < H) {
                const int p = index_at(2 * tid, t, M2), q = index_at(2 * tid + 1, t, M2);
                const double app = As[p * LD + p], aqq = As[q * LD + q];
                const double apq = As[min(p, q) * LD + max(p, q)];
                double c = 1.0, s = 0.0, tt = 0.0;
                if (apq != 0.0) {
                    const double th = (aqq - app) / (2.0 * apq);
                    tt = 1.0 / (fabs(th) + hypot(1.0, th));
                    if (th < 0.0) tt = -tt;
                    c = 1.0 / sqrt(1.0 + tt * tt);
                    s = tt * c;
                }
                cs[4 * tid] = c;
                cs[4 * tid + 1] = s;
                cs[4 * tid + 2] = tt;
                cs[4 * tid + 3] = apq;
                pq[2 * tid] = p;
                pq[2 * tid + 1] = q;
            }
            __syncthreads();
            // A_hat <- J^T A_hat J, one 2x2 pair-block per item
            for (int it = tid; it < C::NITEMS; it += NT) {
                int k1, k2;
                item_pairs<H>(it, k1, k2);
                if (k1 == k2) {
                    const double apq = cs[4 * k1 + 3];
                    if (apq != 0.0) {
                        const int p = pq[2 * k1], q = pq[2 * k1 + 1];
                        const double tt = cs[4 * k1 + 2];
                        As[p * LD + p] -= tt * apq;
                        As[q * LD + q] += tt * apq;
                        As[min(p, q) * LD + max(p, q)] = 0.0;
                    }
                } else {
                    const int p1 = pq[2 * k1], q1 = pq[2 * k1 + 1];
                    const int p2 = pq[2 * k2], q2 = pq[2 * k2 + 1];
                    const double c1 = cs[4 * k1], s1 = cs[4 * k1 + 1];
                    const double c2 = cs[4 * k2], s2 = cs[4 * k2 + 1];
                    const int i11 = min(p1, p2) * LD + max(p1, p2);
                    const int i12 = min(p1, q2) * LD + max(p1, q2);
                    const int i21 = min(q1, p2) * LD + max(q1, p2);
                    const int i22 = min(q1, q2) * LD + max(q1, q2);
                    const double x11 = As[i11], x12 = As[i12], x21 = As[i21], x22 = As[i22];
                    // left: rows p1, q1
                    const double y11 = c1 * x11 - s1 * x21, y21 = s1 * x11 + c1 * x21;
                    const double y12 = c1 * x12 - s1 * x22, y22 = s1 * x12 + c1 * x22;
                    // right: columns p2, q2
                    As[i11] = c2 * y11 - s2 * y12;
                    As[i12] = s2 * y11 + c2 * y12;
                    As[i21] = c2 * y21 - s2 * y22;
                    As[i22] = s2 * y21 + c2 * y22;
                }
            }
            // V_hat <- V_hat J on this thread's 8 position pairs
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int k = 8 * g + j;
                const double c = cs[4 * k], s = cs[4 * k + 1];
                const double e = V[2 * j], o = V[2 * j + 1];
                V[2 * j] = c * e - s * o;
                V[2 * j + 1] = s * e + c * o;
            }
            // move the column content one step along the ring
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
            __syncthreads();
        }
    }

    // ---- results ------------------------------------------------------------
    if (MODE == SUB_PLAIN) {
        double *vo = a.vout + (size_t)pr * M2 * M2;
#pragma unroll
        for (int x = 0; x < 16; ++x) vo[(size_t)(16 * g + x) * M2 + r] = V[x];
        double *dd = a.dout + (size_t)pr * M2 * M2;
        for (int e = tid; e < M2 * M2; e += NT) {
            const int rr = e % M2, cc = e / M2;
            dd[e] = As[min(rr, cc) * LD + max(rr, cc)];
        }
    } else {
        double *vo = a.vout + (size_t)pr * M2 * M2;
#pragma unroll
        for (int x = 0; x < 16; ++x) vo[vperm(r, 16 * g + x, M2)] = V[x];
        if (MODE == SUB_EIG) {
            // A([I,J],[I,J]) <- D_hat
            for (int e = tid; e < M2 * M2; e += NT) {
                const int rr = e % M2, cc = e / M2;
                const double v = As[min(rr, cc) * LD + max(rr, cc)];
                if (cc < B) {
                    if (rr < B) Wii[cc * B + rr] = v;
                } else if (rr < B) {
                    Wij[(cc - B) * B + rr] = v;
                } else {
                    Wjj[(cc - B) * B + (rr - B)] = v;
                }
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
