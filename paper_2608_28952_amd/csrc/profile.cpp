// profile.cpp -- optional per-kernel timing of the solver's hot kernels.
//
// While enabled (jacobi_profile_enable), the drivers record a HIP event pair
// on the launch stream around every launch of the subproblem, pair-tile
// update, Q update and GEMM kernels, together with that launch's algorithmic
// work (flops and HBM bytes the method needs, not what the kernel happens to
// execute).  jacobi_profile_query sums the records of one kernel kind.
#include "jx_prof.hpp"

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

namespace jx {

namespace {
struct Rec {
    int kind;
    hipEvent_t a, b;
    double flops, bytes;
    int flag_slot;   // >= 0: work depends on the skip flags stored at this slot
    int npairs;
    int m2;
};
std::mutex g_mu;
bool g_on = false;
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;
std::vector<int> g_flag_log;  // host copy of skip flags for slot-dependent records

hipEvent_t get_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    JX_HIP(hipEventCreate(&e));
    return e;
}
}  // namespace

bool prof_on() { return g_on; }

ProfScope::ProfScope(int kind, hipStream_t s, double flops, double bytes, int flag_slot, int npairs, int m2)
    : active(g_on), kind(kind), s(s), flops(flops), bytes(bytes), flag_slot(flag_slot), npairs(npairs), m2(m2) {
    if (!active) return;
    std::lock_guard<std::mutex> lk(g_mu);
    a = get_event();
    b = get_event();
    JX_HIP(hipEventRecord(a, s));
}

ProfScope::~ProfScope() noexcept(false) {
    if (!active) return;
    JX_HIP(hipEventRecord(b, s));
    std::lock_guard<std::mutex> lk(g_mu);
    g_recs.push_back(Rec{kind, a, b, flops, bytes, flag_slot, npairs, m2});
}

int prof_flag_base() {
    std::lock_guard<std::mutex> lk(g_mu);
    return (int)g_flag_log.size();
}

void prof_add_flags(const std::vector<int> &flags) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_flag_log.insert(g_flag_log.end(), flags.begin(), flags.end());
}

// Algorithmic work of a pair-tile update launch given the round's flags:
// a tile needs one 2b x 2b x 2b product per rotated side.
static void tile_work(const int *f, int H, int m2, double &flops, double &bytes) {
    const double prod = 2.0 * m2 * (double)m2 * m2;
    const double tile_bytes = 2.0 * m2 * (double)m2 * sizeof(double);
    flops = bytes = 0.0;
    for (int p = 0; p < H; ++p)
        for (int q = p + 1; q < H; ++q) {
            const int sides = (f[p] ? 0 : 1) + (f[q] ? 0 : 1);
            if (!sides) continue;
            flops += sides * prod;
            bytes += tile_bytes;
        }
}

static void qupd_work(const int *f, int H, int m2, double rows, double &flops, double &bytes) {
    flops = bytes = 0.0;
    for (int p = 0; p < H; ++p) {
        if (f[p]) continue;
        flops += 2.0 * rows * m2 * (double)m2;
        bytes += 2.0 * rows * m2 * sizeof(double);
    }
}

}  // namespace jx

using namespace jx;

extern "C" int jacobi_profile_enable(int on) {
    try {
        JX_HIP(hipDeviceSynchronize());
        std::lock_guard<std::mutex> lk(g_mu);
        for (auto &r : g_recs) {
            g_pool.push_back(r.a);
            g_pool.push_back(r.b);
        }
        g_recs.clear();
        g_flag_log.clear();
        g_on = on != 0;
        return 0;
    } catch (const HipFail &) {
        return 3;
    }
}

extern "C" int jacobi_profile_query(int kind, int *launches, double *total_ms, double *flops, double *bytes) {
    try {
        JX_HIP(hipDeviceSynchronize());
        std::lock_guard<std::mutex> lk(g_mu);
        int cnt = 0;
        double ms = 0.0, fl = 0.0, by = 0.0;
        for (const auto &r : g_recs) {
            if (r.kind != kind) continue;
            float t = 0.0f;
            JX_HIP(hipEventElapsedTime(&t, r.a, r.b));
            ++cnt;
            ms += t;
            if (r.flag_slot >= 0 && r.flag_slot + r.npairs <= (int)g_flag_log.size()) {
                double f = 0.0, b = 0.0;
                const int *fl_ = g_flag_log.data() + r.flag_slot;
                if (kind == PROF_UPDATE_A || kind == PROF_UPDATE_A_REST) {  // r.flops: share of the round's tiles
                    tile_work(fl_, r.npairs, r.m2, f, b);
                    const double share = r.flops > 0.0 ? r.flops : 1.0;
                    f *= share;
                    b *= share;
                } else if (kind == PROF_UPDATE_AQ) {  // all tiles, and Q when r.flops (its row count) > 0
                    tile_work(fl_, r.npairs, r.m2, f, b);
                    if (r.flops > 0.0) {
                        double fq = 0.0, bq = 0.0;
                        qupd_work(fl_, r.npairs, r.m2, r.flops, fq, bq);
                        f += fq;
                        b += bq;
                    }
                } else if (kind == PROF_SUBPROBLEM) {  // r.flops / r.bytes: per rotated pair
                    for (int q = 0; q < r.npairs; ++q)
                        if (!fl_[q]) {
                            f += r.flops;
                            b += r.bytes;
                        }
                } else {
                    qupd_work(fl_, r.npairs, r.m2, r.flops, f, b);  // r.flops holds the row count
                }
                fl += f;
                by += b;
            } else if (kind != PROF_UPDATE_A && kind != PROF_UPDATE_A_REST && kind != PROF_UPDATE_AQ) {
                fl += r.flops;
                by += r.bytes;
            }
        }
        if (launches) *launches = cnt;
        if (total_ms) *total_ms = ms;
        if (flops) *flops = fl;
        if (bytes) *bytes = by;
        return 0;
    } catch (const HipFail &) {
        return 3;
    }
}
