// jx_prof.hpp -- hooks of the optional kernel profiler (profile.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "jx_common.hpp"

namespace jx {

enum ProfKind {
    PROF_SUBPROBLEM = 0,
    PROF_UPDATE_A = 1,       // tile updates on the solve's stream (the critical tiles)
    PROF_UPDATE_Q = 2,
    PROF_GEMM = 3,
    PROF_GRAM = 4,
    PROF_UPDATE_A_REST = 5,  // the other tiles, beside the next round's subproblems
    PROF_UPDATE_AQ = 6       // the other tiles and the Q update in one launch (b = 64)
};

bool prof_on();

// Records an event pair around the launches issued during its lifetime.
// flag_slot >= 0: the work is derived later from the skip flags logged at
// that slot (npairs entries); for PROF_UPDATE_Q `flops` then carries the row
// count of Q.
struct ProfScope {
    bool active;
    int kind;
    hipStream_t s;
    hipEvent_t a{}, b{};
    double flops, bytes;
    int flag_slot, npairs, m2;
    ProfScope(int kind, hipStream_t s, double flops, double bytes, int flag_slot = -1, int npairs = 0,
              int m2 = 0);
    ~ProfScope() noexcept(false);
};

int prof_flag_base();
void prof_add_flags(const std::vector<int> &flags);

}  // namespace jx
