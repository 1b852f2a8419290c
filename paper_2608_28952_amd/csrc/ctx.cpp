// ctx.cpp -- the library's per-device context: the second stream that runs
// the rotation work beside the next round's subproblems, the events that
// order the two streams, and pinned host memory for the scalars each sweep
// reads back.  Created once per device (lazily, or by jacobi_init) and kept
// until the process ends, so a solve creates no stream, event or pinned
// buffer of its own.
#include <hip/hip_runtime.h>

#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <utility>

#include "jx_common.hpp"
#include "jx_host.hpp"

namespace jx {

namespace {
std::mutex g_reg_mu;
std::map<int, std::unique_ptr<DeviceCtx>> g_ctx;  // by device ordinal
}  // namespace

DeviceCtx &device_ctx() {
    int dev = 0;
    JX_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_reg_mu);
    auto it = g_ctx.find(dev);
    if (it != g_ctx.end()) return *it->second;
    std::unique_ptr<DeviceCtx> c(new DeviceCtx());
    c->device = dev;
    // default priority; ordering between the two streams of one device only,
    // so the events need no system-scope fence (cache write-back)
    JX_HIP(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
    const unsigned fl = hipEventDisableTiming | hipEventDisableSystemFence;
    for (int i = 0; i < DeviceCtx::NEV; ++i) JX_HIP(hipEventCreateWithFlags(&c->ev[i], fl));
    void *p = nullptr;
    JX_HIP(hipHostMalloc(&p, DeviceCtx::PINNED_BYTES, hipHostMallocDefault));
    c->pinned = static_cast<char *>(p);
    DeviceCtx &ref = *c;
    g_ctx[dev] = std::move(c);
    return ref;
}

void ensure_lds_limit(const void *func, int bytes) {
    static std::mutex mu;
    static std::set<std::pair<int, const void *>> done;
    int dev = 0;
    JX_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(mu);
    if (done.count({dev, func})) return;
    JX_HIP(hipFuncSetAttribute(func, hipFuncAttributeMaxDynamicSharedMemorySize, bytes));
    done.insert({dev, func});
}

}  // namespace jx
