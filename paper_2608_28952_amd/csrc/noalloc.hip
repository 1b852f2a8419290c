// noalloc.hip -- jacobi_eig_noalloc: jacobi_eig with its workspace in a
// fixed device array of this library instead of caller- or library-allocated
// memory, for callers that cannot allocate device memory.
//
// `scratch` below is a __device__ array: every GPU the library runs on holds
// its own copy at its own address, from the code object's load until the
// process ends.  Host code never uses the array's name as an address (on the
// host it is only a stand-in); set-up records, per device, the address that
// hipGetSymbolAddress returns, and the solver receives that address as its
// workspace.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>

#include "jx_common.hpp"
#include "jx_host.hpp"

namespace jx {

namespace {

constexpr size_t NOALLOC_BYTES = (size_t)64 << 20;  // 64 MiB per device

__device__ __align__(256) char scratch[NOALLOC_BYTES];

std::mutex g_mu;
std::map<int, void *> g_scratch;  // device ordinal -> device address of `scratch`

}  // namespace

// Set-up for the current device (once per device; later calls return the
// recorded address).  Returns the device address of that device's array.
void *noalloc_setup() {
    int dev = 0;
    JX_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_scratch.find(dev);
    if (it != g_scratch.end()) return it->second;
    void *ptr = nullptr;
    JX_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) {
        set_error("hipGetSymbolAddress returned a null address for the scratch array");
        throw HipFail{hipErrorInvalidSymbol};
    }
    g_scratch[dev] = ptr;
    return ptr;
}

size_t noalloc_bytes() { return NOALLOC_BYTES; }

}  // namespace jx

using namespace jx;

extern "C" {

size_t jacobi_eig_noalloc_max_bytes(void) { return NOALLOC_BYTES; }

int jacobi_eig_noalloc(int n, const double *dA, int lda, char uplo, double *dW, double *dQ, int ldq,
                       const double *dQ0, int ldq0, const jacobi_opts *opts, jacobi_info *info,
                       jacobi_stream_t stream) {
    if (info) *info = jacobi_info{};
    if (n > 1) {
        const size_t need = jacobi_eig_workspace(n, opts);
        if (need > NOALLOC_BYTES) {  // (0: invalid options, reported by jacobi_eig)
            set_error("jacobi_eig_noalloc: order " + std::to_string(n) + " with these options needs " +
                      std::to_string(need) + " bytes of workspace; the static scratch array holds " +
                      std::to_string(NOALLOC_BYTES));
            if (info) info->status = -1;
            return -1;
        }
    }
    void *ws = nullptr;
    try {
        (void)device_ctx();  // set-up on the first call on this device (jacobi_init does it earlier)
        ws = noalloc_setup();
    } catch (const HipFail &) {
        if (info) info->status = 3;
        return 3;
    }
    return jacobi_eig(n, dA, lda, uplo, dW, dQ, ldq, dQ0, ldq0, ws, NOALLOC_BYTES, opts, info, stream);
}

}  // extern "C"
