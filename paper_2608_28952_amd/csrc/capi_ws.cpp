// capi_ws.cpp -- extern "C" entry points of the learned warm start
// (include/jacobi.h, jws_*): argument checks and dispatch to k_mlp.hip and
// k_cayley.hip.  All calls enqueue on `stream` and return without waiting.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>

#include "jx_common.hpp"
#include "jx_mlp.hpp"

using namespace jx;

namespace {

template <class F>
int ws_guard(const char *name, int bad_arg, F &&f) {
    set_error("");
    if (bad_arg != 0) {
        set_error(std::string(name) + ": invalid argument " + std::to_string(-bad_arg));
        return bad_arg;
    }
    try {
        f();
        return 0;
    } catch (const HipFail &) {
        return 3;
    }
}

}  // namespace

extern "C" {

size_t jws_param_count(void) { return mlp::NPARAM; }

size_t jws_acts_bytes(int batch) {
    return batch > 0 ? sizeof(uint16_t) * mlp::act_off(batch, mlp::ACT_END) : 0;
}

int jws_mlp_forward(int batch, const float *dTheta, const uint16_t *dWbf16, const float *dBias, float *dOut,
                    uint16_t *dActs, jacobi_stream_t stream) {
    const int bad = batch < 0 ? -1 : (batch > 0 && !dTheta) ? -2 : (batch > 0 && !dWbf16) ? -3
                  : (batch > 0 && !dBias) ? -4 : (batch > 0 && !dOut) ? -5 : (batch > 0 && !dActs) ? -6 : 0;
    return ws_guard("jws_mlp_forward", bad, [&] {
        if (batch > 0) mlp_forward(batch, dTheta, dWbf16, dBias, dOut, dActs, (hipStream_t)stream);
    });
}

int jws_mlp_backward(int batch, const uint16_t *dActs, const float *dGradOut, const uint16_t *dWbf16, float *dGradW,
                     float *dGradB, jacobi_stream_t stream) {
    const int bad = batch < 0 ? -1 : (batch > 0 && !dActs) ? -2 : (batch > 0 && !dGradOut) ? -3
                  : (batch > 0 && !dWbf16) ? -4 : (batch > 0 && !dGradW) ? -5 : (batch > 0 && !dGradB) ? -6 : 0;
    return ws_guard("jws_mlp_backward", bad, [&] {
        if (batch > 0) mlp_backward(batch, dActs, dGradOut, dWbf16, dGradW, dGradB, (hipStream_t)stream);
    });
}

int jws_mse(int batch, const float *dOut, const float *dTarget, float *dGradOut, double *dLoss,
            jacobi_stream_t stream) {
    const int bad = batch <= 0 ? -1 : !dOut ? -2 : !dTarget ? -3 : !dLoss ? -5 : 0;
    return ws_guard("jws_mse", bad, [&] {
        mlp_mse((size_t)batch * mlp::NOUT, dOut, dTarget, dGradOut, dLoss, (hipStream_t)stream);
    });
}

int jws_adam_step(int nparams, float *dMaster, uint16_t *dWbf16, const float *dGrad, float *dM, float *dV, float lr,
                  float beta1, float beta2, float eps, int step, jacobi_stream_t stream) {
    const int bad = nparams < 0 ? -1 : !dMaster ? -2 : !dWbf16 ? -3 : !dGrad ? -4 : !dM ? -5 : !dV ? -6
                  : !(lr >= 0.f) ? -7 : !(beta1 >= 0.f && beta1 < 1.f) ? -8 : !(beta2 >= 0.f && beta2 < 1.f) ? -9
                  : !(eps > 0.f) ? -10 : step < 1 ? -11 : 0;
    return ws_guard("jws_adam_step", bad, [&] {
        const float c1 = (float)(1.0 - std::pow((double)beta1, step));
        const float c2 = (float)(1.0 - std::pow((double)beta2, step));
        if (nparams > 0) mlp_adam(nparams, dMaster, dWbf16, dGrad, dM, dV, lr, beta1, beta2, eps, c1, c2, (hipStream_t)stream);
    });
}

int jws_to_bf16(size_t count, const float *dSrc, uint16_t *dDst, jacobi_stream_t stream) {
    const int bad = (count > 0 && !dSrc) ? -2 : (count > 0 && !dDst) ? -3 : 0;
    return ws_guard("jws_to_bf16", bad, [&] { mlp_to_bf16(count, dSrc, dDst, (hipStream_t)stream); });
}

int jws_skew_from_coords(int batch, int n, const float *dCoords, const float *dMean, const float *dStd, double *dS,
                         jacobi_stream_t stream) {
    const int bad = batch < 0 ? -1 : (n < 1 || n > 256) ? -2 : (batch > 0 && !dCoords) ? -3 : (batch > 0 && !dS) ? -6 : 0;
    return ws_guard("jws_skew_from_coords", bad, [&] {
        skew_from_coords(batch, n, dCoords, dMean, dStd, dS, (hipStream_t)stream);
    });
}

int jws_cayley_batched(int batch, int n, const double *dS, const double *dQref, double *dQ0, jacobi_stream_t stream) {
    const int bad = batch < 0 ? -1 : (n < 1 || n > 64) ? -2 : (batch > 0 && !dS) ? -3 : (batch > 0 && !dQref) ? -4
                  : (batch > 0 && !dQ0) ? -5 : 0;
    return ws_guard("jws_cayley_batched", bad, [&] { cayley_batched(batch, n, dS, dQref, dQ0, (hipStream_t)stream); });
}

}  // extern "C"
