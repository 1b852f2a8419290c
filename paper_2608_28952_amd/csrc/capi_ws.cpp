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

int jws_family_matrices(int count, int n, int k, const double *dTheta, const double *dA0, const double *dB, double *dA,
                        jacobi_stream_t stream) {
    const int bad = count < 0 ? -1 : n < 1 ? -2 : k < 0 ? -3 : (count > 0 && k > 0 && !dTheta) ? -4
                  : (count > 0 && !dA0) ? -5 : (count > 0 && k > 0 && !dB) ? -6 : (count > 0 && !dA) ? -7 : 0;
    return ws_guard("jws_family_matrices", bad,
                    [&] { family_matrices(count, n, k, dTheta, dA0, dB, dA, (hipStream_t)stream); });
}

int jws_canonical_targets(int count, int n, const double *dQ, const double *dQref, float *dCoords, int *dKeep,
                          double maxabs, jacobi_stream_t stream) {
    const int bad = count < 0 ? -1 : (n < 2 || n > 64) ? -2 : (count > 0 && !dQ) ? -3 : (count > 0 && !dQref) ? -4
                  : (count > 0 && !dCoords) ? -5 : (count > 0 && !dKeep) ? -6 : !(maxabs > 0.0) ? -7 : 0;
    return ws_guard("jws_canonical_targets", bad,
                    [&] { canonical_targets(count, n, dQ, dQref, dCoords, dKeep, maxabs, (hipStream_t)stream); });
}

size_t jws_column_stats_work(int rows, int cols) {
    if (rows <= 0 || cols <= 0) return 0;
    return sizeof(double) * 2 * (size_t)cols * (size_t)((rows + STATS_CHUNK - 1) / STATS_CHUNK);
}

int jws_column_stats(int rows, int cols, const float *dX, const int *dKeep, int kept, float eps, float *dMean,
                     float *dStd, double *dWork, jacobi_stream_t stream) {
    const int bad = rows < 0 ? -1 : cols < 0 ? -2 : (rows > 0 && !dX) ? -3 : (rows > 0 && !dKeep) ? -4
                  : (kept < 0 || kept > rows) ? -5 : !(eps >= 0.f) ? -6 : (cols > 0 && !dMean) ? -7
                  : (cols > 0 && !dStd) ? -8 : (rows > 0 && cols > 0 && !dWork) ? -9 : 0;
    return ws_guard("jws_column_stats", bad, [&] {
        column_stats(rows, cols, dX, dKeep, kept, eps, dMean, dStd, dWork, STATS_CHUNK, (hipStream_t)stream);
    });
}

int jws_gather_standardize(int kept, const int *dIdx, int xcols, const float *dX, int tcols, const float *dT,
                           const float *dMean, const float *dStd, float *dXo, float *dTo, jacobi_stream_t stream) {
    const int bad = kept < 0 ? -1 : (kept > 0 && !dIdx) ? -2 : xcols < 0 ? -3 : (kept > 0 && xcols > 0 && !dX) ? -4
                  : tcols < 0 ? -5 : (kept > 0 && tcols > 0 && !dT) ? -6 : (tcols > 0 && !dMean) ? -7
                  : (tcols > 0 && !dStd) ? -8 : (kept > 0 && xcols > 0 && !dXo) ? -9
                  : (kept > 0 && tcols > 0 && !dTo) ? -10 : 0;
    return ws_guard("jws_gather_standardize", bad, [&] {
        gather_standardize(kept, xcols, tcols, dIdx, dX, dT, dMean, dStd, dXo, dTo, (hipStream_t)stream);
    });
}

}  // extern "C"
