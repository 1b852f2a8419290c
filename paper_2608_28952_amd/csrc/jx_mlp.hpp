// jx_mlp.hpp -- sizes and buffer layouts of the learned warm start's network
// (k_mlp.hip, k_cayley.hip, capi_ws.cpp).
#pragma once

#include <cstddef>
#include <cstdint>

#include "jx_common.hpp"

namespace jx {
namespace mlp {

constexpr int NIN = 8, K1 = 16, H = 256, NOUT = 2016;  // NOUT = 64 * 63 / 2
constexpr size_t OFF_W1 = 0;
constexpr size_t OFF_W2 = OFF_W1 + (size_t)K1 * H;
constexpr size_t OFF_W3 = OFF_W2 + (size_t)H * H;
constexpr size_t OFF_B1 = OFF_W3 + (size_t)H * NOUT;
constexpr size_t OFF_B2 = OFF_B1 + H;
constexpr size_t OFF_B3 = OFF_B2 + H;
constexpr size_t NPARAM = OFF_B3 + NOUT;

enum Act { ACT_X0 = 0, ACT_Z1, ACT_H1, ACT_Z2, ACT_H2, ACT_DZ2, ACT_DZ1, ACT_DY, ACT_END };
// element offset of activation slot `a` for a batch of B samples
constexpr size_t act_off(int B, int a) {
    return (size_t)B * (a == ACT_X0 ? 0 : (size_t)K1 + (size_t)H * (a - 1) + (a == ACT_END ? (size_t)NOUT - H : 0));
}

}  // namespace mlp

void mlp_forward(int B, const float *theta, const uint16_t *Wb, const float *bias, float *out, uint16_t *acts,
                 hipStream_t s);
void mlp_backward(int B, const uint16_t *acts, const float *dY, const uint16_t *Wb, float *gW, float *gB,
                  hipStream_t s);
void mlp_mse(size_t count, const float *Y, const float *T, float *grad, double *loss, hipStream_t s);
void mlp_adam(int count, float *p, uint16_t *pb, const float *g, float *m, float *v, float lr, float b1, float b2,
              float eps, float c1, float c2, hipStream_t s);
void mlp_to_bf16(size_t count, const float *src, uint16_t *dst, hipStream_t s);
void skew_from_coords(int batch, int n, const float *coords, const float *mean, const float *stdv, double *S,
                      hipStream_t s);
void cayley_batched(int batch, int n, const double *S, const double *Qref, double *Q0, hipStream_t s);
// k_canon.hip: training data
void family_matrices(int count, int n, int k, const double *theta, const double *A0, const double *B, double *A,
                     hipStream_t s);
void canonical_targets(int count, int n, const double *Q, const double *Qref, float *coords, int *keep,
                       double maxabs, hipStream_t s);
constexpr int STATS_CHUNK = 1024;  // rows per partial sum of column_stats
void column_stats(int rows, int cols, const float *X, const int *keep, int nkeep, float eps, float *mean,
                  float *stdv, double *part, int chunk, hipStream_t s);
void gather_standardize(int kept, int xcols, int tcols, const int *idx, const float *X, const float *T,
                        const float *mean, const float *stdv, float *Xo, float *To, hipStream_t s);

}  // namespace jx
