// Internal declarations of the spectral-window network kernels (cnn.hip).
#pragma once
#include "common.h"

namespace scsf {

// flat parameter layout: W1[16,6,3,3] b1[16] W2[32,16,3,3] b2[32] W3[64,2048] b3[64] W4[3,64] b4[3]
constexpr int64_t kW1 = 0, kB1 = 864, kW2 = 880, kB2 = 5488, kW3 = 5520, kB3 = 136592;
constexpr int64_t kW4 = 136656, kB4 = 136848, kNetParams = 136851;

// activations per sample: a1 16*16*16, a2 32*8*8, a3 64, y 3; input 6*16*16
hipError_t cnn_forward(const float *params, const float *x, int n, float *a1, float *a2,
                       float *a3, float *y, hipStream_t st);
hipError_t cnn_forward_bf16(const float *params, const float *x, int n, uint16_t *pbf,
                            uint16_t *xbf, uint16_t *a1, uint16_t *a2, uint16_t *a3, uint16_t *ybf,
                            float *y, hipStream_t st);
hipError_t cnn_loss_grad(const float *params, const float *x, const float *t, int n, float *a1,
                         float *a2, float *a3, float *y, float *d, float *da3, float *da2,
                         float *da1, float *grad, double *loss, hipStream_t st);
hipError_t cnn_adam(float *params, const float *grad, float *m, float *v, int step, float lr,
                    hipStream_t st);
hipError_t cnn_init(float *params, uint64_t seed, hipStream_t st);
hipError_t cnn_input(const double *feats, int n, int C, int p0, float *x, hipStream_t st);
hipError_t cnn_labels(const double *ritz, int n, int k, int L, const double *beta, float *t,
                      hipStream_t st);
hipError_t cnn_hints(const float *y, int n, double *hints, hipStream_t st);

}  // namespace scsf
