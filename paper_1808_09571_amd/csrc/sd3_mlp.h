// Host-side launchers of the ranker training kernels (sd3_mlp.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sd3_common.h"

namespace sd3 {

// Activation and gradient scratch for a batch of n samples (device).
struct MlpScratch {
    float *h1, *h2, *h3;  // [n][64] post-ReLU activations
    float *d1, *d2, *d3;  // [n][64] gradients w.r.t. pre-activations
    float *y, *dy;        // [n]
};

void mlp_forward(const float *params, const float *x, int64_t n, MlpScratch &s, float *y,
                 hipStream_t st);
void mlp_loss_grad(const float *params, const float *x, const float *t, int64_t n, MlpScratch &s,
                   float *loss, float *grad, hipStream_t st);
void adam_step(float *p, const float *g, float *m, float *v, int64_t n, int step, float lr,
               float b1, float b2, float eps, hipStream_t st);

}  // namespace sd3
