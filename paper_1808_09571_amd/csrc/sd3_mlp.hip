// Training kernels of the tile-pair ranker MLP (10 -> 64 -> 64 -> 64 -> 1, ReLU,
// FP32): forward pass with stored activations, mean-squared-error loss,
// backward pass (data and weight gradients) and the Adam update.  The layers
// are small, so every output is one thread's dot product (VALU); the weight
// gradients sum over the batch in chunks of 256 samples with one atomic add
// per chunk and weight.
#include "sd3_mlp.h"

namespace sd3 {

// Y[i][o] = b[o] + sum_k W[o][k] X[i][k]   (ReLU if relu)
__global__ void k_mlp_lin(const float *X, int64_t n, int K, const float *W, const float *b,
                          int nout, float *Y, int relu) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n * nout) return;
    int64_t i = t / nout;
    int o = (int)(t % nout);
    float acc = b[o];
    const float *x = X + i * K;
    const float *w = W + (int64_t)o * K;
    for (int k = 0; k < K; k++) acc += w[k] * x[k];
    Y[t] = relu ? fmaxf(acc, 0.0f) : acc;
}

// dY[i] = 2 (y_i - t_i) / n; loss += (y_i - t_i)^2 / n
__global__ void k_mlp_mse(const float *y, const float *tgt, int64_t n, float *dy, float *loss) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    float e = 0.0f;
    if (i < n) {
        float d = y[i] - tgt[i];
        dy[i] = 2.0f * d / (float)n;
        e = d * d / (float)n;
    }
    e = wave_sum(e);
    if (lane_id() == 0 && e != 0.0f) atomicAdd(loss, e);
}

// dX[i][k] = (sum_o dY[i][o] W[o][k]) * (H[i][k] > 0)
__global__ void k_mlp_bwd_data(const float *dY, int64_t n, int nout, const float *W, int K,
                               const float *H, float *dX) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= n * K) return;
    int64_t i = t / K;
    int k = (int)(t % K);
    float acc = 0.0f;
    for (int o = 0; o < nout; o++) acc += dY[i * nout + o] * W[(int64_t)o * K + k];
    dX[t] = H[t] > 0.0f ? acc : 0.0f;
}

// gW[o][k] += sum_i dY[i][o] X[i][k]; gb[o] += sum_i dY[i][o]
// (thread = (chunk of 256 samples, o, k); k == K stands for the bias)
__global__ void k_mlp_bwd_weight(const float *dY, const float *X, int64_t n, int nout, int K,
                                 float *gW, float *gb) {
    int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int64_t per = (int64_t)nout * (K + 1);
    int64_t chunk = t / per;
    int r = (int)(t % per);
    int o = r / (K + 1), k = r % (K + 1);
    int64_t i0 = chunk * 256;
    if (i0 >= n) return;
    int64_t i1 = min(n, i0 + 256);
    float acc = 0.0f;
    for (int64_t i = i0; i < i1; i++) acc += dY[i * nout + o] * (k < K ? X[i * K + k] : 1.0f);
    if (k < K) atomicAdd(&gW[(int64_t)o * K + k], acc);
    else atomicAdd(&gb[o], acc);
}

__global__ void k_mlp_zero(float *p, int64_t n) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// Adam (Kingma & Ba 2015) with bias-corrected moments.
__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.0f - b1) * gi;
    float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

static unsigned g256(int64_t n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

void mlp_forward(const float *P, const float *X, int64_t n, MlpScratch &s, float *y,
                 hipStream_t st) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mlp_lin, dim3(g256(n * MLP_H)), dim3(256), 0, st, X, n, MLP_IN, P + MLP_W1,
                       P + MLP_B1, MLP_H, s.h1, 1);
    hipLaunchKernelGGL(k_mlp_lin, dim3(g256(n * MLP_H)), dim3(256), 0, st, s.h1, n, MLP_H,
                       P + MLP_W2, P + MLP_B2, MLP_H, s.h2, 1);
    hipLaunchKernelGGL(k_mlp_lin, dim3(g256(n * MLP_H)), dim3(256), 0, st, s.h2, n, MLP_H,
                       P + MLP_W3, P + MLP_B3, MLP_H, s.h3, 1);
    hipLaunchKernelGGL(k_mlp_lin, dim3(g256(n)), dim3(256), 0, st, s.h3, n, MLP_H, P + MLP_W4,
                       P + MLP_B4, 1, y, 0);
}

void mlp_loss_grad(const float *P, const float *X, const float *T, int64_t n, MlpScratch &s,
                   float *loss, float *G, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_zero, dim3(g256(MLP_NPARAM)), dim3(256), 0, st, G, (int64_t)MLP_NPARAM);
    hipLaunchKernelGGL(k_mlp_zero, dim3(1), dim3(64), 0, st, loss, (int64_t)1);
    if (n <= 0) return;
    mlp_forward(P, X, n, s, s.y, st);
    hipLaunchKernelGGL(k_mlp_mse, dim3(g256(n)), dim3(256), 0, st, s.y, T, n, s.dy, loss);
    int64_t nch = (n + 255) / 256;
    // head: gw4, gb4; then d(pre3)
    hipLaunchKernelGGL(k_mlp_bwd_weight, dim3(g256(nch * (MLP_H + 1))), dim3(256), 0, st, s.dy,
                       s.h3, n, 1, MLP_H, G + MLP_W4, G + MLP_B4);
    hipLaunchKernelGGL(k_mlp_bwd_data, dim3(g256(n * MLP_H)), dim3(256), 0, st, s.dy, n, 1,
                       P + MLP_W4, MLP_H, s.h3, s.d3);
    // layer 3
    hipLaunchKernelGGL(k_mlp_bwd_weight, dim3(g256(nch * MLP_H * (MLP_H + 1))), dim3(256), 0, st,
                       s.d3, s.h2, n, MLP_H, MLP_H, G + MLP_W3, G + MLP_B3);
    hipLaunchKernelGGL(k_mlp_bwd_data, dim3(g256(n * MLP_H)), dim3(256), 0, st, s.d3, n, MLP_H,
                       P + MLP_W3, MLP_H, s.h2, s.d2);
    // layer 2
    hipLaunchKernelGGL(k_mlp_bwd_weight, dim3(g256(nch * MLP_H * (MLP_H + 1))), dim3(256), 0, st,
                       s.d2, s.h1, n, MLP_H, MLP_H, G + MLP_W2, G + MLP_B2);
    hipLaunchKernelGGL(k_mlp_bwd_data, dim3(g256(n * MLP_H)), dim3(256), 0, st, s.d2, n, MLP_H,
                       P + MLP_W2, MLP_H, s.h1, s.d1);
    // layer 1
    hipLaunchKernelGGL(k_mlp_bwd_weight, dim3(g256(nch * MLP_H * (MLP_IN + 1))), dim3(256), 0, st,
                       s.d1, X, n, MLP_H, MLP_IN, G + MLP_W1, G + MLP_B1);
}

void adam_step(float *p, const float *g, float *m, float *v, int64_t n, int step, float lr,
               float b1, float b2, float eps, hipStream_t st) {
    if (n <= 0) return;
    float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(g256(n)), dim3(256), 0, st, p, g, m, v, n, lr, b1, b2, eps, c1,
                       c2);
}

}  // namespace sd3
