// ECG misfit (Sec. 2.4 Eq. (inverse_ecg), rectangle rule in time) and the Adam
// update used to fit the model parameters (Sec. 2.4).
#include <math.h>

#include "gbp_internal.h"

namespace {

// Single block, fixed reduction order (deterministic).
__global__ void __launch_bounds__(1024)
    k_loss(const float* __restrict__ e, const float* __restrict__ t, int n,
           float* __restrict__ loss, float* __restrict__ grad) {
    __shared__ float sh[1024];
    const float inv = 1.f / (float)n;
    float acc = 0.f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const float d = e[i] - t[i];
        acc += d * d;
        if (grad) grad[i] = 2.f * d * inv;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = sh[0] * inv;
}

// One block per instance.
__global__ void __launch_bounds__(1024)
    k_loss_batched(const float* __restrict__ e, const float* __restrict__ t, int n_per,
                   float* __restrict__ loss, float* __restrict__ grad) {
    __shared__ float sh[1024];
    const size_t base = (size_t)blockIdx.x * n_per;
    const float inv = 1.f / (float)n_per;
    float acc = 0.f;
    for (int i = threadIdx.x; i < n_per; i += blockDim.x) {
        const float d = e[base + i] - t[base + i];
        acc += d * d;
        if (grad) grad[base + i] = 2.f * d * inv;
    }
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[blockIdx.x] = sh[0] * inv;
}

// Adam with the step number in device memory (bias corrections computed here).
__global__ void k_adam_dev(float* __restrict__ p, const float* __restrict__ g,
                           float* __restrict__ m, float* __restrict__ v, int n, float lr, float b1,
                           float b2, float eps, const int* __restrict__ step, float lo, float hi,
                           int clamp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float k = (float)max(*step, 1);
    const float c1 = 1.f / (1.f - powf(b1, k));
    const float c2 = 1.f / (1.f - powf(b2, k));
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float x = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    if (clamp) x = fminf(fmaxf(x, lo), hi);
    p[i] = x;
}

__global__ void k_counter_add(int* c, int d) {
    if (threadIdx.x == 0) *c += d;
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int n, float lr, float b1, float b2, float eps,
                       float c1, float c2, float lo, float hi, int clamp) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float x = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
    if (clamp) x = fminf(fmaxf(x, lo), hi);
    p[i] = x;
}

}  // namespace

extern "C" int gbp_ecg_loss(const float* ecg, const float* target, int n, float* loss,
                            float* dL_decg, void* stream) {
    if (!ecg || !target || !loss || n <= 0) {
        gbp_set_error("ecg_loss: bad arguments");
        return GBP_ERR_ARG;
    }
    k_loss<<<1, 1024, 0, (hipStream_t)stream>>>(ecg, target, n, loss, dL_decg);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}

extern "C" int gbp_adam_step(float* param, const float* grad, float* m, float* v, int n, float lr,
                             float beta1, float beta2, float eps, int step, float lo, float hi,
                             void* stream) {
    if (!param || !grad || !m || !v || n < 0 || step < 1) {
        gbp_set_error("adam_step: bad arguments");
        return GBP_ERR_ARG;
    }
    if (n == 0) return GBP_OK;
    const float c1 = (float)(1.0 / (1.0 - pow((double)beta1, step)));
    const float c2 = (float)(1.0 / (1.0 - pow((double)beta2, step)));
    k_adam<<<gbp_blocks(n, 256), 256, 0, (hipStream_t)stream>>>(param, grad, m, v, n, lr, beta1,
                                                                beta2, eps, c1, c2, lo, hi,
                                                                lo < hi ? 1 : 0);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}

extern "C" int gbp_ecg_loss_batched(const float* ecg, const float* target, int n_inst, int n_per,
                                    float* loss, float* dL_decg, void* stream) {
    if (!ecg || !target || !loss || n_inst < 1 || n_per < 1) {
        gbp_set_error("ecg_loss_batched: bad arguments");
        return GBP_ERR_ARG;
    }
    k_loss_batched<<<n_inst, 1024, 0, (hipStream_t)stream>>>(ecg, target, n_per, loss, dL_decg);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}

extern "C" int gbp_adam_step_dev(float* param, const float* grad, float* m, float* v, int n,
                                 float lr, float beta1, float beta2, float eps, const int* step,
                                 float lo, float hi, void* stream) {
    if (!param || !grad || !m || !v || !step || n < 0) {
        gbp_set_error("adam_step_dev: bad arguments");
        return GBP_ERR_ARG;
    }
    if (n == 0) return GBP_OK;
    k_adam_dev<<<gbp_blocks(n, 256), 256, 0, (hipStream_t)stream>>>(param, grad, m, v, n, lr, beta1,
                                                                    beta2, eps, step, lo, hi,
                                                                    lo < hi ? 1 : 0);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}

extern "C" int gbp_counter_add(int* counter, int delta, void* stream) {
    if (!counter) {
        gbp_set_error("counter is NULL");
        return GBP_ERR_ARG;
    }
    k_counter_add<<<1, 64, 0, (hipStream_t)stream>>>(counter, delta);
    GBP_LAUNCH_CHECK();
    return GBP_OK;
}
