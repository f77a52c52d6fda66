// Kernels of the schedule cost model: a small fully connected network
// (Linear + ReLU layers, masked mean-squared error on log-times, Adam),
// trained on the GPU.  The shapes are tiny (inputs 7, hidden 64, outputs
// 48, batches of a few thousand), so these kernels are latency-bound
// elementwise / reduction kernels; every reduction runs in a fixed order so
// training is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace starmm {

namespace {

constexpr int kT = 256;

// Y[b, o] = act(sum_i X[b, i] W[o, i] + bias[o]).
__global__ void __launch_bounds__(kT)
k_linear_fwd(int64_t batch, int64_t in, int64_t out, const float* __restrict__ X, const float* __restrict__ W,
             const float* __restrict__ bias, float* __restrict__ Y, int relu) {
    const int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (idx >= batch * out) return;
    const int64_t b = idx / out, o = idx % out;
    float acc = bias ? bias[o] : 0.0f;
    const float* x = X + b * in;
    const float* w = W + o * in;
    for (int64_t i = 0; i < in; ++i) acc = fmaf(x[i], w[i], acc);
    Y[idx] = (relu && acc < 0.0f) ? 0.0f : acc;
}

// dZ = dY * [Y > 0] (ReLU) or dY; stored for the two reductions below.
__global__ void __launch_bounds__(kT)
k_act_bwd(int64_t total, const float* __restrict__ Y, const float* __restrict__ dY, float* __restrict__ dZ, int relu) {
    const int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (idx >= total) return;
    dZ[idx] = (relu && !(Y[idx] > 0.0f)) ? 0.0f : dY[idx];
}

// dX[b, i] = sum_o dZ[b, o] W[o, i].
__global__ void __launch_bounds__(kT)
k_linear_bwd_x(int64_t batch, int64_t in, int64_t out, const float* __restrict__ dZ, const float* __restrict__ W,
               float* __restrict__ dX) {
    const int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (idx >= batch * in) return;
    const int64_t b = idx / in, i = idx % in;
    float acc = 0.0f;
    for (int64_t o = 0; o < out; ++o) acc = fmaf(dZ[b * out + o], W[o * in + i], acc);
    dX[idx] = acc;
}

// dW[o, i] = sum_b dZ[b, o] X[b, i] and db[o] = sum_b dZ[b, o]: one workgroup
// per (o, i) pair (i == in means the bias); each thread sums a strided
// subset of the batch, then a fixed-shape tree in LDS combines them.
__global__ void __launch_bounds__(kT)
k_linear_bwd_w(int64_t batch, int64_t in, int64_t out, const float* __restrict__ dZ, const float* __restrict__ X,
               float* __restrict__ dW, float* __restrict__ db) {
    __shared__ float red[kT];
    const int64_t o = blockIdx.x / (in + 1), i = blockIdx.x % (in + 1);
    float acc = 0.0f;
    for (int64_t b = threadIdx.x; b < batch; b += kT) {
        const float g = dZ[b * out + o];
        acc = fmaf(g, i < in ? X[b * in + i] : 1.0f, acc);
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int w = kT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (i < in)
            dW[o * in + i] = red[0];
        else if (db)
            db[o] = red[0];
    }
}

// Masked mean-squared error: loss = sum mask (P - T)^2 / max(1, sum mask),
// dP = 2 mask (P - T) / max(1, sum mask).  One workgroup (fixed order).
__global__ void __launch_bounds__(kT)
k_masked_mse(int64_t total, const float* __restrict__ P, const float* __restrict__ T, const float* __restrict__ M,
             float* __restrict__ loss, float* __restrict__ dP) {
    __shared__ float red_e[kT], red_n[kT];
    float e = 0.0f, cnt = 0.0f;
    for (int64_t j = threadIdx.x; j < total; j += kT) {
        const float mk = M[j];
        const float d = P[j] - T[j];
        e = fmaf(mk * d, d, e);
        cnt += mk;
    }
    red_e[threadIdx.x] = e;
    red_n[threadIdx.x] = cnt;
    __syncthreads();
    for (int w = kT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red_e[threadIdx.x] += red_e[threadIdx.x + w];
            red_n[threadIdx.x] += red_n[threadIdx.x + w];
        }
        __syncthreads();
    }
    const float denom = red_n[0] > 1.0f ? red_n[0] : 1.0f;
    if (threadIdx.x == 0 && loss) *loss = red_e[0] / denom;
    if (dP)
        for (int64_t j = threadIdx.x; j < total; j += kT) dP[j] = 2.0f * M[j] * (P[j] - T[j]) / denom;
}

// Adam (Kingma & Ba) with bias correction, step >= 1.
__global__ void __launch_bounds__(kT)
k_adam(int64_t count, float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
       float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t idx = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (idx >= count) return;
    const float gi = g[idx];
    const float mi = b1 * m[idx] + (1.0f - b1) * gi;
    const float vi = b2 * v[idx] + (1.0f - b2) * gi * gi;
    m[idx] = mi;
    v[idx] = vi;
    p[idx] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

unsigned blocks(int64_t n) { return (unsigned)((n + kT - 1) / kT); }

mm_status done(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        set_last_error(std::string(what) + ": " + hipGetErrorString(e));
        return MM_ERR_HIP;
    }
    return MM_OK;
}

}  // namespace

}  // namespace starmm

using namespace starmm;

extern "C" {

mm_status mm_mlp_linear_forward(int64_t batch, int64_t in, int64_t out, const float* X, const float* W,
                                const float* bias, float* Y, int32_t relu, void* stream) {
    if (batch < 0 || in < 0 || out < 0) return MM_ERR_INVALID_ARG;
    if (batch * out == 0) return MM_OK;
    if (!W && in > 0) return MM_ERR_INVALID_ARG;
    if ((!X && in > 0) || !Y) return MM_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps("mlp", st);
    hipLaunchKernelGGL(k_linear_fwd, dim3(blocks(batch * out)), dim3(kT), 0, st, batch, in, out, X, W, bias, Y,
                       (int)relu);
    return done("mm_mlp_linear_forward");
}

mm_status mm_mlp_linear_backward(int64_t batch, int64_t in, int64_t out, const float* X, const float* W,
                                 const float* Y, const float* dY, float* dZ, float* dX, float* dW, float* db,
                                 int32_t relu, void* stream) {
    if (batch < 0 || in < 0 || out < 0) return MM_ERR_INVALID_ARG;
    if (!Y || !dY || !dZ || !dW || (in > 0 && (!X || !W))) return MM_ERR_INVALID_ARG;
    if (out == 0) return MM_OK;
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps("mlp", st);
    if (batch > 0)
        hipLaunchKernelGGL(k_act_bwd, dim3(blocks(batch * out)), dim3(kT), 0, st, batch * out, Y, dY, dZ, (int)relu);
    if (dX && batch * in > 0)
        hipLaunchKernelGGL(k_linear_bwd_x, dim3(blocks(batch * in)), dim3(kT), 0, st, batch, in, out, dZ, W, dX);
    hipLaunchKernelGGL(k_linear_bwd_w, dim3((unsigned)(out * (in + 1))), dim3(kT), 0, st, batch, in, out, dZ, X, dW,
                       db);
    return done("mm_mlp_linear_backward");
}

mm_status mm_mlp_masked_mse(int64_t total, const float* P, const float* T, const float* M, float* loss, float* dP,
                            void* stream) {
    if (total < 0 || (total > 0 && (!P || !T || !M))) return MM_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps("mlp", st);
    hipLaunchKernelGGL(k_masked_mse, dim3(1), dim3(kT), 0, st, total, P, T, M, loss, dP);
    return done("mm_mlp_masked_mse");
}

mm_status mm_mlp_adam(int64_t count, float* param, const float* grad, float* m1, float* m2, float lr, float beta1,
                      float beta2, float eps, int32_t step, void* stream) {
    if (count < 0 || step < 1 || (count > 0 && (!param || !grad || !m1 || !m2))) return MM_ERR_INVALID_ARG;
    if (count == 0) return MM_OK;
    float c1 = 1.0f, c2 = 1.0f, p1 = 1.0f, p2 = 1.0f;
    for (int32_t s = 0; s < step && s < 100000; ++s) {
        p1 *= beta1;
        p2 *= beta2;
    }
    c1 = 1.0f - p1;
    c2 = 1.0f - p2;
    hipStream_t st = (hipStream_t)stream;
    ProfScope ps("mlp", st);
    hipLaunchKernelGGL(k_adam, dim3(blocks(count)), dim3(kT), 0, st, count, param, grad, m1, m2, lr, beta1, beta2, eps,
                       c1, c2);
    return done("mm_mlp_adam");
}

}  // extern "C"
