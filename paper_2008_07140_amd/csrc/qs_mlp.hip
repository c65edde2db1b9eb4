// Cost-model network F -> H -> H -> 1 (ReLU, FP32) on the GPU: forward,
// exact backward pass and Adam steps.  Parameters are packed as
//   W1[H][F], b1[H], W2[H][H], b2[H], W3[H], b3
// and the loss is the mean squared error over the samples of a batch.
//
// One workgroup runs a training step: its parameters and gradients live in
// LDS, each thread takes one sample (forward, then backward with gradient
// accumulation by LDS atomics), and the threads then update the parameters
// with Adam.  The network is tiny; a step is a few microseconds.
#include <hip/hip_runtime.h>

#include "qs_internal.h"
#include "qs_mlp.h"

namespace qs {

namespace {

constexpr int kT = 256;

__device__ __forceinline__ int nparams(int f, int h) { return h * f + h + h * h + h + h + 1; }

// forward of one sample; returns y and keeps z1 / z2 (pre-activations)
template <int H>
__device__ float forward(const float *P, int f, const float *x, float *z1, float *z2)
{
    const float *W1 = P, *b1 = W1 + H * f, *W2 = b1 + H, *b2 = W2 + H * H, *W3 = b2 + H, *b3 = W3 + H;
#pragma unroll 4
    for (int j = 0; j < H; ++j) {
        float acc = b1[j];
        for (int k = 0; k < f; ++k) acc += W1[j * f + k] * x[k];
        z1[j] = acc;
    }
#pragma unroll 4
    for (int j = 0; j < H; ++j) {
        float acc = b2[j];
        for (int k = 0; k < H; ++k) acc += W2[j * H + k] * fmaxf(z1[k], 0.f);
        z2[j] = acc;
    }
    float y = b3[0];
    for (int k = 0; k < H; ++k) y += W3[k] * fmaxf(z2[k], 0.f);
    return y;
}

// backward of one sample, gradient of scale * (y - t)^2 added to G
template <int H>
__device__ void backward(const float *P, int f, const float *x, const float *z1, const float *z2, float dy,
                         float *G)
{
    const float *W2 = P + H * f + H, *W3 = W2 + H * H + H;
    float *gW1 = G, *gb1 = gW1 + H * f, *gW2 = gb1 + H, *gb2 = gW2 + H * H, *gW3 = gb2 + H, *gb3 = gW3 + H;
    atomicAdd(gb3, dy);
    float d2[H];
#pragma unroll
    for (int k = 0; k < H; ++k) {
        const float a2 = fmaxf(z2[k], 0.f);
        atomicAdd(gW3 + k, dy * a2);
        d2[k] = z2[k] > 0.f ? dy * W3[k] : 0.f;
    }
    for (int j = 0; j < H; ++j) {
        if (d2[j] == 0.f) continue;
        atomicAdd(gb2 + j, d2[j]);
        for (int k = 0; k < H; ++k) {
            const float a1 = fmaxf(z1[k], 0.f);
            if (a1 != 0.f) atomicAdd(gW2 + j * H + k, d2[j] * a1);
        }
    }
    for (int k = 0; k < H; ++k) {
        if (z1[k] <= 0.f) continue;
        float acc = 0.f;
#pragma unroll 8
        for (int j = 0; j < H; ++j) acc += W2[j * H + k] * d2[j];
        if (acc == 0.f) continue;
        atomicAdd(gb1 + k, acc);
        for (int c = 0; c < f; ++c) atomicAdd(gW1 + k * f + c, acc * x[c]);
    }
}

template <int H>
__global__ __launch_bounds__(kT) void k_mlp_forward(const float *params, int f, const float *x, int64_t n,
                                                    float *y)
{
    extern __shared__ float P[];
    const int np = nparams(f, H);
    for (int k = threadIdx.x; k < np; k += kT) P[k] = params[k];
    __syncthreads();
    float z1[H], z2[H];
    for (int64_t i = int64_t(blockIdx.x) * kT + threadIdx.x; i < n; i += int64_t(gridDim.x) * kT)
        y[i] = forward<H>(P, f, x + i * f, z1, z2);
}

// Gradient of the mean loss over all n samples (one workgroup), loss into *loss.
template <int H>
__global__ __launch_bounds__(kT) void k_mlp_grad(const float *params, int f, const float *x, const float *t,
                                                 int64_t n, float *grad, float *loss)
{
    extern __shared__ float sh[];
    const int np = nparams(f, H);
    float *P = sh, *G = sh + np;
    __shared__ float lsum;
    for (int k = threadIdx.x; k < np; k += kT) {
        P[k] = params[k];
        G[k] = 0.f;
    }
    if (threadIdx.x == 0) lsum = 0.f;
    __syncthreads();
    float z1[H], z2[H];
    for (int64_t i = threadIdx.x; i < n; i += kT) {
        const float y = forward<H>(P, f, x + i * f, z1, z2);
        const float e = y - t[i];
        atomicAdd(&lsum, e * e / float(n));
        backward<H>(P, f, x + i * f, z1, z2, 2.f * e / float(n), G);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < np; k += kT) grad[k] = G[k];
    if (threadIdx.x == 0) *loss = lsum;
}

// `steps` Adam steps on minibatches idx[s * batch .. s * batch + batch).
template <int H>
__global__ __launch_bounds__(kT) void k_mlp_train(float *params, float *mom, float *vel, int f, const float *x,
                                                  const float *t, const int *idx, int batch, int steps,
                                                  int step0, float lr, float *loss)
{
    extern __shared__ float sh[];
    const int np = nparams(f, H);
    float *P = sh, *G = sh + np;
    __shared__ float lsum;
    for (int k = threadIdx.x; k < np; k += kT) P[k] = params[k];
    float z1[H], z2[H];
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    for (int s = 0; s < steps; ++s) {
        for (int k = threadIdx.x; k < np; k += kT) G[k] = 0.f;
        if (threadIdx.x == 0) lsum = 0.f;
        __syncthreads();
        for (int b = threadIdx.x; b < batch; b += kT) {
            const int i = idx[int64_t(s) * batch + b];
            const float y = forward<H>(P, f, x + int64_t(i) * f, z1, z2);
            const float e = y - t[i];
            atomicAdd(&lsum, e * e / float(batch));
            backward<H>(P, f, x + int64_t(i) * f, z1, z2, 2.f * e / float(batch), G);
        }
        __syncthreads();
        const float c1 = 1.f - powf(b1, float(step0 + s + 1)), c2 = 1.f - powf(b2, float(step0 + s + 1));
        for (int k = threadIdx.x; k < np; k += kT) {
            const float g = G[k];
            const float mk = b1 * mom[k] + (1.f - b1) * g;
            const float vk = b2 * vel[k] + (1.f - b2) * g * g;
            mom[k] = mk;
            vel[k] = vk;
            P[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
        }
        __syncthreads();
    }
    for (int k = threadIdx.x; k < np; k += kT) params[k] = P[k];
    if (threadIdx.x == 0) *loss = lsum;
}

}  // namespace

size_t mlp_num_params(int f, int h) { return size_t(h) * f + h + size_t(h) * h + h + h + 1; }

hipError_t launch_mlp_forward(const float *params, int f, int h, const float *x, int64_t n, float *y,
                              hipStream_t st)
{
    if (h != kMlpHidden) return hipErrorInvalidValue;
    const size_t lds = mlp_num_params(f, h) * sizeof(float);
    int64_t grid = (n + kT - 1) / kT;
    if (grid < 1) grid = 1;
    if (grid > 1024) grid = 1024;
    hipLaunchKernelGGL(k_mlp_forward<kMlpHidden>, dim3(unsigned(grid)), dim3(kT), lds, st, params, f, x, n, y);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *params, int f, int h, const float *x, const float *t, int64_t n,
                           float *grad, float *loss, hipStream_t st)
{
    if (h != kMlpHidden) return hipErrorInvalidValue;
    const size_t lds = 2 * mlp_num_params(f, h) * sizeof(float);
    hipLaunchKernelGGL(k_mlp_grad<kMlpHidden>, dim3(1), dim3(kT), lds, st, params, f, x, t, n, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_train(float *params, float *mom, float *vel, int f, int h, const float *x, const float *t,
                            const int *idx, int batch, int steps, int step0, float lr, float *loss,
                            hipStream_t st)
{
    if (h != kMlpHidden) return hipErrorInvalidValue;
    const size_t lds = 2 * mlp_num_params(f, h) * sizeof(float);
    hipLaunchKernelGGL(k_mlp_train<kMlpHidden>, dim3(1), dim3(kT), lds, st, params, mom, vel, f, x, t, idx, batch,
                       steps, step0, lr, loss);
    return hipGetLastError();
}

}  // namespace qs
