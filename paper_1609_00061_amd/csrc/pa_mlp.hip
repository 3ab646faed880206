// Learned contraction-order cost model: a small MLP (F -> H -> H -> 1, ReLU)
// predicting the log2 duration of one pairwise generalized array
// multiplication step from features of its index groups.  Forward, backward
// (mean-squared error) and Adam update are hand-written gfx950 kernels; all
// reductions over the batch run in a fixed order, so gradients are
// deterministic.
//
// Parameter layout (float32, contiguous):
//   W1[H][F], b1[H], W2[H][H], b2[H], W3[H], b3
#include <hip/hip_runtime.h>

#include "pa_mlp.h"

namespace pa {

constexpr int kF = kMlpFeatures, kH = kMlpHidden;
constexpr int oW1 = 0, ob1 = oW1 + kH * kF, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH, ob3 = oW3 + kH;
static_assert(ob3 + 1 == kMlpParams, "parameter layout");

// Forward for one sample per thread; weights staged in LDS (read as
// broadcasts).  With `acts` the pre-activations of both hidden layers are
// stored for the backward pass.
__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ X, int64_t n,
                                                     const float *__restrict__ P, float *__restrict__ Y,
                                                     float *__restrict__ acts) {
    __shared__ float w[kMlpParams];
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) w[i] = P[i];
    __syncthreads();
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
        float x[kF];
#pragma unroll
        for (int f = 0; f < kF; ++f) x[f] = X[s * kF + f];
        float h1[kH];   // fully unrolled loops keep h1 in registers
#pragma unroll
        for (int j = 0; j < kH; ++j) {
            float a = w[ob1 + j];
#pragma unroll
            for (int f = 0; f < kF; ++f) a = fmaf(w[oW1 + j * kF + f], x[f], a);
            if (acts) acts[s * 2 * kH + j] = a;
            h1[j] = fmaxf(a, 0.0f);
        }
        float y = w[ob3];
        for (int j = 0; j < kH; ++j) {
            float a = w[ob2 + j];
#pragma unroll
            for (int i = 0; i < kH; ++i) a = fmaf(w[oW2 + j * kH + i], h1[i], a);
            if (acts) acts[s * 2 * kH + kH + j] = a;
            y = fmaf(w[oW3 + j], fmaxf(a, 0.0f), y);
        }
        Y[s] = y;
    }
}

// Per-sample backward of L = (1/n) sum (y - t)^2: dY, and the gradients of
// the hidden pre-activations (stored per sample, reduced by k_mlp_wgrad).
__global__ __launch_bounds__(256) void k_mlp_backward(const float *__restrict__ Y, const float *__restrict__ T,
                                                      int64_t n, const float *__restrict__ P,
                                                      const float *__restrict__ acts, float *__restrict__ dacts,
                                                      float *__restrict__ dY) {
    __shared__ float w[kMlpParams];
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) w[i] = P[i];
    __syncthreads();
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
        const float dy = 2.0f * (Y[s] - T[s]) / (float)n;
        dY[s] = dy;
        const float *a1 = acts + s * 2 * kH, *a2 = a1 + kH;
        float g2[kH];
#pragma unroll
        for (int j = 0; j < kH; ++j) {
            g2[j] = a2[j] > 0.0f ? dy * w[oW3 + j] : 0.0f;
            dacts[s * 2 * kH + kH + j] = g2[j];
        }
        for (int i = 0; i < kH; ++i) {
            float g = 0.0f;
#pragma unroll
            for (int j = 0; j < kH; ++j) g = fmaf(w[oW2 + j * kH + i], g2[j], g);
            dacts[s * 2 * kH + i] = a1[i] > 0.0f ? g : 0.0f;
        }
    }
}

// Weight gradients: one thread per parameter, summing over the batch in
// sample order (deterministic).
__global__ __launch_bounds__(256) void k_mlp_wgrad(const float *__restrict__ X, int64_t n,
                                                   const float *__restrict__ acts, const float *__restrict__ dacts,
                                                   const float *__restrict__ dY, float *__restrict__ G) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    float g = 0.0f;
    if (p < ob1) {                                   // W1[j][f]: dact1[j] * x[f]
        const int j = p / kF, f = p % kF;
        for (int64_t s = 0; s < n; ++s) g = fmaf(dacts[s * 2 * kH + j], X[s * kF + f], g);
    } else if (p < oW2) {                            // b1[j]
        const int j = p - ob1;
        for (int64_t s = 0; s < n; ++s) g += dacts[s * 2 * kH + j];
    } else if (p < ob2) {                            // W2[j][i]: dact2[j] * relu(act1[i])
        const int q = p - oW2, j = q / kH, i = q % kH;
        for (int64_t s = 0; s < n; ++s) g = fmaf(dacts[s * 2 * kH + kH + j], fmaxf(acts[s * 2 * kH + i], 0.0f), g);
    } else if (p < oW3) {                            // b2[j]
        const int j = p - ob2;
        for (int64_t s = 0; s < n; ++s) g += dacts[s * 2 * kH + kH + j];
    } else if (p < ob3) {                            // W3[j]: dy * relu(act2[j])
        const int j = p - oW3;
        for (int64_t s = 0; s < n; ++s) g = fmaf(dY[s], fmaxf(acts[s * 2 * kH + kH + j], 0.0f), g);
    } else {                                         // b3
        for (int64_t s = 0; s < n; ++s) g += dY[s];
    }
    G[p] = g;
}

// Mean-squared error of the last forward, summed in sample order by one block.
__global__ void k_mlp_loss(const float *__restrict__ Y, const float *__restrict__ T, int64_t n, float *loss) {
    __shared__ double part[256];
    double acc = 0.0;
    for (int64_t s = threadIdx.x; s < n; s += blockDim.x) {
        const double d = (double)Y[s] - (double)T[s];
        acc += d * d;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)blockDim.x; ++i) t += part[i];
        *loss = (float)(t / (double)n);
    }
}

// Adam (Kingma & Ba, 2015) with bias correction; step counts from 1.
__global__ void k_mlp_adam(float *__restrict__ P, const float *__restrict__ G, float *__restrict__ M,
                           float *__restrict__ V, float lr, float b1, float b2, float eps, int step) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    const float g = G[p];
    const float m = b1 * M[p] + (1.0f - b1) * g;
    const float v = b2 * V[p] + (1.0f - b2) * g * g;
    M[p] = m;
    V[p] = v;
    const float mh = m / (1.0f - powf(b1, (float)step));
    const float vh = v / (1.0f - powf(b2, (float)step));
    P[p] -= lr * mh / (sqrtf(vh) + eps);
}

static dim3 blocks_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return dim3((unsigned)b);
}

hipError_t mlp_forward(const float *X, int64_t n, const float *P, float *Y, float *acts, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, blocks_for(n), dim3(256), 0, s, X, n, P, Y, acts);
    return hipGetLastError();
}

hipError_t mlp_grad(const float *X, const float *T, int64_t n, const float *P, float *Y, float *acts, float *dacts,
                    float *dY, float *G, float *loss, hipStream_t s) {
    if (n <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mlp_forward, blocks_for(n), dim3(256), 0, s, X, n, P, Y, acts);
    hipLaunchKernelGGL(k_mlp_backward, blocks_for(n), dim3(256), 0, s, Y, T, n, P, acts, dacts, dY);
    hipLaunchKernelGGL(k_mlp_wgrad, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, X, n, acts, dacts, dY, G);
    if (loss) hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(256), 0, s, Y, T, n, loss);
    return hipGetLastError();
}

hipError_t mlp_adam(float *P, const float *G, float *M, float *V, float lr, float b1, float b2, float eps, int step,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, P, G, M, V, lr, b1, b2, eps, step);
    return hipGetLastError();
}

}  // namespace pa
