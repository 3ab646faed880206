// Learned contraction-order cost model: shapes, kernel launchers, the step
// feature map and the model object behind the pa_model_* entry points.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace pa {

constexpr int kMlpFeatures = 16;
constexpr int kMlpHidden = 64;
constexpr int kMlpParams = kMlpHidden * kMlpFeatures + kMlpHidden + kMlpHidden * kMlpHidden + kMlpHidden + kMlpHidden + 1;

hipError_t mlp_forward(const float *X, int64_t n, const float *P, float *Y, float *acts, hipStream_t s);
hipError_t mlp_grad(const float *X, const float *T, int64_t n, const float *P, float *Y, float *acts, float *dacts,
                    float *dY, float *G, float *loss, hipStream_t s);
hipError_t mlp_adam(float *P, const float *G, float *M, float *V, float lr, float b1, float b2, float eps, int step,
                    hipStream_t s);

struct SysInfo;

// Features of the pairwise step that multiplies the clusters of relation
// sets s1 and s2 (their intermediate packs, and the pack of their union).
void step_features(const SysInfo &si, uint32_t s1, uint32_t s2, float *f);

}  // namespace pa

struct pa_model {
    int device = 0;
    float *P = nullptr, *M = nullptr, *V = nullptr, *G = nullptr, *loss = nullptr;
    int adam_step = 0;
    double level_us = 6.0;   // launch cost of one tree level charged by the learned order
    // per-batch scratch, grown on demand
    int64_t cap = 0;
    float *Y = nullptr, *acts = nullptr, *dacts = nullptr, *dY = nullptr;
    ~pa_model();
};
