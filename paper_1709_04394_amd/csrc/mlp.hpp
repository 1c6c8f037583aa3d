// mlp.hpp -- parameters and launchers of the weight-predicting MLP.
#pragma once

#include "common.hpp"

namespace mcs {

constexpr int kMlpParams = 4417;  // 2-64-64-1: 128 + 64 + 4096 + 64 + 64 + 1

struct MlpHyper {
    float lr, beta1, beta2, eps;
};

int mlp_chunks(int n);
hipError_t launch_mlp_grad(const float *params, const float *X, const float *Y, int n, float *part, float *grad,
                           float *loss, hipStream_t s);
// steps: kMlpParams + 1 per-slot Adam step counts, zeroed by the setup
hipError_t launch_mlp_train_setup(float *m, float *v, int *steps, hipStream_t s);
hipError_t launch_mlp_epoch(float *params, const float *X, const float *Y, int n, float *part, float *m, float *v,
                            int *steps, float *loss_log, const MlpHyper &hp, hipStream_t s);
hipError_t launch_mlp_predict(const float *params, const float *X, int n, float *Y, hipStream_t s);
hipError_t launch_mlp_init(float *params, uint64_t seed, hipStream_t s);
hipError_t launch_mlp_features(int L, float *X, hipStream_t s);

}  // namespace mcs
