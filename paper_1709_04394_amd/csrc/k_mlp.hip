// k_mlp.hip -- the small MLP that predicts initial multicanonical weights:
// x (2) -> tanh (64) -> tanh (64) -> linear (1), FP32, mean-squared error,
// full-batch Adam.  Parameters are flattened as W1 [64][2], b1 [64],
// W2 [64][64], b2 [64], W3 [1][64], b3 [1] (4417 floats).
//
// k_mlp_fwdbwd: one workgroup of 256 threads per chunk of 32 samples, the
//   parameters and the chunk's activations in LDS; forward, loss, backward,
//   and the chunk's gradient written to its own slot (no atomics).
// k_mlp_adam:   one thread per parameter: gradient = chunk slots summed in
//   chunk order, then the bias-corrected Adam update.
#include <cmath>

#include "internal.hpp"
#include "mlp.hpp"

namespace mcs {

constexpr int H = 64, CH = 32;  // hidden width, samples per workgroup
constexpr int TPS = 256 / CH, UPT = H / TPS;  // threads per sample, hidden units per thread
constexpr int oW1 = 0, ob1 = oW1 + H * 2, oW2 = ob1 + H, ob2 = oW2 + H * H, oW3 = ob2 + H, ob3 = oW3 + H;
static_assert(ob3 + 1 == kMlpParams, "parameter layout");

__global__ __launch_bounds__(256) void k_mlp_fwdbwd(const float *params, const float *X, const float *Y, int n,
                                                    float *part /* [nchunks][kMlpParams + 1] */)
{
    __shared__ float P[kMlpParams];
    __shared__ float h1[CH][H + 1], h2[CH][H + 1], d2[CH][H + 1], d1[CH][H + 1];
    __shared__ float xs[CH][2], dys[CH], l2[CH];
    const int tid = threadIdx.x, chunk = blockIdx.x;
    for (int i = tid; i < kMlpParams; i += blockDim.x) P[i] = params[i];
    if (tid < CH) {
        const int s = chunk * CH + tid;
        xs[tid][0] = s < n ? X[2 * s] : 0.f;
        xs[tid][1] = s < n ? X[2 * s + 1] : 0.f;
    }
    __syncthreads();
    const int s = tid / TPS, q = tid % TPS;  // sample, group of UPT hidden units
    const int gs = chunk * CH + s;
    const bool live = gs < n;
    // layer 1
#pragma unroll 4
    for (int jj = 0; jj < UPT; ++jj) {
        const int j = UPT * q + jj;
        const float z = P[oW1 + 2 * j] * xs[s][0] + P[oW1 + 2 * j + 1] * xs[s][1] + P[ob1 + j];
        h1[s][j] = tanhf(z);
    }
    __syncthreads();
    // layer 2
    for (int jj = 0; jj < UPT; ++jj) {
        const int j = UPT * q + jj;
        float z = P[ob2 + j];
        for (int i = 0; i < H; ++i) z += P[oW2 + H * j + i] * h1[s][i];
        h2[s][j] = tanhf(z);
    }
    __syncthreads();
    // output, residual, dL/dy = 2 (y - t) / n
    if (q == 0) {
        float y = P[ob3];
        for (int j = 0; j < H; ++j) y += P[oW3 + j] * h2[s][j];
        const float r = live ? y - Y[gs] : 0.f;
        dys[s] = 2.f * r / (float)n;
        l2[s] = r * r;
    }
    __syncthreads();
    for (int jj = 0; jj < UPT; ++jj) {
        const int j = UPT * q + jj;
        d2[s][j] = dys[s] * P[oW3 + j] * (1.f - h2[s][j] * h2[s][j]);
    }
    __syncthreads();
    for (int ii = 0; ii < UPT; ++ii) {
        const int i = UPT * q + ii;
        float g = 0.f;
        for (int j = 0; j < H; ++j) g += d2[s][j] * P[oW2 + H * j + i];
        d1[s][i] = g * (1.f - h1[s][i] * h1[s][i]);
    }
    __syncthreads();
    // this chunk's gradient, summed over its samples in order
    float *out = part + (size_t)chunk * (kMlpParams + 1);
    for (int e = tid; e < H * H; e += blockDim.x) {
        const int j = e / H, i = e % H;
        float g = 0.f;
        for (int t = 0; t < CH; ++t) g += d2[t][j] * h1[t][i];
        out[oW2 + e] = g;
    }
    for (int e = tid; e < H * 2; e += blockDim.x) {
        const int j = e / 2, c = e % 2;
        float g = 0.f;
        for (int t = 0; t < CH; ++t) g += d1[t][j] * xs[t][c];
        out[oW1 + e] = g;
    }
    if (tid < H) {
        float g1 = 0.f, g2 = 0.f, g3 = 0.f;
        for (int t = 0; t < CH; ++t) {
            g1 += d1[t][tid];
            g2 += d2[t][tid];
            g3 += dys[t] * h2[t][tid];
        }
        out[ob1 + tid] = g1;
        out[ob2 + tid] = g2;
        out[oW3 + tid] = g3;
    }
    if (tid == 0) {
        float g = 0.f, l = 0.f;
        for (int t = 0; t < CH; ++t) {
            g += dys[t];
            l += l2[t];
        }
        out[ob3] = g;
        out[kMlpParams] = l;
    }
}

// Sum the chunk slots in order; mode 0: write gradient and loss; mode 1:
// Adam step t on params with moments m, v, and log the loss.  Each slot p
// (a parameter, or the loss at p = kMlpParams) keeps its own step count in
// steps[p] and advances it itself, so no other thread reads it and no extra
// launch per epoch is needed (all counts are equal between epochs).
__global__ void k_mlp_adam(const float *part, int nchunks, int n, float *params, float *m, float *v, int *steps,
                           float *grad_out, float *loss_out, MlpHyper hp, int mode)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kMlpParams) return;
    float g = 0.f;
    for (int c = 0; c < nchunks; ++c) g += part[(size_t)c * (kMlpParams + 1) + p];
    if (mode == 0) {
        if (p == kMlpParams) *loss_out = g / (float)n;
        else grad_out[p] = g;
        return;
    }
    const int t = steps[p] + 1;
    steps[p] = t;
    if (p == kMlpParams) {
        loss_out[t - 1] = g / (float)n;
        return;
    }
    const float mm = hp.beta1 * m[p] + (1.f - hp.beta1) * g;
    const float vv = hp.beta2 * v[p] + (1.f - hp.beta2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / (1.f - powf(hp.beta1, (float)t));
    const float vh = vv / (1.f - powf(hp.beta2, (float)t));
    params[p] -= hp.lr * mh / (sqrtf(vh) + hp.eps);
}

__global__ void k_mlp_predict(const float *params, const float *X, int n, float *Y)
{
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const float x0 = X[2 * s], x1 = X[2 * s + 1];
    float h1[H];
    for (int j = 0; j < H; ++j) h1[j] = tanhf(params[oW1 + 2 * j] * x0 + params[oW1 + 2 * j + 1] * x1 + params[ob1 + j]);
    float y = params[ob3];
    for (int j = 0; j < H; ++j) {
        float z = params[ob2 + j];
        for (int i = 0; i < H; ++i) z += params[oW2 + H * j + i] * h1[i];
        y += params[oW3 + j] * tanhf(z);
    }
    Y[s] = y;
}

__global__ void k_zero_f32(float *p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.f;
}

__global__ void k_zero_i32(int *p, int n)
{
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}

int mlp_chunks(int n) { return (n + CH - 1) / CH; }

hipError_t launch_mlp_grad(const float *params, const float *X, const float *Y, int n, float *part, float *grad,
                           float *loss, hipStream_t s)
{
    const int nc = mlp_chunks(n);
    hipLaunchKernelGGL(k_mlp_fwdbwd, dim3(nc), dim3(256), 0, s, params, X, Y, n, part);
    MlpHyper hp{};
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 256) / 256), dim3(256), 0, s, part, nc, n, (float *)nullptr,
                       (float *)nullptr, (float *)nullptr, (int *)nullptr, grad, loss, hp, 0);
    return hipGetLastError();
}

hipError_t launch_mlp_train_setup(float *m, float *v, int *steps, hipStream_t s)
{
    hipLaunchKernelGGL(k_zero_f32, dim3(32), dim3(256), 0, s, m, kMlpParams);
    hipLaunchKernelGGL(k_zero_f32, dim3(32), dim3(256), 0, s, v, kMlpParams);
    hipLaunchKernelGGL(k_zero_i32, dim3(32), dim3(256), 0, s, steps, kMlpParams + 1);
    return hipGetLastError();
}

hipError_t launch_mlp_epoch(float *params, const float *X, const float *Y, int n, float *part, float *m, float *v,
                            int *steps, float *loss_log, const MlpHyper &hp, hipStream_t s)
{
    const int nc = mlp_chunks(n);
    hipLaunchKernelGGL(k_mlp_fwdbwd, dim3(nc), dim3(256), 0, s, params, X, Y, n, part);
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 256) / 256), dim3(256), 0, s, part, nc, n, params, m, v, steps,
                       (float *)nullptr, loss_log, hp, 1);
    return hipGetLastError();
}

// Inputs of the window levels k = 0 .. N/2 of an L x L lattice:
// x = (E/N + 1, 32/L - 1) with E = 4k - 2N, in FP64 rounded to FP32.
__global__ void k_mlp_features(int L, float *X)
{
    const int N = L * L, K = N / 2;
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k > K) return;
    const double E = 4.0 * k - 2.0 * N;
    X[2 * k] = (float)(E / (double)N + 1.0);
    X[2 * k + 1] = (float)(32.0 / (double)L - 1.0);
}

hipError_t launch_mlp_features(int L, float *X, hipStream_t s)
{
    const int n = L * L / 2 + 1;
    hipLaunchKernelGGL(k_mlp_features, dim3((n + 255) / 256), dim3(256), 0, s, L, X);
    return hipGetLastError();
}

hipError_t launch_mlp_predict(const float *params, const float *X, int n, float *Y, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_predict, dim3((n + 127) / 128), dim3(128), 0, s, params, X, n, Y);
    return hipGetLastError();
}

}  // namespace mcs

namespace mcs {

// Xavier-uniform weights from Philox: parameter idx draws word (idx mod 4) of
// Philox(ctr = (idx / 4, 0, 0, TAG_MLP_INIT << 24)); u = (r >> 8) 2^-24 and
// w = (2u - 1) a in FP64 (a = sqrt(6 / (fan_in + fan_out)) from the host),
// rounded once to FP32; biases zero.
__global__ void k_mlp_init(float *params, uint32_t k0, uint32_t k1, double a1, double a2, double a3)
{
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= kMlpParams) return;
    double a = 0.0;
    if (idx < ob1) a = a1;
    else if (idx >= oW2 && idx < ob2) a = a2;
    else if (idx >= oW3 && idx < ob3) a = a3;
    if (a == 0.0) {
        params[idx] = 0.f;
        return;
    }
    const uint4 b = philox(make_uint4((uint32_t)idx >> 2, 0u, 0u, ctr_w3(kTagMlpInit, 0, 0)), k0, k1);
    const uint32_t r = (idx & 3) == 0 ? b.x : (idx & 3) == 1 ? b.y : (idx & 3) == 2 ? b.z : b.w;
    const double u = (double)(r >> 8) * (1.0 / 16777216.0);
    params[idx] = (float)((2.0 * u - 1.0) * a);
}

hipError_t launch_mlp_init(float *params, uint64_t seed, hipStream_t s)
{
    const double a1 = std::sqrt(6.0 / (2 + H)), a2 = std::sqrt(6.0 / (H + H)), a3 = std::sqrt(6.0 / (H + 1));
    hipLaunchKernelGGL(k_mlp_init, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, params, (uint32_t)seed,
                       (uint32_t)(seed >> 32), a1, a2, a3);
    return hipGetLastError();
}

}  // namespace mcs
