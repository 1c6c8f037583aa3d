// mlp_driver.hip -- C ABI of the weight-predicting MLP: init, gradient,
// training (all epochs recorded into one hipGraph), prediction.
#include <cmath>
#include <vector>

#include "internal.hpp"
#include "mlp.hpp"

using namespace mcs;

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Entropy per site of independent flipped spins at density x, 0 at x = 0.
double gas_entropy(double x) { return x <= 0.0 ? 0.0 : -x * std::log(x) - (1.0 - x) * std::log1p(-x); }

// Output baseline of level k of an N-site lattice: h(k / 2N) - h(1/4); the
// network fits the entropy deficit minus this (the ground-state singularity
// of g(E) is the flipped-spin gas's x ln x).
double baseline(int k, int N) { return gas_entropy((double)k / (2.0 * N)) - gas_entropy(0.25); }

struct MlpLayout {
    size_t part = 0, m = 0, v = 0, step = 0, loss = 0, total = 0;
};

MlpLayout mlp_layout(int n)
{
    MlpLayout l;
    size_t off = 0;
    l.part = off, off += align256((size_t)mlp_chunks(n) * (kMlpParams + 1) * 4);
    l.m = off, off += align256((size_t)kMlpParams * 4);
    l.v = off, off += align256((size_t)kMlpParams * 4);
    l.step = off, off += align256((size_t)(kMlpParams + 1) * 4);
    l.loss = off, off += 256;
    l.total = off;
    return l;
}

}  // namespace

extern "C" {

int32_t mc_mlp_param_count(void) { return kMlpParams; }

size_t mc_mlp_workspace_bytes(int32_t n) { return n < 1 ? 0 : mlp_layout(n).total; }

int mc_mlp_init(mc_ctx *ctx, float *params, uint64_t seed, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    if (!params) return fail(ctx, MC_E_INVAL, "params is NULL");
    int rc = set_device(ctx);
    if (rc) return rc;
    return device_check(ctx, launch_mlp_init(params, seed, (hipStream_t)stream), "mc_mlp_init");
}

int mc_mlp_grad(mc_ctx *ctx, const float *params, const float *X, const float *Y, int32_t n, float *grad, float *loss,
                void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    if (!params || !X || !Y || !grad || !loss) return fail(ctx, MC_E_INVAL, "a pointer argument is NULL");
    if (n < 1 || n > (1 << 24)) return fail(ctx, MC_E_RANGE, "n must be 1..2^24");
    const MlpLayout l = mlp_layout(n);
    if (!ws || ws_bytes < l.total) return fail(ctx, MC_E_WORKSPACE, "workspace needs %zu bytes", l.total);
    int rc = set_device(ctx);
    if (rc) return rc;
    char *w = (char *)ws;
    return device_check(ctx,
                        launch_mlp_grad(params, X, Y, n, (float *)(w + l.part), grad, loss, (hipStream_t)stream),
                        "mc_mlp_grad");
}

int mc_mlp_train(mc_ctx *ctx, const mc_mlp_args *a, const float *X, const float *Y, int32_t n, float *params,
                 float *loss_log, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    if (!a || !params || !X || !Y || !loss_log) return fail(ctx, MC_E_INVAL, "a pointer argument is NULL");
    if (n < 1 || n > (1 << 24) || a->epochs < 0 || a->epochs > 10000000) return fail(ctx, MC_E_RANGE, "n or epochs");
    if (!(a->lr > 0.f) || !(a->beta1 >= 0.f && a->beta1 < 1.f) || !(a->beta2 >= 0.f && a->beta2 < 1.f) ||
        !(a->eps > 0.f))
        return fail(ctx, MC_E_RANGE, "Adam hyper-parameters out of range");
    const MlpLayout l = mlp_layout(n);
    if (!ws || ws_bytes < l.total) return fail(ctx, MC_E_WORKSPACE, "workspace needs %zu bytes", l.total);
    int rc = set_device(ctx);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream, cap = nullptr;
    if ((rc = capture_stream(ctx, &cap))) return rc;
    char *w = (char *)ws;
    float *part = (float *)(w + l.part), *m = (float *)(w + l.m), *v = (float *)(w + l.v);
    int *step = (int *)(w + l.step);
    const MlpHyper hp{a->lr, a->beta1, a->beta2, a->eps};
    hipError_t e = launch_mlp_train_setup(m, v, step, s);
    // a graph of up to kChunk epochs, replayed: the step counts live in
    // device memory, so every replay continues where the last one stopped
    constexpr int kChunk = 500;
    auto run_graph = [&](int epochs, int times) -> hipError_t {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        hipError_t r = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        for (int ep = 0; ep < epochs && r == hipSuccess; ++ep)
            r = launch_mlp_epoch(params, X, Y, n, part, m, v, step, loss_log, hp, cap);
        const hipError_t ec = hipStreamEndCapture(cap, &graph);
        if (r == hipSuccess) r = ec;
        if (r == hipSuccess) r = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        for (int t = 0; t < times && r == hipSuccess; ++t) r = hipGraphLaunch(exec, s);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        return r;
    };
    const int full = a->epochs / kChunk, rest = a->epochs % kChunk;
    if (e == hipSuccess && full > 0) e = run_graph(kChunk, full);
    if (e == hipSuccess && rest > 0) e = run_graph(rest, 1);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return device_check(ctx, e, "mc_mlp_train");
}

int mc_mlp_predict(mc_ctx *ctx, const float *params, const float *X, int32_t n, float *Y, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    if (!params || !X || !Y) return fail(ctx, MC_E_INVAL, "a pointer argument is NULL");
    if (n < 0 || n > (1 << 26)) return fail(ctx, MC_E_RANGE, "n out of range");
    if (n == 0) return MC_OK;
    int rc = set_device(ctx);
    if (rc) return rc;
    return device_check(ctx, launch_mlp_predict(params, X, n, Y, (hipStream_t)stream), "mc_mlp_predict");
}

int mc_mlp_training_set(mc_ctx *ctx, int32_t nL, const int32_t *Ls, const double *const *lnW, float *X, float *Y,
                        int32_t cap, int32_t *n_out)
{
    if (!ctx) return MC_E_INVAL;
    if (nL < 1 || !Ls || !lnW || !X || !Y || !n_out) return fail(ctx, MC_E_INVAL, "a pointer argument is NULL or nL < 1");
    int64_t n = 0;
    for (int i = 0; i < nL; ++i) {
        const int L = Ls[i];
        if (L < 4 || L > 1024 || L % 2) return fail(ctx, MC_E_SHAPE, "Ls[%d] = %d: need an even L in 4..1024", i, L);
        if (!lnW[i]) return fail(ctx, MC_E_INVAL, "lnW[%d] is NULL", i);
        const int K = L * L / 2;
        for (int k = 0; k <= K; ++k)
            if (k != 1 && !std::isfinite(lnW[i][k])) return fail(ctx, MC_E_RANGE, "lnW[%d][%d] is not finite", i, k);
        n += K;  // K + 1 levels minus the empty one
    }
    if (n > cap) return fail(ctx, MC_E_RANGE, "%lld samples do not fit in cap = %d", (long long)n, cap);
    int64_t j = 0;
    for (int i = 0; i < nL; ++i) {
        const int L = Ls[i], N = L * L, K = N / 2;
        const double ref = lnW[i][K];
        for (int k = 0; k <= K; ++k) {
            if (k == 1) continue;
            const double E = 4.0 * k - 2.0 * N;
            X[2 * j] = (float)(E / (double)N + 1.0);
            X[2 * j + 1] = (float)(32.0 / (double)L - 1.0);
            Y[j] = (float)(-(lnW[i][k] - ref) / (double)N - baseline(k, N));
            ++j;
        }
    }
    *n_out = (int32_t)n;
    return MC_OK;
}

size_t mc_mlp_lnw_workspace_bytes(int32_t L)
{
    if (L < 4 || L > 1024 || L % 2) return 0;
    const size_t n = (size_t)L * L / 2 + 1;
    return align256(n * 8) + align256(n * 4);
}

int mc_mlp_lnw_init(mc_ctx *ctx, const float *params, int32_t L, double *lnW_out, int32_t *used_fallback, void *ws,
                    size_t ws_bytes, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    if (!params || !lnW_out || !used_fallback) return fail(ctx, MC_E_INVAL, "a pointer argument is NULL");
    if (L < 4 || L > 1024 || L % 2) return fail(ctx, MC_E_SHAPE, "L = %d: need an even L in 4..1024", L);
    const size_t need = mc_mlp_lnw_workspace_bytes(L);
    if (!ws || ws_bytes < need) return fail(ctx, MC_E_WORKSPACE, "workspace needs %zu bytes", need);
    int rc = set_device(ctx);
    if (rc) return rc;
    const int N = L * L, K = N / 2;
    float *X = (float *)ws, *Yd = (float *)((char *)ws + align256((size_t)(K + 1) * 8));
    hipStream_t s = (hipStream_t)stream;
    std::vector<float> y((size_t)K + 1);
    hipError_t e = launch_mlp_features(L, X, s);
    if (e == hipSuccess) e = launch_mlp_predict(params, X, K + 1, Yd, s);
    if (e == hipSuccess) e = hipMemcpyAsync(y.data(), Yd, y.size() * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if ((rc = device_check(ctx, e, "mc_mlp_lnw_init"))) return rc;
    bool finite = true;
    for (int k = 0; k <= K; ++k) finite = finite && std::isfinite(y[(size_t)k]);
    *used_fallback = finite ? 0 : 1;
    const double ref = finite ? -(double)N * ((double)y[(size_t)K] + baseline(K, N)) : 0.0;
    for (int k = 0; k <= K; ++k)
        lnW_out[k] = finite ? -(double)N * ((double)y[(size_t)k] + baseline(k, N)) - ref : 0.0;
    return MC_OK;
}

}  // extern "C"
