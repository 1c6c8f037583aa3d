// mlp_driver.hip -- C ABI of the weight-predicting MLP: init, gradient,
// training (all epochs recorded into one hipGraph), prediction.
#include <cmath>

#include "internal.hpp"
#include "mlp.hpp"

using namespace mcs;

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

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
    l.step = off, off += 256;
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
                        launch_mlp_grad(params, X, Y, n, (float *)(w + l.part), grad, loss, (int *)(w + l.step),
                                        (hipStream_t)stream),
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
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess && a->epochs > 0) {
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        for (int ep = 0; ep < a->epochs && e == hipSuccess; ++ep)
            e = launch_mlp_epoch(params, X, Y, n, part, m, v, step, loss_log, hp, cap);
        hipError_t ec = hipStreamEndCapture(cap, &graph);
        if (e == hipSuccess) e = ec;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e == hipSuccess) e = hipGraphLaunch(exec, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
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

}  // extern "C"
