// noalloc.hip -- mc_sweep_noalloc: mc_sweep with the fused kernels' scratch
// in a fixed device array of the library instead of a caller workspace, for
// callers that cannot allocate device memory (code under graph capture, tight
// serving loops, harnesses that forbid allocation).
//
// The array lives in this file's device image; each device that runs the
// library holds its own copy until the process ends.  Host code never uses
// the array's name as an address: its device address is read once per device
// with hipGetSymbolAddress and kept here.
#include <mutex>

#include "internal.hpp"

namespace mcs {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// The device address of this device's copy of the array (the context's
// device must be current).
static int static_scratch(mc_ctx *ctx, void **out)
{
    if (ctx->device >= kMaxDevices) return fail(ctx, MC_E_DEVICE, "device %d: static scratch supports devices below %d", ctx->device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[ctx->device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return device_check(ctx, e, "hipGetSymbolAddress(static scratch)");
        if (!p) return fail(ctx, MC_E_DEVICE, "hipGetSymbolAddress(static scratch) gave a null address");
        g_scratch_ptr[ctx->device] = p;
    }
    *out = g_scratch_ptr[ctx->device];
    return MC_OK;
}

}  // namespace mcs

using namespace mcs;

extern "C" {

size_t mc_static_scratch_bytes(void) { return kStaticScratchBytes; }

int mc_sweep_noalloc(mc_ctx *ctx, const mc_geom *geom, void *spins, const int8_t *J, const mc_sweep_args *args,
                     int64_t *EM, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    int rc = check_sweep_args(ctx, geom, spins, args);
    if (rc) return rc;
    const size_t need = fused_workspace_bytes(to_geom(geom), geom->layout);
    if (need > kStaticScratchBytes)
        return fail(ctx, MC_E_RANGE,
                    "the fused sweep of this geometry needs %zu bytes of scratch; the static scratch holds %zu "
                    "(use mc_sweep with a workspace)",
                    need, (size_t)kStaticScratchBytes);
    if (args->nsweeps == 0) return MC_OK;
    if ((rc = set_device(ctx))) return rc;
    void *ws = nullptr;
    if (need > 0 && (rc = static_scratch(ctx, &ws))) return rc;
    return sweep_dispatch(ctx, geom, spins, J, args, EM, need > 0 ? ws : nullptr, need, (hipStream_t)stream);
}

}  // extern "C"
