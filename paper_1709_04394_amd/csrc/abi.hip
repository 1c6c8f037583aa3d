// abi.hip -- the extern "C" entry points of libmcspin: argument checking,
// FP64 acceptance tables on the host, and dispatch to the kernels.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/mcspin.h"
#include "common.hpp"
#include "internal.hpp"

using namespace mcs;

namespace mcs {

int fail(mc_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->last_error = buf;
    }
    return code;
}

int device_check(mc_ctx *ctx, hipError_t e, const char *what)
{
    if (e == hipSuccess) return MC_OK;
    return fail(ctx, MC_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int set_device(mc_ctx *ctx)
{
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || ctx->device >= n)
        return fail(ctx, MC_E_DEVICE, "HIP device %d not available", ctx->device);
    return device_check(ctx, hipSetDevice(ctx->device), "hipSetDevice");
}

int capture_stream(mc_ctx *ctx, hipStream_t *out)
{
    if (!ctx->capture) {
        hipError_t e = hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking);
        if (e != hipSuccess) {
            ctx->capture = nullptr;
            return device_check(ctx, e, "hipStreamCreateWithFlags");
        }
    }
    *out = ctx->capture;
    return MC_OK;
}

int check_geom(mc_ctx *ctx, const mc_geom *g, bool need_count)
{
    if (!g) return fail(ctx, MC_E_INVAL, "geom is NULL");
    if (g->dims != 2 && g->dims != 3) return fail(ctx, MC_E_SHAPE, "dims must be 2 or 3 (got %d)", g->dims);
    if (g->layout != MC_INT8 && g->layout != MC_MSC64) return fail(ctx, MC_E_INVAL, "unknown layout %d", g->layout);
    const int Lz = g->dims == 3 ? g->Lz : 1;
    if (g->dims == 2 && g->Lz != 1) return fail(ctx, MC_E_SHAPE, "Lz must be 1 for dims = 2 (got %d)", g->Lz);
    int ext[3] = {g->Lx, g->Ly, Lz};
    for (int d = 0; d < g->dims; ++d) {
        if (ext[d] < 4 || (ext[d] & 1))
            return fail(ctx, MC_E_SHAPE, "extent %d of dimension %d must be even and >= 4", ext[d], d);
        if (ext[d] > (1 << 20)) return fail(ctx, MC_E_SHAPE, "extent %d too large", ext[d]);
    }
    const double N = (double)g->Lx * g->Ly * Lz;
    if (N > 4294967296.0) return fail(ctx, MC_E_SHAPE, "more than 2^32 sites per lattice");
    if (need_count && (g->count < 1)) return fail(ctx, MC_E_RANGE, "count must be >= 1 (got %d)", g->count);
    // the lattice index is a launch dimension of at most 65535 workgroups
    if (need_count && g->count > 65535) return fail(ctx, MC_E_RANGE, "count must be <= 65535 (got %d)", g->count);
    if (need_count && (double)g->count * N * (g->layout == MC_MSC64 ? 8.0 : 1.0) > 1.0e12)
        return fail(ctx, MC_E_RANGE, "lattice buffer too large");
    // replica ids must fit 32 bits (checked by the callers that know replica0)
    return MC_OK;
}

Geom to_geom(const mc_geom *g)
{
    Geom o;
    o.dims = g->dims;
    o.Lx = g->Lx;
    o.Ly = g->Ly;
    o.Lz = g->dims == 3 ? g->Lz : 1;
    o.N = (int64_t)o.Lx * o.Ly * o.Lz;
    o.count = g->count;
    return o;
}

// Acceptance tables, FP64 on the host, once per call.  An entry is
// ceil(p 2^32): r < p for r = r32 / 2^32 is exactly r32 < ceil(p 2^32).
//   Metropolis (Eq. metropolis-canonical): p = exp(-beta dE), dE = 4k.
//   Heat-bath (Eq. heatbath): p(+ | h) = 1 / (1 + exp(-2 beta h)).
SweepTables build_tables(double beta)
{
    SweepTables t;
    for (int k = 0; k < 4; ++k) {
        const double p = std::exp(-beta * (double)(4 * k));
        t.met[k] = split_thr((uint64_t)std::ceil(std::ldexp(p, 32)));
    }
    for (int h = -6; h <= 6; ++h) {
        const double e = std::exp(-2.0 * beta * (double)h);
        const double p = 1.0 / (1.0 + e);
        t.hb[h + 6] = split_thr((uint64_t)std::ceil(std::ldexp(p, 32)));
    }
    return t;
}

int check_sweep_args(mc_ctx *ctx, const mc_geom *geom, const void *spins, const mc_sweep_args *args)
{
    int rc = check_geom(ctx, geom, true);
    if (rc) return rc;
    if (!spins) return fail(ctx, MC_E_INVAL, "spins is NULL");
    if (!args) return fail(ctx, MC_E_INVAL, "args is NULL");
    if (args->rule != MC_METROPOLIS && args->rule != MC_HEATBATH)
        return fail(ctx, MC_E_INVAL, "unknown rule %d", args->rule);
    if (!(args->beta >= 0.0) || std::isinf(args->beta))
        return fail(ctx, MC_E_RANGE, "beta must be finite and >= 0");
    if (args->nsweeps < 0) return fail(ctx, MC_E_RANGE, "nsweeps must be >= 0");
    if (args->sweep0 + (uint64_t)args->nsweeps >= (1ull << 55))
        return fail(ctx, MC_E_RANGE, "sweep numbers must stay below 2^55");
    const uint64_t lanes = geom->layout == MC_MSC64 ? 64 : 1;
    if ((uint64_t)args->replica0 + lanes * (uint64_t)geom->count > 4294967296ull)
        return fail(ctx, MC_E_RANGE, "replica ids exceed 32 bits");
    return MC_OK;
}

int sweep_dispatch(mc_ctx *ctx, const mc_geom *geom, void *spins, const int8_t *J, const mc_sweep_args *args,
                   int64_t *EM, void *ws, size_t ws_bytes, hipStream_t s)
{
    SweepCall c;
    c.g = to_geom(geom);
    c.J = J;
    c.rule = args->rule;
    c.seed_lo = (uint32_t)args->seed;
    c.seed_hi = (uint32_t)(args->seed >> 32);
    c.replica0 = args->replica0;
    c.tab = build_tables(args->beta);
    c.per_lattice = 0;
    c.tabs = nullptr;
    const int64_t lanes = geom->layout == MC_MSC64 ? 64 : 1;
    const int64_t em_stride = 2 * (int64_t)geom->count * lanes;
    return run_sweeps(ctx, c, geom->layout, spins, args->sweep0, args->nsweeps, EM, em_stride, ws, ws_bytes, s);
}

}  // namespace mcs

// ============================================================================
extern "C" {

int mc_abi_version(void) { return MC_ABI_VERSION; }

const char *mc_strerror(int code)
{
    switch (code) {
    case MC_OK: return "success";
    case MC_E_INVAL: return "invalid argument";
    case MC_E_SHAPE: return "unsupported lattice shape";
    case MC_E_RANGE: return "argument out of range";
    case MC_E_LAYOUT: return "unsupported layout/rule combination";
    case MC_E_WORKSPACE: return "workspace missing or too small";
    case MC_E_DEVICE: return "HIP device error";
    case MC_E_NOTCONV: return "multicanonical iteration did not converge";
    case MC_E_IO: return "file could not be opened, read or written";
    default: return "unknown error code";
    }
}

int mc_ctx_create(mc_ctx **out, int device)
{
    // Host state only: the device is first touched by the first call that
    // enqueues work (after that call's argument checks).
    if (!out) return MC_E_INVAL;
    *out = nullptr;
    if (device < 0) return MC_E_INVAL;
    mc_ctx *c = new (std::nothrow) mc_ctx;
    if (!c) return MC_E_DEVICE;
    c->device = device;
    *out = c;
    return MC_OK;
}

void mc_ctx_destroy(mc_ctx *ctx) { delete ctx; }

const char *mc_ctx_last_error(const mc_ctx *ctx) { return ctx ? ctx->last_error.c_str() : "no context"; }

int mc_init(mc_ctx *ctx, const mc_geom *geom, void *spins, int32_t start, uint64_t seed, uint32_t replica0,
            void *stream)
{
    if (!ctx) return MC_E_INVAL;
    int rc = check_geom(ctx, geom, true);
    if (rc) return rc;
    if (!spins) return fail(ctx, MC_E_INVAL, "spins is NULL");
    if (start != MC_COLD && start != MC_HOT) return fail(ctx, MC_E_INVAL, "start must be MC_COLD or MC_HOT");
    const uint64_t lanes = geom->layout == MC_MSC64 ? 64 : 1;
    if ((uint64_t)replica0 + lanes * (uint64_t)geom->count > 4294967296ull)
        return fail(ctx, MC_E_RANGE, "replica ids exceed 32 bits");
    if ((rc = set_device(ctx))) return rc;
    const Geom g = to_geom(geom);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = geom->layout == MC_INT8 ? launch_init_int8(g, (int8_t *)spins, start, seed, replica0, s)
                                           : launch_init_msc64(g, (uint64_t *)spins, start, seed, replica0, s);
    return device_check(ctx, e, "mc_init launch");
}

int mc_couplings(mc_ctx *ctx, const mc_geom *geom, int8_t *J, uint64_t seed, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    int rc = check_geom(ctx, geom, false);
    if (rc) return rc;
    if (!J) return fail(ctx, MC_E_INVAL, "J is NULL");
    if ((double)geom->dims * geom->Lx * geom->Ly * (geom->dims == 3 ? geom->Lz : 1) > 4294967296.0 * 16)
        return fail(ctx, MC_E_SHAPE, "too many bonds");
    if ((rc = set_device(ctx))) return rc;
    return device_check(ctx, launch_couplings(to_geom(geom), J, seed, (hipStream_t)stream), "mc_couplings launch");
}

size_t mc_sweep_workspace_bytes(const mc_geom *geom)
{
    if (!geom || check_geom(nullptr, geom, true) != MC_OK) return 0;
    return fused_workspace_bytes(to_geom(geom), geom->layout);
}

int mc_sweep(mc_ctx *ctx, const mc_geom *geom, void *spins, const int8_t *J, const mc_sweep_args *args,
             int64_t *EM, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    int rc = check_sweep_args(ctx, geom, spins, args);
    if (rc) return rc;
    if (args->nsweeps == 0) return MC_OK;
    if ((rc = set_device(ctx))) return rc;
    return sweep_dispatch(ctx, geom, spins, J, args, EM, ws, ws_bytes, (hipStream_t)stream);
}

int mc_sweep_betas(mc_ctx *ctx, const mc_geom *geom, void *spins, const int8_t *J, const mc_sweep_args *args,
                   const double *betas, int64_t *EM, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    int rc = check_geom(ctx, geom, true);
    if (rc) return rc;
    if (!betas) return fail(ctx, MC_E_INVAL, "betas is NULL");
    if (geom->layout != MC_INT8) return fail(ctx, MC_E_LAYOUT, "per-lattice temperatures need MC_INT8");
    for (int l = 0; l < geom->count; ++l)
        if (!(betas[l] >= 0.0) || std::isinf(betas[l])) return fail(ctx, MC_E_RANGE, "betas[%d] out of range", l);
    mc_sweep_args a1 = args ? *args : mc_sweep_args{};
    if (!args) return fail(ctx, MC_E_INVAL, "args is NULL");
    a1.beta = betas[0];
    // common argument checks (spins, rule, counts) through the single-beta path's rules
    if (!spins) return fail(ctx, MC_E_INVAL, "spins is NULL");
    if (a1.rule != MC_METROPOLIS && a1.rule != MC_HEATBATH) return fail(ctx, MC_E_INVAL, "unknown rule %d", a1.rule);
    if (a1.nsweeps < 0) return fail(ctx, MC_E_RANGE, "nsweeps must be >= 0");
    if (a1.sweep0 + (uint64_t)a1.nsweeps >= (1ull << 55)) return fail(ctx, MC_E_RANGE, "sweep numbers must stay below 2^55");
    if ((uint64_t)a1.replica0 + (uint64_t)geom->count > 4294967296ull)
        return fail(ctx, MC_E_RANGE, "replica ids exceed 32 bits");
    if (a1.nsweeps == 0) return MC_OK;
    if ((rc = set_device(ctx))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const int64_t em_stride = 2 * (int64_t)geom->count;
    std::vector<SweepTables> tabs((size_t)geom->count);
    for (int l = 0; l < geom->count; ++l) tabs[(size_t)l] = build_tables(betas[l]);
    SweepCall c;
    c.g = to_geom(geom);
    c.J = J;
    c.rule = a1.rule;
    c.seed_lo = (uint32_t)a1.seed;
    c.seed_hi = (uint32_t)(a1.seed >> 32);
    c.replica0 = a1.replica0;
    c.tab = tabs[0];
    c.per_lattice = 1;
    c.tabs = tabs.data();
    return run_sweeps_betas(ctx, c, (int8_t *)spins, a1.sweep0, a1.nsweeps, EM, em_stride, ws, ws_bytes, s);
}

int mc_measure(mc_ctx *ctx, const mc_geom *geom, const void *spins, const int8_t *J, int64_t *EM, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    int rc = check_geom(ctx, geom, true);
    if (rc) return rc;
    if (!spins || !EM) return fail(ctx, MC_E_INVAL, "spins or EM is NULL");
    if ((rc = set_device(ctx))) return rc;
    const Geom g = to_geom(geom);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = geom->layout == MC_INT8 ? launch_measure_int8(g, (const int8_t *)spins, J, EM, s)
                                           : launch_measure_msc64(g, (const uint64_t *)spins, J, EM, s);
    return device_check(ctx, e, "mc_measure launch");
}

}  // extern "C"
