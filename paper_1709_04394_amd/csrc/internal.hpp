// internal.hpp -- host-side helpers shared by the ABI translation units.
#pragma once

#include <cstdarg>
#include <cstddef>

#include "../../include/mcspin.h"
#include "common.hpp"

namespace mcs {

int fail(mc_ctx *ctx, int code, const char *fmt, ...);
int device_check(mc_ctx *ctx, hipError_t e, const char *what);
int set_device(mc_ctx *ctx);
int check_geom(mc_ctx *ctx, const mc_geom *g, bool need_count);
Geom to_geom(const mc_geom *g);
SweepTables build_tables(double beta);

// Sweep driver: chooses the fused single-pass kernel when the geometry and the
// workspace allow it, the generic two-launch half-sweeps otherwise.
size_t fused_workspace_bytes(const Geom &g, int layout);
int run_sweeps(mc_ctx *ctx, const SweepCall &c, int layout, void *spins, uint64_t sweep0, int nsweeps,
               int64_t *EM, int64_t em_stride, void *ws, size_t ws_bytes, hipStream_t s);

}  // namespace mcs
