// sweep_driver.hip -- sequencing of half-sweeps, fused sweeps and per-sweep
// measurement for mc_sweep.
#include "internal.hpp"

namespace mcs {

size_t fused_workspace_bytes(const Geom &g, int layout)
{
    (void)g;
    (void)layout;
    return 0;
}

int run_sweeps(mc_ctx *ctx, const SweepCall &c, int layout, void *spins, uint64_t sweep0, int nsweeps,
               int64_t *EM, int64_t em_stride, void *ws, size_t ws_bytes, hipStream_t s)
{
    (void)ws;
    (void)ws_bytes;
    for (int t = 0; t < nsweeps; ++t) {
        const uint64_t sweep = sweep0 + (uint64_t)t;
        hipError_t e = hipSuccess;
        for (int phase = 0; phase < 2 && e == hipSuccess; ++phase)
            e = layout == MC_INT8 ? launch_phase_int8(c, (int8_t *)spins, sweep, phase, s)
                                  : launch_phase_msc64(c, (uint64_t *)spins, sweep, phase, s);
        if (e == hipSuccess && EM)
            e = layout == MC_INT8 ? launch_measure_int8(c.g, (const int8_t *)spins, c.J, EM + t * em_stride, s)
                                  : launch_measure_msc64(c.g, (const uint64_t *)spins, c.J, EM + t * em_stride, s);
        if (e != hipSuccess) return device_check(ctx, e, "mc_sweep launch");
    }
    return MC_OK;
}

}  // namespace mcs
