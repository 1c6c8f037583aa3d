// internal.hpp -- host-side helpers shared by the ABI translation units.
#pragma once

#include <atomic>
#include <cstdarg>
#include <cstddef>
#include <map>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/mcspin.h"
#include "common.hpp"
#include "em_slots.hpp"

namespace mcs {

// Launch shape of the fused sweeps: band height (2D) or tile side in y and z
// (3D), sweeps per launch and threads per workgroup.  Any choice gives the
// same results.
// Size of the device array behind mc_sweep_noalloc (one copy per device).
constexpr size_t kStaticScratchBytes = (size_t)20 << 20;

struct TilePlan {
    int H = 16;
    int K = 2;
    int threads = 512;
};

}  // namespace mcs

namespace mcs {

// An instantiated graph kept for reuse, with the bytes of every input that
// shaped it: a later call with the same inputs launches it again as it is.
struct GraphCache {
    std::vector<unsigned char> key;
    hipGraphExec_t exec = nullptr;
    void reset()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        exec = nullptr;
        key.clear();
    }
    ~GraphCache() { reset(); }
};

}  // namespace mcs

struct mc_ctx {
    int device = 0;
    std::string last_error;
    // tuned launch shapes keyed by (dims, Lx, Ly, Lz, count)
    std::map<std::tuple<int, int, int, int, int>, mcs::TilePlan> tile_plans;
    // population annealing: replicas per workgroup of the sweep kernel, keyed
    // by the lattice extent L (set or tuned; absent means the built-in rule)
    std::map<int, int> pa_groups;
    // stream on which launch sequences are recorded into hipGraphs (created
    // on first use, default priority, destroyed with the context)
    hipStream_t capture = nullptr;
    // the last population-annealing graph (mc_pa_anneal) and tempering graph
    // (mc_pt_run)
    mcs::GraphCache pa_graph, pt_graph;
    ~mc_ctx()
    {
        pa_graph.reset();
        pt_graph.reset();
        if (capture) (void)hipStreamDestroy(capture);
    }
};

namespace mcs {

// Raises one kernel's dynamic-LDS limit, once per device (the attribute
// belongs to the device's copy of the kernel).  One function-local static
// per kernel instance; safe when several host threads launch at once.
class LdsLimit {
  public:
    hipError_t ensure(const void *kernel, int bytes)
    {
        int dev = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return e;
        const uint64_t bit = dev >= 0 && dev < 64 ? (uint64_t)1 << dev : 0;
        if (bit && (done_.load(std::memory_order_acquire) & bit)) return hipSuccess;
        e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e == hipSuccess && bit) done_.fetch_or(bit, std::memory_order_release);
        return e;
    }

  private:
    std::atomic<uint64_t> done_{0};
};

int fail(mc_ctx *ctx, int code, const char *fmt, ...);
int device_check(mc_ctx *ctx, hipError_t e, const char *what);
int set_device(mc_ctx *ctx);
int capture_stream(mc_ctx *ctx, hipStream_t *out);
int check_geom(mc_ctx *ctx, const mc_geom *g, bool need_count);
Geom to_geom(const mc_geom *g);
SweepTables build_tables(double beta);
// mc_sweep's argument checks (everything but the pointers to J, EM and ws),
// and its dispatch once they have passed and the device is current.
int check_sweep_args(mc_ctx *ctx, const mc_geom *geom, const void *spins, const mc_sweep_args *args);
int sweep_dispatch(mc_ctx *ctx, const mc_geom *geom, void *spins, const int8_t *J, const mc_sweep_args *args,
                   int64_t *EM, void *ws, size_t ws_bytes, hipStream_t s);

// fused 2D kernel (k_tile2d.hip)
bool tile2d_supported(const SweepCall &c, int layout);
size_t tile2d_lds_bytes(int Lx, int H, int K);
// One fused launch of k sweeps (k = 0: conversion only).  src / dst are int8
// lattices or, with in_packed / out_packed, the packed rows of the LDS layout
// (per lattice Ly rows of 2 Lx/64 words, even-x array first); src != dst.
// With em.slots set, a launch of k >= 1 sweeps stores every band's (E, M)
// after each sweep in slots [k][count][tiles][2]; with em.red_in set, its
// first workgroups add up the red_K sweeps of band sums of the previous launch
// (same band height) into EM [red_sweep0 + j][count][2] (em_slots.hpp).
hipError_t launch_tile2d(const SweepCall &c, const void *src, int in_packed, void *dst, int out_packed,
                         uint64_t sweep0, int k, int H, int threads, const EmSlots &em, hipStream_t s);
// Adds up K sweeps of per-tile sums (slots as above, tiles per lattice) into
// EM [sweep0 + j][count][2].
hipError_t launch_em_slots(const int64_t *slots, int tiles, int count, int K, int64_t *EM, int64_t em_stride,
                           int64_t sweep0, hipStream_t s);
size_t tile2d_slot_bytes(const Geom &g);
TilePlan default_tile_plan(const Geom &g);

// fused 3D kernel (k_tile3d.hip)
bool tile3d_supported(const SweepCall &c, int layout);
size_t tile3d_lds_bytes(int Lx, int H, int K, bool hasJ);
// E, M as for the 2D kernel, one slot per H x H tile.
hipError_t launch_tile3d(const SweepCall &c, const void *src, int in_packed, void *dst, int out_packed,
                         const uint32_t *Jp, uint64_t sweep0, int k, int H, int threads, const EmSlots &em,
                         hipStream_t s);
size_t tile3d_slot_bytes(const Geom &g);
hipError_t launch_pack_couplings(const Geom &g, const int8_t *J, uint32_t *Jp, hipStream_t s);

// int8 lattices with 32-site rows, bit-packed whole in one workgroup's LDS
// (k_small_bits.hip)
bool small_bits_supported(const SweepCall &c, int layout);
hipError_t launch_small_bits(const SweepCall &c, int8_t *spins, uint64_t sweep0, int nsweeps, int64_t *EM,
                             int64_t em_stride, hipStream_t s);

// small int8 lattices held whole in one workgroup's LDS (k_small.hip)
bool small_supported(const SweepCall &c, int layout);
hipError_t launch_small(const SweepCall &c, int8_t *spins, uint64_t sweep0, int nsweeps, int64_t *EM,
                        int64_t em_stride, hipStream_t s);

// 64-lane multi-spin-coded half-sweep with fused per-lane E, M (k_msc.hip)
bool msc_fast_supported(const SweepCall &c, int layout);
hipError_t launch_msc_phase(const SweepCall &c, uint64_t *words, uint64_t sweep, int phase, int64_t *EM,
                            hipStream_t s);

// Whole lattices in one workgroup's LDS (population annealing, tempering):
// the extents they take, LDS words per row and parity, and lattices per
// workgroup (set on the context, tuned, or the built-in rule).
bool pa_L_ok(int L);
int pa_words_per_row(int L);
int pa_group_for(const mc_ctx *ctx, int L);

// double-checkerboard multi-hit sweeps (k_dcb.hip): one launch updates every
// tile of one coarse colour of the packed lattices in place
size_t dcb_lds_bytes(int T);
// part: this sweep's (E, M) slots [count][(L/T)^2][2], or nullptr; prev: the
// previous sweep's slots, added up by the first workgroup of each lattice
hipError_t launch_dcb_phase(uint32_t *packed, int L, int T, int count, int coarse, int hits, uint32_t replica0,
                            uint64_t sweep, uint32_t seed_lo, uint32_t seed_hi, const SweepTables &tab, int64_t *part,
                            const EmSlots &prev, hipStream_t s);

// +-J spin glasses multi-spin coded across 64 disorder realisations with one
// random number per site shared by the coded copies (k_sg_msc.hip)
bool sg_msc_supported(const Geom &g);
hipError_t launch_couplings_msc64(const Geom &g, uint64_t *J, uint64_t seed, uint32_t realisation0, hipStream_t s);
hipError_t launch_sg_msc_phase(const Geom &g, int rule, const SweepTables &tab, uint64_t *words, const uint64_t *J,
                               uint32_t seed_lo, uint32_t seed_hi, uint32_t replica0, uint64_t sweep, int phase,
                               int64_t *EM, hipStream_t s);

// Sweep driver: chooses the fused kernel when the geometry and the workspace
// allow it, the generic two-launch half-sweeps otherwise.
size_t fused_workspace_bytes(const Geom &g, int layout);
int run_sweeps(mc_ctx *ctx, const SweepCall &c, int layout, void *spins, uint64_t sweep0, int nsweeps,
               int64_t *EM, int64_t em_stride, void *ws, size_t ws_bytes, hipStream_t s);
// Per-lattice temperatures (c.per_lattice, c.tabs): the fused kernels when
// the geometry, plan and workspace allow, else each lattice alone.
int run_sweeps_betas(mc_ctx *ctx, const SweepCall &c, int8_t *spins, uint64_t sweep0, int nsweeps, int64_t *EM,
                     int64_t em_stride, void *ws, size_t ws_bytes, hipStream_t s);

}  // namespace mcs
