// sweep_driver.hip -- sequencing of half-sweeps, fused multi-sweep launches
// and per-sweep measurement for mc_sweep, and the launch-shape autotuner.
#include <algorithm>
#include <vector>

#include "internal.hpp"

namespace mcs {

// Bytes of one packed copy of all lattices: one bit per spin.
static size_t packed_bytes(const Geom &g)
{
    return (size_t)g.count * (size_t)g.Ly * (size_t)(g.dims == 3 ? g.Lz : 1) * (size_t)(g.Lx / 8);
}

static bool fused2d_geom(const Geom &g, int layout)
{
    return layout == MC_INT8 && g.dims == 2 && g.Lx % 64 == 0 && g.Lx <= 16384;
}

static bool fused3d_geom(const Geom &g, int layout)
{
    return layout == MC_INT8 && g.dims == 3 && g.Lx % 64 == 0 && g.Lx <= 4096 && g.Ly >= 4 && g.Lz >= 4;
}

// Two packed copies (ping-pong between the launches of one call), in 3D the
// couplings in packed form (three directions, whether or not a call has
// couplings), then two arrays of per-tile (E, M) sums (ping-pong likewise).
// The 2D packed copies end on a multiple of 16 bytes (Lx / 4 bytes per row
// pair); in 3D the slots start on the next multiple of 256.
static size_t fused_slots_offset(const Geom &g)
{
    if (g.dims == 2) return 2 * packed_bytes(g);
    Geom one = g;
    one.count = 1;
    return (2 * packed_bytes(g) + 3 * packed_bytes(one) + 255) & ~(size_t)255;
}

size_t fused_workspace_bytes(const Geom &g, int layout)
{
    if (fused2d_geom(g, layout)) return fused_slots_offset(g) + 2 * tile2d_slot_bytes(g);
    if (fused3d_geom(g, layout)) return fused_slots_offset(g) + 2 * tile3d_slot_bytes(g);
    return 0;
}

// Default launch shape of the 2D kernel: enough bands to give every CU work,
// sweeps per launch limited so the redone halo stays small.
TilePlan default_tile_plan(const Geom &g)
{
    TilePlan p;
    if (g.dims == 3) {
        // 16 x 16 tiles give a 256^3 lattice one tile per CU; two sweeps per
        // launch, reduced until the tile fits LDS with room for couplings.
        // Threads: with one tile per CU a wide workgroup (768) evens out the
        // shrinking half-sweeps best; with several tiles per CU narrower
        // workgroups run side by side on a CU instead of one after another
        // (1024 threads leave room for one workgroup per CU): 256^3 x 4 at
        // 256 threads takes 39 us per sweep against 62 us at 1024.
        p.H = std::min(16, std::min(g.Ly, g.Lz));
        p.K = 2;
        while (p.K > 1 && tile3d_lds_bytes(g.Lx, p.H, p.K, true) > 98304) --p.K;
        while (p.H > 1 && tile3d_lds_bytes(g.Lx, p.H, p.K, true) > 98304) p.H /= 2;
        constexpr int64_t kCUs = 256;
        const int64_t tiles = (int64_t)g.count * ((g.Ly + p.H - 1) / p.H) * ((g.Lz + p.H - 1) / p.H);
        p.threads = tiles >= 4 * kCUs ? 256 : tiles >= 2 * kCUs ? 512 : 768;
        return p;
    }
    const int want_tiles = 256;
    const int64_t per = std::max<int64_t>(1, (int64_t)want_tiles / std::max(1, g.count));
    int H = (int)std::max<int64_t>(4, g.Ly / per);
    H = std::min(H, 64);
    H = std::min(H, g.Ly);
    p.H = H;
    p.K = H >= 16 ? 2 : 1;
    while (p.K > 1 && tile2d_lds_bytes(g.Lx, p.H, p.K) > 65536) --p.K;
    while (p.H > 4 && tile2d_lds_bytes(g.Lx, p.H, p.K) > 65536) p.H /= 2;
    const int tasks = (p.H + 2 * p.K) * (g.Lx / 64);
    p.threads = std::min(1024, std::max(64, ((tasks + 63) / 64) * 64));
    while (g.Lx / 64 > p.threads && (g.Lx / 64) % p.threads) p.threads += 64;
    return p;
}

// A row of Wd = Lx/64 words is spread over the threads; when it is wider than
// the workgroup every thread must take the same number of words, because the
// tie queue's fill level is kept wave-uniform by all lanes taking part in the
// same ballots.  3D tiles are H x H rows (y, z); their LDS (with room for
// couplings) must fit in 96 KB.  The band height (2D) or tile side (3D) has a
// floor, 4 or 2, for which the workspace's per-tile (E, M) slots are sized.
static bool plan_ok(const Geom &g, const TilePlan &p)
{
    const int Wd = g.Lx / 64;
    if (p.H < 1 || p.K < 1 || p.threads < 64 || p.threads > 1024 || p.threads % 64 != 0) return false;
    if (g.dims == 3)
        return p.H >= 2 && p.K <= 4 && Wd <= p.threads && p.H <= std::min(g.Ly, g.Lz) &&
               tile3d_lds_bytes(g.Lx, p.H, p.K, true) <= 98304;
    return p.H >= 4 && p.K <= 8 && (Wd <= p.threads || Wd % p.threads == 0) &&
           tile2d_lds_bytes(g.Lx, std::min(p.H, g.Ly), p.K) <= 65536;
}

static std::tuple<int, int, int, int, int> plan_key(const Geom &g)
{
    return std::make_tuple(g.dims, g.Lx, g.Ly, g.dims == 3 ? g.Lz : 1, g.count);
}

static TilePlan plan_for(mc_ctx *ctx, const Geom &g)
{
    auto it = ctx->tile_plans.find(plan_key(g));
    if (it != ctx->tile_plans.end()) return it->second;
    return default_tile_plan(g);
}

// Split n >= 1 sweeps into launches of at most K sweeps, sizes as equal as
// possible; at least two launches (a launch never writes its own input), the
// second of zero sweeps when n = 1.
static std::vector<int> split_launches(int n, int K)
{
    if (n == 1) return {1, 0};
    const int m = std::max(2, (n + K - 1) / K);
    std::vector<int> sizes(m, n / m);
    for (int i = 0; i < n % m; ++i) sizes[i] += 1;
    return sizes;
}

// Launch i reads the caller's int8 lattices (i = 0) or packed copy (i - 1) & 1
// of the workspace, and writes packed copy i & 1 or, for the last launch, the
// caller's lattices.  With EM, launch i also stores its per-tile sums in slot
// array i & 1 and adds up those of launch i - 1 into EM; a small kernel adds
// up the last launch's.
static int run_fused(mc_ctx *ctx, const SweepCall &c, const TilePlan &p, int8_t *spins, char *ws, uint64_t sweep0,
                     int nsweeps, int64_t *EM, int64_t em_stride, hipStream_t s)
{
    hipError_t e = hipSuccess;
    const bool three = c.g.dims == 3;
    const std::vector<int> sizes = split_launches(nsweeps, p.K);
    char *pk[2] = {ws, ws + packed_bytes(c.g)};
    uint32_t *Jp = nullptr;
    if (three && c.J) {
        Jp = (uint32_t *)(ws + 2 * packed_bytes(c.g));
        e = launch_pack_couplings(c.g, c.J, Jp, s);
    }
    char *slots = ws + fused_slots_offset(c.g);
    const size_t slot_bytes = three ? tile3d_slot_bytes(c.g) : tile2d_slot_bytes(c.g);
    int64_t *slot[2] = {(int64_t *)slots, (int64_t *)(slots + slot_bytes)};
    int tiles;
    if (three) {
        tiles = ((c.g.Ly + p.H - 1) / p.H) * ((c.g.Lz + p.H - 1) / p.H);
    } else {
        const int H = std::min(p.H, c.g.Ly);
        tiles = (c.g.Ly + H - 1) / H;
    }
    EmSlots pend;  // tile sums not yet added up
    pend.EM = EM;
    pend.em_stride = em_stride;
    int done = 0;
    const size_t m = sizes.size();
    for (size_t i = 0; i < m && e == hipSuccess; ++i) {
        const bool first = i == 0, last = i + 1 == m;
        const void *src = first ? (const void *)spins : (const void *)pk[(i - 1) & 1];
        void *dst = last ? (void *)spins : (void *)pk[i & 1];
        EmSlots em = pend;
        em.slots = EM ? slot[i & 1] : nullptr;
        if (three)
            e = launch_tile3d(c, src, first ? 0 : 1, dst, last ? 0 : 1, Jp, sweep0 + (uint64_t)done, sizes[i], p.H,
                              p.threads, em, s);
        else
            e = launch_tile2d(c, src, first ? 0 : 1, dst, last ? 0 : 1, sweep0 + (uint64_t)done, sizes[i],
                              std::min(p.H, c.g.Ly), p.threads, em, s);
        pend.red_in = EM && sizes[i] > 0 ? slot[i & 1] : nullptr;
        pend.red_K = EM ? sizes[i] : 0;
        pend.red_sweep0 = done;
        done += sizes[i];
    }
    if (e == hipSuccess && pend.red_in)
        e = launch_em_slots(pend.red_in, tiles, c.g.count, pend.red_K, EM, em_stride, pend.red_sweep0, s);
    return device_check(ctx, e, "mc_sweep fused launch");
}

// Which kernel family runs a call, in order of preference: the fused tiles
// (given a large enough workspace and a usable plan), the bit-packed whole
// lattice, the int8 whole lattice, the multi-spin-coded kernel, the generic
// half-sweeps.
static int sweep_path(mc_ctx *ctx, const SweepCall &c, int layout, bool have_ws, size_t ws_bytes)
{
    if ((tile2d_supported(c, layout) || tile3d_supported(c, layout)) && have_ws &&
        ws_bytes >= fused_workspace_bytes(c.g, layout) && plan_ok(c.g, plan_for(ctx, c.g)))
        return c.g.dims == 2 ? MC_PATH_FUSED_2D : MC_PATH_FUSED_3D;
    if (small_bits_supported(c, layout)) return MC_PATH_SMALL_BITS;
    if (small_supported(c, layout)) return MC_PATH_SMALL;
    if (msc_fast_supported(c, layout)) return MC_PATH_MSC64;
    return MC_PATH_GENERIC;
}

// The kernel family of a call with per-lattice temperatures: the fused
// tiles carry one table per lattice; every other family runs the lattices
// one at a time, each alone with its own table and no workspace.
static SweepCall single_lattice(const SweepCall &c, int l)
{
    SweepCall c1 = c;
    c1.g.count = 1;
    c1.replica0 = c.replica0 + (uint32_t)l;
    if (c.per_lattice) c1.tab = c.tabs[l];
    c1.per_lattice = 0;
    c1.tabs = nullptr;
    return c1;
}

static int betas_path(mc_ctx *ctx, const SweepCall &c, bool have_ws, size_t ws_bytes)
{
    const int p = sweep_path(ctx, c, MC_INT8, have_ws, ws_bytes);
    if (p == MC_PATH_FUSED_2D || p == MC_PATH_FUSED_3D) return p;
    SweepCall c1 = c;
    c1.g.count = 1;
    c1.per_lattice = 0;
    c1.tabs = nullptr;
    return sweep_path(ctx, c1, MC_INT8, false, 0);
}

int run_sweeps_betas(mc_ctx *ctx, const SweepCall &c, int8_t *spins, uint64_t sweep0, int nsweeps, int64_t *EM,
                     int64_t em_stride, void *ws, size_t ws_bytes, hipStream_t s)
{
    const int p = betas_path(ctx, c, ws != nullptr, ws_bytes);
    if (p == MC_PATH_FUSED_2D || p == MC_PATH_FUSED_3D)
        return run_fused(ctx, c, plan_for(ctx, c.g), spins, (char *)ws, sweep0, nsweeps, EM, em_stride, s);
    for (int l = 0; l < c.g.count; ++l) {
        const int rc = run_sweeps(ctx, single_lattice(c, l), MC_INT8, spins + (int64_t)l * c.g.N, sweep0, nsweeps,
                                  EM ? EM + 2 * l : nullptr, em_stride, nullptr, 0, s);
        if (rc) return rc;
    }
    return MC_OK;
}

int run_sweeps(mc_ctx *ctx, const SweepCall &c, int layout, void *spins, uint64_t sweep0, int nsweeps,
               int64_t *EM, int64_t em_stride, void *ws, size_t ws_bytes, hipStream_t s)
{
    const int path = sweep_path(ctx, c, layout, ws != nullptr, ws_bytes);
    // only the fused tiles read per-lattice tables; any other family would
    // apply the first lattice's table to all of them
    if (c.per_lattice && path != MC_PATH_FUSED_2D && path != MC_PATH_FUSED_3D)
        return fail(ctx, MC_E_LAYOUT, "per-lattice temperatures reached a kernel without per-lattice tables");
    switch (path) {
    case MC_PATH_FUSED_2D:
    case MC_PATH_FUSED_3D:
        return run_fused(ctx, c, plan_for(ctx, c.g), (int8_t *)spins, (char *)ws, sweep0, nsweeps, EM, em_stride, s);
    case MC_PATH_SMALL_BITS:
        return device_check(ctx, launch_small_bits(c, (int8_t *)spins, sweep0, nsweeps, EM, em_stride, s),
                            "mc_sweep small bit-packed lattice launch");
    case MC_PATH_SMALL:
        return device_check(ctx, launch_small(c, (int8_t *)spins, sweep0, nsweeps, EM, em_stride, s),
                            "mc_sweep small-lattice launch");
    case MC_PATH_MSC64: {
        hipError_t e = EM ? launch_fill_i64(EM, (int64_t)nsweeps * em_stride, 0, s) : hipSuccess;
        for (int t = 0; t < nsweeps && e == hipSuccess; ++t)
            for (int phase = 0; phase < 2 && e == hipSuccess; ++phase)
                e = launch_msc_phase(c, (uint64_t *)spins, sweep0 + (uint64_t)t, phase, EM ? EM + t * em_stride : nullptr,
                                     s);
        return device_check(ctx, e, "mc_sweep multi-spin launch");
    }
    default:
        break;
    }
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

using namespace mcs;

extern "C" {

int mc_sweep_path(mc_ctx *ctx, const mc_geom *geom, int32_t rule, int32_t has_couplings, int32_t per_lattice,
                  size_t ws_bytes, int32_t *path)
{
    if (!ctx) return MC_E_INVAL;
    int rc = check_geom(ctx, geom, true);
    if (rc) return rc;
    if (!path) return fail(ctx, MC_E_INVAL, "path is NULL");
    if (rule != MC_METROPOLIS && rule != MC_HEATBATH) return fail(ctx, MC_E_INVAL, "unknown rule %d", rule);
    if (per_lattice && geom->layout != MC_INT8) return fail(ctx, MC_E_LAYOUT, "per-lattice temperatures need MC_INT8");
    // the selection reads only the shape, the rule and whether couplings and
    // per-lattice tables are present, never their contents
    static const int8_t some_coupling = 1;
    SweepCall c{};
    c.g = to_geom(geom);
    c.J = has_couplings ? &some_coupling : nullptr;
    c.rule = rule;
    c.per_lattice = per_lattice ? 1 : 0;
    *path = per_lattice ? betas_path(ctx, c, ws_bytes > 0, ws_bytes) : sweep_path(ctx, c, geom->layout, ws_bytes > 0, ws_bytes);
    return MC_OK;
}

int mc_set_tile_plan(mc_ctx *ctx, const mc_geom *geom, int32_t H, int32_t K, int32_t threads)
{
    if (!ctx) return MC_E_INVAL;
    int rc = check_geom(ctx, geom, true);
    if (rc) return rc;
    const Geom g = to_geom(geom);
    TilePlan p;
    p.H = H;
    p.K = K;
    p.threads = threads;
    if (!plan_ok(g, p)) return fail(ctx, MC_E_RANGE, "tile plan H=%d K=%d threads=%d not usable", H, K, threads);
    ctx->tile_plans[plan_key(g)] = p;
    return MC_OK;
}

int mc_get_tile_plan(mc_ctx *ctx, const mc_geom *geom, int32_t *H, int32_t *K, int32_t *threads)
{
    if (!ctx || !H || !K || !threads) return MC_E_INVAL;
    int rc = check_geom(ctx, geom, true);
    if (rc) return rc;
    const TilePlan p = plan_for(ctx, to_geom(geom));
    *H = p.H;
    *K = p.K;
    *threads = p.threads;
    return MC_OK;
}

int mc_tune_sweep(mc_ctx *ctx, const mc_geom *geom, void *scratch_a, void *scratch_b, double beta, int32_t sweeps,
                  void *stream)
{
    return mc_tune_sweep_rule(ctx, geom, MC_METROPOLIS, scratch_a, scratch_b, beta, sweeps, stream);
}

int mc_tune_sweep_rule(mc_ctx *ctx, const mc_geom *geom, int32_t rule, void *scratch_a, void *scratch_b, double beta,
                       int32_t sweeps, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    int rc = check_geom(ctx, geom, true);
    if (rc) return rc;
    if (!scratch_a || !scratch_b) return fail(ctx, MC_E_INVAL, "scratch buffers are NULL");
    if (rule != MC_METROPOLIS && rule != MC_HEATBATH) return fail(ctx, MC_E_INVAL, "unknown rule %d", rule);
    if (!(beta >= 0.0) || sweeps < 1 || sweeps > 1000) return fail(ctx, MC_E_RANGE, "beta or sweeps out of range");
    const Geom g = to_geom(geom);
    SweepCall c;
    c.g = g;
    c.J = nullptr;
    c.rule = rule;
    c.seed_lo = 1;
    c.seed_hi = 0;
    c.replica0 = 0;
    c.tab = build_tables(beta);
    c.per_lattice = 0;
    c.tabs = nullptr;
    const bool three = g.dims == 3;
    if (!(three ? tile3d_supported(c, geom->layout) : tile2d_supported(c, geom->layout)))
        return fail(ctx, MC_E_LAYOUT, "no tunable kernel for this geometry and rule");
    if ((rc = set_device(ctx))) return rc;
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(ctx, MC_E_DEVICE, "hipEventCreate failed");
    }
    auto launch = [&](const void *src, int inp, void *dst, int outp, uint64_t sweep0, int K, const TilePlan &p,
                      bool measure) {
        // the tile sums go to the unused half of scratch_b and are not added
        // up (the plans differ in the measuring launches only)
        EmSlots te;
        te.slots = measure ? (int64_t *)((char *)scratch_b + (size_t)g.count * (size_t)g.N / 2) : nullptr;
        if (three) return launch_tile3d(c, src, inp, dst, outp, nullptr, sweep0, K, p.H, p.threads, te, s);
        return launch_tile2d(c, src, inp, dst, outp, sweep0, K, std::min(p.H, g.Ly), p.threads, te, s);
    };
    // a hot lattice, packed into scratch_b
    TilePlan conv = default_tile_plan(g);
    hipError_t e = launch_init_int8(g, (int8_t *)scratch_a, 1, 1, 0, s);
    if (e == hipSuccess) e = launch(scratch_a, 0, scratch_b, 1, 0, 0, conv, false);
    TilePlan best = default_tile_plan(g);
    float best_ms = 1e30f;
    std::vector<int> Hs, Ks, Ts;
    if (three) {
        Hs = {4, 6, 8, 12, 16, 24, 32};
        Ks = {1, 2, 3, 4};
        Ts = {64, 128, 256, 512, 1024};
    } else {
        Hs = {4, 8, 12, 16, 24, 32, 48, 64, 96, 128};
        Ks = {1, 2, 3, 4, 6, 8};
        Ts = {256, 512, 1024};
    }
    for (int H : Hs) {
        if (H > g.Ly || (three && H > g.Lz)) continue;
        for (int K : Ks)
            for (int T : Ts) {
                TilePlan p;
                p.H = H;
                p.K = K;
                p.threads = T;
                if (!plan_ok(g, p) || e != hipSuccess) continue;
                const int Hy = std::min(p.H, g.Ly);
                const int64_t tiles =
                    three ? (int64_t)((g.Ly + H - 1) / H) * ((g.Lz + H - 1) / H) : (int64_t)((g.Ly + Hy - 1) / Hy);
                if ((size_t)K * (size_t)g.count * (size_t)tiles * 16 > (size_t)g.count * (size_t)g.N / 2)
                    continue;  // tile sums larger than half of scratch_b
                int n = std::max(sweeps, 2 * K);
                n -= n % (2 * K);
                // the steady state of a long measured call: packed -> packed
                // launches between the two scratch buffers, measuring E, M; a
                // warm-up launch, then the best of two timed runs
                e = launch(scratch_b, 1, scratch_a, 1, 0, K, p, true);
                float ms = 1e30f;
                for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
                    e = hipEventRecord(e0, s);
                    for (int i = 0; i < n / K && e == hipSuccess; ++i)
                        e = launch((i & 1) ? scratch_b : scratch_a, 1, (i & 1) ? scratch_a : scratch_b, 1,
                                   (uint64_t)i * K, K, p, true);
                    if (e == hipSuccess) e = hipEventRecord(e1, s);
                    if (e == hipSuccess) e = hipEventSynchronize(e1);
                    float t = 0;
                    if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
                    ms = std::min(ms, t / (float)n);
                }
                if (e != hipSuccess) break;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = p;
                }
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return device_check(ctx, e, "mc_tune_sweep");
    ctx->tile_plans[plan_key(g)] = best;
    return MC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Double-checkerboard sweeps with k hits per tile (a different Markov chain
// from mc_sweep's): the caller's int8 lattices are packed into the workspace
// once, every sweep is two in-place launches (one per coarse colour of the
// tiles), and the last step unpacks them.
extern "C" {

// The packed lattices, then two arrays of (E, M) slots (consecutive sweeps
// alternate) for the smallest tile's count, each rounded up to 256 bytes.
static size_t dcb_slot_bytes(const mc_geom *geom)
{
    const size_t b = (size_t)geom->count * (size_t)(geom->Lx / 64) * (size_t)(geom->Lx / 64) * 2 * 8;
    return (b + 255) & ~(size_t)255;
}

size_t mc_dcb_workspace_bytes(const mc_geom *geom)
{
    if (!geom || check_geom(nullptr, geom, true) != MC_OK) return 0;
    if (geom->dims != 2 || geom->layout != MC_INT8 || geom->Lx != geom->Ly || geom->Lx % 64 ||
        geom->Lx > 16384)
        return 0;
    return ((packed_bytes(to_geom(geom)) + 255) & ~(size_t)255) + 2 * dcb_slot_bytes(geom);
}

int mc_sweep_dcb(mc_ctx *ctx, const mc_geom *geom, void *spins, const mc_sweep_args *args, int32_t tile,
                 int32_t hits, int64_t *EM, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    int rc = check_sweep_args(ctx, geom, spins, args);
    if (rc) return rc;
    if (geom->dims != 2 || geom->layout != MC_INT8)
        return fail(ctx, MC_E_LAYOUT, "the double checkerboard takes 2D int8 lattices");
    if (args->rule != MC_METROPOLIS) return fail(ctx, MC_E_LAYOUT, "the double checkerboard runs Metropolis updates");
    const int L = geom->Lx;
    if (geom->Ly != L || L % 64 || L > 16384)
        return fail(ctx, MC_E_SHAPE, "the double checkerboard takes L x L lattices, L a multiple of 64 up to 16384");
    if (tile != 64 && tile != 128 && tile != 256 && tile != 512)
        return fail(ctx, MC_E_SHAPE, "tile must be 64, 128, 256 or 512 (got %d)", tile);
    if (L % tile || ((L / tile) & 1))
        return fail(ctx, MC_E_SHAPE, "L / tile must be an even integer (L = %d, tile = %d)", L, tile);
    if (hits < 1 || hits > 1000) return fail(ctx, MC_E_RANGE, "hits must be 1..1000 (got %d)", hits);
    if ((args->sweep0 + (uint64_t)args->nsweeps) * (uint64_t)hits >= (1ull << 55))
        return fail(ctx, MC_E_RANGE, "sweep numbers times hits must stay below 2^55");
    const Geom g = to_geom(geom);
    const size_t need = mc_dcb_workspace_bytes(geom);
    if (!ws || ws_bytes < need) return fail(ctx, MC_E_WORKSPACE, "workspace needs %zu bytes", need);
    char *slots = (char *)ws + ((packed_bytes(g) + 255) & ~(size_t)255);
    int64_t *part[2] = {(int64_t *)slots, (int64_t *)(slots + dcb_slot_bytes(geom))};
    if (args->nsweeps == 0) return MC_OK;
    if ((rc = set_device(ctx))) return rc;
    hipStream_t s = (hipStream_t)stream;
    SweepCall c;
    c.g = g;
    c.J = nullptr;
    c.rule = MC_METROPOLIS;
    c.seed_lo = (uint32_t)args->seed;
    c.seed_hi = (uint32_t)(args->seed >> 32);
    c.replica0 = args->replica0;
    c.tab = build_tables(args->beta);
    c.per_lattice = 0;
    c.tabs = nullptr;
    // conversions between int8 and packed rows: band launches of no sweeps
    const TilePlan conv = default_tile_plan(g);
    const int H = std::min(conv.H, g.Ly);
    hipError_t e = launch_tile2d(c, spins, 0, ws, 1, 0, 0, H, conv.threads, EmSlots(), s);
    // sweep t stores its tiles' (E, M) in part[t & 1]; the colour-0 launch of
    // sweep t + 1 adds them up into EM row t, a small kernel those of the last
    const int tiles = (L / tile) * (L / tile);
    for (int t = 0; t < args->nsweeps && e == hipSuccess; ++t) {
        EmSlots prev;
        if (EM && t > 0) {
            prev.red_in = part[(t - 1) & 1];
            prev.red_K = 1;
            prev.red_sweep0 = t - 1;
            prev.EM = EM;
            prev.em_stride = 2 * (int64_t)g.count;
        }
        for (int P = 0; P < 2 && e == hipSuccess; ++P)
            e = launch_dcb_phase((uint32_t *)ws, L, tile, g.count, P, hits, c.replica0, args->sweep0 + (uint64_t)t,
                                 c.seed_lo, c.seed_hi, c.tab, EM ? part[t & 1] : nullptr, P == 0 ? prev : EmSlots(), s);
    }
    if (EM && e == hipSuccess)
        e = launch_em_slots(part[(args->nsweeps - 1) & 1], tiles, g.count, 1, EM, 2 * (int64_t)g.count,
                            args->nsweeps - 1, s);
    if (e == hipSuccess) e = launch_tile2d(c, ws, 1, spins, 0, 0, 0, H, conv.threads, EmSlots(), s);
    return device_check(ctx, e, "mc_sweep_dcb");
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Spin glasses multi-spin coded across disorder realisations (64 per word),
// one random number per site shared by the coded realisations.
extern "C" {

int mc_couplings_msc64(mc_ctx *ctx, const mc_geom *geom, uint64_t *J, uint64_t seed, uint32_t realisation0,
                       void *stream)
{
    if (!ctx) return MC_E_INVAL;
    int rc = check_geom(ctx, geom, true);
    if (rc) return rc;
    if (geom->layout != MC_MSC64) return fail(ctx, MC_E_LAYOUT, "coupling words need MC_MSC64");
    if (!J) return fail(ctx, MC_E_INVAL, "J is NULL");
    if ((uint64_t)realisation0 + 64ull * (uint64_t)geom->count > 4294967296ull)
        return fail(ctx, MC_E_RANGE, "realisation ids exceed 32 bits");
    const Geom g = to_geom(geom);
    if ((double)g.dims * (double)g.N > 4294967296.0 * 16) return fail(ctx, MC_E_SHAPE, "too many bonds");
    if ((rc = set_device(ctx))) return rc;
    return device_check(ctx, launch_couplings_msc64(g, J, seed, realisation0, (hipStream_t)stream),
                        "mc_couplings_msc64 launch");
}

int mc_sweep_sg_msc64(mc_ctx *ctx, const mc_geom *geom, uint64_t *spins, const uint64_t *J, const mc_sweep_args *args,
                      int64_t *EM, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    int rc = check_sweep_args(ctx, geom, spins, args);
    if (rc) return rc;
    if (geom->layout != MC_MSC64) return fail(ctx, MC_E_LAYOUT, "realisation coding needs MC_MSC64");
    if (!J) return fail(ctx, MC_E_INVAL, "J is NULL");
    const Geom g = to_geom(geom);
    if (!sg_msc_supported(g))
        return fail(ctx, MC_E_SHAPE, "the sites of one colour must be a multiple of 64 (N = %lld)", (long long)g.N);
    if (args->nsweeps == 0) return MC_OK;
    if ((rc = set_device(ctx))) return rc;
    hipStream_t s = (hipStream_t)stream;
    const SweepTables tab = build_tables(args->beta);
    const int64_t em_stride = 2 * 64 * (int64_t)g.count;
    hipError_t e = EM ? launch_fill_i64(EM, (int64_t)args->nsweeps * em_stride, 0, s) : hipSuccess;
    for (int t = 0; t < args->nsweeps && e == hipSuccess; ++t)
        for (int phase = 0; phase < 2 && e == hipSuccess; ++phase)
            e = launch_sg_msc_phase(g, args->rule, tab, spins, J, (uint32_t)args->seed, (uint32_t)(args->seed >> 32),
                                    args->replica0, args->sweep0 + (uint64_t)t, phase,
                                    EM ? EM + t * em_stride : nullptr, s);
    return device_check(ctx, e, "mc_sweep_sg_msc64");
}

}  // extern "C"
