// tempering.hip -- parallel tempering (Sec. "Parallel Tempering", Eq. pt):
// the replica-exchange step on the host (mc_pt_exchange), and whole runs of
// sweeps and exchanges on the device (mc_pt_run, kernels in k_pt.hip).
// Host side: the replica-exchange step.  An exchange touches a few
// scalars per pair of temperatures; the replicas' configurations never move
// (temperatures are exchanged, as the paper recommends when replicas live
// apart).  The energies come from the sweeps' fused measurement (mc_sweep /
// mc_sweep_betas per-sweep E), so no extra pass over the lattices is needed.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"
#include "pt.hpp"

using namespace mcs;

namespace {

// Philox4x32-10 (the same generator the kernels use), for a few host draws.
void philox_host(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c[0];
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c[2];
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0, y2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = y0;
        c[1] = (uint32_t)p1;
        c[2] = y2;
        c[3] = (uint32_t)p0;
    }
}

// r32 of pair i in round t: word (i mod 4) of Philox(ctr = (i / 4, 0, t,
// TAG_EXCHANGE << 24 | t >> 32)).
uint32_t pair_draw(uint64_t seed, uint32_t i, uint64_t round)
{
    uint32_t c[4] = {i >> 2, 0u, (uint32_t)round, ctr_w3(kTagExchange, 0, round)};
    philox_host(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    return c[i & 3u];
}

}  // namespace

extern "C" {

int mc_pt_exchange(mc_ctx *ctx, int32_t n_temps, const double *beta, const int64_t *E, int32_t *temp_of,
                   int32_t *replica_at, uint64_t seed, uint64_t round, int64_t *accepted)
{
    if (!ctx) return MC_E_INVAL;
    if (n_temps < 2 || n_temps > (1 << 20)) return fail(ctx, MC_E_RANGE, "n_temps must be 2..2^20 (got %d)", n_temps);
    if (!beta || !E || !temp_of || !replica_at || !accepted) return fail(ctx, MC_E_INVAL, "a pointer argument is NULL");
    if (round >= (1ull << 55)) return fail(ctx, MC_E_RANGE, "round numbers must stay below 2^55");
    for (int i = 0; i < n_temps; ++i) {
        if (!(beta[i] >= 0.0) || std::isinf(beta[i])) return fail(ctx, MC_E_RANGE, "beta[%d] out of range", i);
        if (i > 0 && !(beta[i] > beta[i - 1]))
            return fail(ctx, MC_E_RANGE, "beta must increase strictly (beta[%d] <= beta[%d])", i, i - 1);
        if (E[i] > (1ll << 52) || E[i] < -(1ll << 52)) return fail(ctx, MC_E_RANGE, "|E[%d]| exceeds 2^52", i);
    }
    // the two maps must be inverse permutations of 0..n_temps-1
    std::vector<char> seen((size_t)n_temps, 0);
    for (int i = 0; i < n_temps; ++i) {
        const int32_t a = replica_at[i];
        if (a < 0 || a >= n_temps || seen[(size_t)a] || temp_of[a] != i)
            return fail(ctx, MC_E_INVAL, "replica_at / temp_of are not inverse permutations (at temperature %d)", i);
        seen[(size_t)a] = 1;
    }
    for (int i = (int)(round & 1u); i + 1 < n_temps; i += 2) {
        const int32_t a = replica_at[i], b = replica_at[i + 1];
        // min(1, exp((beta_i - beta_{i+1}) (E_a - E_b))) as an integer test on
        // a 32-bit draw, exactly as the sweeps' acceptance tables
        const double x = (beta[i] - beta[i + 1]) * (double)(E[a] - E[b]);
        bool acc = x >= 0.0;
        if (!acc) {
            const uint64_t T = (uint64_t)std::ceil(std::ldexp(std::exp(x), 32));
            acc = (uint64_t)pair_draw(seed, (uint32_t)i, round) < T;
        }
        if (acc) {
            replica_at[i] = b;
            replica_at[i + 1] = a;
            temp_of[a] = i + 1;
            temp_of[b] = i;
            accepted[i] += 1;
        }
    }
    return MC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// mc_pt_run: rounds of sweeps and exchanges on the device.

namespace {

size_t pt_align(size_t b) { return (b + 255) & ~(size_t)255; }

struct PtLayout {
    size_t thr = 0, xtab = 0, temp_of = 0, replica_at = 0, E = 0, accepted = 0, E_at = 0, total = 0;
};

int64_t pt_mmax(int L) { return (int64_t)L * L; }  // (E_a - E_b) / 4 <= 4N / 4

PtLayout pt_layout(const mc_pt_args *a)
{
    PtLayout l;
    const size_t nT = (size_t)a->n_temps, count = nT * (size_t)a->n_sets;
    size_t off = 0;
    l.thr = off, off += pt_align(nT * 2 * sizeof(Thr));
    l.xtab = off, off += pt_align((nT - 1) * (size_t)(pt_mmax(a->L) + 1) * 8);
    l.temp_of = off, off += pt_align(count * 4);
    l.replica_at = off, off += pt_align(count * 4);
    l.E = off, off += pt_align(count * 4);
    l.accepted = off, off += pt_align((size_t)a->n_sets * (nT - 1) * 8);
    l.E_at = off, off += pt_align((size_t)a->rounds * count * 8);
    l.total = off;
    return l;
}

int check_pt(mc_ctx *ctx, const mc_pt_args *a)
{
    if (!a) return fail(ctx, MC_E_INVAL, "args is NULL");
    if (!pa_L_ok(a->L))
        return fail(ctx, MC_E_SHAPE, "L=%d: tempering takes L in {4,8,16,32,64} or a multiple of 64 up to 512", a->L);
    if (a->n_temps < 2 || a->n_temps > kPtMaxTemps)
        return fail(ctx, MC_E_RANGE, "n_temps must be 2..%d (got %d)", kPtMaxTemps, a->n_temps);
    if (a->n_sets < 1 || (int64_t)a->n_sets * a->n_temps > 65535 * (int64_t)1)
        return fail(ctx, MC_E_RANGE, "n_sets * n_temps must be 1..65535");
    if (!a->beta) return fail(ctx, MC_E_INVAL, "beta is NULL");
    for (int i = 0; i < a->n_temps; ++i) {
        if (!(a->beta[i] >= 0.0) || std::isinf(a->beta[i])) return fail(ctx, MC_E_RANGE, "beta[%d] out of range", i);
        if (i > 0 && !(a->beta[i] > a->beta[i - 1]))
            return fail(ctx, MC_E_RANGE, "beta must increase strictly (beta[%d] <= beta[%d])", i, i - 1);
    }
    if (a->theta < 1 || a->rounds < 0) return fail(ctx, MC_E_RANGE, "theta must be >= 1 and rounds >= 0");
    if (a->round0 + (uint64_t)a->rounds >= (1ull << 40))
        return fail(ctx, MC_E_RANGE, "round numbers must stay below 2^40");
    if ((a->round0 + (uint64_t)a->rounds) * (uint64_t)a->theta >= (1ull << 55))
        return fail(ctx, MC_E_RANGE, "sweep numbers must stay below 2^55");
    return MC_OK;
}

}  // namespace

extern "C" {

size_t mc_pt_workspace_bytes(const mc_pt_args *args)
{
    if (check_pt(nullptr, args) != MC_OK) return 0;
    return pt_layout(args).total;
}

int mc_pt_run(mc_ctx *ctx, const mc_pt_args *a, int8_t *spins, int32_t *temp_of, int32_t *replica_at,
              int64_t *accepted, int64_t *E_at, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    int rc = check_pt(ctx, a);
    if (rc) return rc;
    if (!spins || !temp_of || !replica_at || !accepted) return fail(ctx, MC_E_INVAL, "a pointer argument is NULL");
    const int nT = a->n_temps, nS = a->n_sets, count = nT * nS;
    for (int s_ = 0; s_ < nS; ++s_) {
        const int32_t *tof = temp_of + (size_t)s_ * nT, *rat = replica_at + (size_t)s_ * nT;
        std::vector<char> seen((size_t)nT, 0);
        for (int i = 0; i < nT; ++i) {
            const int32_t r = rat[i];
            if (r < 0 || r >= nT || seen[(size_t)r] || tof[r] != i)
                return fail(ctx, MC_E_INVAL, "set %d: replica_at / temp_of are not inverse permutations", s_);
            seen[(size_t)r] = 1;
        }
    }
    const PtLayout lay = pt_layout(a);
    if (!ws || ws_bytes < lay.total) return fail(ctx, MC_E_WORKSPACE, "workspace needs %zu bytes", lay.total);
    if ((rc = set_device(ctx))) return rc;
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;

    // host FP64 tables: Metropolis thresholds per temperature, exchange
    // thresholds per pair and energy difference 4m (m = 1 .. N), both
    // ceil(p 2^32) with libm exp, exactly as mc_pt_exchange computes them
    std::vector<Thr> thr((size_t)nT * 2);
    for (int i = 0; i < nT; ++i) {
        const SweepTables t = build_tables(a->beta[i]);
        thr[2 * (size_t)i] = t.met[1];
        thr[2 * (size_t)i + 1] = t.met[2];
    }
    const int64_t mmax = pt_mmax(a->L);
    std::vector<uint64_t> xt((size_t)(nT - 1) * (size_t)(mmax + 1), 0);
    for (int i = 0; i + 1 < nT; ++i)
        for (int64_t m = 1; m <= mmax; ++m) {
            const double x = (a->beta[i] - a->beta[i + 1]) * (double)(4 * m);
            xt[(size_t)i * (mmax + 1) + (size_t)m] = (uint64_t)std::ceil(std::ldexp(std::exp(x), 32));
        }
    hipError_t e = hipMemcpyAsync(w + lay.thr, thr.data(), thr.size() * sizeof(Thr), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(w + lay.xtab, xt.data(), xt.size() * 8, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(w + lay.temp_of, temp_of, (size_t)count * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(w + lay.replica_at, replica_at, (size_t)count * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(w + lay.accepted, accepted, (size_t)nS * (nT - 1) * 8, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return device_check(ctx, e, "mc_pt_run setup");

    PtSweepArgs sw{};
    sw.spins = spins;
    sw.L = a->L;
    sw.Wb = std::min(32, a->L / 2);
    sw.nwr = pa_words_per_row(a->L);
    sw.G = pa_group_for(ctx, a->L);
    sw.count = count;
    sw.temp_of = (const int32_t *)(w + lay.temp_of);
    sw.thr = (const Thr *)(w + lay.thr);
    sw.E = (int32_t *)(w + lay.E);
    sw.theta = a->theta;
    sw.seed_lo = (uint32_t)a->seed;
    sw.seed_hi = (uint32_t)(a->seed >> 32);
    PtExchangeArgs ex{};
    ex.n_temps = nT;
    ex.temp_of = (int32_t *)(w + lay.temp_of);
    ex.replica_at = (int32_t *)(w + lay.replica_at);
    ex.E = sw.E;
    ex.xtab = (const uint64_t *)(w + lay.xtab);
    ex.mmax = (int)mmax;
    ex.accepted = (int64_t *)(w + lay.accepted);
    ex.seed_lo = sw.seed_lo;
    ex.seed_hi = sw.seed_hi;

    // every round as one graph, kept in the context for a call with the same
    // inputs (arguments, schedule, buffers, launch shape)
    std::vector<unsigned char> key;
    auto put = [&key](const void *p, size_t n) {
        key.insert(key.end(), (const unsigned char *)p, (const unsigned char *)p + n);
    };
    const int64_t fields[8] = {ctx->device, a->L, nT, nS, a->theta, (int64_t)a->seed, (int64_t)a->round0, a->rounds};
    put(fields, sizeof fields);
    put(a->beta, sizeof(double) * (size_t)nT);
    put(&spins, sizeof spins);
    put(&ws, sizeof ws);
    const int64_t want_E = E_at != nullptr;
    put(&want_E, sizeof want_E);
    put(&sw.G, sizeof sw.G);
    const bool reuse = ctx->pt_graph.exec && ctx->pt_graph.key == key;
    if (!reuse && a->rounds > 0) {
        ctx->pt_graph.reset();
        hipStream_t cap = nullptr;
        if ((rc = capture_stream(ctx, &cap))) return rc;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        for (int r = 0; r < a->rounds && e == hipSuccess; ++r) {
            const uint64_t round = a->round0 + (uint64_t)r;
            sw.sweep0 = round * (uint64_t)a->theta;
            ex.round = round;
            ex.E_at = E_at ? (int64_t *)(w + lay.E_at) + (size_t)r * count : nullptr;
            e = launch_pt_round(sw, ex, nS, cap);
        }
        const hipError_t ec = hipStreamEndCapture(cap, &graph);
        if (e == hipSuccess) e = ec;
        if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            if (exec) (void)hipGraphExecDestroy(exec);
            return device_check(ctx, e, "mc_pt_run graph");
        }
        ctx->pt_graph.exec = exec;
        ctx->pt_graph.key = key;
    }
    if (a->rounds > 0) e = hipGraphLaunch(ctx->pt_graph.exec, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(temp_of, w + lay.temp_of, (size_t)count * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(replica_at, w + lay.replica_at, (size_t)count * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(accepted, w + lay.accepted, (size_t)nS * (nT - 1) * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess && E_at && a->rounds > 0)
        e = hipMemcpyAsync(E_at, w + lay.E_at, (size_t)a->rounds * count * 8, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        ctx->pt_graph.reset();
        return device_check(ctx, e, "mc_pt_run");
    }
    return MC_OK;
}

}  // extern "C"
