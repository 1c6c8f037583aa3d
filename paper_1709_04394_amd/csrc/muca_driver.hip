// muca_driver.hip -- host side of the multicanonical method: acceptance
// tables from ln W (FP64, libm exp), the weight recursion (libm log), the
// flatness test, and the production run.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"
#include "muca.hpp"

using namespace mcs;

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct MucaLayout {
    size_t table = 0, hist = 0, H = 0, E = 0, prep = 0, prep_bytes = 0, total = 0;
};

constexpr int kPrepGroups = 16;  // walker groups of the preparation sweeps

MucaLayout muca_layout(int L, int W)
{
    const size_t nlev = (size_t)L * L / 2 + 1, nb = (size_t)(W + 63) / 64;
    MucaLayout m;
    size_t off = 0;
    m.table = off, off += align256(nlev * 16);
    m.hist = off, off += align256(nb * nlev * 4);
    m.H = off, off += align256(nlev * 8);
    m.E = off, off += align256((size_t)W * 8);
    // fused-sweep scratch for the largest preparation group
    const int G = std::min(kPrepGroups, W);
    Geom g{2, L, L, 1, (int64_t)L * L, (W + G - 1) / G};
    m.prep_bytes = fused_workspace_bytes(g, MC_INT8);
    m.prep = off, off += align256(m.prep_bytes);
    m.total = off;
    return m;
}

// Inverse temperature of preparation group g: -d ln W / dE of the initial
// weights by the central difference over levels k_g - 1, k_g + 1 (dE = 8),
// k_g = round((g + 1/2) K / G) clamped to 2 .. K - 1, and at least 0.
double prep_beta(int L, int W, int g, const std::vector<double> &lnW)
{
    const int K = L * L / 2, G = std::min(kPrepGroups, W);
    int k = ((2 * g + 1) * K + G) / (2 * G);
    k = std::min(std::max(k, 2), K - 1);
    return std::max(0.0, -(lnW[(size_t)k + 1] - lnW[(size_t)k - 1]) / 8.0);
}

// T[k][d] = ceil(min(1, exp(lnW[k+d] - lnW[k])) 2^32) (at least 1), stored as
// T - 1 so that r32 < T is r32 <= entry; directions d = -2, -1, +1, +2.
void muca_table(int L, const double *lnW, std::vector<uint32_t> &T)
{
    const int K = L * L / 2;
    static const int dk[4] = {-2, -1, 1, 2};
    T.assign((size_t)(K + 1) * 4, 0u);
    for (int k = 0; k <= K; ++k)
        for (int d = 0; d < 4; ++d) {
            const int k2 = k + dk[d];
            if (k2 < 0 || k2 > K) continue;
            const double x = lnW[k2] - lnW[k];
            const double p = x >= 0.0 ? 1.0 : std::exp(x);
            uint64_t v = (uint64_t)std::ceil(std::ldexp(p, 32));
            if (v == 0) v = 1;
            T[(size_t)k * 4 + d] = (uint32_t)(v - 1);
        }
}

int check_LW(mc_ctx *ctx, int L, int W)
{
    if (!muca_L_supported(L))
        return fail(ctx, MC_E_SHAPE, "L=%d: multicanonical walkers take L in {4,8,12,16,24,32,48,64,96,128}", L);
    if (W < 1 || W > (1 << 24)) return fail(ctx, MC_E_RANGE, "walkers must be 1..2^24");
    return MC_OK;
}

// nsweeps sweeps of every walker; counts added to the device histogram H
int run_muca_sweeps(mc_ctx *ctx, int L, int W, int8_t *spins, int64_t *E, const std::vector<uint32_t> &T,
                    uint64_t seed, uint64_t sweep0, int nsweeps, int record, int64_t *H, char *ws, const MucaLayout &lay,
                    hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(ws + lay.table, T.data(), T.size() * 4, hipMemcpyHostToDevice, s);
    MucaArgs a;
    a.spins = spins;
    a.E = E;
    a.table = (const uint32_t *)(ws + lay.table);
    a.hist = (uint32_t *)(ws + lay.hist);
    a.H = H;
    a.W = W;
    a.seed_lo = (uint32_t)seed;
    a.seed_hi = (uint32_t)(seed >> 32);
    a.record = record;
    // per-workgroup 32-bit counts stay below 2^32: at most 64 N sweeps' worth
    const int chunk = (int)std::max<int64_t>(1, (int64_t)4294967295ll / (64ll * L * L));
    for (int done = 0; done < nsweeps && e == hipSuccess;) {
        const int n = std::min(chunk, nsweeps - done);
        a.sweep0 = sweep0 + (uint64_t)done;
        a.nsweeps = n;
        e = launch_muca_sweeps(a, L, s);
        done += n;
    }
    // the table upload reads host memory owned by the caller's frame
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return device_check(ctx, e, "multicanonical sweeps");
}

int copy_to_host(mc_ctx *ctx, void *dst, const void *src, size_t bytes, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return device_check(ctx, e, "device to host copy");
}

// One step of the weight recursion (Eq. weight_modification) in logs:
// W^(n+1) = W^(n) / H^(n) where H > 0, then ln W(E = 0) = 0 (level K).
void recursion_step(int K, double *lnW, const int64_t *H)
{
    for (int k = 0; k <= K; ++k)
        if (H[k] > 0) lnW[k] = lnW[k] - std::log((double)H[k]);
    const double ref = lnW[K];
    for (int k = 0; k <= K; ++k) lnW[k] = lnW[k] - ref;
}

double flatness(int L, const std::vector<int64_t> &H)
{
    // all levels of the window but k = 1 (E = -2N + 4 has no state)
    int64_t mn = -1, mx = 0;
    for (size_t k = 0; k < H.size(); ++k) {
        if (k == 1) continue;
        mn = mn < 0 ? H[k] : std::min(mn, H[k]);
        mx = std::max(mx, H[k]);
    }
    (void)L;
    return mx > 0 ? (double)mn / (double)mx : 0.0;
}

}  // namespace

extern "C" {

size_t mc_muca_workspace_bytes(int32_t L, int32_t walkers)
{
    if (!muca_L_supported(L) || walkers < 1) return 0;
    return muca_layout(L, walkers).total;
}

int mc_muca_start(mc_ctx *ctx, int32_t L, int32_t walkers, uint64_t seed, int32_t start, int8_t *spins, int64_t *E,
                  void *stream)
{
    if (!ctx) return MC_E_INVAL;
    int rc = check_LW(ctx, L, walkers);
    if (rc) return rc;
    if (!spins || !E) return fail(ctx, MC_E_INVAL, "spins or E is NULL");
    if (start != MC_MUCA_HOT && start != MC_MUCA_STRATIFIED) return fail(ctx, MC_E_INVAL, "unknown start %d", start);
    if ((rc = set_device(ctx))) return rc;
    return device_check(ctx, launch_muca_start(spins, E, L, walkers, seed, start, (hipStream_t)stream),
                        "mc_muca_start");
}

int mc_muca_sweeps(mc_ctx *ctx, int32_t L, int32_t walkers, int8_t *spins, int64_t *E, const double *lnW,
                   uint64_t seed, uint64_t sweep0, int32_t nsweeps, int32_t record, int64_t *H, void *ws,
                   size_t ws_bytes, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    int rc = check_LW(ctx, L, walkers);
    if (rc) return rc;
    if (!spins || !E || !lnW || (record && !H)) return fail(ctx, MC_E_INVAL, "a pointer argument is NULL");
    if (nsweeps < 0) return fail(ctx, MC_E_RANGE, "nsweeps must be >= 0");
    const int K = L * L / 2;
    for (int k = 0; k <= K; ++k)
        if (!std::isfinite(lnW[k])) return fail(ctx, MC_E_RANGE, "lnW[%d] is not finite", k);
    const MucaLayout lay = muca_layout(L, walkers);
    if (!ws || ws_bytes < lay.total) return fail(ctx, MC_E_WORKSPACE, "workspace needs %zu bytes", lay.total);
    if ((rc = set_device(ctx))) return rc;
    std::vector<uint32_t> T;
    muca_table(L, lnW, T);
    return run_muca_sweeps(ctx, L, walkers, spins, E, T, seed, sweep0, nsweeps, record, H, (char *)ws, lay,
                           (hipStream_t)stream);
}

int mc_muca_run(mc_ctx *ctx, const mc_muca_args *a, const double *lnW_init, int8_t *spins, double *lnW_out,
                int64_t *H_out, double *lng_out, double *flat_out, mc_muca_stats *stats, void *ws, size_t ws_bytes,
                void *stream)
{
    if (!ctx) return MC_E_INVAL;
    if (!a) return fail(ctx, MC_E_INVAL, "args is NULL");
    int rc = check_LW(ctx, a->L, a->walkers);
    if (rc) return rc;
    if (!spins || !lnW_out || !H_out || !lng_out || !stats) return fail(ctx, MC_E_INVAL, "an output is NULL");
    if (a->eq_sweeps < 0 || a->rec_sweeps < 1 || a->max_iter < 0 || a->prod_sweeps < 0 || !(a->flat > 0.0) ||
        a->flat > 1.0)
        return fail(ctx, MC_E_RANGE, "sweep counts or flatness out of range");
    if (a->start != MC_MUCA_HOT && a->start != MC_MUCA_STRATIFIED) return fail(ctx, MC_E_INVAL, "unknown start");
    if (a->rec_max < 0 || a->rec_max > (1 << 24)) return fail(ctx, MC_E_RANGE, "rec_max out of range");
    if (a->eq_scale < 0 || a->eq_scale > 64) return fail(ctx, MC_E_RANGE, "eq_scale out of range");
    if (a->prep_sweeps < 0 || a->rec_rule < 0 || a->rec_rule > 1)
        return fail(ctx, MC_E_RANGE, "prep_sweeps or rec_rule out of range");
    // each preparation group is one sweep call of up to 65535 lattices
    if (a->prep_sweeps > 0 && (a->walkers + kPrepGroups - 1) / kPrepGroups > 65535)
        return fail(ctx, MC_E_RANGE, "prep_sweeps needs walkers <= %d", kPrepGroups * 65535);
    const int L = a->L, W = a->walkers, K = L * L / 2;
    const MucaLayout lay = muca_layout(L, W);
    if (!ws || ws_bytes < lay.total) return fail(ctx, MC_E_WORKSPACE, "workspace needs %zu bytes", lay.total);
    std::vector<double> lnW((size_t)K + 1, 0.0);
    if (lnW_init)
        for (int k = 0; k <= K; ++k) {
            if (!std::isfinite(lnW_init[k])) return fail(ctx, MC_E_RANGE, "lnW_init[%d] is not finite", k);
            lnW[(size_t)k] = lnW_init[k];
        }
    if ((rc = set_device(ctx))) return rc;
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    int64_t *E = (int64_t *)(w + lay.E), *Hd = (int64_t *)(w + lay.H);
    rc = device_check(ctx, launch_muca_start(spins, E, L, W, a->seed, a->start, s), "walker start");
    if (rc) return rc;
    if (a->prep_sweeps > 0) {
        // walkers thermalised to the initial weights: group g runs canonical
        // Metropolis sweeps at the weights' inverse temperature there
        const int G = std::min(kPrepGroups, W);
        for (int g = 0; g < G; ++g) {
            const int w0 = (int)((int64_t)g * W / G), w1 = (int)((int64_t)(g + 1) * W / G);
            SweepCall c;
            c.g = Geom{2, L, L, 1, (int64_t)L * L, w1 - w0};
            c.J = nullptr;
            c.rule = MC_METROPOLIS;
            c.seed_lo = (uint32_t)a->seed;
            c.seed_hi = (uint32_t)(a->seed >> 32);
            c.replica0 = (uint32_t)w0;
            c.tab = build_tables(prep_beta(L, W, g, lnW));
            c.per_lattice = 0;
            c.tabs = nullptr;
            if ((rc = run_sweeps(ctx, c, MC_INT8, spins + (int64_t)w0 * L * L, 0, a->prep_sweeps, nullptr, 0,
                                 w + lay.prep, lay.prep_bytes, s)))
                return rc;
        }
        if ((rc = device_check(ctx, launch_muca_settle(spins, E, L, W, s), "walker settle"))) return rc;
    }
    std::vector<uint32_t> T;
    std::vector<int64_t> H((size_t)K + 1);
    uint64_t sweep = 0;
    int it = 0;
    bool converged = false;
    double ratio = 0.0;
    int R = a->rec_sweeps;
    const int Rmax = std::max(a->rec_max, a->rec_sweeps);
    double prev = 0.0;
    while (it < a->max_iter) {
        muca_table(L, lnW.data(), T);
        const int neq = a->eq_sweeps + a->eq_scale * R;
        if ((rc = run_muca_sweeps(ctx, L, W, spins, E, T, a->seed, sweep, neq, 0, nullptr, w, lay, s))) return rc;
        sweep += (uint64_t)neq;
        if ((rc = device_check(ctx, launch_fill_i64(Hd, K + 1, 0, s), "histogram clear"))) return rc;
        if ((rc = run_muca_sweeps(ctx, L, W, spins, E, T, a->seed, sweep, R, 1, Hd, w, lay, s))) return rc;
        sweep += (uint64_t)R;
        if ((rc = copy_to_host(ctx, H.data(), Hd, H.size() * 8, s))) return rc;
        ++it;
        ratio = flatness(L, H);
        if (flat_out) flat_out[it - 1] = ratio;
        if (a->progress) a->progress(a->progress_user, it, ratio, (int64_t)sweep);
        if (ratio >= a->flat) {
            converged = true;
            break;
        }
        // longer iterations once the histogram reaches the whole window
        bool covered = true;
        for (int k = 0; k <= K; ++k)
            if (k != 1 && H[(size_t)k] == 0) covered = false;
        if (covered && (a->rec_rule == 0 || ratio <= prev)) R = std::min(2 * R, Rmax);
        prev = covered ? ratio : 0.0;
        recursion_step(K, lnW.data(), H.data());
    }
    stats->iterations = it;
    stats->converged = converged ? 1 : 0;
    stats->sweeps_per_walker = (int64_t)sweep;
    stats->min_over_max = ratio;
    std::fill(H.begin(), H.end(), 0);
    if (a->prod_sweeps > 0) {
        muca_table(L, lnW.data(), T);
        if ((rc = device_check(ctx, launch_fill_i64(Hd, K + 1, 0, s), "histogram clear"))) return rc;
        // in chunks, so that a progress callback hears from long runs
        const int chunk = 1000;
        for (int done = 0; done < a->prod_sweeps;) {
            const int n = std::min(chunk, a->prod_sweeps - done);
            if ((rc = run_muca_sweeps(ctx, L, W, spins, E, T, a->seed, sweep + (uint64_t)done, n, 1, Hd, w, lay, s)))
                return rc;
            done += n;
            if (a->progress) a->progress(a->progress_user, 0, -1.0, (int64_t)done);
        }
        if ((rc = copy_to_host(ctx, H.data(), Hd, H.size() * 8, s))) return rc;
    }
    for (int k = 0; k <= K; ++k) {
        lnW_out[k] = lnW[(size_t)k];
        H_out[k] = H[(size_t)k];
        lng_out[k] = H[(size_t)k] > 0 ? std::log((double)H[(size_t)k]) - lnW[(size_t)k] : -INFINITY;
    }
    return converged ? MC_OK : fail(ctx, MC_E_NOTCONV, "not flat after %d iterations (min/max %.3f)", it, ratio);
}

int mc_muca_update(mc_ctx *ctx, int32_t L, const double *lnW, const int64_t *H, double *lnW_out, double *flat_out)
{
    if (!ctx) return MC_E_INVAL;
    if (!muca_L_supported(L))
        return fail(ctx, MC_E_SHAPE, "L=%d: multicanonical walkers take L in {4,8,12,16,24,32,48,64,96,128}", L);
    if (!lnW || !H || !lnW_out) return fail(ctx, MC_E_INVAL, "a pointer argument is NULL");
    const int K = L * L / 2;
    for (int k = 0; k <= K; ++k) {
        if (!std::isfinite(lnW[k])) return fail(ctx, MC_E_RANGE, "lnW[%d] is not finite", k);
        if (H[k] < 0) return fail(ctx, MC_E_RANGE, "H[%d] is negative", k);
    }
    std::vector<double> w(lnW, lnW + K + 1);  // lnW_out may be lnW
    std::vector<int64_t> h(H, H + K + 1);
    recursion_step(K, w.data(), h.data());
    std::copy(w.begin(), w.end(), lnW_out);
    if (flat_out) *flat_out = flatness(L, h);
    return MC_OK;
}

}  // extern "C"
