// wl_driver.hip -- host side of Wang-Landau sampling in energy windows (Sec.
// "Wang-Landau update"): argument checks, the exponential factors (FP64, libm
// exp), the stage loop (flatness of every walker of a window, averaging, ln f
// halved), and the matching of the windows' pieces on their overlaps; and the
// multicanonical recursion in the same windows (Sec. "Multicanonical
// simulations"), on the same sweeps with ln f = 0.
#include <algorithm>
#include <cmath>
#include <vector>

#include "internal.hpp"
#include "muca.hpp"
#include "wl.hpp"

using namespace mcs;

namespace {

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

struct WlLayout {
    size_t G = 0, H = 0, flat = 0, ok = 0, lo = 0, hi = 0, inc = 0, active = 0, mask = 0, xtab = 0, total = 0;
};

WlLayout wl_layout(int nwin, int M, int wmax)
{
    const size_t W = (size_t)nwin * M;
    WlLayout l;
    size_t off = 0;
    l.G = off, off += align256(W * wmax * 8);
    l.H = off, off += align256(W * wmax * 4);
    l.flat = off, off += align256(W * 4);
    l.ok = off, off += align256(W * 4);
    l.lo = off, off += align256((size_t)nwin * 4);
    l.hi = off, off += align256((size_t)nwin * 4);
    l.inc = off, off += align256((size_t)nwin * 8);
    l.active = off, off += align256((size_t)nwin);
    l.mask = off, off += align256((size_t)nwin);
    l.xtab = off, off += align256((size_t)kWlTab * 8);
    l.total = off;
    return l;
}

// exp(-n), n = 0..22, then exp(-a 2^-8), exp(-a 2^-16), exp(-a 2^-24),
// exp(-a 2^-32), a = 0..255 (libm exp, FP64)
void wl_exp_table(std::vector<double> &t)
{
    t.assign(kWlTab, 0.0);
    for (int n = 0; n < kWlExpN; ++n) t[(size_t)n] = std::exp(-(double)n);
    for (int a = 0; a < 256; ++a) {
        t[(size_t)kWlExpN + a] = std::exp(-(double)a / 256.0);
        t[(size_t)kWlExpN + 256 + a] = std::exp(-(double)a / 65536.0);
        t[(size_t)kWlExpN + 512 + a] = std::exp(-(double)a / 16777216.0);
        t[(size_t)kWlExpN + 768 + a] = std::exp(-(double)a / 4294967296.0);
    }
}

// Windows: 0 <= lo < hi <= N/2 (at least two levels), at most kWlMaxWidth
// levels; with `cover`, consecutive windows overlap on a level with states,
// start at 0 and end at N/2.
int check_windows(mc_ctx *ctx, int L, int nwin, const int32_t *lo, const int32_t *hi, bool cover, int *wmax)
{
    if (!muca_L_supported(L))
        return fail(ctx, MC_E_SHAPE, "L=%d: the walkers take L in {4,8,12,16,24,32,48,64,96,128}", L);
    if (nwin < 1 || nwin > 65535) return fail(ctx, MC_E_RANGE, "nwin must be 1..65535");
    if (!lo || !hi) return fail(ctx, MC_E_INVAL, "lo or hi is NULL");
    const int K = L * L / 2;
    int w = 0;
    for (int i = 0; i < nwin; ++i) {
        if (lo[i] < 0 || hi[i] > K || hi[i] - lo[i] < 1)
            return fail(ctx, MC_E_RANGE, "window %d: need 0 <= lo < hi <= %d (got %d, %d)", i, K, lo[i], hi[i]);
        if (hi[i] - lo[i] + 1 > kWlMaxWidth)
            return fail(ctx, MC_E_RANGE, "window %d spans %d levels (at most %d)", i, hi[i] - lo[i] + 1, kWlMaxWidth);
        w = std::max(w, hi[i] - lo[i] + 1);
        if (cover && i > 0) {
            const int a = lo[i], b = hi[i - 1];
            if (a <= lo[i - 1] || hi[i] <= b || a > b || (a == 1 && b == 1))
                return fail(ctx, MC_E_RANGE, "windows %d and %d must overlap on a level with states", i - 1, i);
        }
    }
    if (cover && (lo[0] != 0 || hi[nwin - 1] != K))
        return fail(ctx, MC_E_RANGE, "the windows must cover the levels 0..%d", K);
    *wmax = w;
    return MC_OK;
}

int check_walkers(mc_ctx *ctx, int nwin, int M)
{
    if (M < 64 || M % 64 || (int64_t)nwin * M > (1 << 24))
        return fail(ctx, MC_E_RANGE, "walkers per window must be a multiple of 64, nwin * walkers <= 2^24");
    return MC_OK;
}

int upload(mc_ctx *ctx, void *dst, const void *src, size_t bytes, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, s);
    // the source is host memory of the caller's frame
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return device_check(ctx, e, "host to device copy");
}

int download(mc_ctx *ctx, void *dst, const void *src, size_t bytes, hipStream_t s)
{
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return device_check(ctx, e, "device to host copy");
}

// one ln g over [0, K] from the windows' pieces: window i + 1 shifted by the
// mean of (previous, shifted) - (own) over the overlap levels with states;
// level k from window i up to the middle of each overlap; ln g(0) = ln 2,
// ln g(1) = -inf
void wl_match(int K, int nwin, const int32_t *lo, const int32_t *hi, const double *pieces, int wmax, double *out)
{
    std::vector<double> prev(pieces, pieces + (hi[0] - lo[0] + 1)), cur;
    for (int k = lo[0]; k <= hi[0]; ++k) out[k] = prev[(size_t)(k - lo[0])];
    for (int i = 1; i < nwin; ++i) {
        const double *p = pieces + (size_t)i * wmax;
        cur.assign(p, p + (hi[i] - lo[i] + 1));
        double sum = 0.0;
        int cnt = 0;
        for (int k = lo[i]; k <= hi[i - 1]; ++k) {
            if (k == 1) continue;
            sum = sum + (prev[(size_t)(k - lo[i - 1])] - cur[(size_t)(k - lo[i])]);
            ++cnt;
        }
        const double shift = sum / (double)cnt;
        for (double &v : cur) v = v + shift;
        const int mid = (lo[i] + hi[i - 1]) / 2;
        for (int k = mid + 1; k <= hi[i]; ++k) out[k] = cur[(size_t)(k - lo[i])];
        prev.swap(cur);
    }
    const double o0 = out[0], ln2 = std::log(2.0);
    for (int k = 0; k <= K; ++k) out[k] = (out[k] - o0) + ln2;
    if (K >= 1) out[1] = -INFINITY;
}

}  // namespace

extern "C" {

size_t mc_wl_workspace_bytes(const mc_wl_args *a)
{
    if (!a || !a->lo || !a->hi || a->nwin < 1 || a->walkers < 1) return 0;
    int w = 0;
    for (int i = 0; i < a->nwin; ++i) w = std::max(w, a->hi[i] - a->lo[i] + 1);
    if (w < 2 || w > kWlMaxWidth) return 0;
    return wl_layout(a->nwin, a->walkers, w).total;
}

int mc_win_drive(mc_ctx *ctx, int32_t L, int32_t nwin, const int32_t *lo, const int32_t *hi, int32_t walkers,
                 uint64_t seed, int32_t max_pass, int8_t *spins, int64_t *E, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    int wmax = 0;
    int rc = check_windows(ctx, L, nwin, lo, hi, false, &wmax);
    if (rc) return rc;
    if ((rc = check_walkers(ctx, nwin, walkers))) return rc;
    if (!spins || !E) return fail(ctx, MC_E_INVAL, "spins or E is NULL");
    if (max_pass < 1) return fail(ctx, MC_E_RANGE, "max_pass must be >= 1");
    const WlLayout lay = wl_layout(nwin, walkers, wmax);
    if (!ws || ws_bytes < lay.total) return fail(ctx, MC_E_WORKSPACE, "workspace needs %zu bytes", lay.total);
    if ((rc = set_device(ctx))) return rc;
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    const int W = nwin * walkers;
    if ((rc = upload(ctx, w + lay.lo, lo, (size_t)nwin * 4, s))) return rc;
    rc = device_check(ctx, launch_win_drive(spins, E, (int32_t *)(w + lay.ok), (const int32_t *)(w + lay.lo), L, W,
                                            walkers, max_pass, seed, s), "window drive");
    if (rc) return rc;
    std::vector<int32_t> ok((size_t)W);
    if ((rc = download(ctx, ok.data(), w + lay.ok, (size_t)W * 4, s))) return rc;
    for (int i = 0; i < W; ++i)
        if (!ok[(size_t)i]) return fail(ctx, MC_E_NOTCONV, "walker %d did not reach its window in %d passes", i, max_pass);
    return MC_OK;
}

int mc_wl_sweeps(mc_ctx *ctx, int32_t L, int32_t nwin, const int32_t *lo, const int32_t *hi, int32_t walkers,
                 const int64_t *inc, const uint8_t *active, double flat, uint64_t seed, uint64_t sweep0,
                 int32_t nsweeps, int8_t *spins, int64_t *E, int64_t *G, uint32_t *H, int32_t *flags, void *ws,
                 size_t ws_bytes, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    int wmax = 0;
    int rc = check_windows(ctx, L, nwin, lo, hi, false, &wmax);
    if (rc) return rc;
    if ((rc = check_walkers(ctx, nwin, walkers))) return rc;
    if (!inc || !active || !spins || !E || !G || !H || !flags) return fail(ctx, MC_E_INVAL, "a pointer is NULL");
    if (nsweeps < 0) return fail(ctx, MC_E_RANGE, "nsweeps must be >= 0");
    if (!(flat > 0.0) || flat > 1.0) return fail(ctx, MC_E_RANGE, "flat must be in (0, 1]");
    for (int i = 0; i < nwin; ++i)
        if (inc[i] < 0 || inc[i] > (1ll << 32)) return fail(ctx, MC_E_RANGE, "inc[%d] out of 0..2^32", i);
    const WlLayout lay = wl_layout(nwin, walkers, wmax);
    if (!ws || ws_bytes < lay.total) return fail(ctx, MC_E_WORKSPACE, "workspace needs %zu bytes", lay.total);
    if ((rc = set_device(ctx))) return rc;
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    std::vector<double> xt;
    wl_exp_table(xt);
    if ((rc = upload(ctx, w + lay.lo, lo, (size_t)nwin * 4, s))) return rc;
    if ((rc = upload(ctx, w + lay.hi, hi, (size_t)nwin * 4, s))) return rc;
    if ((rc = upload(ctx, w + lay.inc, inc, (size_t)nwin * 8, s))) return rc;
    if ((rc = upload(ctx, w + lay.active, active, (size_t)nwin, s))) return rc;
    if ((rc = upload(ctx, w + lay.xtab, xt.data(), xt.size() * 8, s))) return rc;
    if (nsweeps == 0) return MC_OK;
    WlArgs a;
    a.spins = spins;
    a.E = E;
    a.G = G;
    a.H = H;
    a.flat = flags;
    a.lo = (const int32_t *)(w + lay.lo);
    a.hi = (const int32_t *)(w + lay.hi);
    a.inc = (const int64_t *)(w + lay.inc);
    a.active = (const uint8_t *)(w + lay.active);
    a.xtab = (const double *)(w + lay.xtab);
    a.flat_ratio = flat;
    a.M = walkers;
    a.wmax = wmax;
    a.seed_lo = (uint32_t)seed;
    a.seed_hi = (uint32_t)(seed >> 32);
    a.sweep0 = sweep0;
    a.nsweeps = nsweeps;
    return device_check(ctx, launch_wl_sweeps(a, L, nwin * walkers, s), "Wang-Landau sweeps");
}

int mc_wl_run(mc_ctx *ctx, const mc_wl_args *a, int8_t *spins, int64_t *E, double *pieces, double *lng,
              mc_wl_window_stats *stats, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    if (!a) return fail(ctx, MC_E_INVAL, "args is NULL");
    int wmax = 0;
    int rc = check_windows(ctx, a->L, a->nwin, a->lo, a->hi, true, &wmax);
    if (rc) return rc;
    if ((rc = check_walkers(ctx, a->nwin, a->walkers))) return rc;
    if (!spins || !E || !pieces || !lng || !stats) return fail(ctx, MC_E_INVAL, "an output is NULL");
    if (a->check_sweeps < 1 || a->max_sweeps < 0 || a->max_pass < 1)
        return fail(ctx, MC_E_RANGE, "check_sweeps, max_sweeps or max_pass out of range");
    if (!(a->flat > 0.0) || a->flat > 1.0) return fail(ctx, MC_E_RANGE, "flat must be in (0, 1]");
    if (!(a->lnf_final >= std::ldexp(1.0, -32)) || a->lnf_final > 1.0)
        return fail(ctx, MC_E_RANGE, "lnf_final must be in [2^-32, 1]");
    const int L = a->L, nwin = a->nwin, M = a->walkers, W = nwin * M, K = L * L / 2;
    const WlLayout lay = wl_layout(nwin, M, wmax);
    if (!ws || ws_bytes < lay.total) return fail(ctx, MC_E_WORKSPACE, "workspace needs %zu bytes", lay.total);
    if ((rc = mc_win_drive(ctx, L, nwin, a->lo, a->hi, M, a->seed, a->max_pass, spins, E, ws, ws_bytes, stream)))
        return rc;
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    int64_t *G = (int64_t *)(w + lay.G);
    uint32_t *H = (uint32_t *)(w + lay.H);
    int32_t *flags = (int32_t *)(w + lay.flat);
    if ((rc = device_check(ctx, launch_fill_i64(G, (int64_t)W * wmax, 0, s), "estimate clear"))) return rc;
    // the counts are cleared as int64 words (two counts each, padding included)
    if ((rc = device_check(ctx, launch_fill_i64((int64_t *)H, ((int64_t)W * wmax + 1) / 2, 0, s), "count clear")))
        return rc;
    std::vector<int> stage((size_t)nwin, 0);
    std::vector<uint8_t> active((size_t)nwin, 1), mask((size_t)nwin, 0);
    std::vector<int64_t> inc((size_t)nwin), sweeps((size_t)nwin, 0), in_stage((size_t)nwin, 0);
    std::vector<int32_t> fl((size_t)W);
    int64_t sweep = 0;
    auto any_active = [&]() { return std::any_of(active.begin(), active.end(), [](uint8_t v) { return v != 0; }); };
    while (any_active() && sweep < a->max_sweeps) {
        for (int i = 0; i < nwin; ++i) {
            inc[(size_t)i] = (int64_t)((1ull << 32) >> stage[(size_t)i]);
            // a walker's visits of one level within a stage are 32-bit counts
            if (active[(size_t)i] && (in_stage[(size_t)i] + a->check_sweeps) * (int64_t)L * L > 0xFFFFFFFFll)
                return fail(ctx, MC_E_RANGE, "window %d: a stage of %lld sweeps would overflow the visit counts", i,
                            (long long)in_stage[(size_t)i]);
        }
        if ((rc = mc_wl_sweeps(ctx, L, nwin, a->lo, a->hi, M, inc.data(), active.data(), a->flat, a->seed,
                               (uint64_t)sweep, a->check_sweeps, spins, E, G, H, flags, ws, ws_bytes, stream)))
            return rc;
        sweep += a->check_sweeps;
        if ((rc = download(ctx, fl.data(), flags, (size_t)W * 4, s))) return rc;
        bool avg = false;
        for (int i = 0; i < nwin; ++i) {
            mask[(size_t)i] = 0;
            if (!active[(size_t)i]) continue;
            sweeps[(size_t)i] += a->check_sweeps;
            in_stage[(size_t)i] += a->check_sweeps;
            bool all = true;
            for (int m = 0; m < M && all; ++m) all = fl[(size_t)i * M + m] != 0;
            if (!all) continue;
            mask[(size_t)i] = 1;
            avg = true;
            in_stage[(size_t)i] = 0;
            ++stage[(size_t)i];
            if (std::ldexp(1.0, -stage[(size_t)i]) < a->lnf_final) active[(size_t)i] = 0;
        }
        if (avg) {
            if ((rc = upload(ctx, w + lay.mask, mask.data(), (size_t)nwin, s))) return rc;
            if ((rc = device_check(ctx, launch_wl_average(G, H, (const int32_t *)(w + lay.lo),
                                                          (const int32_t *)(w + lay.hi), (const uint8_t *)(w + lay.mask),
                                                          nwin, M, wmax, s), "estimate average")))
                return rc;
        }
        if (a->progress) {
            int done = 0;
            for (int i = 0; i < nwin; ++i) done += !active[(size_t)i];
            a->progress(a->progress_user, done, *std::min_element(stage.begin(), stage.end()), sweep);
        }
    }
    // windows still running: their current average
    bool left = false;
    for (int i = 0; i < nwin; ++i) {
        mask[(size_t)i] = active[(size_t)i];
        left = left || active[(size_t)i];
    }
    if (left) {
        if ((rc = upload(ctx, w + lay.mask, mask.data(), (size_t)nwin, s))) return rc;
        if ((rc = device_check(ctx, launch_wl_average(G, H, (const int32_t *)(w + lay.lo), (const int32_t *)(w + lay.hi),
                                                      (const uint8_t *)(w + lay.mask), nwin, M, wmax, s),
                               "estimate average")))
            return rc;
    }
    std::vector<int64_t> row((size_t)wmax);
    for (int i = 0; i < nwin; ++i) {
        if ((rc = download(ctx, row.data(), G + (size_t)i * M * wmax, (size_t)wmax * 8, s))) return rc;
        for (int j = 0; j < wmax; ++j)
            pieces[(size_t)i * wmax + j] = j <= a->hi[i] - a->lo[i] ? (double)row[(size_t)j] / 4294967296.0 : 0.0;
        stats[i].stages = stage[(size_t)i];
        stats[i].converged = active[(size_t)i] ? 0 : 1;
        stats[i].sweeps = sweeps[(size_t)i];
    }
    wl_match(K, nwin, a->lo, a->hi, pieces, wmax, lng);
    return left ? fail(ctx, MC_E_NOTCONV, "windows still above lnf_final after %lld sweeps", (long long)sweep) : MC_OK;
}

}  // extern "C"

extern "C" {

size_t mc_muca_windows_workspace_bytes(const mc_muca_win_args *a)
{
    if (!a) return 0;
    mc_wl_args w{};
    w.nwin = a->nwin;
    w.lo = a->lo;
    w.hi = a->hi;
    w.walkers = a->walkers;
    return mc_wl_workspace_bytes(&w);
}

int mc_muca_windows_run(mc_ctx *ctx, const mc_muca_win_args *a, int8_t *spins, int64_t *E, double *pieces,
                        double *lng, mc_muca_win_stats *stats, void *ws, size_t ws_bytes, void *stream)
{
    if (!ctx) return MC_E_INVAL;
    if (!a) return fail(ctx, MC_E_INVAL, "args is NULL");
    int wmax = 0;
    int rc = check_windows(ctx, a->L, a->nwin, a->lo, a->hi, true, &wmax);
    if (rc) return rc;
    if ((rc = check_walkers(ctx, a->nwin, a->walkers))) return rc;
    if (!spins || !E || !pieces || !lng || !stats) return fail(ctx, MC_E_INVAL, "an output is NULL");
    if (a->eq_sweeps < 0 || a->rec_sweeps < 1 || a->max_iter < 0 || a->max_pass < 1)
        return fail(ctx, MC_E_RANGE, "eq_sweeps, rec_sweeps, max_iter or max_pass out of range");
    if (!(a->flat > 0.0) || a->flat > 1.0) return fail(ctx, MC_E_RANGE, "flat must be in (0, 1]");
    const int L = a->L, nwin = a->nwin, M = a->walkers, W = nwin * M, K = L * L / 2;
    const WlLayout lay = wl_layout(nwin, M, wmax);
    if (!ws || ws_bytes < lay.total) return fail(ctx, MC_E_WORKSPACE, "workspace needs %zu bytes", lay.total);
    if ((rc = mc_win_drive(ctx, L, nwin, a->lo, a->hi, M, a->seed, a->max_pass, spins, E, ws, ws_bytes, stream)))
        return rc;
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)ws;
    int64_t *G = (int64_t *)(w + lay.G);
    uint32_t *H = (uint32_t *)(w + lay.H);
    int32_t *flags = (int32_t *)(w + lay.flat);
    const int64_t hwords = ((int64_t)W * wmax + 1) / 2;
    if ((rc = device_check(ctx, launch_fill_i64(G, (int64_t)W * wmax, 0, s), "weight clear"))) return rc;
    if ((rc = device_check(ctx, launch_fill_i64((int64_t *)H, hwords, 0, s), "count clear"))) return rc;
    std::vector<uint8_t> active((size_t)nwin, 1);
    std::vector<int64_t> zero((size_t)nwin, 0), Gh((size_t)W * wmax, 0), sumH((size_t)wmax);
    std::vector<uint32_t> Hh((size_t)W * wmax);
    std::vector<int> iters((size_t)nwin, 0);
    std::vector<char> done((size_t)nwin, 0);
    int64_t sweep = 0;
    // the piece of window i from its pooled counts and weights
    auto piece = [&](int i) {
        const int n = a->hi[i] - a->lo[i] + 1;
        for (int j = 0; j < wmax; ++j) {
            double v = 0.0;
            if (j < n && sumH[(size_t)j] > 0)
                v = std::log((double)sumH[(size_t)j]) + (double)Gh[(size_t)i * M * wmax + j] / 4294967296.0;
            pieces[(size_t)i * wmax + j] = v;
        }
    };
    auto pool = [&](int i) {
        const int n = a->hi[i] - a->lo[i] + 1;
        for (int j = 0; j < n; ++j) {
            int64_t t = 0;
            for (int m = 0; m < M; ++m) t += Hh[((size_t)i * M + m) * wmax + j];
            sumH[(size_t)j] = t;
        }
    };
    for (int it = 0; it < a->max_iter; ++it) {
        if (std::none_of(active.begin(), active.end(), [](uint8_t v) { return v != 0; })) break;
        if ((rc = mc_wl_sweeps(ctx, L, nwin, a->lo, a->hi, M, zero.data(), active.data(), a->flat, a->seed,
                               (uint64_t)sweep, a->eq_sweeps, spins, E, G, H, flags, ws, ws_bytes, stream)))
            return rc;
        sweep += a->eq_sweeps;
        if ((rc = device_check(ctx, launch_fill_i64((int64_t *)H, hwords, 0, s), "count clear"))) return rc;
        if ((rc = mc_wl_sweeps(ctx, L, nwin, a->lo, a->hi, M, zero.data(), active.data(), a->flat, a->seed,
                               (uint64_t)sweep, a->rec_sweeps, spins, E, G, H, flags, ws, ws_bytes, stream)))
            return rc;
        sweep += a->rec_sweeps;
        if ((rc = download(ctx, Hh.data(), H, Hh.size() * 4, s))) return rc;
        bool changed = false;
        for (int i = 0; i < nwin; ++i) {
            if (!active[(size_t)i]) continue;
            ++iters[(size_t)i];
            const int lo = a->lo[i], n = a->hi[i] - lo + 1;
            pool(i);
            int64_t mn = -1, mx = 0;
            for (int j = 0; j < n; ++j) {
                if (lo + j == 1) continue;
                mn = mn < 0 ? sumH[(size_t)j] : std::min(mn, sumH[(size_t)j]);
                mx = std::max(mx, sumH[(size_t)j]);
            }
            if ((double)mn >= a->flat * (double)mx) {
                piece(i);
                done[(size_t)i] = 1;
                active[(size_t)i] = 0;
                continue;
            }
            // ln W <- ln W - ln H where H > 0, i.e. G += round(ln H 2^32);
            // then the minimum over the levels with states to 0
            int64_t *g = Gh.data() + (size_t)i * M * wmax;
            for (int j = 0; j < n; ++j)
                if (sumH[(size_t)j] > 0)
                    g[j] += (int64_t)std::floor(std::log((double)sumH[(size_t)j]) * 4294967296.0 + 0.5);
            int64_t gmin = INT64_MAX;
            for (int j = 0; j < n; ++j)
                if (lo + j != 1) gmin = std::min(gmin, g[j]);
            for (int j = 0; j < n; ++j) g[j] -= gmin;
            for (int m = 1; m < M; ++m) std::copy(g, g + wmax, g + (size_t)m * wmax);
            changed = true;
        }
        if (changed && (rc = upload(ctx, G, Gh.data(), Gh.size() * 8, s))) return rc;
        if (a->progress) {
            int nd = 0;
            for (int i = 0; i < nwin; ++i) nd += done[(size_t)i];
            a->progress(a->progress_user, nd, it + 1, sweep);
        }
    }
    bool left = false;
    for (int i = 0; i < nwin; ++i) {
        if (!done[(size_t)i]) {
            // not flat: the last recursion's weights, -ln W = G 2^-32
            const int n = a->hi[i] - a->lo[i] + 1;
            for (int j = 0; j < wmax; ++j)
                pieces[(size_t)i * wmax + j] = j < n ? (double)Gh[(size_t)i * M * wmax + j] / 4294967296.0 : 0.0;
            left = true;
        }
        stats[i].iterations = iters[(size_t)i];
        stats[i].converged = done[(size_t)i] ? 1 : 0;
    }
    wl_match(K, nwin, a->lo, a->hi, pieces, wmax, lng);
    return left ? fail(ctx, MC_E_NOTCONV, "windows not flat after %d iterations", a->max_iter) : MC_OK;
}

}  // extern "C"
