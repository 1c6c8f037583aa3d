// k_wl.hip -- Wang-Landau sampling of 2D L x L ferromagnets in energy windows
// (Sec. "Wang-Landau update": g(E) multiplied by f at every visit, moves
// accepted with min[1, g(E)/g(E')]; windows sampled by separate walkers, a
// move out of the window rejected and the current level counted again, the
// walkers' estimates averaged before f is reduced).
//
// One lane is one walker and a workgroup is 64 walkers of one window, visiting
// the sites in the multicanonical walkers' sequential order with their random
// numbers.  Every walker keeps its own estimate G[k] of ln g (integers in units
// of 2^-32, so ln f = 2^-s adds exactly) and its own visit counts over the
// window's levels, both in LDS as [level][lane] for the whole call.  The
// acceptance probability exp(-(G[k'] - G[k]) 2^-32) is a fixed-order product of
// five tabulated factors (exp(-n) and one per byte of the fraction), so the
// device evaluates no transcendental; the integer test r32 < ceil(p 2^32)
// follows.  At the end of a call each walker shifts its estimate to a minimum
// of 0 over the levels with states and reports whether its histogram is flat.
#include <algorithm>

#include "internal.hpp"
#include "muca.hpp"
#include "muca_rows.hpp"
#include "wl.hpp"

namespace mcs {

// ceil(exp(-x 2^-32) 2^32), at least 1, for x > 0
__device__ __forceinline__ uint64_t wl_threshold(uint64_t x, const double *xt)
{
    const uint64_t n = x >> 32;
    if (n >= (uint64_t)kWlExpN) return 1;
    const uint32_t f = (uint32_t)x;
    double p = xt[n];
    p = p * xt[kWlExpN + (f >> 24)];
    p = p * xt[kWlExpN + 256 + ((f >> 16) & 255u)];
    p = p * xt[kWlExpN + 512 + ((f >> 8) & 255u)];
    p = p * xt[kWlExpN + 768 + (f & 255u)];
    const uint64_t T = (uint64_t)__builtin_ceil(p * 4294967296.0);
    return T < 1 ? 1 : T;
}

template <int L>
__global__ __launch_bounds__(64) void k_wl(WlArgs a)
{
    constexpr int N = L * L, NW = (L + 31) / 32;
    extern __shared__ __align__(16) unsigned char wl_lds[];
    double *xt = (double *)wl_lds;
    int64_t *Gl = (int64_t *)(xt + kWlTab);                   // [n][64]
    uint32_t *Hl = (uint32_t *)(Gl + (size_t)a.wmax * 64);    // [n][64]
    const int lane = threadIdx.x;
    const int w0 = blockIdx.x * 64, win = w0 / a.M;
    if (!a.active[win]) return;
    const int lo = a.lo[win], hi = a.hi[win], n = hi - lo + 1;
    const int w = w0 + lane;
    for (int i = lane; i < kWlTab; i += 64) xt[i] = a.xtab[i];
    int64_t *Gg = a.G + (int64_t)w * a.wmax;
    uint32_t *Hg = a.H + (int64_t)w * a.wmax;
    for (int j = 0; j < n; ++j) {
        Gl[j * 64 + lane] = Gg[j];
        Hl[j * 64 + lane] = Hg[j];
    }
    __syncthreads();
    const int64_t inc = a.inc[win];
    int8_t *sp = a.spins + (int64_t)w * N;
    int k = (int)((a.E[w] + 2 * N) / 4);
    for (int t = 0; t < a.nsweeps; ++t) {
        const uint64_t sweep = a.sweep0 + (uint64_t)t;
        const uint32_t w3 = ctr_w3(kTagMuca, 0, sweep);
        uint32_t up[NW], cur[NW], dn[NW], row0[NW];
        load_row<L>(sp, L - 1, up);
        load_row<L>(sp, 0, cur);
        load_row<L>(sp, 1 % L, dn);
        for (int y = 0; y < L; ++y) {
            uint4 blk = make_uint4(0, 0, 0, 0);
#pragma unroll
            for (int x = 0; x < L; ++x) {
                if (x % 4 == 0)
                    blk = philox(make_uint4((uint32_t)(x + L * y) >> 2, (uint32_t)w, (uint32_t)sweep, w3), a.seed_lo,
                                 a.seed_hi);
                const uint32_t r = (x % 4 == 0) ? blk.x : (x % 4 == 1) ? blk.y : (x % 4 == 2) ? blk.z : blk.w;
                const uint32_t s = bit_at<L>(cur, x);
                const uint32_t nl = bit_at<L>(cur, (x + L - 1) % L), nr = bit_at<L>(cur, (x + 1) % L);
                const uint32_t nu = bit_at<L>(up, x), nd = bit_at<L>(dn, x);
                const int anti = (int)((s ^ nl) + (s ^ nr) + (s ^ nu) + (s ^ nd));
                const int dl = 2 - anti;  // level change if the spin flips
                const int k2 = k + dl;
                bool acc;
                if (dl == 0) acc = true;
                else if (k2 < lo || k2 > hi) acc = false;  // out of the window: counted again
                else {
                    const int64_t d = Gl[(k2 - lo) * 64 + lane] - Gl[(k - lo) * 64 + lane];
                    acc = d <= 0 || (uint64_t)r < wl_threshold((uint64_t)d, xt);
                }
                if (acc) {
                    cur[x / 32] ^= 1u << (x % 32);
                    k = k2;
                }
                Gl[(k - lo) * 64 + lane] += inc;
                Hl[(k - lo) * 64 + lane] += 1u;
            }
            store_row<L>(sp, y, cur);
            if (y == 0) {
#pragma unroll
                for (int i = 0; i < NW; ++i) row0[i] = cur[i];
            }
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                up[i] = cur[i];
                cur[i] = dn[i];
            }
            if (y + 2 < L) load_row<L>(sp, y + 2, dn);
            else {
#pragma unroll
                for (int i = 0; i < NW; ++i) dn[i] = row0[i];
            }
        }
    }
    a.E[w] = 4 * (int64_t)k - 2 * N;
    // the estimate's minimum over the levels with states (all but level 1)
    // to 0; flatness: min H >= flat * mean H over those levels
    int64_t mn = INT64_MAX;
    uint32_t hmin = 0xFFFFFFFFu;
    uint64_t hsum = 0;
    int cnt = 0;
    for (int j = 0; j < n; ++j) {
        if (lo + j == 1) continue;
        mn = min(mn, Gl[j * 64 + lane]);
        const uint32_t h = Hl[j * 64 + lane];
        hmin = min(hmin, h);
        hsum += h;
        ++cnt;
    }
    for (int j = 0; j < n; ++j) {
        Gg[j] = Gl[j * 64 + lane] - mn;
        Hg[j] = Hl[j * 64 + lane];
    }
    a.flat[w] = (double)hmin * (double)cnt >= a.flat_ratio * (double)hsum ? 1 : 0;
}

// Walkers into their windows: from the ground state, typewriter passes taking
// a flip iff the walker is below its window, the flip raises its level and
// the top bit of word (i mod 4) of Philox(WINDOW, i div 4, w, pass) is set,
// until the level reaches lo.  One thread per walker.
__global__ void k_win_drive(int8_t *spins, int64_t *E, int32_t *ok, const int32_t *lo, int L, int W, int M,
                            int max_pass, uint32_t k0, uint32_t k1)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W) return;
    const int N = L * L;
    int8_t *s = spins + (int64_t)w * N;
    const int klo = lo[w / M];
    int k = 0;
    for (int i = 0; i < N; ++i) s[i] = 1;
    for (int pass = 0; pass < max_pass && k < klo; ++pass)
        for (int y = 0; y < L && k < klo; ++y)
            for (int x = 0; x < L && k < klo; ++x) {
                const int i = x + L * y;
                const int h = s[(x + 1) % L + L * y] + s[(x + L - 1) % L + L * y] + s[x + L * ((y + 1) % L)] +
                              s[x + L * ((y + L - 1) % L)];
                const int dl = s[i] * h / 2;
                if (dl <= 0) continue;
                const uint4 b = philox(make_uint4((uint32_t)i >> 2, (uint32_t)w, (uint32_t)pass,
                                                  ctr_w3(kTagWindow, 0, (uint64_t)pass)), k0, k1);
                const uint32_t r = (i & 3) == 0 ? b.x : (i & 3) == 1 ? b.y : (i & 3) == 2 ? b.z : b.w;
                if (r >> 31) {
                    s[i] = (int8_t)-s[i];
                    k += dl;
                }
            }
    E[w] = 4 * (int64_t)k - 2 * N;
    ok[w] = k >= klo ? 1 : 0;
}

// Average of a window's walker estimates: floor of the integer mean per level,
// shifted to a minimum of 0 over the levels with states, given to every walker
// of the window, whose visit counts are cleared.  One workgroup per window
// with mask[window] set.
__global__ __launch_bounds__(256) void k_wl_average(int64_t *G, uint32_t *H, const int32_t *lo, const int32_t *hi,
                                                    const uint8_t *mask, int M, int wmax)
{
    const int win = blockIdx.x;
    if (!mask[win]) return;
    __shared__ int64_t avg[kWlMaxWidth];
    __shared__ int64_t shift;
    const int klo = lo[win], n = hi[win] - klo + 1;
    const int64_t w0 = (int64_t)win * M;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        int64_t sum = 0;
        for (int m = 0; m < M; ++m) sum += G[(w0 + m) * wmax + j];
        int64_t q = sum / M;
        if (sum % M != 0 && sum < 0) --q;  // floor
        avg[j] = q;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t mn = INT64_MAX;
        for (int j = 0; j < n; ++j)
            if (klo + j != 1) mn = min(mn, avg[j]);
        shift = mn;
    }
    __syncthreads();
    for (int64_t idx = threadIdx.x; idx < (int64_t)M * n; idx += blockDim.x) {
        const int64_t m = idx / n;
        const int j = (int)(idx - m * n);
        G[(w0 + m) * wmax + j] = avg[j] - shift;
        H[(w0 + m) * wmax + j] = 0u;
    }
}

template <int L>
static hipError_t launch_wl_L(const WlArgs &a, int W, hipStream_t s)
{
    const size_t lds = (size_t)kWlTab * 8 + (size_t)a.wmax * 64 * 12;
    static LdsLimit lim;
    const hipError_t e = lim.ensure((const void *)k_wl<L>, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_wl<L>, dim3(W / 64), dim3(64), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_wl_sweeps(const WlArgs &a, int L, int W, hipStream_t s)
{
    switch (L) {
    case 4: return launch_wl_L<4>(a, W, s);
    case 8: return launch_wl_L<8>(a, W, s);
    case 12: return launch_wl_L<12>(a, W, s);
    case 16: return launch_wl_L<16>(a, W, s);
    case 24: return launch_wl_L<24>(a, W, s);
    case 32: return launch_wl_L<32>(a, W, s);
    case 48: return launch_wl_L<48>(a, W, s);
    case 64: return launch_wl_L<64>(a, W, s);
    case 96: return launch_wl_L<96>(a, W, s);
    case 128: return launch_wl_L<128>(a, W, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_win_drive(int8_t *spins, int64_t *E, int32_t *ok, const int32_t *lo, int L, int W, int M,
                            int max_pass, uint64_t seed, hipStream_t s)
{
    hipLaunchKernelGGL(k_win_drive, dim3((W + 63) / 64), dim3(64), 0, s, spins, E, ok, lo, L, W, M, max_pass,
                       (uint32_t)seed, (uint32_t)(seed >> 32));
    return hipGetLastError();
}

hipError_t launch_wl_average(int64_t *G, uint32_t *H, const int32_t *lo, const int32_t *hi, const uint8_t *mask,
                             int nwin, int M, int wmax, hipStream_t s)
{
    hipLaunchKernelGGL(k_wl_average, dim3(nwin), dim3(256), 0, s, G, H, lo, hi, mask, M, wmax);
    return hipGetLastError();
}

}  // namespace mcs
