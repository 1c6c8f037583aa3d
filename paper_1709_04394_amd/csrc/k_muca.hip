// k_muca.hip -- parallel-walker multicanonical sweeps (Sec. "Multicanonical
// simulations": p walkers share one weight function, their histograms are
// added; Eq. muca, Eq. weight_modification) for 2D L x L ferromagnets.
//
// One lane is one walker; 64 walkers form a wave and visit the same site at
// the same time (the paper's shared site sequence), each with its own random
// numbers.  A walker's rows are bit-packed in registers while it sweeps them
// in sequential (typewriter) order; the rows of the whole lattice stay int8 in
// global memory and stream through once per sweep.  The acceptance table
// T[level][direction] (FP64 host values as 32-bit thresholds) sits in LDS
// (131 KB at L = 128, within gfx950's 160 KB), so the dependent chain of one
// update is a few bit operations, one LDS read and a compare.  Moves that
// would leave the energy window [-2N, 0] are rejected and the current level
// is counted again.
#include <algorithm>

#include "internal.hpp"
#include "muca.hpp"
#include "muca_rows.hpp"

namespace mcs {

template <int L>
__global__ __launch_bounds__(64) void k_muca(MucaArgs a)
{
    constexpr int N = L * L, NW = (L + 31) / 32, K = N / 2;
    extern __shared__ uint32_t tab[];  // [(K + 1) * 4] thresholds minus one
    const int lane = threadIdx.x;
    for (int i = lane; i < (K + 1) * 4; i += 64) tab[i] = a.table[i];
    __syncthreads();
    const int w = blockIdx.x * 64 + lane;
    if (w >= a.W) return;
    int8_t *sp = a.spins + (int64_t)w * N;
    int k = (int)((a.E[w] + 2 * N) / 4);
    uint32_t *hist = a.hist + (int64_t)blockIdx.x * (K + 1);
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
                const int dl = 2 - anti;  // level change if the spin flips (dE = 4 dl)
                const int k2 = k + dl;
                bool acc;
                if (dl == 0) acc = true;
                else acc = k2 <= K && r <= tab[4 * k + (dl < 0 ? dl + 2 : dl + 1)];
                if (acc) {
                    cur[x / 32] ^= 1u << (x % 32);
                    k = k2;
                }
                if (a.record) atomicAdd(&hist[k], 1u);
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
}

// ---------------------------------------------------------------------------
// k_muca_w<L>: the same walk for L a multiple of 32, organised around the one
// serial dependence of an update (the acceptance of the site to its left and
// the walker's level), so that little else is on that chain:
//  * the row being swept is held as 32-bit words rotated so the active word is
//    always at index 0, and its 32 updates are unrolled with fixed bit
//    positions;
//  * per word, the unsatisfied-bond count against the up, down and right
//    neighbours (all in their old state, except the wrap-around of a one-word
//    row) is summed for all 32 bits at once in two bit planes; the left
//    neighbour, updated one step earlier, gives the count for either outcome
//    of that step (a0 if it was rejected, a1 if accepted);
//  * the threshold for either outcome (row of the level it leaves, entry of
//    its count) is read from LDS one update ahead, so the dependent chain of
//    an update is a few selects and compares; no branches;
//  * the histogram is counted in LDS, two 16-bit counts per word, and flushed
//    to the workgroup's slice before a count can reach 2^16;
//  * the row two ahead is loaded while the current row is swept.
// It draws the same random numbers, takes the same decisions and records the
// same levels as k_muca<L>.
template <int L>
__device__ __forceinline__ void load_row_raw(const int8_t *sp, int y, uint4 (&raw)[L / 16])
{
    const uint4 *p = (const uint4 *)(sp + y * L);
#pragma unroll
    for (int i = 0; i < L / 16; ++i) raw[i] = p[i];
}

template <int L>
__device__ __forceinline__ void pack_raw(const uint4 (&raw)[L / 16], uint32_t (&row)[L / 32])
{
#pragma unroll
    for (int i = 0; i < L / 32; ++i) {
        const uint4 a = raw[2 * i], b = raw[2 * i + 1];
        row[i] = pack4(a.x) | pack4(a.y) << 4 | pack4(a.z) << 8 | pack4(a.w) << 12 | pack4(b.x) << 16 |
                 pack4(b.y) << 20 | pack4(b.z) << 24 | pack4(b.w) << 28;
    }
}

template <int L>
__device__ __forceinline__ void store_row_w(int8_t *sp, int y, const uint32_t (&row)[L / 32])
{
    uint4 *p = (uint4 *)(sp + y * L);
#pragma unroll
    for (int i = 0; i < L / 32; ++i) {
        const uint32_t v = row[i];
        p[2 * i] = make_uint4(unpack4(v & 0xFu), unpack4((v >> 4) & 0xFu), unpack4((v >> 8) & 0xFu),
                              unpack4((v >> 12) & 0xFu));
        p[2 * i + 1] = make_uint4(unpack4((v >> 16) & 0xFu), unpack4((v >> 20) & 0xFu), unpack4((v >> 24) & 0xFu),
                                  unpack4(v >> 28));
    }
}

// Adds the LDS counts (two 16-bit levels per word) to the workgroup's slice and
// clears them.  The workgroup is one wave; the barriers order the lanes' LDS
// accesses around the exchange.
__device__ __forceinline__ void flush_hist16(uint32_t *h16, uint32_t *gh, int nh, int K, int lane)
{
    __syncthreads();
    for (int i = lane; i < nh; i += 64) {
        const uint32_t v = h16[i];
        if (v) {
            h16[i] = 0u;
            if (v & 0xFFFFu) atomicAdd(&gh[2 * i], v & 0xFFFFu);
            if ((v >> 16) && 2 * i + 1 <= K) atomicAdd(&gh[2 * i + 1], v >> 16);
        }
    }
    __syncthreads();
}

// Table entry of an update with unsatisfied-bond count a (dl = 2 - a):
// entries 0..3 are dl = -2, -1, +1, +2, i.e. a = 4, 3, 1, 0 (a = 2 is always
// accepted; its entry is never used).
__device__ __forceinline__ int entry_of(int a)
{
    return 3 - a + ((a + 5) >> 3);
}

template <int L>
__global__ __launch_bounds__(64) void k_muca_w(MucaArgs a)
{
    static_assert(L % 32 == 0, "whole 32-bit words per row");
    constexpr int N = L * L, NW = L / 32, K = N / 2, NH = K / 2 + 1;
    // rows between flushes: 64 walkers x L updates per row, below 2^16 per level
    constexpr int FL = 65535 / (64 * L);
    static_assert(FL >= 1, "flush interval");
    extern __shared__ __align__(16) uint32_t lds[];
    const uint32_t *tab = lds;  // [K + 1][4] thresholds minus one for dl = -2, -1, +1, +2
    uint32_t *h16 = lds + 4 * (K + 1);
    const int lane = threadIdx.x;
    for (int i = lane; i < 4 * (K + 1); i += 64) lds[i] = a.table[i];
    for (int i = lane; i < NH; i += 64) h16[i] = 0u;
    __syncthreads();
    // lanes past the last walker follow walker W - 1 without storing anything,
    // so the wave stays whole for the histogram flushes
    const int wr = blockIdx.x * 64 + lane;
    const bool live = wr < a.W;
    const int w = live ? wr : a.W - 1;
    int8_t *sp = a.spins + (int64_t)w * N;
    uint32_t *gh = a.hist + (int64_t)blockIdx.x * (K + 1);
    const uint32_t rec = (a.record && live) ? 1u : 0u;
    // chain state: level before the previous update (kp), its dl and acceptance
    int kp = (int)((a.E[w] + 2 * N) / 4), dlp = 0;
    bool accp = false;
    for (int t = 0; t < a.nsweeps; ++t) {
        const uint64_t sweep = a.sweep0 + (uint64_t)t;
        const uint32_t w3 = ctr_w3(kTagMuca, 0, sweep);
        uint32_t U[NW], C[NW], D[NW], R0[NW];
        uint4 raw[L / 16];
        load_row_raw<L>(sp, L - 1, raw);
        pack_raw<L>(raw, U);
        load_row_raw<L>(sp, 0, raw);
        pack_raw<L>(raw, C);
        load_row_raw<L>(sp, 1, raw);
        pack_raw<L>(raw, D);
        int rows_since_flush = 0;
        for (int y = 0; y < L; ++y) {
            const bool pre = y + 2 < L;
            if (pre) load_row_raw<L>(sp, y + 2, raw);
            for (int wi = 0; wi < NW; ++wi) {
                const uint32_t c0 = C[0], u = U[0], d = D[0];
                const uint32_t lb = C[NW - 1] >> 31;  // site x - 1 of bit 0 (final value)
                const uint32_t rb = NW > 1 ? (C[NW > 1 ? 1 : 0] & 1u) : 0u;
                const uint32_t X = c0 ^ u, Y = c0 ^ d, Z = c0 ^ ((c0 >> 1) | (rb << 31));
                const uint32_t p0 = X ^ Y ^ Z, p1 = (X & Y) | (X & Z) | (Y & Z);
                const uint32_t lw = c0 ^ ((c0 << 1) | lb);
                const uint32_t ctr0 = (uint32_t)(L * y + 32 * wi) >> 2;
                uint32_t F = 0u;
                uint4 blk = make_uint4(0u, 0u, 0u, 0u);
                // counts of bit 0 (its left neighbour is final: one outcome)
                int a0 = (int)((p0 & 1u) + ((p1 & 1u) << 1) + (lw & 1u)), a1 = a0;
                // thresholds of bit 0 for both outcomes of the previous update
                uint32_t T0 = tab[4 * kp + entry_of(a0)];
                const int kq = kp + dlp;
                uint32_t T1 = tab[4 * (kq < K ? kq : K) + entry_of(a1)];
#pragma unroll
                for (int b = 0; b < 32; ++b) {
                    if ((b & 3) == 0)
                        blk = philox(make_uint4(ctr0 + (uint32_t)(b >> 2), (uint32_t)w, (uint32_t)sweep, w3), a.seed_lo,
                                     a.seed_hi);
                    const uint32_t r = (b & 3) == 0 ? blk.x : (b & 3) == 1 ? blk.y : (b & 3) == 2 ? blk.z : blk.w;
                    // both outcomes of the previous update, off the chain
                    const int kA = kp + dlp;
                    const bool ab0 = (a0 == 2) || (kp + 2 - a0 <= K && r <= T0);
                    const bool ab1 = (a1 == 2) || (kA + 2 - a1 <= K && r <= T1);
                    // on the chain: the previous update's acceptance selects
                    const int kb = accp ? kA : kp;
                    const bool ab = accp ? ab1 : ab0;
                    const int dlb = 2 - (accp ? a1 : a0);
                    const int kn = kb + dlb;
                    // counts of the next bit for both outcomes of this update, and
                    // their thresholds (read now, used next step)
                    if (b < 31) {
                        int Pn;
                        if (NW == 1 && b + 1 == 31) {
                            // one-word row: the right neighbour of bit 31 is bit 0, already updated
                            Pn = (int)((X >> 31) + (Y >> 31) + ((c0 >> 31) ^ ((c0 ^ F) & 1u)));
                        } else {
                            Pn = (int)(((p0 >> (b + 1)) & 1u) + (((p1 >> (b + 1)) & 1u) << 1));
                        }
                        const int ln = (int)((lw >> (b + 1)) & 1u);
                        a0 = Pn + ln;
                        a1 = Pn + 1 - ln;
                        T0 = tab[4 * kb + entry_of(a0)];
                        T1 = tab[4 * (kn < K ? kn : K) + entry_of(a1)];
                    }
                    const int ka = ab ? kn : kb;
                    atomicAdd(&h16[ka >> 1], rec << ((ka & 1) << 4));
                    F |= ab ? (1u << b) : 0u;
                    kp = kb;
                    dlp = dlb;
                    accp = ab;
                }
                // rotate: the processed word goes last, the next word to index 0
                const uint32_t cn = c0 ^ F;
#pragma unroll
                for (int i = 0; i + 1 < NW; ++i) {
                    C[i] = C[i + 1];
                    U[i] = U[i + 1];
                    D[i] = D[i + 1];
                }
                C[NW - 1] = cn;
                U[NW - 1] = u;
                D[NW - 1] = d;
            }
            if (live) store_row_w<L>(sp, y, C);
            if (y == 0) {
#pragma unroll
                for (int i = 0; i < NW; ++i) R0[i] = C[i];
            }
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                U[i] = C[i];
                C[i] = D[i];
            }
            if (pre) pack_raw<L>(raw, D);
            else {
#pragma unroll
                for (int i = 0; i < NW; ++i) D[i] = R0[i];
            }
            if (a.record && (++rows_since_flush == FL || y == L - 1)) {
                flush_hist16(h16, gh, NH, K, lane);
                rows_since_flush = 0;
            }
        }
    }
    const int kf = kp + (accp ? dlp : 0);
    if (live) a.E[w] = 4 * (int64_t)kf - 2 * N;
}

// Walker start: hot start keyed by the walker index (already written by the
// init kernel), energy, and a flip of the odd sub-lattice when E > 0 (E -> -E).
__global__ void k_muca_start(int8_t *spins, int64_t *E, int L, int W)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W) return;
    const int N = L * L;
    int8_t *s = spins + (int64_t)w * N;
    int64_t e = 0;
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            const int si = s[x + L * y];
            e -= si * (s[(x + 1) % L + L * y] + s[x + L * ((y + 1) % L)]);
        }
    if (e > 0) {
        for (int y = 0; y < L; ++y)
            for (int x = 0; x < L; ++x)
                if ((x + y) & 1) s[x + L * y] = (int8_t)-s[x + L * y];
        e = -e;
    }
    E[w] = e;
}

// H[k] += sum over workgroup slices of their counts (fixed order).
__global__ void k_muca_merge(const uint32_t *slices, int nslices, int nlev, int64_t *H)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nlev) return;
    int64_t s = 0;
    for (int b = 0; b < nslices; ++b) s += slices[(int64_t)b * nlev + k];
    H[k] += s;
}

__global__ void k_fill_u32(uint32_t *p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

template <int L>
static hipError_t launch_muca_L(const MucaArgs &a, hipStream_t s)
{
    constexpr int K = L * L / 2;
    if constexpr (L % 32 == 0) {
        const size_t lds = (size_t)(K + 1) * 16 + (size_t)(K / 2 + 1) * 4;
        static LdsLimit lim;
        const hipError_t e = lim.ensure((const void *)k_muca_w<L>, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_muca_w<L>, dim3((a.W + 63) / 64), dim3(64), lds, s, a);
    } else {
        const size_t lds = (size_t)(K + 1) * 4 * 4;
        static LdsLimit lim;
        const hipError_t e = lim.ensure((const void *)k_muca<L>, (int)lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_muca<L>, dim3((a.W + 63) / 64), dim3(64), lds, s, a);
    }
    return hipGetLastError();
}

bool muca_L_supported(int L)
{
    switch (L) {
    case 4: case 8: case 12: case 16: case 24: case 32: case 48: case 64: case 96: case 128: return true;
    default: return false;
    }
}

hipError_t launch_muca_sweeps(const MucaArgs &a, int L, hipStream_t s)
{
    const int nlev = L * L / 2 + 1, nb = (a.W + 63) / 64;
    if (a.record) hipLaunchKernelGGL(k_fill_u32, dim3(256), dim3(256), 0, s, a.hist, (int64_t)nb * nlev);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (L) {
    case 4: e = launch_muca_L<4>(a, s); break;
    case 8: e = launch_muca_L<8>(a, s); break;
    case 12: e = launch_muca_L<12>(a, s); break;
    case 16: e = launch_muca_L<16>(a, s); break;
    case 24: e = launch_muca_L<24>(a, s); break;
    case 32: e = launch_muca_L<32>(a, s); break;
    case 48: e = launch_muca_L<48>(a, s); break;
    case 64: e = launch_muca_L<64>(a, s); break;
    case 96: e = launch_muca_L<96>(a, s); break;
    case 128: e = launch_muca_L<128>(a, s); break;
    default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    if (a.record) hipLaunchKernelGGL(k_muca_merge, dim3((nlev + 255) / 256), dim3(256), 0, s, a.hist, nb, nlev, a.H);
    return hipGetLastError();
}

// Level of disorder of walker w of W in the stratified start: the largest c
// in 0..128 with (257 - 2c)^2 * 2W > 65536 (2W - 2w - 1), i.e. 128 (1 -
// sqrt(1 - (w + 1/2)/W)) rounded, found by bisection in integer arithmetic
// (the condition is monotone in c).
__device__ __forceinline__ uint32_t strat_level(int64_t w, int64_t W)
{
    int lo = 0, hi = 128;
    const int64_t b = 65536ll * (2 * W - 2 * w - 1);
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        const int64_t a = (int64_t)(257 - 2 * mid) * (257 - 2 * mid) * 2 * W;
        if (a > b) lo = mid;
        else hi = mid - 1;
    }
    return (uint32_t)lo;
}

// Walker lattices: site i of walker w is -1 iff byte (i mod 16) of
// Philox(i/16, w, 0, TAG_INIT) >= 256 - c_w, c_w = 128 (hot start) or the
// stratified level.  Threads: x = group of 16 sites, y strides over walkers.
__global__ void k_muca_init(int8_t *spins, int L, int W, int stratified, uint32_t k0, uint32_t k1)
{
    const int N = L * L, groups = (N + 15) / 16;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= groups) return;
    for (int w = blockIdx.y; w < W; w += gridDim.y) {
        const uint32_t c = stratified ? strat_level(w, W) : 128u;
        const uint4 b = philox(make_uint4((uint32_t)g, (uint32_t)w, 0u, ctr_w3(kTagInit, 0, 0)), k0, k1);
        int8_t *s = spins + (int64_t)w * N;
        for (int k = 0; k < 16 && 16 * g + k < N; ++k) s[16 * g + k] = byte_of(b, (uint32_t)k) >= 256u - c ? -1 : 1;
    }
}

hipError_t launch_muca_settle(int8_t *spins, int64_t *E, int L, int W, hipStream_t s)
{
    hipLaunchKernelGGL(k_muca_start, dim3((W + 63) / 64), dim3(64), 0, s, spins, E, L, W);
    return hipGetLastError();
}

hipError_t launch_muca_start(int8_t *spins, int64_t *E, int L, int W, uint64_t seed, int start, hipStream_t s)
{
    const int groups = (L * L + 15) / 16;
    dim3 grid((unsigned)((groups + 255) / 256), (unsigned)std::min(W, 65535));
    hipLaunchKernelGGL(k_muca_init, grid, dim3(256), 0, s, spins, L, W, start, (uint32_t)seed, (uint32_t)(seed >> 32));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_muca_start, dim3((W + 63) / 64), dim3(64), 0, s, spins, E, L, W);
    return hipGetLastError();
}

}  // namespace mcs
