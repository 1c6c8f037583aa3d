// k_sg_msc.hip -- checkerboard half-sweep of +-J spin glasses multi-spin
// coded across 64 disorder realisations (Sec. "Disordered systems": the bits
// of a word are 64 realisations, each with its own couplings, and the coded
// copies share one random number per site, the choice the section reports
// for spin-glass codes).
//
// One lane per site, 64 realisations per word: the neighbour words and the
// per-realisation coupling words give every realisation's class (unsatisfied
// bonds for Metropolis, neighbours with J s_j = -1 for heat-bath) as a
// bit-sliced count.  The site's single 32-bit draw (the byte-lazy stream of
// the word lattice's replica id) is compared once with each class threshold,
// and the per-class outcomes are spread over the realisations of that class
// with one-hot class words.  A tie (top byte equal to a threshold's that a
// present class needs) draws the low 24 bits once for all realisations.
// Per-sweep E and M per realisation come from the odd half-sweep through the
// 64 x 64 bit transpose across the wave, as in the 64-replica kernel.
#include "internal.hpp"

namespace mcs {

struct SgMscArgs {
    uint64_t *w;          // [count][N] spin words, bit b = realisation 64 l + b (set <=> s = -1)
    const uint64_t *J;    // [count][dims][N] coupling words of bond (i, i + e_d) (set <=> J < 0)
    int Lx, Ly, Lz;
    int64_t N;
    uint32_t seed_lo, seed_hi, replica0;
    uint32_t sweep_lo, w3, w3lo;
    int c;                // colour of this half-sweep
    // class thresholds (top byte, low 24 bits; T = 2^32 encoded as top 256):
    // Metropolis class a = unsatisfied bonds < z/2, T of dE = 2z - 4a;
    // heat-bath class d = neighbours with J s_j = -1, T of h = z - 2d
    uint32_t top[8], low[8];
    int64_t *EM;          // this sweep's [count * 64][2], or nullptr
};

template <int D>
__device__ __forceinline__ uint32_t sg_xor_lane(uint32_t x)
{
    if constexpr (D == 32)
        return (uint32_t)__shfl_xor((int)x, 32, 64);
    else
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, (D << 10) | 0x1F);
}

template <int D>
__device__ __forceinline__ uint64_t sg_transpose_stage(uint64_t v, int lane)
{
    constexpr uint64_t M = D == 32 ? 0x00000000FFFFFFFFull
                         : D == 16 ? 0x0000FFFF0000FFFFull
                         : D == 8  ? 0x00FF00FF00FF00FFull
                         : D == 4  ? 0x0F0F0F0F0F0F0F0Full
                         : D == 2  ? 0x3333333333333333ull
                                   : 0x5555555555555555ull;
    const uint32_t lo = sg_xor_lane<D>((uint32_t)v), hi = sg_xor_lane<D>((uint32_t)(v >> 32));
    const uint64_t p = ((uint64_t)hi << 32) | lo;
    const uint64_t sel = (lane & D) ? ~0ull : 0ull;
    const uint64_t keep = M ^ sel;
    const uint64_t up = p << D, down = p >> D;
    const uint64_t t = up ^ ((up ^ down) & sel);
    return (v & keep) | (t & ~keep);
}

// 64 x 64 bit transpose across the wave (lane s ends with bit b = bit s of
// lane b's word)
__device__ __forceinline__ uint64_t sg_transpose64(uint64_t v, int lane)
{
    v = sg_transpose_stage<32>(v, lane);
    v = sg_transpose_stage<16>(v, lane);
    v = sg_transpose_stage<8>(v, lane);
    v = sg_transpose_stage<4>(v, lane);
    v = sg_transpose_stage<2>(v, lane);
    return sg_transpose_stage<1>(v, lane);
}

// bit-sliced count (c0, c1, c2) of set bits among n words (n = 4 or 6)
template <int Z>
__device__ __forceinline__ void count_bits(const uint64_t (&x)[6], uint64_t &c0, uint64_t &c1, uint64_t &c2)
{
    const uint64_t s1 = x[0] ^ x[1] ^ x[2];
    const uint64_t k1 = (x[0] & x[1]) | (x[0] & x[2]) | (x[1] & x[2]);
    if constexpr (Z == 6) {
        const uint64_t s2 = x[3] ^ x[4] ^ x[5];
        const uint64_t k2 = (x[3] & x[4]) | (x[3] & x[5]) | (x[4] & x[5]);
        c0 = s1 ^ s2;
        const uint64_t kk = s1 & s2;
        c1 = k1 ^ k2 ^ kk;
        c2 = (k1 & k2) | (k1 & kk) | (k2 & kk);
    } else {
        c0 = s1 ^ x[3];
        const uint64_t kk = s1 & x[3];
        c1 = k1 ^ kk;
        c2 = k1 & kk;
    }
}

template <int DIMS, bool MEASURE, bool HB>
__global__ __launch_bounds__(256) void k_sg_msc(SgMscArgs a)
{
    __shared__ long long red[2][64];
    constexpr int Z = 2 * DIMS;
    constexpr int NC = HB ? 7 : DIMS;  // heat-bath d = 0..6; Metropolis a = 0 .. z/2 - 1
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l = blockIdx.y;
    if (MEASURE && tid < 128) red[tid >> 6][tid & 63] = 0;
    __syncthreads();
    uint64_t *w = a.w + (int64_t)l * a.N;
    const uint64_t *Jl = a.J + (int64_t)l * DIMS * a.N;
    const int hx = a.Lx >> 1;
    const int64_t tasks = (a.N >> 1) >> 6;
    const uint32_t rep = a.replica0 + (uint32_t)l;  // the shared stream of the 64 realisations
    long long e_acc = 0, m_acc = 0;
    for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < tasks; t += (int64_t)gridDim.x * 4) {
        // lane: same-colour site j = 64 t + lane
        const int64_t j = (t << 6) + lane;
        const int64_t row = j / hx;
        const int m = (int)(j - row * hx);
        const int y = (int)(row % a.Ly), z = (int)(row / a.Ly);
        const int par = (a.c + y + z) & 1;
        const int x = 2 * m + par;
        const int64_t rbase = row * a.Lx;
        const int64_t i = rbase + x;
        const int xp = x + 1 == a.Lx ? 0 : x + 1, xm = x == 0 ? a.Lx - 1 : x - 1;
        const int64_t plane = (int64_t)a.Ly * a.Lx;
        const int64_t ryp = (int64_t)(y + 1 == a.Ly ? 0 : y + 1) * a.Lx + (int64_t)z * plane;
        const int64_t rym = (int64_t)(y == 0 ? a.Ly - 1 : y - 1) * a.Lx + (int64_t)z * plane;
        const uint64_t S = w[i];
        uint64_t n[6] = {0, 0, 0, 0, 0, 0}, jw[6] = {0, 0, 0, 0, 0, 0};
        n[0] = w[rbase + xp], jw[0] = Jl[i];
        n[1] = w[rbase + xm], jw[1] = Jl[rbase + xm];
        n[2] = w[ryp + x], jw[2] = Jl[a.N + i];
        n[3] = w[rym + x], jw[3] = Jl[a.N + rym + x];
        if (DIMS == 3) {
            const int64_t rzp = (z + 1 == a.Lz ? 0 : z + 1) * plane + (int64_t)y * a.Lx;
            const int64_t rzm = (z == 0 ? a.Lz - 1 : z - 1) * plane + (int64_t)y * a.Lx;
            n[4] = w[rzp + x], jw[4] = Jl[2 * a.N + i];
            n[5] = w[rzm + x], jw[5] = Jl[2 * a.N + rzm + x];
        }
        // wk: bit set <=> J s_j = -1 for that realisation; Metropolis counts
        // unsatisfied bonds wk ^ S, heat-bath counts wk
        uint64_t wk[6], xk[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            wk[k] = n[k] ^ jw[k];
            xk[k] = HB ? wk[k] : (wk[k] ^ S);
        }
        uint64_t c0, c1, c2;
        count_bits<Z>(xk, c0, c1, c2);
        const uint64_t ge = HB ? 0ull : (DIMS == 3 ? (c2 | (c1 & c0)) : (c2 | c1));
        uint64_t onehot[7];
        {
            const uint64_t n0 = ~c0, n1 = ~c1, n2 = ~c2;
            onehot[0] = n2 & n1 & n0;
            onehot[1] = n2 & n1 & c0;
            onehot[2] = n2 & c1 & n0;
            onehot[3] = n2 & c1 & c0;
            onehot[4] = c2 & n1 & n0;
            onehot[5] = c2 & n1 & c0;
            onehot[6] = c2 & c1 & n0;
        }
        // the site's one draw: top byte from block j / 16 (bit k = bit j mod 16
        // of half-word k), compared once with each class threshold
        const uint4 B = philox(make_uint4((uint32_t)(j >> 4), rep, a.sweep_lo, a.w3), a.seed_lo, a.seed_hi);
        const uint32_t top = byte_of(B, (uint32_t)(j & 15));
        uint64_t acc = ge, pend = 0ull;
#pragma unroll
        for (int d = 0; d < NC; ++d) {
            const uint32_t td = a.top[d];
            if (top < td) acc |= onehot[d];
            else if (top == td) pend |= onehot[d];
        }
        if (!HB) pend &= ~ge;
        if (pend) {
            const uint4 lo = philox(make_uint4((uint32_t)j, rep, a.sweep_lo, a.w3lo), a.seed_lo, a.seed_hi);
            const uint32_t low = lo.x & 0xFFFFFFu;
#pragma unroll
            for (int d = 0; d < NC; ++d)
                if (top == a.top[d] && low < a.low[d]) acc |= onehot[d] & pend;
        }
        // Metropolis: flip the accepted realisations; heat-bath: s' = +1
        // (bit clear) where r < T
        const uint64_t Sn = HB ? ~acc : (S ^ acc);
        w[i] = Sn;
        if (MEASURE) {
            // odd sites: the realisations' bond counts after the update; both
            // sites of the pair (this odd site and its even partner of the
            // same row position) for M
            uint64_t u[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) u[k] = Sn ^ wk[k];
            uint64_t u0, u1, u2;
            count_bits<Z>(u, u0, u1, u2);
            const uint64_t pw = par == 1 ? n[1] : n[0];
            const uint64_t d0 = Sn ^ pw, d1 = Sn & pw;
            const uint64_t U0 = sg_transpose64(u0, lane), U1 = sg_transpose64(u1, lane),
                           U2 = sg_transpose64(u2, lane);
            const uint64_t D0 = sg_transpose64(d0, lane), D1 = sg_transpose64(d1, lane);
            const int ub = __popcll(U0) + 2 * __popcll(U1) + 4 * __popcll(U2);
            const int db = __popcll(D0) + 2 * __popcll(D1);
            e_acc += 2 * ub - 64 * Z;
            m_acc += 128 - 2 * db;
        }
    }
    if (MEASURE) {
        atomicAdd((unsigned long long *)&red[0][lane], (unsigned long long)e_acc);
        atomicAdd((unsigned long long *)&red[1][lane], (unsigned long long)m_acc);
        __syncthreads();
        if (tid < 128) {
            const int q = tid >> 6, b = tid & 63;
            atomicAdd((unsigned long long *)&a.EM[2 * (64 * (int64_t)l + b) + q], (unsigned long long)red[q][b]);
        }
    }
}

// Couplings of realisations realisation0 + 64 l + b, bit b of word (l, d, i):
// set iff byte (b' mod 16) of Philox(ctr = (b' / 16, realisation, 0,
// TAG_COUPLING << 24)) is >= 128, b' = d N + i (the int8 couplings' stream
// with counter word 1 = the realisation).  One thread per (bond group of 16,
// lattice), 64 realisations in a loop.
__global__ void k_couplings_msc64(uint64_t *J, int64_t bonds, uint32_t realisation0, uint32_t k0, uint32_t k1)
{
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int l = blockIdx.y;
    if (g * 16 >= bonds) return;
    uint64_t out[16] = {};
    for (int b = 0; b < 64; ++b) {
        const uint32_t rz = realisation0 + 64u * (uint32_t)l + (uint32_t)b;
        const uint4 blk = philox(make_uint4((uint32_t)g, rz, 0u, ctr_w3(kTagCoupling, 0, 0)), k0, k1);
#pragma unroll
        for (int k = 0; k < 16; ++k) out[k] |= (uint64_t)(top_bit_of(blk, (uint32_t)k)) << b;
    }
    uint64_t *Jl = J + (int64_t)l * bonds;
    for (int k = 0; k < 16 && g * 16 + k < bonds; ++k) Jl[g * 16 + k] = out[k];
}

hipError_t launch_couplings_msc64(const Geom &g, uint64_t *J, uint64_t seed, uint32_t realisation0, hipStream_t s)
{
    const int64_t bonds = (int64_t)g.dims * g.N;
    const int64_t groups = (bonds + 15) / 16;
    dim3 grid((unsigned)((groups + 255) / 256), (unsigned)g.count);
    hipLaunchKernelGGL(k_couplings_msc64, grid, dim3(256), 0, s, J, bonds, realisation0, (uint32_t)seed,
                       (uint32_t)(seed >> 32));
    return hipGetLastError();
}

bool sg_msc_supported(const Geom &g) { return (g.dims == 2 || g.dims == 3) && ((g.N >> 1) % 64) == 0; }

template <int D, bool HB>
static hipError_t launch_sg_t(const SgMscArgs &a, int count, hipStream_t s)
{
    const int64_t tasks = (a.N >> 1) >> 6;
    int64_t blocks = (tasks + 3) / 4;
    if (blocks > 1024) blocks = 1024;
    dim3 grid((unsigned)blocks, (unsigned)count);
    if (a.EM) hipLaunchKernelGGL((k_sg_msc<D, true, HB>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_sg_msc<D, false, HB>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sg_msc_phase(const Geom &g, int rule, const SweepTables &tab, uint64_t *words, const uint64_t *J,
                               uint32_t seed_lo, uint32_t seed_hi, uint32_t replica0, uint64_t sweep, int phase,
                               int64_t *EM, hipStream_t s)
{
    SgMscArgs a;
    a.w = words;
    a.J = J;
    a.Lx = g.Lx;
    a.Ly = g.Ly;
    a.Lz = g.dims == 3 ? g.Lz : 1;
    a.N = g.N;
    a.seed_lo = seed_lo;
    a.seed_hi = seed_hi;
    a.replica0 = replica0;
    a.sweep_lo = (uint32_t)sweep;
    a.w3 = ctr_w3(kTagSweep, (uint32_t)phase, sweep);
    a.w3lo = ctr_w3(kTagSweepLo, (uint32_t)phase, sweep);
    a.c = phase;
    const int z = 2 * g.dims;
    for (int cl = 0; cl < 8; ++cl) {
        Thr th{0u, 0u};
        if (rule == 0) {
            if (2 * cl < z) th = tab.met[z / 2 - cl];  // dE = 2z - 4a
        } else if (cl <= z) {
            th = tab.hb[z - 2 * cl + 6];               // h = z - 2d
        }
        a.top[cl] = th.top;
        a.low[cl] = th.low;
    }
    a.EM = phase == 1 ? EM : nullptr;
    if (g.dims == 2) return rule ? launch_sg_t<2, true>(a, g.count, s) : launch_sg_t<2, false>(a, g.count, s);
    return rule ? launch_sg_t<3, true>(a, g.count, s) : launch_sg_t<3, false>(a, g.count, s);
}

}  // namespace mcs
