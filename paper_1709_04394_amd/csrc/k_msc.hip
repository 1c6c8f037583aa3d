// k_msc.hip -- checkerboard half-sweep of 64-lane multi-spin-coded lattices
// (Sec. "Checkerboard scheme": multi-spin coding packs 64 independent
// replicas into the bits of one word) for 2D and 3D lattices with Lx a
// multiple of 128, Ising or +-J couplings, Metropolis or heat-bath.
//
// Design (gfx950):
//  * A wave takes 64 consecutive same-colour sites of one row (one site per
//    lane) and all 64 replicas of each (the bits of the site's word).  The
//    neighbour words give per-replica classes as bit-sliced counters
//    (carry-save adders over the 4 or 6 bond masks), so one lane updates 64
//    replicas with word operations.
//  * Every replica has its own random stream: lane b draws the Philox blocks
//    of replica b for the 4 groups of 16 sites the wave covers, whose
//    half-words are the random bit-planes of those sites (the stream the int8
//    kernels use, so lane b of the word lattice equals the int8 run of that
//    replica bit for bit).  A 64 x 64 bit transpose across the lanes
//    (xor-shuffles at distances 32 .. 1) turns "replica b, 64 sites" into
//    "site s, 64 replicas"; then each lane compares its site's 64 replicas
//    against the class thresholds bit-serially.  Ties (top byte equal) draw
//    their low 24 bits in place.
//  * Per-sweep E and M per replica are summed in the odd half-sweep: the
//    bond and down-spin count planes of the 64 sites are transposed back so
//    that lane b adds up replica b; one atomic per replica and workgroup.
#include "internal.hpp"

namespace mcs {

struct MscArgs {
    uint64_t *w;
    const int8_t *J;  // [dims][N] or nullptr
    int Lx, Ly, Lz;
    int64_t N;
    uint32_t seed_lo, seed_hi, replica0;
    uint32_t sweep_lo, w3, w3lo;
    int c;  // colour of this half-sweep
    // class thresholds (top byte, low 24 bits; T = 2^32 as 255 * 2^24 + 2^24):
    // Metropolis class a = unsatisfied bonds, T of dE = 2z - 4a (a < z/2);
    // heat-bath class d = neighbours with J s_j = -1, T of h = z - 2d
    uint32_t top[8], low[8];
    int64_t *EM;  // this sweep's [count * 64][2], or nullptr
};

// Lane exchange at xor distance D: ds_swizzle in its xor mode (and mask 0x1F,
// xor mask D; within groups of 32 lanes) for D <= 16, a permute across the
// wave for D = 32.
template <int D>
__device__ __forceinline__ uint32_t xor_lane(uint32_t x)
{
    if constexpr (D == 32)
        return (uint32_t)__shfl_xor((int)x, 32, 64);
    else
        return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, (D << 10) | 0x1F);
}

// One stage of the transpose: lanes i and i ^ D swap d-bit blocks.  The lane
// with bit D clear keeps the low block of each 2D-bit group and takes its
// partner's low block into the high position; the other lane keeps the high
// block and takes its partner's high block into the low position.  The select
// is a per-lane mask, not a branch (the two lanes of a pair take different
// sides).
template <int D>
__device__ __forceinline__ uint64_t transpose_stage(uint64_t v, int lane)
{
    constexpr uint64_t M = D == 32 ? 0x00000000FFFFFFFFull
                         : D == 16 ? 0x0000FFFF0000FFFFull
                         : D == 8  ? 0x00FF00FF00FF00FFull
                         : D == 4  ? 0x0F0F0F0F0F0F0F0Full
                         : D == 2  ? 0x3333333333333333ull
                                   : 0x5555555555555555ull;
    const uint32_t lo = xor_lane<D>((uint32_t)v), hi = xor_lane<D>((uint32_t)(v >> 32));
    const uint64_t p = ((uint64_t)hi << 32) | lo;
    const uint64_t sel = (lane & D) ? ~0ull : 0ull;
    const uint64_t keep = M ^ sel;                      // M on the low side, ~M on the high side
    const uint64_t up = p << D, down = p >> D;
    const uint64_t t = up ^ ((up ^ down) & sel);        // partner's block moved into place
    return (v & keep) | (t & ~keep);
}

// 64 x 64 bit transpose across the wave: on entry lane b holds row b, on exit
// lane s holds column s (bit b of the result = bit s of lane b's row).
__device__ __forceinline__ uint64_t transpose64(uint64_t v, int lane)
{
    v = transpose_stage<32>(v, lane);
    v = transpose_stage<16>(v, lane);
    v = transpose_stage<8>(v, lane);
    v = transpose_stage<4>(v, lane);
    v = transpose_stage<2>(v, lane);
    return transpose_stage<1>(v, lane);
}

template <int DIMS, bool MEASURE, bool HB, bool HASJ>
__global__ __launch_bounds__(256) void k_msc(MscArgs a)
{
    __shared__ uint32_t tlow[8];
    __shared__ long long red[2][64];
    constexpr int Z = 2 * DIMS;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l = blockIdx.y;
    if (tid < 8) tlow[tid] = a.low[tid];
    if (MEASURE && tid < 128) red[tid >> 6][tid & 63] = 0;
    __syncthreads();
    uint64_t *w = a.w + (int64_t)l * a.N;
    const int hx = a.Lx >> 1;
    const int64_t tasks = (a.N >> 1) >> 6;
    const uint32_t rep = a.replica0 + 64u * (uint32_t)l + (uint32_t)lane;
    long long e_acc = 0, m_acc = 0;
    for (int64_t t = (int64_t)blockIdx.x * 4 + wave; t < tasks; t += (int64_t)gridDim.x * 4) {
        const int64_t j0 = t << 6;
        const int64_t row = j0 / hx;
        const int m0 = (int)(j0 - row * hx);
        const int y = (int)(row % a.Ly), z = (int)(row / a.Ly);
        const int par = (a.c + y + z) & 1;
        const int x = 2 * (m0 + lane) + par;
        const int64_t rbase = row * a.Lx;
        const int64_t i = rbase + x;
        const int xp = x + 1 == a.Lx ? 0 : x + 1, xm = x == 0 ? a.Lx - 1 : x - 1;
        const int64_t ryp = (int64_t)(y + 1 == a.Ly ? 0 : y + 1) * a.Lx + (int64_t)z * a.Ly * a.Lx;
        const int64_t rym = (int64_t)(y == 0 ? a.Ly - 1 : y - 1) * a.Lx + (int64_t)z * a.Ly * a.Lx;
        const uint64_t S = w[i];
        uint64_t n[6];
        int64_t bi[6];
        n[0] = w[rbase + xp], bi[0] = i;
        n[1] = w[rbase + xm], bi[1] = rbase + xm;
        n[2] = w[ryp + x], bi[2] = a.N + i;
        n[3] = w[rym + x], bi[3] = a.N + rym + x;
        if (DIMS == 3) {
            const int64_t plane = (int64_t)a.Ly * a.Lx;
            const int64_t rzp = (z + 1 == a.Lz ? 0 : z + 1) * plane + (int64_t)y * a.Lx;
            const int64_t rzm = (z == 0 ? a.Lz - 1 : z - 1) * plane + (int64_t)y * a.Lx;
            n[4] = w[rzp + x], bi[4] = 2 * a.N + i;
            n[5] = w[rzm + x], bi[5] = 2 * a.N + rzm + x;
        }
        // wk: bit set <=> J s_j = -1 for replica b
        uint64_t wk[6];
#pragma unroll
        for (int k = 0; k < Z; ++k) wk[k] = n[k] ^ ((HASJ && a.J[bi[k]] < 0) ? ~0ull : 0ull);
        uint64_t xk[6];
#pragma unroll
        for (int k = 0; k < Z; ++k) xk[k] = HB ? wk[k] : (wk[k] ^ S);
        uint64_t c0, c1, c2;
        {
            const uint64_t s1 = xk[0] ^ xk[1] ^ xk[2];
            const uint64_t k1 = (xk[0] & xk[1]) | (xk[0] & xk[2]) | (xk[1] & xk[2]);
            if (DIMS == 3) {
                const uint64_t s2 = xk[3] ^ xk[4] ^ xk[5];
                const uint64_t k2 = (xk[3] & xk[4]) | (xk[3] & xk[5]) | (xk[4] & xk[5]);
                c0 = s1 ^ s2;
                const uint64_t kk = s1 & s2;
                c1 = k1 ^ k2 ^ kk;
                c2 = (k1 & k2) | (k1 & kk) | (k2 & kk);
            } else {
                c0 = s1 ^ xk[3];
                const uint64_t kk = s1 & xk[3];
                c1 = k1 ^ kk;
                c2 = k1 & kk;
            }
        }
        // Metropolis: a >= z/2 gives dE <= 0
        const uint64_t ge = HB ? 0ull : (DIMS == 3 ? (c2 | (c1 & c0)) : (c2 | c1));
        // random planes: lane = replica, 4 groups of 16 sites -> transpose
        uint4 B[4];
#pragma unroll
        for (int g = 0; g < 4; ++g)
            B[g] = philox(make_uint4((uint32_t)((j0 >> 4) + g), rep, a.sweep_lo, a.w3), a.seed_lo, a.seed_hi);
        // One indicator word per class (heat-bath d = 0..6; Metropolis a below
        // z/2, larger a being accepted outright); a plane's threshold word is the
        // OR of the indicators of the classes whose threshold has that bit, the
        // bits being uniform (argument block), so only the indicator words stay
        // live across the planes.
        constexpr int NC = HB ? 7 : DIMS;  // Metropolis: a = 0 .. z/2 - 1
        uint64_t onehot[7];
        uint32_t tp[7];
        {
            const uint64_t n0 = ~c0, n1 = ~c1, n2 = ~c2;
            onehot[0] = n2 & n1 & n0;
            onehot[1] = n2 & n1 & c0;
            onehot[2] = n2 & c1 & n0;
            onehot[3] = n2 & c1 & c0;
            onehot[4] = c2 & n1 & n0;
            onehot[5] = c2 & n1 & c0;
            onehot[6] = c2 & c1 & n0;
            // the thresholds' top bytes, marked as redefined per task so the plane
            // masks below are formed where used, not hoisted out of the task loop
            // into scalar registers (where they would spill)
#pragma unroll
            for (int d = 0; d < NC; ++d) {
                tp[d] = a.top[d];
                asm volatile("" : "+s"(tp[d]));
            }
        }
        uint64_t lt = 0ull, eq = ~0ull;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const uint64_t rowk = (uint64_t)plane_pair(B[0], B[1], k) | ((uint64_t)plane_pair(B[2], B[3], k) << 32);
            const uint64_t X = transpose64(rowk, lane);
            uint32_t tlo = 0u, thi = 0u;
#pragma unroll
            for (int d = 0; d < NC; ++d) {
                const uint32_t m = ((tp[d] >> k) & 1u) ? ~0u : 0u;
                tlo |= (uint32_t)onehot[d] & m;
                thi |= (uint32_t)(onehot[d] >> 32) & m;
            }
            const uint64_t T = ((uint64_t)thi << 32) | tlo;
            lt = (~X & T) | (~X & lt) | (T & lt);
            eq = eq & ~(X ^ T);
        }
        uint64_t acc = HB ? ~lt : (ge | lt);
        uint64_t pend = HB ? eq : (eq & ~ge);
        const uint32_t j = (uint32_t)(j0 + lane);
        while (pend) {
            const int b = __builtin_ctzll(pend);
            pend &= pend - 1ull;
            const uint32_t cls = (uint32_t)((c0 >> b) & 1ull) | ((uint32_t)((c1 >> b) & 1ull) << 1) |
                                 ((uint32_t)((c2 >> b) & 1ull) << 2);
            const uint4 lo = philox(make_uint4(j, a.replica0 + 64u * (uint32_t)l + (uint32_t)b, a.sweep_lo, a.w3lo),
                                    a.seed_lo, a.seed_hi);
            // Metropolis: flip; heat-bath: the provisional -1 becomes +1
            if ((lo.x & 0xFFFFFFu) < tlow[cls]) acc ^= (HB ? 1ull : 0ull) << b, acc |= (HB ? 0ull : 1ull) << b;
        }
        const uint64_t Sn = HB ? acc : (S ^ acc);
        w[i] = Sn;
        if (MEASURE) {
            // odd sites: their bonds after the update; both sites of the pair
            // (this odd site and the even site at the same row position) for M
            uint64_t u[6];
#pragma unroll
            for (int k = 0; k < Z; ++k) u[k] = Sn ^ wk[k];
            uint64_t u0, u1, u2;
            const uint64_t s1 = u[0] ^ u[1] ^ u[2];
            const uint64_t k1 = (u[0] & u[1]) | (u[0] & u[2]) | (u[1] & u[2]);
            if (DIMS == 3) {
                const uint64_t s2 = u[3] ^ u[4] ^ u[5];
                const uint64_t k2 = (u[3] & u[4]) | (u[3] & u[5]) | (u[4] & u[5]);
                u0 = s1 ^ s2;
                const uint64_t kk = s1 & s2;
                u1 = k1 ^ k2 ^ kk;
                u2 = (k1 & k2) | (k1 & kk) | (k2 & kk);
            } else {
                u0 = s1 ^ u[3];
                const uint64_t kk = s1 & u[3];
                u1 = k1 ^ kk;
                u2 = k1 & kk;
            }
            const uint64_t pw = par == 1 ? n[1] : n[0];  // the even site 2m + (1 - par)
            const uint64_t d0 = Sn ^ pw, d1 = Sn & pw;
            const uint64_t U0 = transpose64(u0, lane), U1 = transpose64(u1, lane), U2 = transpose64(u2, lane);
            const uint64_t D0 = transpose64(d0, lane), D1 = transpose64(d1, lane);
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

bool msc_fast_supported(const SweepCall &c, int layout)
{
    return layout == MC_MSC64 && (c.g.dims == 2 || c.g.dims == 3) && c.g.Lx % 128 == 0 && c.g.Lx <= 65536 &&
           c.g.N <= (int64_t)1 << 32;
}

template <int D, bool HB, bool HJ>
static hipError_t launch_msc_t(const MscArgs &a, int count, hipStream_t s)
{
    const int64_t tasks = (a.N >> 1) >> 6;
    int64_t blocks = (tasks + 3) / 4;
    if (blocks > 1024) blocks = 1024;
    dim3 grid((unsigned)blocks, (unsigned)count);
    if (a.EM) hipLaunchKernelGGL((k_msc<D, true, HB, HJ>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_msc<D, false, HB, HJ>), grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// One half-sweep (colour c) of every word lattice; EM: this sweep's per-lane
// (E, M), accumulated (cleared by the caller), in the odd half-sweep only.
hipError_t launch_msc_phase(const SweepCall &c, uint64_t *words, uint64_t sweep, int phase, int64_t *EM,
                            hipStream_t s)
{
    MscArgs a;
    a.w = words;
    a.J = c.J;
    a.Lx = c.g.Lx;
    a.Ly = c.g.Ly;
    a.Lz = c.g.dims == 3 ? c.g.Lz : 1;
    a.N = c.g.N;
    a.seed_lo = c.seed_lo;
    a.seed_hi = c.seed_hi;
    a.replica0 = c.replica0;
    a.sweep_lo = (uint32_t)sweep;
    a.w3 = ctr_w3(kTagSweep, (uint32_t)phase, sweep);
    a.w3lo = ctr_w3(kTagSweepLo, (uint32_t)phase, sweep);
    a.c = phase;
    const int z = 2 * c.g.dims;
    for (int cl = 0; cl < 8; ++cl) {
        Thr th{0u, 0u};
        if (c.rule == 0) {
            if (2 * cl < z) th = c.tab.met[z / 2 - cl];   // dE = 2z - 4a
        } else if (cl <= z) {
            th = c.tab.hb[z - 2 * cl + 6];                // h = z - 2d
        }
        if (th.top >= 256u) th = Thr{255u, 1u << 24};
        a.top[cl] = th.top;
        a.low[cl] = th.low;
    }
    a.EM = phase == 1 ? EM : nullptr;
    const bool hb = c.rule == 1, hj = c.J != nullptr;
    if (c.g.dims == 2) {
        if (hb) return hj ? launch_msc_t<2, true, true>(a, c.g.count, s) : launch_msc_t<2, true, false>(a, c.g.count, s);
        return hj ? launch_msc_t<2, false, true>(a, c.g.count, s) : launch_msc_t<2, false, false>(a, c.g.count, s);
    }
    if (hb) return hj ? launch_msc_t<3, true, true>(a, c.g.count, s) : launch_msc_t<3, true, false>(a, c.g.count, s);
    return hj ? launch_msc_t<3, false, true>(a, c.g.count, s) : launch_msc_t<3, false, false>(a, c.g.count, s);
}

}  // namespace mcs
