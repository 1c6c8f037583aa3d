// k_small_bits.hip -- checkerboard sweeps of small int8 lattices whose rows are
// 32 sites long (Lx = 32), 2D or 3D, J = 1 or +-J, Metropolis or heat-bath
// (Sec. "Checkerboard scheme"; Sec. "Disordered systems"), with the whole
// lattice bit-packed in one workgroup's LDS and every sweep of a call in one
// launch.
//
// Layout: row r = y + Ly z is two 16-bit words, one per x parity p (bit i =
// site x = 2i + p), set bit = spin -1.  Couplings likewise, one word per
// direction, parity and row (bit set = J -1, bond from the site to its + e_d
// neighbour).  In a half-sweep of colour c the sites of row r to update are
// its parity p = (c + y + z) mod 2 word; their x neighbours are the other
// parity word of the same row shifted by one, their y and z neighbours the
// parity p words of the adjacent rows.  Only colour-c words are written and
// only colour-(1-c) words are read, so the threads of a half-sweep (one per
// row) never race.
//
// Randomness is that of the generic half-sweep: site j = 16 r + i of colour c
// draws byte i of Philox(j / 16 = r, replica, sweep, SWEEP | c), so one block
// per row gives the eight random bit-planes of its 16 sites (plane k = half-word
// k of the block), and a tie with the threshold's top byte draws the low 24
// bits from Philox(j, ..., SWEEP_LO | c).  Per site the class (unsatisfied
// bonds for Metropolis, neighbours with J s = -1 for heat-bath) is a 3-bit
// bit-sliced count; the threshold planes are selected per class and compared
// bit-serially against the random planes.  E and M are recounted after each
// sweep from the bonds' popcounts.
#include "internal.hpp"

namespace mcs {

struct SmallBitsArgs {
    int8_t *spins;
    const int8_t *J;  // [dims][N] or nullptr
    Geom g;
    uint32_t seed_lo, seed_hi, replica0;
    uint64_t sweep0;
    int nsweeps;
    // class thresholds (top byte, low 24 bits; T = 2^32 as 255 * 2^24 + 2^24)
    uint32_t top[8], low[8];
    int64_t *EM;  // [nsweeps][count][2] or nullptr
    int64_t em_stride;
};

__device__ __forceinline__ uint32_t rotl16(uint32_t v)
{
    return ((v << 1) | (v >> 15)) & 0xFFFFu;
}

__device__ __forceinline__ uint32_t rotr16(uint32_t v)
{
    return ((v >> 1) | (v << 15)) & 0xFFFFu;
}

// Sign bits of 32 int8 spins (one row) -> even-x and odd-x 16-bit words.
__device__ __forceinline__ void pack_row32(const int8_t *p, uint32_t &ev, uint32_t &od)
{
    const uint4 *q = (const uint4 *)p;
    ev = od = 0u;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const uint4 v = q[h];
        const uint32_t d[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int x0 = 16 * h + 4 * t;  // bytes x0 .. x0 + 3
            ev |= ((d[t] >> 7) & 1u) << (x0 / 2);
            od |= ((d[t] >> 15) & 1u) << (x0 / 2);
            ev |= ((d[t] >> 23) & 1u) << (x0 / 2 + 1);
            od |= ((d[t] >> 31) & 1u) << (x0 / 2 + 1);
        }
    }
}

__device__ __forceinline__ void unpack_row32(int8_t *p, uint32_t ev, uint32_t od)
{
    uint4 *q = (uint4 *)p;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        uint32_t d[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int i = 8 * h + 2 * t;  // parity index of bytes x = 2i .. 2i + 3
            const uint32_t b0 = (ev >> i) & 1u, b1 = (od >> i) & 1u, b2 = (ev >> (i + 1)) & 1u,
                           b3 = (od >> (i + 1)) & 1u;
            d[t] = (b0 ? 0xFFu : 0x01u) | (b1 ? 0xFF00u : 0x0100u) | (b2 ? 0xFF0000u : 0x010000u) |
                   (b3 ? 0xFF000000u : 0x01000000u);
        }
        q[h] = make_uint4(d[0], d[1], d[2], d[3]);
    }
}

// Row r = y + Ly z: the parity of (y + z) and the indices of its four (2D:
// two) neighbouring rows.
struct RowGeo {
    int yz;  // (y + z) & 1
    int ryp, rym, rzp, rzm;
};

__device__ __forceinline__ RowGeo row_geo(int r, int Ly, int Lz)
{
    const int y = r % Ly, z = r / Ly;
    RowGeo g;
    g.yz = (y + z) & 1;
    g.ryp = y + 1 == Ly ? r - y : r + 1;
    g.rym = y == 0 ? r + Ly - 1 : r - 1;
    g.rzp = z + 1 == Lz ? r - (Lz - 1) * Ly : r + Ly;
    g.rzm = z == 0 ? r + (Lz - 1) * Ly : r - Ly;
    return g;
}

template <int DIMS, bool HB, bool HASJ>
__global__ __launch_bounds__(1024) void k_small_bits(SmallBitsArgs a)
{
    constexpr int Z = 2 * DIMS;
    extern __shared__ uint32_t sm[];  // S[2][R], then J[DIMS][2][R]
    __shared__ __align__(16) uint32_t tm[8][8];  // [plane][class]: all ones iff bit set in the class's top byte
    __shared__ uint32_t tlow[8];
    __shared__ long long red[2][16];
    const int tid = threadIdx.x, nt = blockDim.x, l = blockIdx.x;
    const int Ly = a.g.Ly, Lz = DIMS == 3 ? a.g.Lz : 1, R = Ly * Lz;
    const int64_t N = (int64_t)32 * R;
    uint32_t *S = sm;           // S[p * R + r]
    uint32_t *Jb = sm + 2 * R;  // Jb[(d * 2 + p) * R + r]
    if (tid < 64) tm[tid >> 3][tid & 7] = ((a.top[tid & 7] >> (tid >> 3)) & 1u) ? ~0u : 0u;
    if (tid < 8) tlow[tid] = a.low[tid];
    const int8_t *src = a.spins + (int64_t)l * N;
    for (int r = tid; r < R; r += nt) {
        uint32_t ev, od;
        pack_row32(src + 32 * (int64_t)r, ev, od);
        S[r] = ev;
        S[R + r] = od;
        if (HASJ)
            for (int d = 0; d < DIMS; ++d) {
                pack_row32(a.J + (int64_t)d * N + 32 * (int64_t)r, ev, od);
                Jb[(2 * d) * R + r] = ev;
                Jb[(2 * d + 1) * R + r] = od;
            }
    }
    __syncthreads();
    const uint32_t rep = a.replica0 + (uint32_t)l;
    // geometry of this thread's first row (the only one when R <= threads)
    const RowGeo g0 = row_geo(tid < R ? tid : 0, Ly, Lz);
    for (int t = 0; t < a.nsweeps; ++t) {
        const uint64_t sweep = a.sweep0 + (uint64_t)t;
        for (int c = 0; c < 2; ++c) {
            const uint32_t w3 = ctr_w3(kTagSweep, (uint32_t)c, sweep), w3lo = ctr_w3(kTagSweepLo, (uint32_t)c, sweep);
            for (int r = tid; r < R; r += nt) {
                const RowGeo rg = r == tid ? g0 : row_geo(r, Ly, Lz);
                const int p = (c + rg.yz) & 1;
                const int op = p ? R : 0, oq = p ? 0 : R;  // word offsets of parity p and 1 - p
                const uint32_t s = S[op + r], o = S[oq + r];
                // x neighbours: the other parity word shifted by one, selected
                // without branching (neighbouring rows of a wave differ in p)
                const uint32_t ol = rotl16(o), orr = rotr16(o);
                uint32_t nb[6], jb[6];
                nb[0] = p ? o : ol;   // x - 1
                nb[1] = p ? orr : o;  // x + 1
                nb[2] = S[op + rg.ryp];
                nb[3] = S[op + rg.rym];
                if (HASJ) {
                    const uint32_t j0o = Jb[oq + r];
                    jb[0] = p ? j0o : rotl16(j0o);  // bond to x - 1: J_x of site x - 1
                    jb[1] = Jb[op + r];             // bond to x + 1: J_x of this site
                    jb[2] = Jb[2 * R + op + r];
                    jb[3] = Jb[2 * R + op + rg.rym];
                }
                if (DIMS == 3) {
                    nb[4] = S[op + rg.rzp];
                    nb[5] = S[op + rg.rzm];
                    if (HASJ) {
                        jb[4] = Jb[4 * R + op + r];
                        jb[5] = Jb[4 * R + op + rg.rzm];
                    }
                }
                // per-bond indicator: heat-bath J s_j = -1, Metropolis unsatisfied
                uint32_t xk[6];
#pragma unroll
                for (int k = 0; k < Z; ++k) {
                    const uint32_t w = HASJ ? (nb[k] ^ jb[k]) : nb[k];
                    xk[k] = HB ? w : (w ^ s);
                }
                uint32_t c0, c1, c2;
                {
                    const uint32_t s1 = xk[0] ^ xk[1] ^ xk[2];
                    const uint32_t k1 = (xk[0] & xk[1]) | (xk[0] & xk[2]) | (xk[1] & xk[2]);
                    if (DIMS == 3) {
                        const uint32_t s2 = xk[3] ^ xk[4] ^ xk[5];
                        const uint32_t k2 = (xk[3] & xk[4]) | (xk[3] & xk[5]) | (xk[4] & xk[5]);
                        c0 = s1 ^ s2;
                        const uint32_t kk = s1 & s2;
                        c1 = k1 ^ k2 ^ kk;
                        c2 = (k1 & k2) | (k1 & kk) | (k2 & kk);
                    } else {
                        c0 = s1 ^ xk[3];
                        const uint32_t kk = s1 & xk[3];
                        c1 = k1 ^ kk;
                        c2 = k1 & kk;
                    }
                }
                // Metropolis: a >= z/2 gives dE <= 0
                const uint32_t ge = HB ? 0u : (DIMS == 3 ? (c2 | (c1 & c0)) : (c2 | c1));
                const uint4 blk = philox(make_uint4((uint32_t)r, rep, (uint32_t)sweep, w3), a.seed_lo, a.seed_hi);
                uint32_t lt = 0u, eq = 0xFFFFu;
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const uint32_t wk = (k >> 1) == 0 ? blk.x : (k >> 1) == 1 ? blk.y : (k >> 1) == 2 ? blk.z : blk.w;
                    const uint32_t X = (k & 1) ? (wk >> 16) : (wk & 0xFFFFu);
                    const uint4 ml = *(const uint4 *)&tm[k][0];
                    uint32_t T;
                    if (HB) {
                        const uint4 mh = *(const uint4 *)&tm[k][4];
                        const uint32_t m01 = (c0 & ml.y) | (~c0 & ml.x), m23 = (c0 & ml.w) | (~c0 & ml.z);
                        const uint32_t m45 = (c0 & mh.y) | (~c0 & mh.x);
                        const uint32_t lo4 = (c1 & m23) | (~c1 & m01), hi4 = (c1 & mh.z) | (~c1 & m45);
                        T = (c2 & hi4) | (~c2 & lo4);
                    } else if (DIMS == 3) {
                        const uint32_t m01 = (c0 & ml.y) | (~c0 & ml.x);
                        T = (c1 & ml.z) | (~c1 & m01);
                    } else {
                        T = (c0 & ml.y) | (~c0 & ml.x);
                    }
                    lt = (~X & T) | (~X & lt) | (T & lt);
                    eq = eq & ~(X ^ T);
                }
                // heat-bath: up where r < T; Metropolis: flip where accepted
                uint32_t acc = HB ? lt : ((ge | lt) & 0xFFFFu);
                uint32_t pend = HB ? (eq & 0xFFFFu) : (eq & ~ge & 0xFFFFu);
                while (pend) {
                    const int b = __builtin_ctz(pend);
                    pend &= pend - 1u;
                    const uint32_t cls = ((c0 >> b) & 1u) | (((c1 >> b) & 1u) << 1) | (((c2 >> b) & 1u) << 2);
                    const uint4 lo =
                        philox(make_uint4(16u * (uint32_t)r + (uint32_t)b, rep, (uint32_t)sweep, w3lo), a.seed_lo,
                               a.seed_hi);
                    if ((lo.x & 0xFFFFFFu) < tlow[cls]) acc |= 1u << b;
                }
                S[op + r] = HB ? (~acc & 0xFFFFu) : (s ^ acc);
            }
            __syncthreads();
        }
        if (a.EM) {
            // E = 2 (unsatisfied bonds) - DIMS N, M = N - 2 (down spins)
            long long unsat = 0, down = 0;
            for (int r = tid; r < R; r += nt) {
                const RowGeo rg = r == tid ? g0 : row_geo(r, Ly, Lz);
                const uint32_t s0 = S[r], s1 = S[R + r];
                const uint32_t j00 = HASJ ? Jb[r] : 0u, j01 = HASJ ? Jb[R + r] : 0u;
                // + x bonds: even site 2i to odd i, odd site 2i + 1 to even i + 1
                uint32_t u = __popc((s0 ^ s1 ^ j00) & 0xFFFFu) + __popc((s1 ^ rotr16(s0) ^ j01) & 0xFFFFu);
#pragma unroll
                for (int p = 0; p < 2; ++p) {
                    const uint32_t sp = p ? s1 : s0;
                    u += __popc((sp ^ S[p * R + rg.ryp] ^ (HASJ ? Jb[(2 + p) * R + r] : 0u)) & 0xFFFFu);
                    if (DIMS == 3)
                        u += __popc((sp ^ S[p * R + rg.rzp] ^ (HASJ ? Jb[(4 + p) * R + r] : 0u)) & 0xFFFFu);
                }
                unsat += u;
                down += __popc(s0) + __popc(s1);
            }
            unsat = wave_sum(unsat);
            down = wave_sum(down);
            if ((tid & 63) == 0) {
                red[0][tid >> 6] = unsat;
                red[1][tid >> 6] = down;
            }
            __syncthreads();
            if (tid == 0) {
                long long U = 0, D = 0;
                for (int w = 0; w < (nt >> 6); ++w) {
                    U += red[0][w];
                    D += red[1][w];
                }
                a.EM[t * a.em_stride + 2 * l] = 2 * U - (long long)DIMS * N;
                a.EM[t * a.em_stride + 2 * l + 1] = N - 2 * D;
            }
            __syncthreads();
        }
    }
    int8_t *dst = a.spins + (int64_t)l * N;
    for (int r = tid; r < R; r += nt) unpack_row32(dst + 32 * (int64_t)r, S[r], S[R + r]);
}

static size_t small_bits_lds_bytes(const Geom &g, bool hasJ)
{
    const size_t R = (size_t)g.Ly * (g.dims == 3 ? (size_t)g.Lz : 1);
    return 4 * R * (2 + (hasJ ? 2 * (size_t)g.dims : 0));
}

bool small_bits_supported(const SweepCall &c, int layout)
{
    return layout == MC_INT8 && !c.per_lattice && c.g.Lx == 32 && (c.g.dims == 2 || c.g.dims == 3) &&
           small_bits_lds_bytes(c.g, c.J != nullptr) <= 128 * 1024;
}

template <int DIMS, bool HB, bool HASJ>
static hipError_t launch_sb(const SmallBitsArgs &a, size_t lds, hipStream_t s)
{
    static LdsLimit lim;
    {
        const hipError_t e = lim.ensure((const void *)k_small_bits<DIMS, HB, HASJ>, 128 * 1024);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_small_bits<DIMS, HB, HASJ>), dim3((unsigned)a.g.count), dim3(1024), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_small_bits(const SweepCall &c, int8_t *spins, uint64_t sweep0, int nsweeps, int64_t *EM,
                             int64_t em_stride, hipStream_t s)
{
    SmallBitsArgs a;
    a.spins = spins;
    a.J = c.J;
    a.g = c.g;
    a.seed_lo = c.seed_lo;
    a.seed_hi = c.seed_hi;
    a.replica0 = c.replica0;
    a.sweep0 = sweep0;
    a.nsweeps = nsweeps;
    a.EM = EM;
    a.em_stride = em_stride;
    // class cl: Metropolis a = cl unsatisfied bonds, dE = 2 z - 4 a (only
    // a < z / 2 needs a draw); heat-bath d = cl neighbours with J s = -1,
    // h = z - 2 d
    const int z = 2 * c.g.dims;
    for (int cl = 0; cl < 8; ++cl) {
        Thr th{0u, 0u};
        if (c.rule == 0) {
            if (cl < z / 2) th = c.tab.met[z / 2 - cl];
        } else if (cl <= z) {
            th = c.tab.hb[z - 2 * cl + 6];
        }
        if (th.top >= 256u) th = Thr{255u, 1u << 24};  // T = 2^32
        a.top[cl] = th.top;
        a.low[cl] = th.low;
    }
    const size_t lds = small_bits_lds_bytes(c.g, c.J != nullptr);
    const bool hb = c.rule == 1, hj = c.J != nullptr;
    if (c.g.dims == 3) {
        if (hb) return hj ? launch_sb<3, true, true>(a, lds, s) : launch_sb<3, true, false>(a, lds, s);
        return hj ? launch_sb<3, false, true>(a, lds, s) : launch_sb<3, false, false>(a, lds, s);
    }
    if (hb) return hj ? launch_sb<2, true, true>(a, lds, s) : launch_sb<2, true, false>(a, lds, s);
    return hj ? launch_sb<2, false, true>(a, lds, s) : launch_sb<2, false, false>(a, lds, s);
}

}  // namespace mcs
