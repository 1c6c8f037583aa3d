// k_small.hip -- checkerboard sweeps of small int8 lattices held whole in one
// workgroup's LDS (spins, and the couplings of a +-J model), any dimension,
// Metropolis or heat-bath (Sec. "Checkerboard scheme"; Sec. "Disordered
// systems").  One workgroup per lattice runs every sweep of a call in a single
// launch with barriers between the steps of a half-sweep, so a lattice of a
// few ten thousand sites is not bound by launch latency.
//
// Randomness and decisions are those of the generic half-sweep: site j of
// colour c draws byte (j mod 16) of Philox(j/16, replica, sweep, SWEEP | c)
// and, on a tie with the threshold's top byte, the low 24 bits from
// Philox(j, ..., SWEEP_LO | c).
//
// A half-sweep is two steps.  First every Philox block of the colour is drawn
// once into LDS (one block serves 16 sites).  Then consecutive threads take
// consecutive sites, so the byte-wide neighbour reads of a wave fall on
// consecutive LDS addresses; site coordinates advance by fixed increments, not
// by division.  E and M are kept as running totals: one full measurement at
// the start, then the energy and magnetisation changes of the accepted flips
// of each sweep (Delta E = 2 s h, Delta M = -2 s), reduced in the workgroup.
#include "internal.hpp"

namespace mcs {

struct SmallArgs {
    int8_t *spins;
    const int8_t *J;  // [dims][N] or nullptr
    Geom g;
    int rule;
    uint32_t seed_lo, seed_hi, replica0;
    uint64_t sweep0;
    int nsweeps;
    SweepTables tab;
    int64_t *EM;  // [nsweeps][count][2] or nullptr
    int64_t em_stride;
};

__host__ __device__ __forceinline__ int64_t pad16(int64_t n)
{
    return (n + 15) & ~(int64_t)15;
}

// LDS layout: spins [pad16(N)], couplings [pad16(dims N)] if any, then one
// Philox block (16 B) per 16 sites of a colour.
__host__ __device__ __forceinline__ int64_t small_rnd_offset(const Geom &g, bool hasJ)
{
    return pad16(g.N) + (hasJ ? pad16((int64_t)g.dims * g.N) : 0);
}

__host__ __device__ __forceinline__ int64_t small_groups(const Geom &g)
{
    return ((g.N >> 1) + 15) >> 4;
}

// byte_of(b, pos) by masks: the bits of the eight half-words at position pos
// are gathered at even offsets (low half-words) and at 16 + even offsets
// (high half-words), then interleaved.
__device__ __forceinline__ uint32_t plane_byte(const uint4 &b, uint32_t pos)
{
    const uint32_t m = 0x00010001u;
    uint32_t a = (b.x >> pos) & m;
    a |= ((b.y >> pos) & m) << 2;
    a |= ((b.z >> pos) & m) << 4;
    a |= ((b.w >> pos) & m) << 6;
    return (a & 0x55u) | ((a >> 15) & 0xAAu);
}

// r32 < T with T split as (top byte, low 24 bits); the low bits are drawn only
// on a tie with the top byte.
__device__ __forceinline__ bool below_lazy(uint32_t byte, uint32_t top, uint32_t low, uint32_t k0, uint32_t k1,
                                           uint32_t j, uint32_t rep, uint32_t sweep_lo, uint32_t w3lo)
{
    if (byte != top) return byte < top;
    const uint4 lo = philox(make_uint4(j, rep, sweep_lo, w3lo), k0, k1);
    return (lo.x & 0xFFFFFFu) < low;
}

template <bool HASJ>
__global__ __launch_bounds__(1024) void k_small(SmallArgs a)
{
    extern __shared__ __align__(16) int8_t sm[];
    __shared__ long long red[2][2][16];
    // thresholds in LDS: a lane-indexed read of the argument block would be a
    // memory load per site.  Entries 0..3 Metropolis (dE / 4), 4..16 heat-bath
    // (h + 6).
    __shared__ uint32_t thr_top[17], thr_low[17];
    const Geom &g = a.g;
    const int l = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x, wave = tid >> 6, nwaves = nt >> 6;
    const int N = (int)g.N, Lx = g.Lx, Ly = g.Ly, Lz = g.dims == 3 ? g.Lz : 1;
    const int plane = Lx * Ly;
    int8_t *s = sm;
    const int8_t *J0 = sm + pad16(N), *J1 = J0 + N, *J2 = J1 + N;
    uint4 *rnd = (uint4 *)(sm + small_rnd_offset(g, HASJ));
    const int8_t *src = a.spins + (int64_t)l * N;
    if (tid < 17) {
        const Thr t = tid < 4 ? a.tab.met[tid] : a.tab.hb[tid - 4];
        thr_top[tid] = t.top;
        thr_low[tid] = t.low;
    }
    for (int i = tid; i < N; i += nt) s[i] = src[i];
    if (HASJ)
        for (int i = tid; i < g.dims * N; i += nt) sm[pad16(N) + i] = a.J[i];
    __syncthreads();

    // running E and M, held by thread 0 after the initial reduction
    long long E = 0, M = 0;
    if (a.EM) {
        // E = -sum_i s_i sum_d J_d(i) s_{i + e_d}, M = sum_i s_i
        long long e = 0, mm = 0;
        for (int i = tid; i < N; i += nt) {
            const int x = i % Lx, r = i / Lx, y = r % Ly, z = r / Ly;
            const int si = s[i];
            const int xp = x + 1 == Lx ? i - x : i + 1;
            const int yp = y + 1 == Ly ? i - (Ly - 1) * Lx : i + Lx;
            int b = (HASJ ? J0[i] : 1) * s[xp] + (HASJ ? J1[i] : 1) * s[yp];
            if (g.dims == 3) {
                const int zp = z + 1 == Lz ? i - (Lz - 1) * plane : i + plane;
                b += (HASJ ? J2[i] : 1) * s[zp];
            }
            e -= si * b;
            mm += si;
        }
        e = wave_sum(e);
        mm = wave_sum(mm);
        if ((tid & 63) == 0) {
            red[0][0][wave] = e;
            red[0][1][wave] = mm;
        }
        __syncthreads();
        if (tid == 0)
            for (int w = 0; w < nwaves; ++w) {
                E += red[0][0][w];
                M += red[0][1][w];
            }
        __syncthreads();
    }

    const uint32_t rep = a.replica0 + (uint32_t)l;
    const int hx = Lx >> 1, half = N >> 1, groups = (int)small_groups(g);
    // coordinates of this thread's first site j = tid (j = m + hx (y + Ly z)),
    // and the increments for a step of nt sites
    const int m0 = tid % hx, row0 = tid / hx, y0 = row0 % Ly, z0 = row0 / Ly;
    const int dm = nt % hx, drow = nt / hx, dy = drow % Ly, dz = drow / Ly;
    for (int t = 0; t < a.nsweeps; ++t) {
        const uint64_t sweep = a.sweep0 + (uint64_t)t;
        int de = 0, dmg = 0;
        for (int c = 0; c < 2; ++c) {
            const uint32_t w3 = ctr_w3(kTagSweep, (uint32_t)c, sweep), w3lo = ctr_w3(kTagSweepLo, (uint32_t)c, sweep);
            for (int gi = tid; gi < groups; gi += nt)
                rnd[gi] = philox(make_uint4((uint32_t)gi, rep, (uint32_t)sweep, w3), a.seed_lo, a.seed_hi);
            __syncthreads();
            int m = m0, y = y0, z = z0;
            for (int j = tid; j < half; j += nt) {
                const int x = 2 * m + ((c + y + z) & 1);
                const int rb = Lx * (y + Ly * z);
                const int i = rb + x;
                const int ixp = x + 1 == Lx ? rb : i + 1;
                const int ixm = x == 0 ? rb + Lx - 1 : i - 1;
                const int iyp = y + 1 == Ly ? i - (Ly - 1) * Lx : i + Lx;
                const int iym = y == 0 ? i + (Ly - 1) * Lx : i - Lx;
                int h;
                if (HASJ) h = J0[i] * s[ixp] + J0[ixm] * s[ixm] + J1[i] * s[iyp] + J1[iym] * s[iym];
                else h = s[ixp] + s[ixm] + s[iyp] + s[iym];
                if (g.dims == 3) {
                    const int izp = z + 1 == Lz ? i - (Lz - 1) * plane : i + plane;
                    const int izm = z == 0 ? i + (Lz - 1) * plane : i - plane;
                    h += HASJ ? J2[i] * s[izp] + J2[izm] * s[izm] : s[izp] + s[izm];
                }
                const int si = s[i];
                const uint32_t byte = plane_byte(rnd[j >> 4], (uint32_t)(j & 15));
                bool flip;
                if (a.rule == 0) {
                    const int dE = 2 * si * h;
                    const int q = dE > 0 ? dE >> 2 : 0;
                    flip = dE <= 0 || below_lazy(byte, thr_top[q], thr_low[q], a.seed_lo, a.seed_hi, (uint32_t)j, rep,
                                                 (uint32_t)sweep, w3lo);
                } else {
                    const int q = h + 10;
                    const bool up = below_lazy(byte, thr_top[q], thr_low[q], a.seed_lo, a.seed_hi, (uint32_t)j, rep,
                                               (uint32_t)sweep, w3lo);
                    flip = up != (si > 0);
                }
                if (flip) {
                    s[i] = (int8_t)-si;
                    de += 2 * si * h;
                    dmg -= 2 * si;
                }
                m += dm;
                const int carry = m >= hx ? 1 : 0;
                if (carry) m -= hx;
                y += dy + carry;
                if (y >= Ly) {
                    y -= Ly;
                    ++z;
                }
                z += dz;
            }
            if (c == 1 && a.EM) {
                const int we = wave_sum_i(de), wm = wave_sum_i(dmg);
                if ((tid & 63) == 0) {
                    red[t & 1][0][wave] = we;
                    red[t & 1][1][wave] = wm;
                }
            }
            __syncthreads();
        }
        // red[t & 1] is next written two sweeps on, after further barriers
        if (a.EM && tid == 0) {
            for (int w = 0; w < nwaves; ++w) {
                E += red[t & 1][0][w];
                M += red[t & 1][1][w];
            }
            a.EM[t * a.em_stride + 2 * l] = E;
            a.EM[t * a.em_stride + 2 * l + 1] = M;
        }
    }
    int8_t *dst = a.spins + (int64_t)l * N;
    for (int i = tid; i < N; i += nt) dst[i] = s[i];
}

size_t small_lds_bytes(const Geom &g, bool hasJ)
{
    return (size_t)(small_rnd_offset(g, hasJ) + 16 * small_groups(g));
}

bool small_supported(const SweepCall &c, int layout)
{
    return layout == MC_INT8 && !c.per_lattice && c.g.N <= (1 << 20) &&
           small_lds_bytes(c.g, c.J != nullptr) <= 150 * 1024;
}

hipError_t launch_small(const SweepCall &c, int8_t *spins, uint64_t sweep0, int nsweeps, int64_t *EM,
                        int64_t em_stride, hipStream_t s)
{
    SmallArgs a;
    a.spins = spins;
    a.J = c.J;
    a.g = c.g;
    a.rule = c.rule;
    a.seed_lo = c.seed_lo;
    a.seed_hi = c.seed_hi;
    a.replica0 = c.replica0;
    a.sweep0 = sweep0;
    a.nsweeps = nsweeps;
    a.tab = c.tab;
    a.EM = EM;
    a.em_stride = em_stride;
    const bool hj = c.J != nullptr;
    const size_t lds = small_lds_bytes(c.g, hj);
    static LdsLimit lim[2];
    {
        const hipError_t e =
            lim[hj ? 1 : 0].ensure(hj ? (const void *)k_small<true> : (const void *)k_small<false>, 150 * 1024);
        if (e != hipSuccess) return e;
    }
    if (hj) hipLaunchKernelGGL(k_small<true>, dim3((unsigned)c.g.count), dim3(1024), lds, s, a);
    else hipLaunchKernelGGL(k_small<false>, dim3((unsigned)c.g.count), dim3(1024), lds, s, a);
    return hipGetLastError();
}

}  // namespace mcs
