// k_small.hip -- checkerboard sweeps of small int8 lattices held whole in one
// workgroup's LDS (spins, and the couplings of a +-J model), any dimension,
// Metropolis or heat-bath (Sec. "Checkerboard scheme"; Sec. "Disordered
// systems").  One workgroup per lattice runs every sweep of a call in a single
// launch with a barrier between half-sweeps, so a lattice of a few ten
// thousand sites is not bound by launch latency; E and M of each sweep are
// reduced in the workgroup and stored without atomics.
//
// Randomness and decisions are those of the generic half-sweep: site j of
// colour c draws byte (j mod 16) of Philox(j/16, replica, sweep, SWEEP | c)
// and, on a tie with the threshold's top byte, the low 24 bits from
// Philox(j, ..., SWEEP_LO | c).
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

__device__ __forceinline__ bool below_lazy(uint32_t byte, const Thr &t, uint32_t k0, uint32_t k1, uint32_t j,
                                           uint32_t rep, uint32_t sweep_lo, uint32_t w3lo)
{
    if (byte != t.top) return byte < t.top;
    const uint4 lo = philox(make_uint4(j, rep, sweep_lo, w3lo), k0, k1);
    return (lo.x & 0xFFFFFFu) < t.low;
}

template <bool HASJ>
__global__ __launch_bounds__(1024) void k_small(SmallArgs a)
{
    extern __shared__ int8_t sm[];
    __shared__ long long red[2][16];
    const Geom &g = a.g;
    const int l = blockIdx.x;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int N = (int)g.N;
    int8_t *s = sm;
    int8_t *Js = sm + ((N + 15) & ~15);
    const int8_t *src = a.spins + (int64_t)l * N;
    for (int i = tid; i < N; i += nt) s[i] = src[i];
    if (HASJ)
        for (int i = tid; i < g.dims * N; i += nt) Js[i] = a.J[i];
    __syncthreads();
    const uint32_t rep = a.replica0 + (uint32_t)l;
    const int hx = g.Lx >> 1, half = N >> 1, groups = (half + 15) >> 4;
    const int Lz = g.dims == 3 ? g.Lz : 1;
    for (int t = 0; t < a.nsweeps; ++t) {
        const uint64_t sweep = a.sweep0 + (uint64_t)t;
        for (int c = 0; c < 2; ++c) {
            const uint32_t w3 = ctr_w3(kTagSweep, (uint32_t)c, sweep), w3lo = ctr_w3(kTagSweepLo, (uint32_t)c, sweep);
            for (int gi = tid; gi < groups; gi += nt) {
                const uint4 blk = philox(make_uint4((uint32_t)gi, rep, (uint32_t)sweep, w3), a.seed_lo, a.seed_hi);
                int j = 16 * gi;
                int row = j / hx, m = j - row * hx;
                for (int k = 0; k < 16 && j < half; ++k, ++j) {
                    const int y = row % g.Ly, z = row / g.Ly;
                    const int x = 2 * m + ((c + y + z) & 1);
                    const int i = x + g.Lx * row;
                    const int xp = x + 1 == g.Lx ? 0 : x + 1, xm = x == 0 ? g.Lx - 1 : x - 1;
                    const int rb = g.Lx * row;
                    const int ryp = g.Lx * ((y + 1 == g.Ly ? 0 : y + 1) + g.Ly * z);
                    const int rym = g.Lx * ((y == 0 ? g.Ly - 1 : y - 1) + g.Ly * z);
                    int h;
                    if (HASJ) {
                        h = Js[i] * s[rb + xp] + Js[rb + xm] * s[rb + xm] + Js[N + i] * s[ryp + x] +
                            Js[N + rym + x] * s[rym + x];
                    } else {
                        h = s[rb + xp] + s[rb + xm] + s[ryp + x] + s[rym + x];
                    }
                    if (g.dims == 3) {
                        const int plane = g.Lx * g.Ly;
                        const int rzp = g.Lx * y + plane * (z + 1 == Lz ? 0 : z + 1);
                        const int rzm = g.Lx * y + plane * (z == 0 ? Lz - 1 : z - 1);
                        h += HASJ ? Js[2 * N + i] * s[rzp + x] + Js[2 * N + rzm + x] * s[rzm + x]
                                  : s[rzp + x] + s[rzm + x];
                    }
                    const int si = s[i];
                    const uint32_t byte = byte_of(blk, (uint32_t)k);
                    if (a.rule == 0) {
                        const int dE = 2 * si * h;
                        bool acc = dE <= 0;
                        if (!acc) acc = below_lazy(byte, a.tab.met[dE >> 2], a.seed_lo, a.seed_hi, (uint32_t)j, rep,
                                                   (uint32_t)sweep, w3lo);
                        if (acc) s[i] = (int8_t)-si;
                    } else {
                        const bool up = below_lazy(byte, a.tab.hb[h + 6], a.seed_lo, a.seed_hi, (uint32_t)j, rep,
                                                   (uint32_t)sweep, w3lo);
                        s[i] = up ? (int8_t)1 : (int8_t)-1;
                    }
                    if (++m == hx) {
                        m = 0;
                        ++row;
                    }
                }
            }
            __syncthreads();
        }
        if (a.EM) {
            // E = -sum_i s_i sum_d J_d(i) s_{i + e_d}, M = sum_i s_i
            long long e = 0, mm = 0;
            for (int i = tid; i < N; i += nt) {
                const int x = i % g.Lx, r = i / g.Lx, y = r % g.Ly, z = r / g.Ly;
                const int si = s[i];
                const int xp = x + 1 == g.Lx ? 0 : x + 1;
                const int iy = x + g.Lx * ((y + 1 == g.Ly ? 0 : y + 1) + g.Ly * z);
                int b = (HASJ ? Js[i] : 1) * s[xp + g.Lx * r] + (HASJ ? Js[N + i] : 1) * s[iy];
                if (g.dims == 3) {
                    const int iz = x + g.Lx * (y + g.Ly * (z + 1 == Lz ? 0 : z + 1));
                    b += (HASJ ? Js[2 * N + i] : 1) * s[iz];
                }
                e -= si * b;
                mm += si;
            }
            e = wave_sum(e);
            mm = wave_sum(mm);
            if ((tid & 63) == 0) {
                red[0][tid >> 6] = e;
                red[1][tid >> 6] = mm;
            }
            __syncthreads();
            if (tid == 0) {
                long long te = 0, tm = 0;
                for (int w = 0; w < (nt >> 6); ++w) {
                    te += red[0][w];
                    tm += red[1][w];
                }
                a.EM[t * a.em_stride + 2 * l] = te;
                a.EM[t * a.em_stride + 2 * l + 1] = tm;
            }
            __syncthreads();
        }
    }
    int8_t *dst = a.spins + (int64_t)l * N;
    for (int i = tid; i < N; i += nt) dst[i] = s[i];
}

size_t small_lds_bytes(const Geom &g, bool hasJ)
{
    return (size_t)((g.N + 15) & ~(int64_t)15) + (hasJ ? (size_t)g.dims * (size_t)g.N : 0);
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
    static bool attr[2] = {false, false};
    if (!attr[hj ? 1 : 0]) {
        const hipError_t e = hipFuncSetAttribute(hj ? (const void *)k_small<true> : (const void *)k_small<false>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
        if (e != hipSuccess) return e;
        attr[hj ? 1 : 0] = true;
    }
    if (hj) hipLaunchKernelGGL(k_small<true>, dim3((unsigned)c.g.count), dim3(1024), lds, s, a);
    else hipLaunchKernelGGL(k_small<false>, dim3((unsigned)c.g.count), dim3(1024), lds, s, a);
    return hipGetLastError();
}

}  // namespace mcs
