// k_basic.hip -- initialisation, couplings, measurement and the generic
// (any even geometry) checkerboard half-sweep kernels for int8 and 64-lane
// multi-spin-coded lattices.
#include "common.hpp"

namespace mcs {

// ----------------------------------------------------------------------------
__global__ void k_fill_i64(int64_t *p, int64_t n, int64_t v)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_i64(int64_t *p, int64_t n, int64_t value, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_i64, dim3((unsigned)blocks), dim3(256), 0, s, p, n, value);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Hot start: site i of replica r is +1 iff byte (i mod 16) of
// Philox(i/16, r, 0, TAG_INIT) < 128.  One thread per 16 consecutive sites.
__global__ void k_init_int8(int8_t *spins, int64_t N, int start, uint32_t k0, uint32_t k1, uint32_t replica0)
{
    const int l = blockIdx.y;
    const int64_t g16 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t i0 = g16 * 16;
    if (i0 >= N) return;
    int8_t *s = spins + (int64_t)l * N;
    uint4 b = make_uint4(0, 0, 0, 0);
    if (start) b = philox(make_uint4((uint32_t)g16, replica0 + (uint32_t)l, 0u, ctr_w3(kTagInit, 0, 0)), k0, k1);
    for (int k = 0; k < 16 && i0 + k < N; ++k)
        s[i0 + k] = (!start || byte_of(b, (uint32_t)k) < 128u) ? (int8_t)1 : (int8_t)-1;
}

hipError_t launch_init_int8(const Geom &g, int8_t *spins, int start, uint64_t seed, uint32_t replica0,
                            hipStream_t s)
{
    const int64_t groups = (g.N + 15) / 16;
    dim3 grid((unsigned)((groups + 255) / 256), (unsigned)g.count);
    hipLaunchKernelGGL(k_init_int8, grid, dim3(256), 0, s, spins, g.N, start, (uint32_t)seed,
                       (uint32_t)(seed >> 32), replica0);
    return hipGetLastError();
}

// MSC64: bit b of word i of word-lattice l is (spin of replica r0 + 64 l + b at
// site i) == -1.  One thread per 16 sites, one Philox block per lane.
__global__ void k_init_msc64(uint64_t *words, int64_t N, int start, uint32_t k0, uint32_t k1, uint32_t replica0)
{
    const int l = blockIdx.y;
    const int64_t g16 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t i0 = g16 * 16;
    if (i0 >= N) return;
    uint64_t w[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) w[k] = 0;
    if (start) {
        for (int b = 0; b < 64; ++b) {
            const uint4 blk = philox(make_uint4((uint32_t)g16, replica0 + 64u * (uint32_t)l + (uint32_t)b, 0u,
                                                ctr_w3(kTagInit, 0, 0)),
                                     k0, k1);
#pragma unroll
            for (int k = 0; k < 16; ++k)
                w[k] |= (uint64_t)(byte_of(blk, (uint32_t)k) >= 128u) << b;
        }
    }
    uint64_t *out = words + (int64_t)l * N;
#pragma unroll
    for (int k = 0; k < 16; ++k)
        if (i0 + k < N) out[i0 + k] = w[k];
}

hipError_t launch_init_msc64(const Geom &g, uint64_t *words, int start, uint64_t seed, uint32_t replica0,
                             hipStream_t s)
{
    const int64_t groups = (g.N + 15) / 16;
    dim3 grid((unsigned)((groups + 63) / 64), (unsigned)g.count);
    hipLaunchKernelGGL(k_init_msc64, grid, dim3(64), 0, s, words, g.N, start, (uint32_t)seed,
                       (uint32_t)(seed >> 32), replica0);
    return hipGetLastError();
}

// Couplings: flat bond index b = d N + i; +1 iff byte (b mod 16) of
// Philox(b/16, 0, 0, TAG_COUPLING) < 128.
__global__ void k_couplings(int8_t *J, int64_t nb, uint32_t k0, uint32_t k1)
{
    const int64_t g16 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t b0 = g16 * 16;
    if (b0 >= nb) return;
    const uint4 blk = philox(make_uint4((uint32_t)g16, 0u, 0u, ctr_w3(kTagCoupling, 0, 0)), k0, k1);
    for (int k = 0; k < 16 && b0 + k < nb; ++k) J[b0 + k] = byte_of(blk, (uint32_t)k) < 128u ? 1 : -1;
}

hipError_t launch_couplings(const Geom &g, int8_t *J, uint64_t seed, hipStream_t s)
{
    const int64_t nb = (int64_t)g.dims * g.N;
    const int64_t groups = (nb + 15) / 16;
    hipLaunchKernelGGL(k_couplings, dim3((unsigned)((groups + 255) / 256)), dim3(256), 0, s, J, nb,
                       (uint32_t)seed, (uint32_t)(seed >> 32));
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Geometry helpers for the generic kernels.
struct Coord {
    int x, y, z;
};

__device__ __forceinline__ int64_t site_of(const Geom &g, int x, int y, int z)
{
    return (int64_t)x + (int64_t)g.Lx * ((int64_t)y + (int64_t)g.Ly * z);
}

// Site of colour c with same-colour index j: row ry = j / (Lx/2) holds Lx/2
// sites of each colour; x = 2 (j mod Lx/2) + parity.
__device__ __forceinline__ Coord coord_of(const Geom &g, int64_t j, int c)
{
    const int hx = g.Lx >> 1;
    const int64_t ry = j / hx;
    const int m = (int)(j - ry * hx);
    Coord q;
    q.y = (int)(ry % g.Ly);
    q.z = (int)(ry / g.Ly);
    q.x = 2 * m + ((c + q.y + q.z) & 1);
    return q;
}

// Neighbour sites and the bonds to them (bond index d N + i of its left end).
__device__ __forceinline__ int neighbours(const Geom &g, Coord q, int64_t *nb, int64_t *bd)
{
    const int xp = q.x + 1 == g.Lx ? 0 : q.x + 1, xm = q.x == 0 ? g.Lx - 1 : q.x - 1;
    const int yp = q.y + 1 == g.Ly ? 0 : q.y + 1, ym = q.y == 0 ? g.Ly - 1 : q.y - 1;
    const int64_t i = site_of(g, q.x, q.y, q.z);
    nb[0] = site_of(g, xp, q.y, q.z); bd[0] = i;
    nb[1] = site_of(g, xm, q.y, q.z); bd[1] = nb[1];
    nb[2] = site_of(g, q.x, yp, q.z); bd[2] = g.N + i;
    nb[3] = site_of(g, q.x, ym, q.z); bd[3] = g.N + nb[3];
    if (g.dims == 3) {
        const int zp = q.z + 1 == g.Lz ? 0 : q.z + 1, zm = q.z == 0 ? g.Lz - 1 : q.z - 1;
        nb[4] = site_of(g, q.x, q.y, zp); bd[4] = 2 * g.N + i;
        nb[5] = site_of(g, q.x, q.y, zm); bd[5] = 2 * g.N + nb[5];
        return 6;
    }
    return 4;
}

__device__ __forceinline__ bool lazy_below(uint32_t byte, uint32_t top, uint32_t low, uint32_t k0, uint32_t k1,
                                           uint32_t j, uint32_t replica, uint32_t sweep_lo, uint32_t w3lo)
{
    if (byte != top) return byte < top;
    const uint4 lo = philox(make_uint4(j, replica, sweep_lo, w3lo), k0, k1);
    return (lo.x & 0xFFFFFFu) < low;
}

// The call's thresholds copied to LDS (entries 0..3 Metropolis by dE / 4,
// 4..16 heat-bath by h + 6): indexing the argument block by a per-lane value
// would be a memory load per site.  Every thread of the block must call this
// (it ends with a barrier).
__device__ __forceinline__ void stage_tables(const SweepTables &t, uint32_t *top, uint32_t *low)
{
    if (threadIdx.x < 17) {
        const Thr v = threadIdx.x < 4 ? t.met[threadIdx.x] : t.hb[threadIdx.x - 4];
        top[threadIdx.x] = v.top;
        low[threadIdx.x] = v.low;
    }
    __syncthreads();
}

// ----------------------------------------------------------------------------
// Generic int8 half-sweep: one thread per 16 consecutive same-colour indices.
__global__ void k_phase_int8(SweepCall c, int8_t *spins, uint32_t sweep_lo, uint32_t w3, uint32_t w3lo, int phase)
{
    const Geom &g = c.g;
    const int l = blockIdx.y;
    const int64_t half = g.N >> 1;
    const int64_t t16 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t j0 = t16 * 16;
    __shared__ uint32_t ttop[17], tlow[17];
    stage_tables(c.tab, ttop, tlow);
    if (j0 >= half) return;
    int8_t *s = spins + (int64_t)l * g.N;
    const uint32_t rep = c.replica0 + (uint32_t)l;
    const uint4 blk = philox(make_uint4((uint32_t)t16, rep, sweep_lo, w3), c.seed_lo, c.seed_hi);
    for (int k = 0; k < 16 && j0 + k < half; ++k) {
        const int64_t j = j0 + k;
        const Coord q = coord_of(g, j, phase);
        const int64_t i = site_of(g, q.x, q.y, q.z);
        int64_t nb[6], bd[6];
        const int nn = neighbours(g, q, nb, bd);
        int h = 0;
        for (int d = 0; d < nn; ++d) h += (c.J ? (int)c.J[bd[d]] : 1) * (int)s[nb[d]];
        const int si = s[i];
        const uint32_t byte = byte_of(blk, (uint32_t)k);
        int8_t out;
        if (c.rule == 0) {
            const int dE = 2 * si * h;
            bool acc = dE <= 0;
            if (!acc) acc = lazy_below(byte, ttop[dE >> 2], tlow[dE >> 2], c.seed_lo, c.seed_hi, (uint32_t)j, rep, sweep_lo, w3lo);
            out = acc ? (int8_t)-si : (int8_t)si;
        } else {
            const bool up = lazy_below(byte, ttop[h + 10], tlow[h + 10], c.seed_lo, c.seed_hi, (uint32_t)j, rep, sweep_lo, w3lo);
            out = up ? (int8_t)1 : (int8_t)-1;
        }
        s[i] = out;
    }
}

hipError_t launch_phase_int8(const SweepCall &c, int8_t *spins, uint64_t sweep, int phase, hipStream_t s)
{
    const int64_t half = c.g.N >> 1;
    const int64_t groups = (half + 15) / 16;
    dim3 grid((unsigned)((groups + 127) / 128), (unsigned)c.g.count);
    hipLaunchKernelGGL(k_phase_int8, grid, dim3(128), 0, s, c, spins, (uint32_t)sweep,
                       ctr_w3(kTagSweep, (uint32_t)phase, sweep), ctr_w3(kTagSweepLo, (uint32_t)phase, sweep), phase);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Generic MSC64 half-sweep.  Per site: unsatisfied-bond masks
// u_d = w_i ^ w_nbr ^ (J < 0 ? ~0 : 0); their per-lane count a (0..6) is kept
// bit-sliced in three words; a lane's energy change is dE = 2 (z - 2 a) and its
// local field h = s_i (z - 2 a).  One thread per 16 same-colour sites, one
// Philox block per lane (replica r0 + 64 l + b).
__device__ __forceinline__ void add_bit(uint64_t &a0, uint64_t &a1, uint64_t &a2, uint64_t u)
{
    const uint64_t c0 = a0 & u;
    a0 ^= u;
    const uint64_t c1 = a1 & c0;
    a1 ^= c0;
    a2 |= c1;
}

__global__ void k_phase_msc64(SweepCall c, uint64_t *words, uint32_t sweep_lo, uint32_t w3, uint32_t w3lo, int phase)
{
    const Geom &g = c.g;
    const int l = blockIdx.y;
    const int64_t half = g.N >> 1;
    const int64_t t16 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t j0 = t16 * 16;
    __shared__ uint32_t ttop[17], tlow[17];
    stage_tables(c.tab, ttop, tlow);
    if (j0 >= half) return;
    uint64_t *w = words + (int64_t)l * g.N;
    const int z = 2 * g.dims;
    uint64_t A0[16], A1[16], A2[16], S[16], F[16];
    int64_t idx[16];
    const int cnt = (int)((half - j0) < 16 ? (half - j0) : 16);
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        A0[k] = A1[k] = A2[k] = S[k] = F[k] = 0;
        idx[k] = -1;
        if (k < cnt) {
            const Coord q = coord_of(g, j0 + k, phase);
            const int64_t i = site_of(g, q.x, q.y, q.z);
            int64_t nb[6], bd[6];
            const int nn = neighbours(g, q, nb, bd);
            const uint64_t wi = w[i];
            for (int d = 0; d < nn; ++d) {
                const uint64_t jm = (c.J && c.J[bd[d]] < 0) ? ~0ull : 0ull;
                add_bit(A0[k], A1[k], A2[k], wi ^ w[nb[d]] ^ jm);
            }
            S[k] = wi;
            idx[k] = i;
        }
    }
    for (int b = 0; b < 64; ++b) {
        const uint32_t rep = c.replica0 + 64u * (uint32_t)l + (uint32_t)b;
        const uint4 blk = philox(make_uint4((uint32_t)t16, rep, sweep_lo, w3), c.seed_lo, c.seed_hi);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k >= cnt) continue;
            const int a = (int)((A0[k] >> b) & 1) | ((int)((A1[k] >> b) & 1) << 1) | ((int)((A2[k] >> b) & 1) << 2);
            const uint32_t byte = byte_of(blk, (uint32_t)k);
            const uint32_t j = (uint32_t)(j0 + k);
            bool flip;
            if (c.rule == 0) {
                const int dE = 2 * (z - 2 * a);
                flip = dE <= 0 || lazy_below(byte, ttop[dE > 0 ? dE >> 2 : 0], tlow[dE > 0 ? dE >> 2 : 0], c.seed_lo, c.seed_hi, j, rep, sweep_lo, w3lo);
            } else {
                const int si = ((S[k] >> b) & 1) ? -1 : 1;
                const int h = si * (z - 2 * a);
                const bool up = lazy_below(byte, ttop[h + 10], tlow[h + 10], c.seed_lo, c.seed_hi, j, rep, sweep_lo, w3lo);
                flip = up != (si > 0);
            }
            F[k] |= (uint64_t)flip << b;
        }
    }
#pragma unroll
    for (int k = 0; k < 16; ++k)
        if (k < cnt) w[idx[k]] = S[k] ^ F[k];
}

hipError_t launch_phase_msc64(const SweepCall &c, uint64_t *words, uint64_t sweep, int phase, hipStream_t s)
{
    const int64_t half = c.g.N >> 1;
    const int64_t groups = (half + 15) / 16;
    dim3 grid((unsigned)((groups + 63) / 64), (unsigned)c.g.count);
    hipLaunchKernelGGL(k_phase_msc64, grid, dim3(64), 0, s, c, words, (uint32_t)sweep,
                       ctr_w3(kTagSweep, (uint32_t)phase, sweep), ctr_w3(kTagSweepLo, (uint32_t)phase, sweep), phase);
    return hipGetLastError();
}

// ----------------------------------------------------------------------------
// Measurement.  int8: E = -sum_i s_i sum_{d} J_d(i) s_{i+e_d}, M = sum s_i,
// block partial sums then one int64 atomic per block and quantity.
__global__ void k_measure_int8(Geom g, const int8_t *spins, const int8_t *J, int64_t *EM)
{
    const int l = blockIdx.y;
    const int8_t *s = spins + (int64_t)l * g.N;
    long long e = 0, m = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < g.N; i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % g.Lx);
        const int64_t r = i / g.Lx;
        const int y = (int)(r % g.Ly);
        const int zc = (int)(r / g.Ly);
        const int si = s[i];
        const int64_t nx = site_of(g, x + 1 == g.Lx ? 0 : x + 1, y, zc);
        const int64_t ny = site_of(g, x, y + 1 == g.Ly ? 0 : y + 1, zc);
        int acc = (J ? J[i] : 1) * s[nx] + (J ? J[g.N + i] : 1) * s[ny];
        if (g.dims == 3) {
            const int64_t nz = site_of(g, x, y, zc + 1 == g.Lz ? 0 : zc + 1);
            acc += (J ? J[2 * g.N + i] : 1) * s[nz];
        }
        e -= si * acc;
        m += si;
    }
    __shared__ long long red[2][16];
    e = wave_sum(e);
    m = wave_sum(m);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) { red[0][wid] = e; red[1][wid] = m; }
    __syncthreads();
    if (threadIdx.x == 0) {
        long long te = 0, tm = 0;
        for (int k = 0; k < (int)(blockDim.x >> 6); ++k) { te += red[0][k]; tm += red[1][k]; }
        atomicAdd((unsigned long long *)&EM[2 * l], (unsigned long long)te);
        atomicAdd((unsigned long long *)&EM[2 * l + 1], (unsigned long long)tm);
    }
}

hipError_t launch_measure_int8(const Geom &g, const int8_t *spins, const int8_t *J, int64_t *EM, hipStream_t s)
{
    hipError_t e = launch_fill_i64(EM, 2 * (int64_t)g.count, 0, s);
    if (e != hipSuccess) return e;
    int64_t blocks = (g.N + 1023) / 1024;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_measure_int8, dim3((unsigned)blocks, (unsigned)g.count), dim3(256), 0, s, g, spins, J, EM);
    return hipGetLastError();
}

// MSC64: thread = lane b of a 64-thread block; every thread reads the same
// words and counts its own bit: unsatisfied bonds n_u and down spins n_d give
// E_b = -(bonds - 2 n_u), M_b = N - 2 n_d.
__global__ void k_measure_msc64(Geom g, const uint64_t *words, const int8_t *J, int64_t *EM)
{
    const int l = blockIdx.y;
    const int b = threadIdx.x;
    const uint64_t *w = words + (int64_t)l * g.N;
    int64_t chunk = (g.N + gridDim.x - 1) / gridDim.x;
    const int64_t i0 = blockIdx.x * chunk;
    int64_t i1 = i0 + chunk;
    if (i1 > g.N) i1 = g.N;
    long long nu = 0, nd = 0;
    for (int64_t i = i0; i < i1; ++i) {
        const int x = (int)(i % g.Lx);
        const int64_t r = i / g.Lx;
        const int y = (int)(r % g.Ly);
        const int zc = (int)(r / g.Ly);
        const uint64_t wi = w[i];
        uint64_t u = wi ^ w[site_of(g, x + 1 == g.Lx ? 0 : x + 1, y, zc)] ^ ((J && J[i] < 0) ? ~0ull : 0ull);
        nu += (u >> b) & 1;
        u = wi ^ w[site_of(g, x, y + 1 == g.Ly ? 0 : y + 1, zc)] ^ ((J && J[g.N + i] < 0) ? ~0ull : 0ull);
        nu += (u >> b) & 1;
        if (g.dims == 3) {
            u = wi ^ w[site_of(g, x, y, zc + 1 == g.Lz ? 0 : zc + 1)] ^ ((J && J[2 * g.N + i] < 0) ? ~0ull : 0ull);
            nu += (u >> b) & 1;
        }
        nd += (wi >> b) & 1;
    }
    const long long nbonds = (long long)(i1 - i0) * g.dims;
    const long long e = -(nbonds - 2 * nu);
    const long long m = (long long)(i1 - i0) - 2 * nd;
    atomicAdd((unsigned long long *)&EM[2 * (64 * (int64_t)l + b)], (unsigned long long)e);
    atomicAdd((unsigned long long *)&EM[2 * (64 * (int64_t)l + b) + 1], (unsigned long long)m);
}

hipError_t launch_measure_msc64(const Geom &g, const uint64_t *words, const int8_t *J, int64_t *EM, hipStream_t s)
{
    hipError_t e = launch_fill_i64(EM, 2 * 64 * (int64_t)g.count, 0, s);
    if (e != hipSuccess) return e;
    int64_t blocks = (g.N + 4095) / 4096;
    if (blocks > 2048) blocks = 2048;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_measure_msc64, dim3((unsigned)blocks, (unsigned)g.count), dim3(64), 0, s, g, words, J, EM);
    return hipGetLastError();
}

}  // namespace mcs
