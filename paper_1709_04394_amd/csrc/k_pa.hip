// k_pa.hip -- population annealing (Sec. "Population annealing", Eq. Q) for
// populations of 2D L x L ferromagnets, several populations (of different L)
// per launch.
//
// One annealing step is five kernels (kernel boundaries order the steps; no
// device-wide fences):
//  k_pa_scan      one wave per block of 64 replicas: weights w_j = exp(-dbeta
//                 (E_j + 2N)) from the step's host table, the block's 64-wide
//                 doubling scan x (the first level of the fixed-order FP64
//                 prefix sum) and its running maximum;
//  k_pa_blocks    one workgroup per population: the block totals' doubling
//                 scans, group totals in sequence, each block's offset
//                 G_q + B_b, C_total, and the running maximum of C at each
//                 block's end;
//  k_pa_resample  one thread per new slot: u from Philox, t = u C_total, parent =
//                 first j with Cmax_j > t, found block by block (binary search
//                 over the block-end maxima in LDS, then the block's own running
//                 maxima plus its offset), integer copy counts;
//  k_pa_place     one workgroup per chunk of 2048 parents: parents in index
//                 order fill slots [P_j, P_j + n_j);
//  k_pa_sweep     gathers each slot's parent into LDS (bit-packed, split by x
//                 parity, periodic in both directions, so a whole lattice lives
//                 in one workgroup and needs no halo), runs theta checkerboard
//                 Metropolis sweeps, and writes the lattice, its energy and the
//                 energy histogram.
// Within a block the sums are those of the whole-array definition (C_i =
// x_i + (G_q + B_b)), and rounding to nearest is monotone, so the running
// maximum of C inside block b is fl(runmax(x) + (G_q + B_b)): the search needs
// no materialised C.
#include "internal.hpp"
#include "lds_lattice.hpp"
#include "pa.hpp"

namespace mcs {

// ----------------------------------------------------------------------------
// Inclusive scan of one wave's 64 doubles in the doubling order
// x_i <- x_i + x_{i-d}, d = 1, 2, ..., 32, from the values before each step.
__device__ __forceinline__ double wave_scan_f64(double v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double t = __shfl_up(v, (unsigned)d, 64);
        if (lane >= d) v = v + t;
    }
    return v;
}

// Inclusive running maximum over one wave (exact in any order).
__device__ __forceinline__ double wave_max_scan_f64(double v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double t = __shfl_up(v, (unsigned)d, 64);
        if (lane >= d) v = fmax(v, t);
    }
    return v;
}

__device__ __forceinline__ int wave_scan_i32(int v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int t = __shfl_up(v, (unsigned)d, 64);
        if (lane >= d) v += t;
    }
    return v;
}

// Block-level step of the scan by the last workgroup of a population (256
// threads): inclusive doubling scans of the block totals within groups of 64
// blocks, group totals in sequence, the offsets G_q + B_b, C_total, and the
// running maximum of C over the block ends.
__device__ void pa_block_level(const PaPop &P, const PaStep &st, int nb)
{
    __shared__ double sB[kPaMaxChunks];  // block totals, scanned within their group
    __shared__ double sM[kPaMaxChunks];  // maximum of C in each block, then running maximum
    __shared__ double G[kPaMaxChunks / 64], GM[kPaMaxChunks / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const int ng = (nb + 63) / 64;
    const double *btot = P.blk, *bxm = P.blk + nb;
    double *boff = P.blk + 2 * nb, *bmax = P.blk + 3 * nb;
    for (int q = wave; q < ng; q += nw) {
        const int b = 64 * q + lane;
        double v = b < nb ? btot[b] : 0.0;
        v = wave_scan_f64(v, lane);
        if (b < nb) sB[b] = v;
    }
    __syncthreads();
    if (tid == 0) {
        double g = 0.0;
        G[0] = 0.0;
        for (int q = 1; q < ng; ++q) {
            g = g + sB[64 * (q - 1) + 63];
            G[q] = g;
        }
    }
    __syncthreads();
    for (int b = tid; b < nb; b += blockDim.x) {
        const int q = b / 64;
        const double off = G[q] + ((b % 64 == 0) ? 0.0 : sB[b - 1]);
        boff[b] = off;
        sM[b] = bxm[b] + off;
        // the last block's recorded total is x_{R-1}
        if (b == nb - 1) P.ctot[st.ctot_idx] = btot[b] + off;
    }
    __syncthreads();
    for (int q = wave; q < ng; q += nw) {
        const int b = 64 * q + lane;
        double v = b < nb ? sM[b] : -1.0;
        v = wave_max_scan_f64(v, lane);
        if (b < nb) sM[b] = v;
    }
    __syncthreads();
    if (tid == 0) {
        double m = -1.0;
        for (int q = 0; q < ng; ++q) {
            GM[q] = m;
            m = fmax(m, sM[64 * q + min(63, nb - 1 - 64 * q)]);
        }
    }
    __syncthreads();
    for (int b = tid; b < nb; b += blockDim.x) bmax[b] = fmax(GM[b / 64], sM[b]);
}

__global__ __launch_bounds__(256) void k_pa_scan(PaStep st)
{
    const PaPop &P = st.pop[blockIdx.y];
    const int R = P.R, N = P.N, nb = (R + 63) / 64;
    const int lane = threadIdx.x & 63, b = (int)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    if (b < nb) {
        const int i = 64 * b + lane;
        double v = 0.0;
        if (i < R) {
            v = st.wtab[(P.E[i] + 2 * N) / 4];
            P.n[i] = 0;
        }
        // lanes past R add zeros, which leaves the valid lanes' sums as the
        // whole-array definition has them (a lane's sum only reads lower
        // lanes), but not the padding lanes' own sums: those are kept out of
        // the maximum, and a partial block is recorded at its last valid lane
        const double x = wave_scan_f64(v, lane);
        const double m = wave_max_scan_f64(i < R ? x : -1.0, lane);
        if (i < R) P.rmx[i] = m;
        if (lane == min(63, R - 1 - 64 * b)) {
            P.blk[b] = x;       // block total (x_{R-1} for a partial last block)
            P.blk[nb + b] = m;  // largest x of the block
        }
    }
}

__global__ __launch_bounds__(256) void k_pa_blocks(PaStep st)
{
    const PaPop &P = st.pop[blockIdx.y];
    pa_block_level(P, st, (P.R + 63) / 64);
}

// Copy placement, one workgroup (256 threads) per chunk of 2048 parents: the
// exclusive scan of the copy numbers n_j in index order gives P_j; slot s
// then holds the largest j with n_j > 0 and P_j <= s.  A chunk's slots are
// [P_j0, P_j0 + its copies), j0 its first parent, and the first of them is
// the first slot of the chunk's first parent with copies, so chunks are
// independent once each has summed the counts before it.  Each parent with
// copies marks its first slot in an LDS window of slots, a running maximum
// over the window fills the rest, and the window is stored contiguously.
constexpr int kPlacePer = 8;      // copy numbers per thread
constexpr int kPlaceWin = 4096;   // slots per LDS window
constexpr int kPlaceThreads = 256;
constexpr int kPlaceChunk = kPlacePer * kPlaceThreads;

__device__ void place_copies(const PaPop &P, int chunk)
{
    const int R = P.R, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int nt = kPlaceThreads, nw = kPlaceThreads / 64, per = kPlaceWin / kPlaceThreads;
    __shared__ int win[kPlaceWin];
    __shared__ int wsum[nw], wmax[nw];
    __shared__ int carry_par;
    const int base = chunk * kPlaceChunk;
    // slots before this chunk: the copies of all earlier parents, read as
    // int4 in batches of eight per thread so that the loads overlap (base is
    // a multiple of 4)
    int before = 0;
    const int4 *n4 = (const int4 *)P.n;
    const int nb4 = base / 4;
    for (int j0 = tid; j0 < nb4; j0 += nt * 8) {
        int4 q[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) q[u] = j0 + u * nt < nb4 ? n4[j0 + u * nt] : make_int4(0, 0, 0, 0);
#pragma unroll
        for (int u = 0; u < 8; ++u) before += q[u].x + q[u].y + q[u].z + q[u].w;
    }
    before = wave_scan_i32(before, lane);
    if (lane == 63) wsum[wave] = before;
    if (tid == 0) carry_par = -1;
    __syncthreads();
    int p0 = 0;
    for (int w = 0; w < nw; ++w) p0 += wsum[w];
    __syncthreads();
    const int i0 = base + tid * kPlacePer;
    int c[kPlacePer];
    int s = 0;
    // the counts of the previous kernel; a full group is 32-byte aligned
    if (i0 + kPlacePer <= R) {
        const int4 *v = (const int4 *)(P.n + i0);
#pragma unroll
        for (int k = 0; k < kPlacePer / 4; ++k) {
            const int4 q = v[k];
            c[4 * k] = q.x;
            c[4 * k + 1] = q.y;
            c[4 * k + 2] = q.z;
            c[4 * k + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kPlacePer; ++k) c[k] = i0 + k < R ? P.n[i0 + k] : 0;
    }
#pragma unroll
    for (int k = 0; k < kPlacePer; ++k) s += c[k];
    const int incl = wave_scan_i32(s, lane);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int pre = 0, total = 0;
    for (int w = 0; w < nw; ++w) {
        if (w < wave) pre += wsum[w];
        total += wsum[w];
    }
    const int first = p0 + pre + incl - s;  // first slot of this thread's parents
    for (int w0 = p0; w0 < p0 + total; w0 += kPlaceWin) {
        const int wn = min(kPlaceWin, p0 + total - w0);
        for (int i = tid; i < kPlaceWin; i += nt) win[i] = -1;
        __syncthreads();
        int pos = first;
#pragma unroll
        for (int k = 0; k < kPlacePer; ++k) {
            if (c[k] > 0 && pos >= w0 && pos < w0 + wn) win[pos - w0] = i0 + k;
            pos += c[k];
        }
        __syncthreads();
        // running maximum over the window: per thread, then across lanes,
        // waves and windows
        int r[per];
        int m = -1;
#pragma unroll
        for (int i = 0; i < per; ++i) {
            m = max(m, win[tid * per + i]);
            r[i] = m;
        }
        int im = m;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int t = __shfl_up(im, (unsigned)d, 64);
            if (lane >= d) im = max(im, t);
        }
        if (lane == 63) wmax[wave] = im;
        int bef = __shfl_up(im, 1u, 64);
        if (lane == 0) bef = -1;
        __syncthreads();
        bef = max(bef, carry_par);
        for (int w = 0; w < wave; ++w) bef = max(bef, wmax[w]);
#pragma unroll
        for (int i = 0; i < per; ++i) win[tid * per + i] = max(bef, r[i]);
        __syncthreads();
        for (int i = tid; i < wn; i += nt) P.newparent[w0 + i] = win[i];
        if (tid == 0) carry_par = win[wn - 1];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_pa_resample(PaStep st)
{
    const int p = blockIdx.y;
    const PaPop &P = st.pop[p];
    const int R = P.R, nb = (R + 63) / 64;
    __shared__ double sbm[kPaMaxChunks];
    const double *boff = P.blk + 2 * nb;
    for (int b = threadIdx.x; b < nb; b += blockDim.x) sbm[b] = P.blk[3 * nb + b];
    const double ct = P.ctot[st.ctot_idx];
    __syncthreads();
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < R) {
        const uint4 r = philox(make_uint4((uint32_t)k, (uint32_t)p, st.step, ctr_w3(kTagResample, 0, st.step)),
                               st.seed_lo, st.seed_hi);
        const uint64_t a = r.x >> 5, b = r.y >> 6;
        const double u = (double)(a * 67108864ull + b) * (1.0 / 9007199254740992.0);
        const double t = u * ct;
        // the first block whose running maximum of C exceeds t
        int lo = 0, hi = nb - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (sbm[mid] > t) hi = mid;
            else lo = mid + 1;
        }
        int parent = R - 1;  // no C exceeds t (t rounded up to C_total)
        if (sbm[lo] > t) {
            // inside block lo every earlier C is <= t, so the parent is the
            // first j with fl(runmax(x)_j + offset) > t; runmax is monotone:
            // first the group of 8, then the element
            const double off = boff[lo];
            const int j0 = 64 * lo, jn = min(64, R - j0);
            const double *rm = P.rmx + j0;
            double ge[8];
#pragma unroll
            for (int g = 0; g < 8; ++g) ge[g] = rm[min(8 * g + 7, jn - 1)];
            int g = 7;
#pragma unroll
            for (int q = 7; q >= 0; --q)
                if (ge[q] + off > t) g = q;
            double e[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) e[q] = rm[min(8 * g + q, jn - 1)];
            int jj = min(8 * g + 7, jn - 1);
#pragma unroll
            for (int q = 7; q >= 0; --q)
                if (8 * g + q < jn && e[q] + off > t) jj = 8 * g + q;
            parent = j0 + jj;
        }
        atomicAdd(&P.n[parent], 1);
    }
}

__global__ __launch_bounds__(kPlaceThreads) void k_pa_place(PaStep st)
{
    const PaPop &P = st.pop[blockIdx.y];
    if ((int)blockIdx.x * kPlaceChunk >= P.R) return;
    place_copies(P, blockIdx.x);
}

// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pa_sweep(PaStep st)
{
    extern __shared__ uint32_t lds[];
    __shared__ int e_lat[64];
    __shared__ LdsTieQueue tq;
    int p = 0;
    while (p + 1 < st.npop && (int)blockIdx.x >= st.pop[p + 1].blk0) ++p;
    const PaPop &P = st.pop[p];
    LdsLattices a;
    a.L = P.L;
    a.N = P.N;
    a.Wb = P.Wb;
    a.nwr = P.nwr;
    const int s0 = ((int)blockIdx.x - P.blk0) * P.G;
    a.ng = min(P.G, P.R - s0);
    a.rep0 = (uint32_t)p * (uint32_t)P.R + (uint32_t)s0;
    a.sweep0 = (uint64_t)(st.step - 1) * (uint64_t)st.theta;
    a.theta = st.theta;
    a.seed_lo = st.seed_lo;
    a.seed_hi = st.seed_hi;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int L = a.L, N = a.N, nwr = a.nwr;
    if (tid < 64) e_lat[tid] = 0;

    // ---- gather the parents and pack
    const int tasks_ld = a.ng * L * nwr;
    for (int t = tid; t < tasks_ld; t += nt) {
        const int g = t / (L * nwr), rem = t - g * L * nwr, r = rem / nwr, w = rem - r * nwr;
        const int slot = s0 + g;
        const int parent = st.identity ? slot : P.newparent[slot];
        pack_lattice_rows(lds, a, g, P.cur + (int64_t)parent * N, r, w);
    }
    __syncthreads();

    sweep_lds_lattices<false>(lds, a, st.t4, st.t8, nullptr, nullptr, tq, e_lat);

    if (tid < a.ng) {
        const int slot = s0 + tid;
        const int e = e_lat[tid];
        P.Enew[slot] = e;
        atomicAdd((unsigned long long *)&P.hist[(int64_t)st.hist_idx * (N + 1) + (e + 2 * N) / 4], 1ull);
    }

    // ---- unpack and store the new population
    for (int t = tid; t < tasks_ld; t += nt) {
        const int g = t / (L * nwr), rem = t - g * L * nwr, r = rem / nwr, w = rem - r * nwr;
        unpack_lattice_rows(lds, a, g, P.nxt + (int64_t)(s0 + g) * N, r, w);
    }
}

// ----------------------------------------------------------------------------
hipError_t launch_pa_step(const PaStep &st, int rmax, int sweep_blocks, hipStream_t s)
{
    if (!st.identity) {
        const int nb = (rmax + 63) / 64;
        hipLaunchKernelGGL(k_pa_scan, dim3((nb + 3) / 4, st.npop), dim3(256), 0, s, st);
        hipLaunchKernelGGL(k_pa_blocks, dim3(1, st.npop), dim3(256), 0, s, st);
        hipLaunchKernelGGL(k_pa_resample, dim3((rmax + 255) / 256, st.npop), dim3(256), 0, s, st);
        hipLaunchKernelGGL(k_pa_place, dim3((rmax + kPlaceChunk - 1) / kPlaceChunk, st.npop), dim3(kPlaceThreads), 0,
                           s, st);
    }
    size_t lds = 0;
    for (int p = 0; p < st.npop; ++p) {
        const size_t b = (size_t)st.pop[p].G * 2 * st.pop[p].L * st.pop[p].nwr * 4;
        if (b > lds) lds = b;
    }
    hipLaunchKernelGGL(k_pa_sweep, dim3(sweep_blocks), dim3(256), lds, s, st);
    return hipGetLastError();
}

}  // namespace mcs
