// k_pa.hip -- population annealing (Sec. "Population annealing", Eq. Q) for
// populations of 2D L x L ferromagnets, several populations (of different L)
// per launch.
//
// One annealing step is three kernels:
//  k_pa_scan      one workgroup per population: weights w_j = exp(-dbeta (E_j +
//                 2N)) from the step's host table, the fixed-order FP64 prefix
//                 sum (64-wide doubling scans by wave shuffles, block totals
//                 scanned the same way, group totals in sequence), C_total, and
//                 the running maximum of C used by the parent search;
//  k_pa_resample  one thread per new slot: u from Philox, t = u C_total, parent =
//                 first j with Cmax_j > t (binary search), integer copy counts;
//                 the last workgroup of each population to finish then places
//                 the copies: exclusive integer scan of the counts, copies of
//                 parent j fill slots [P_j, P_j + n_j);
//  k_pa_sweep     gathers each slot's parent into LDS (bit-packed, split by x
//                 parity, periodic in both directions, so a whole lattice lives
//                 in one workgroup and needs no halo), runs theta checkerboard
//                 Metropolis sweeps, and writes the lattice, its energy and the
//                 energy histogram.
// The scan and the placement read all their inputs into registers in batches
// before storing, so their global-memory round trips overlap.
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

constexpr int kScanBatch = 8;  // blocks of 64 a wave holds in registers at once

__global__ __launch_bounds__(1024) void k_pa_scan(PaStep st)
{
    const PaPop &P = st.pop[blockIdx.x];
    const int R = P.R, N = P.N;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const int nb = (R + 63) / 64, ng = (nb + 63) / 64;
    __shared__ double tch[kPaMaxChunks];  // block totals, then their level-1 scan
    __shared__ double bmx[kPaMaxChunks];  // running maximum at each block's end, then scanned per group
    __shared__ double G[64];              // level-2 exclusive group offsets
    __shared__ double GM[64];             // running maximum before each group
    const int32_t *__restrict__ E = P.E;
    double *__restrict__ x = P.x;
    double *__restrict__ cmax = P.cmax;
    const double *__restrict__ wtab = st.wtab;
    for (int i = tid; i < R; i += blockDim.x) P.n[i] = 0;
    // level 0: blocks of 64 in index order; a wave's blocks are b = wave + k nw
    for (int b0 = wave; b0 < nb; b0 += kScanBatch * nw) {
        int e[kScanBatch];
        double v[kScanBatch];
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) {
            const int i = 64 * (b0 + k * nw) + lane;
            e[k] = (b0 + k * nw < nb && i < R) ? E[i] : INT32_MIN;
        }
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) v[k] = e[k] != INT32_MIN ? wtab[(e[k] + 2 * N) / 4] : 0.0;
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) {
            const int b = b0 + k * nw;
            if (b >= nb) break;
            const double s = wave_scan_f64(v[k], lane);
            const int i = 64 * b + lane;
            if (i < R) x[i] = s;
            if (lane == 63) tch[b] = s;
        }
    }
    __syncthreads();
    // level 1: block totals, 64 at a time
    for (int q = wave; q < ng; q += nw) {
        const int b = 64 * q + lane;
        double v = b < nb ? tch[b] : 0.0;
        v = wave_scan_f64(v, lane);
        if (b < nb) tch[b] = v;
    }
    __syncthreads();
    // level 2: group totals one after the other
    if (tid == 0) {
        double g = 0.0;
        G[0] = 0.0;
        for (int q = 1; q < ng; ++q) {
            g = g + tch[64 * (q - 1) + 63];
            G[q] = g;
        }
    }
    __syncthreads();
    // C_i = x_i + (G_q + B_b); C_total = C_{R-1}; running maximum within each block
    for (int b0 = wave; b0 < nb; b0 += kScanBatch * nw) {
        double xv[kScanBatch];
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) {
            const int i = 64 * (b0 + k * nw) + lane;
            xv[k] = (b0 + k * nw < nb && i < R) ? x[i] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) {
            const int b = b0 + k * nw;
            if (b >= nb) break;
            const int i = 64 * b + lane, q = b / 64;
            const double Bb = (b % 64 == 0) ? 0.0 : tch[b - 1];
            double C = -1.0;
            if (i < R) {
                C = xv[k] + (G[q] + Bb);
                if (i == R - 1) P.ctot[st.ctot_idx] = C;
            }
            const double cm = wave_max_scan_f64(C, lane);
            if (i < R) cmax[i] = cm;
            if (lane == 63) bmx[b] = cm;
        }
    }
    __syncthreads();
    // running maximum over the blocks: within groups of 64 blocks by waves,
    // over the groups in sequence
    for (int q = wave; q < ng; q += nw) {
        const int b = 64 * q + lane;
        double v = b < nb ? bmx[b] : -1.0;
        v = wave_max_scan_f64(v, lane);
        if (b < nb) bmx[b] = v;
    }
    __syncthreads();
    if (tid == 0) {
        double m = -1.0;
        for (int q = 0; q < ng; ++q) {
            GM[q] = m;
            m = fmax(m, bmx[64 * q + min(63, nb - 1 - 64 * q)]);
        }
    }
    __syncthreads();
    // cmax_i = max(running maximum within its block, maximum of all blocks before)
    for (int b0 = wave; b0 < nb; b0 += kScanBatch * nw) {
        double cv[kScanBatch];
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) {
            const int i = 64 * (b0 + k * nw) + lane;
            cv[k] = (b0 + k * nw < nb && i < R) ? cmax[i] : 0.0;
        }
#pragma unroll
        for (int k = 0; k < kScanBatch; ++k) {
            const int b = b0 + k * nw;
            if (b >= nb) break;
            const int i = 64 * b + lane, q = b / 64;
            const double before = fmax(GM[q], (b % 64 == 0) ? -1.0 : bmx[b - 1]);
            if (i < R) cmax[i] = fmax(cv[k], before);
        }
    }
}

// Copy placement by the last workgroup of a population: exclusive scan of the
// copy numbers n_j (in index order), then slots [P_j, P_j + n_j) get parent j.
constexpr int kPlacePer = 64;  // counts per thread: R <= 256 * kPlacePer per pass

__device__ void place_copies(const PaPop &P)
{
    const int R = P.R, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nt = blockDim.x;
    __shared__ int wsum[16];
    __shared__ int carry;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < R; base += nt * kPlacePer) {
        const int i0 = base + tid * kPlacePer;
        int c[kPlacePer];
        int s = 0;
        // the counts were added by other workgroups' atomics and are read after
        // the caller's device-scope fence; a full chunk is 16-byte aligned
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
        int off = carry;
        for (int w = 0; w < wave; ++w) off += wsum[w];
        int pos = off + incl - s;
#pragma unroll
        for (int k = 0; k < kPlacePer; ++k) {
            for (int m = 0; m < c[k]; ++m) P.newparent[pos + m] = i0 + k;
            pos += c[k];
        }
        __syncthreads();
        if (tid == nt - 1) carry = pos;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_pa_resample(PaStep st)
{
    const int p = blockIdx.y;
    const PaPop &P = st.pop[p];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < P.R) {
        const uint4 r = philox(make_uint4((uint32_t)k, (uint32_t)p, st.step, ctr_w3(kTagResample, 0, st.step)),
                               st.seed_lo, st.seed_hi);
        const uint64_t a = r.x >> 5, b = r.y >> 6;
        const double u = (double)(a * 67108864ull + b) * (1.0 / 9007199254740992.0);
        const double t = u * P.ctot[st.ctot_idx];
        int lo = 0, hi = P.R - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (P.cmax[mid] > t) hi = mid;
            else lo = mid + 1;
        }
        atomicAdd(&P.n[lo], 1);
    }
    // the last workgroup of this population to finish places the copies
    __shared__ int last;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const int done = atomicAdd(P.done, 1);
        last = done == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    place_copies(P);
    if (threadIdx.x == 0) *P.done = 0;  // ready for the next step
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
        hipLaunchKernelGGL(k_pa_scan, dim3(st.npop), dim3(1024), 0, s, st);
        hipLaunchKernelGGL(k_pa_resample, dim3((rmax + 255) / 256, st.npop), dim3(256), 0, s, st);
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
