// em_slots.hpp -- per-workgroup (E, M) sums of the fused sweep kernels.
//
// A fused launch runs several sweeps on every tile of a lattice; energy and
// magnetisation of a sweep are sums over all tiles.  Instead of same-address
// int64 atomics (every tile of every XCD adding into one pair, which queue at
// the memory side, most of all at the end of a launch), each workgroup stores
// its share of each sweep in a slot of its own, and the first workgroups of
// the next launch add up the previous launch's slots into EM while they load
// their tile; a small kernel adds up the slots of the last launch of a call.
// Integer sums, so the order does not matter and the results are exact.
#pragma once

#include "common.hpp"

namespace mcs {

// slots:  [K][count][tiles] x (E, M) of the launch that carries it, or nullptr
// red_in: the previous launch's slots (same tiles) to add up, or nullptr;
//         red_K sweeps of them, EM rows red_sweep0 ..
// EM:     [sweep][count][2], em_stride = 2 count
struct EmSlots {
    int64_t *slots = nullptr;
    const int64_t *red_in = nullptr;
    int red_K = 0;
    int64_t red_sweep0 = 0;
    int64_t *EM = nullptr;
    int64_t em_stride = 0;
};

__device__ __forceinline__ longlong2 *em_slot(int64_t *slots, int sweep, int l, int nlat, int tile, int ntile)
{
    return (longlong2 *)slots + ((int64_t)sweep * nlat + l) * ntile + tile;
}

// Workgroup `tile` of lattice l adds up the previous launch's sweeps tile,
// tile + ntile, ...; the first value of its first sweep is fetched here, ahead
// of the tile load, so that the two latencies overlap.
__device__ __forceinline__ void em_prefetch(const EmSlots &e, int tile, int ntile, int l, int nlat, int tid,
                                            long long &pe, long long &pm)
{
    pe = pm = 0;
    if (tile < e.red_K && tid < ntile) {
        const longlong2 v = *em_slot((int64_t *)e.red_in, tile, l, nlat, tid, ntile);
        pe = v.x;
        pm = v.y;
    }
}

// The rest of the sums; called by the whole workgroup (it synchronises), with
// part a __shared__ [2][16] scratch.
__device__ __forceinline__ void em_reduce(const EmSlots &e, int tile, int ntile, int l, int nlat, int tid, int nt,
                                          long long pe, long long pm, long long (*part)[16])
{
    const int wave = tid >> 6, nwaves = nt >> 6;
    for (int j = tile; j < e.red_K; j += ntile) {
        long long se = 0, sm = 0;
        int t = tid;
        if (j == tile) {
            se = pe;
            sm = pm;
            t += nt;
        }
        const longlong2 *src = em_slot((int64_t *)e.red_in, j, l, nlat, 0, ntile);
        for (; t < ntile; t += nt) {
            const longlong2 v = src[t];
            se += v.x;
            sm += v.y;
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            se += __shfl_xor(se, off, 64);
            sm += __shfl_xor(sm, off, 64);
        }
        if ((tid & 63) == 0) {
            part[0][wave] = se;
            part[1][wave] = sm;
        }
        __syncthreads();
        if (tid == 0) {
            long long te = 0, tm = 0;
            for (int i = 0; i < nwaves; ++i) {
                te += part[0][i];
                tm += part[1][i];
            }
            int64_t *em = e.EM + (e.red_sweep0 + j) * e.em_stride + 2 * l;
            em[0] = te;
            em[1] = tm;
        }
        __syncthreads();
    }
}

}  // namespace mcs
