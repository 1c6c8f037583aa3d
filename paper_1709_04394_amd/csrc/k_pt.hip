// k_pt.hip -- parallel tempering (Sec. "Parallel Tempering", Eq. pt) of 2D
// L x L ferromagnets on the device: independent sets of n_temps replicas,
// each replica at the temperature it currently holds.
//
// One round is two kernels:
//  k_pt_sweep     every replica whole in LDS (several per workgroup for small
//                 L), theta checkerboard Metropolis sweeps at the thresholds of
//                 its temperature (looked up through the replica -> temperature
//                 map, so no host round trip is needed between rounds), and its
//                 energy afterwards: the on-the-fly energy the exchange needs;
//  k_pt_exchange  one workgroup per set: records the energy at each
//                 temperature, then proposes the disjoint neighbour pairs of
//                 the round, accepting with min(1, exp((beta_i - beta_{i+1})
//                 (E_a - E_b))) by an integer test against a host FP64 table,
//                 and swaps temperatures in both maps (configurations never
//                 move).
#include "internal.hpp"
#include "lds_lattice.hpp"
#include "pt.hpp"

namespace mcs {

__global__ __launch_bounds__(256) void k_pt_sweep(PtSweepArgs a)
{
    extern __shared__ uint32_t lds[];
    __shared__ int e_lat[64];
    __shared__ Thr t4s[64], t8s[64];
    __shared__ LdsTieQueue tq;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int s0 = (int)blockIdx.x * a.G;
    LdsLattices la;
    la.L = a.L;
    la.N = a.L * a.L;
    la.Wb = a.Wb;
    la.nwr = a.nwr;
    la.ng = min(a.G, a.count - s0);
    la.rep0 = (uint32_t)s0;  // lattice l = set s, replica r is replica id s n_temps + r = l
    la.sweep0 = a.sweep0;
    la.theta = a.theta;
    la.seed_lo = a.seed_lo;
    la.seed_hi = a.seed_hi;
    const int L = la.L, N = la.N, nwr = la.nwr;
    if (tid < 64) e_lat[tid] = 0;
    if (tid < la.ng) {
        const int ti = a.temp_of[s0 + tid];
        t4s[tid] = a.thr[2 * ti];
        t8s[tid] = a.thr[2 * ti + 1];
    }
    const int tasks = la.ng * L * nwr;
    for (int t = tid; t < tasks; t += nt) {
        const int g = t / (L * nwr), rem = t - g * L * nwr, r = rem / nwr, w = rem - r * nwr;
        pack_lattice_rows(lds, la, g, a.spins + (int64_t)(s0 + g) * N, r, w);
    }
    __syncthreads();
    sweep_lds_lattices<true>(lds, la, Thr{}, Thr{}, t4s, t8s, tq, e_lat);
    if (tid < la.ng) a.E[s0 + tid] = e_lat[tid];
    for (int t = tid; t < tasks; t += nt) {
        const int g = t / (L * nwr), rem = t - g * L * nwr, r = rem / nwr, w = rem - r * nwr;
        unpack_lattice_rows(lds, la, g, a.spins + (int64_t)(s0 + g) * N, r, w);
    }
}

__global__ __launch_bounds__(1024) void k_pt_exchange(PtExchangeArgs a)
{
    __shared__ int32_t rep[kPtMaxTemps];
    const int s = blockIdx.x, i = threadIdx.x, nT = a.n_temps;
    int32_t *tof = a.temp_of + (int64_t)s * nT;
    int32_t *rat = a.replica_at + (int64_t)s * nT;
    const int32_t *Es = a.E + (int64_t)s * nT;
    if (i < nT) {
        rep[i] = rat[i];
        if (a.E_at) a.E_at[(int64_t)s * nT + i] = Es[rep[i]];
    }
    __syncthreads();
    if (i + 1 < nT && (uint32_t)(i & 1) == (uint32_t)(a.round & 1u)) {
        const int32_t ra = rep[i], rb = rep[i + 1];
        const int32_t d = Es[ra] - Es[rb];
        // beta_i < beta_{i+1}: the exponent (beta_i - beta_{i+1}) d is >= 0 iff
        // d <= 0; energies of the even torus differ by multiples of 4
        bool acc = d <= 0;
        if (!acc) {
            const uint64_t T = a.xtab[(int64_t)i * (a.mmax + 1) + (d >> 2)];
            const uint4 r = philox(make_uint4((uint32_t)i >> 2, (uint32_t)s, (uint32_t)a.round,
                                              ctr_w3(kTagExchange, 0, a.round)),
                                   a.seed_lo, a.seed_hi);
            const uint32_t w[4] = {r.x, r.y, r.z, r.w};
            acc = (uint64_t)w[i & 3] < T;
        }
        if (acc) {
            rat[i] = rb;
            rat[i + 1] = ra;
            tof[ra] = i + 1;
            tof[rb] = i;
            a.accepted[(int64_t)s * (nT - 1) + i] += 1;
        }
    }
}

hipError_t launch_pt_round(const PtSweepArgs &sw, const PtExchangeArgs &ex, int n_sets, hipStream_t s)
{
    const int blocks = (sw.count + sw.G - 1) / sw.G;
    const size_t lds = (size_t)sw.G * 2 * sw.L * sw.nwr * 4;
    hipLaunchKernelGGL(k_pt_sweep, dim3(blocks), dim3(256), lds, s, sw);
    const int threads = ((ex.n_temps + 63) / 64) * 64;
    hipLaunchKernelGGL(k_pt_exchange, dim3(n_sets), dim3(threads), 0, s, ex);
    return hipGetLastError();
}

}  // namespace mcs
