// pt.hpp -- parameter blocks of the parallel-tempering kernels.
#pragma once

#include "common.hpp"

namespace mcs {

constexpr int kPtMaxTemps = 1024;  // temperatures per set: one exchange workgroup

struct PtSweepArgs {
    int8_t *spins;              // [count][L^2], lattice l = set s, replica r at l = s n_temps + r
    int L, Wb, nwr, G;          // extent, LDS word layout, lattices per workgroup
    int count;                  // n_sets * n_temps
    const int32_t *temp_of;     // [count] temperature index held by lattice l
    const Thr *thr;             // [n_temps][2] Metropolis thresholds dE = 4, 8
    int32_t *E;                 // [count] energy after the sweeps
    uint64_t sweep0;            // round theta
    int theta;
    uint32_t seed_lo, seed_hi;
};

struct PtExchangeArgs {
    int n_temps;
    int32_t *temp_of, *replica_at;  // [n_sets][n_temps]
    const int32_t *E;               // [n_sets][n_temps] by replica
    const uint64_t *xtab;           // [n_temps - 1][mmax + 1]: ceil(exp((beta_i - beta_{i+1}) 4m) 2^32)
    int mmax;                       // largest (E_a - E_b) / 4
    int64_t *accepted;              // [n_sets][n_temps - 1]
    int64_t *E_at;                  // [n_sets][n_temps] of this round, or nullptr
    uint64_t round;
    uint32_t seed_lo, seed_hi;
};

hipError_t launch_pt_round(const PtSweepArgs &sw, const PtExchangeArgs &ex, int n_sets, hipStream_t s);

}  // namespace mcs
