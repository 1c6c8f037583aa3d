// muca.hpp -- parameter block and launchers of the multicanonical kernels.
#pragma once

#include "common.hpp"

namespace mcs {

struct MucaArgs {
    int8_t *spins;          // [W][L*L] int8 walker lattices (in/out)
    int64_t *E;             // [W] walker energies (in/out)
    const uint32_t *table;  // [(K+1)*4] thresholds minus one, direction -2, -1, +1, +2
    uint32_t *hist;         // [ceil(W/64)][K+1] per-workgroup counts (scratch)
    int64_t *H;             // [K+1] histogram the counts are added to
    int W;
    uint32_t seed_lo, seed_hi;
    uint64_t sweep0;
    int nsweeps;
    int record;
};

bool muca_L_supported(int L);
hipError_t launch_muca_sweeps(const MucaArgs &a, int L, hipStream_t s);
hipError_t launch_muca_start(int8_t *spins, int64_t *E, int L, int W, uint64_t seed, int start, hipStream_t s);
hipError_t launch_muca_settle(int8_t *spins, int64_t *E, int L, int W, hipStream_t s);

}  // namespace mcs
