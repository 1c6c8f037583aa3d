// wl.hpp -- parameter blocks and launchers of the Wang-Landau window kernels.
#pragma once

#include "common.hpp"

namespace mcs {

constexpr int kWlExpN = 23;                    // exp(-n), n = 0..22; n >= 23 gives the threshold 1
constexpr int kWlTab = kWlExpN + 4 * 256;       // exp(-n), then the factors of the four bytes
constexpr int kWlMaxWidth = 192;                // levels per window (estimates of 64 walkers in LDS)

struct WlArgs {
    int8_t *spins;          // [W][L*L] walker lattices (in/out)
    int64_t *E;             // [W] walker energies (in/out)
    int64_t *G;             // [W][wmax] ln g estimates in units of 2^-32, level k at k - lo
    uint32_t *H;            // [W][wmax] visit counts of the stage
    int32_t *flat;          // [W] 1 if the walker's histogram is flat after the call
    const int32_t *lo, *hi; // [nwin] window levels
    const int64_t *inc;     // [nwin] ln f in units of 2^-32
    const uint8_t *active;  // [nwin] windows whose walkers sweep
    const double *xtab;     // [kWlTab] exponential factors
    double flat_ratio;
    int M, wmax;            // walkers per window (multiple of 64), estimate row length
    uint32_t seed_lo, seed_hi;
    uint64_t sweep0;
    int nsweeps;
};

hipError_t launch_win_drive(int8_t *spins, int64_t *E, int32_t *ok, const int32_t *lo, int L, int W, int M,
                            int max_pass, uint64_t seed, hipStream_t s);
hipError_t launch_wl_sweeps(const WlArgs &a, int L, int W, hipStream_t s);
hipError_t launch_wl_average(int64_t *G, uint32_t *H, const int32_t *lo, const int32_t *hi, const uint8_t *mask,
                             int nwin, int M, int wmax, hipStream_t s);

}  // namespace mcs
