// pa.hpp -- parameter blocks of the population-annealing kernels.
#pragma once

#include "common.hpp"

namespace mcs {

constexpr int kPaMaxPops = 8;
constexpr int kPaMaxChunks = 1024;  // R <= 64 * 1024 replicas per population

struct PaPop {
    int L, N, R;
    int Wb, nwr;            // bits per LDS word, words per row and parity
    int G;                  // lattices per workgroup in k_pa_sweep
    int blk0;               // first k_pa_sweep block of this population
    const int8_t *cur;      // population before the step [R][N]
    int8_t *nxt;            // population after the step
    const int32_t *E;       // energies of cur
    int32_t *Enew;          // energies of nxt
    double *rmx;            // [R] running maximum of each block's inclusive sums x
    double *blk;            // [4][nb], nb = ceil(R / 64): block totals, largest x of each
                            // block, block offsets G_q + B_b, running maximum of C at block ends
    int32_t *n, *newparent; // [R] copy numbers, parent of each new slot
    int64_t *hist;          // [rows][N + 1]
    double *ctot;           // [nsteps]
};

struct PaStep {
    PaPop pop[kPaMaxPops];
    int npop;
    const double *wtab;     // weights exp(-dbeta 4k), k = 0..N_max, of this step
    uint32_t seed_lo, seed_hi;
    uint32_t step;          // annealing step number i >= 1 (sweeps (i-1) theta + t)
    int theta;
    Thr t4, t8;             // Metropolis thresholds at beta_i
    int hist_idx, ctot_idx;
    int identity;           // 1: no resampling, slot s keeps replica s (measuring pass)
};

hipError_t launch_pa_step(const PaStep &st, int rmax, int sweep_blocks, hipStream_t s);

}  // namespace mcs
