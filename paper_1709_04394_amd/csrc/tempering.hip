// tempering.hip -- the replica-exchange step of parallel tempering (Sec.
// "Parallel Tempering", Eq. pt), on the host.  An exchange touches a few
// scalars per pair of temperatures; the replicas' configurations never move
// (temperatures are exchanged, as the paper recommends when replicas live
// apart).  The energies come from the sweeps' fused measurement (mc_sweep /
// mc_sweep_betas per-sweep E), so no extra pass over the lattices is needed.
#include <cmath>
#include <vector>

#include "internal.hpp"

using namespace mcs;

namespace {

constexpr uint32_t kTagExchange = 9;

// Philox4x32-10 (the same generator the kernels use), for a few host draws.
void philox_host(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c[0];
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c[2];
        const uint32_t y0 = (uint32_t)(p1 >> 32) ^ c[1] ^ k0, y2 = (uint32_t)(p0 >> 32) ^ c[3] ^ k1;
        c[0] = y0;
        c[1] = (uint32_t)p1;
        c[2] = y2;
        c[3] = (uint32_t)p0;
    }
}

// r32 of pair i in round t: word (i mod 4) of Philox(ctr = (i / 4, 0, t,
// TAG_EXCHANGE << 24 | t >> 32)).
uint32_t pair_draw(uint64_t seed, uint32_t i, uint64_t round)
{
    uint32_t c[4] = {i >> 2, 0u, (uint32_t)round, ctr_w3(kTagExchange, 0, round)};
    philox_host(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    return c[i & 3u];
}

}  // namespace

extern "C" {

int mc_pt_exchange(mc_ctx *ctx, int32_t n_temps, const double *beta, const int64_t *E, int32_t *temp_of,
                   int32_t *replica_at, uint64_t seed, uint64_t round, int64_t *accepted)
{
    if (!ctx) return MC_E_INVAL;
    if (n_temps < 2 || n_temps > (1 << 20)) return fail(ctx, MC_E_RANGE, "n_temps must be 2..2^20 (got %d)", n_temps);
    if (!beta || !E || !temp_of || !replica_at || !accepted) return fail(ctx, MC_E_INVAL, "a pointer argument is NULL");
    if (round >= (1ull << 55)) return fail(ctx, MC_E_RANGE, "round numbers must stay below 2^55");
    for (int i = 0; i < n_temps; ++i) {
        if (!(beta[i] >= 0.0) || std::isinf(beta[i])) return fail(ctx, MC_E_RANGE, "beta[%d] out of range", i);
        if (i > 0 && !(beta[i] > beta[i - 1]))
            return fail(ctx, MC_E_RANGE, "beta must increase strictly (beta[%d] <= beta[%d])", i, i - 1);
        if (E[i] > (1ll << 52) || E[i] < -(1ll << 52)) return fail(ctx, MC_E_RANGE, "|E[%d]| exceeds 2^52", i);
    }
    // the two maps must be inverse permutations of 0..n_temps-1
    std::vector<char> seen((size_t)n_temps, 0);
    for (int i = 0; i < n_temps; ++i) {
        const int32_t a = replica_at[i];
        if (a < 0 || a >= n_temps || seen[(size_t)a] || temp_of[a] != i)
            return fail(ctx, MC_E_INVAL, "replica_at / temp_of are not inverse permutations (at temperature %d)", i);
        seen[(size_t)a] = 1;
    }
    for (int i = (int)(round & 1u); i + 1 < n_temps; i += 2) {
        const int32_t a = replica_at[i], b = replica_at[i + 1];
        // min(1, exp((beta_i - beta_{i+1}) (E_a - E_b))) as an integer test on
        // a 32-bit draw, exactly as the sweeps' acceptance tables
        const double x = (beta[i] - beta[i + 1]) * (double)(E[a] - E[b]);
        bool acc = x >= 0.0;
        if (!acc) {
            const uint64_t T = (uint64_t)std::ceil(std::ldexp(std::exp(x), 32));
            acc = (uint64_t)pair_draw(seed, (uint32_t)i, round) < T;
        }
        if (acc) {
            replica_at[i] = b;
            replica_at[i + 1] = a;
            temp_of[a] = i + 1;
            temp_of[b] = i;
            accepted[i] += 1;
        }
    }
    return MC_OK;
}

}  // extern "C"
