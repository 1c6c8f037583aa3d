// muca_rows.hpp -- int8 rows of a walker's lattice packed into 32-bit words
// (bit set <=> s = -1) and back, for the sequential walker kernels.
#pragma once

#include "common.hpp"

namespace mcs {

// Sign bits of four int8 spins -> 4 bits (bit set <=> -1): bytes' bit 7 to
// positions 0, 8, 16, 24, then a multiply gathers them at 21..24.
__device__ __forceinline__ uint32_t pack4(uint32_t d)
{
    const uint32_t m = (d & 0x80808080u) >> 7;
    return (m * 0x00204081u >> 21) & 0xFu;
}

// 4 bits -> four int8 spins (+1 for 0, -1 for 1).
__device__ __forceinline__ uint32_t unpack4(uint32_t nib)
{
    const uint32_t bits = (nib * 0x00204081u) & 0x01010101u;
    return __builtin_amdgcn_perm(0u, 0x0000FF01u, bits);
}

template <int L>
__device__ __forceinline__ void load_row(const int8_t *sp, int y, uint32_t (&row)[(L + 31) / 32])
{
    constexpr int NW = (L + 31) / 32;
    const uint32_t *p = (const uint32_t *)(sp + y * L);
#pragma unroll
    for (int i = 0; i < NW; ++i) row[i] = 0;
#pragma unroll
    for (int q = 0; q < L / 4; ++q) row[(4 * q) / 32] |= pack4(p[q]) << ((4 * q) % 32);
}

template <int L>
__device__ __forceinline__ void store_row(int8_t *sp, int y, const uint32_t (&row)[(L + 31) / 32])
{
    uint32_t *p = (uint32_t *)(sp + y * L);
#pragma unroll
    for (int q = 0; q < L / 4; ++q) p[q] = unpack4((row[(4 * q) / 32] >> ((4 * q) % 32)) & 0xFu);
}

template <int L>
__device__ __forceinline__ uint32_t bit_at(const uint32_t (&row)[(L + 31) / 32], int x)
{
    return (row[x / 32] >> (x % 32)) & 1u;
}

}  // namespace mcs
