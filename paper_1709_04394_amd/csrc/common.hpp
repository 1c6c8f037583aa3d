// common.hpp -- device helpers and internal launcher declarations of libmcspin.
//
// Everything device-side that more than one kernel file needs: the Philox4x32-10
// block function, the random-stream counter layout, the byte-lazy 32-bit draw,
// wave64 reductions, and the parameter structs the host side fills.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcs {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Sec. "Random number generation", counter-based generators):
// ten rounds of  L' = mullo(R, M), R' = mulhi(R, M) ^ k ^ L  on the two word
// pairs, with the 4x32 word permutation and a Weyl key schedule.  The key is
// wave-uniform in every kernel here, so the key schedule runs on the scalar
// unit and each round costs two 32x32->64 multiplies and two 3-input XORs.
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

// gfx950's v_bitop3_b32 evaluates any 3-input boolean function in one
// instruction; the immediate is the truth table f(0xF0, 0xCC, 0xAA) of the
// operands (a, b, c).  BOP3(a, b, c, expr) spells the function with A, B, C.
template <unsigned IMM>
__device__ __forceinline__ uint32_t bop3(uint32_t a, uint32_t b, uint32_t c)
{
    return __builtin_amdgcn_bitop3_b32(a, b, c, (unsigned char)IMM);
}
#define MCS_A 0xF0u
#define MCS_B 0xCCu
#define MCS_C 0xAAu
#define MCS_BOP3(a, b, c, expr) ::mcs::bop3<((expr)&0xFFu)>((a), (b), (c))

__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) { return bop3<0x96u>(a, b, c); }

__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += kPhiloxW0;
            k1 += kPhiloxW1;
        }
        const uint64_t p0 = (uint64_t)kPhiloxM0 * c.x;
        const uint64_t p1 = (uint64_t)kPhiloxM1 * c.z;
        c = make_uint4(xor3((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1, xor3((uint32_t)(p0 >> 32), c.w, k1),
                       (uint32_t)p0);
    }
    return c;
}

// Stream tags (counter word 3, bits 24..31).
enum : uint32_t {
    kTagInit = 1, kTagSweep = 2, kTagCoupling = 3, kTagResample = 4,
    kTagMuca = 5, kTagMlpInit = 6, kTagSweepLo = 7, kTagMucaLo = 8, kTagExchange = 9,
    kTagWindow = 10
};

// Counter word 3: tag << 24 | phase << 23 | (sweep >> 32) & 0x7FFFFF.
__host__ __device__ __forceinline__ uint32_t ctr_w3(uint32_t tag, uint32_t phase, uint64_t sweep)
{
    return (tag << 24) | ((phase & 1u) << 23) | ((uint32_t)(sweep >> 32) & 0x7FFFFFu);
}

// The top byte of the 32-bit draw of item j lives in the Philox block of
// a = j / 16 as eight bit-planes: bit k of the byte is bit (j mod 16) of
// 16-bit half-word k of the block (half-word k = bits 16 (k mod 2) .. +15 of
// word k / 2).  One block thus serves 16 consecutive items, and a pair of
// blocks gives 32 items' planes as eight 32-bit words (plane_pair below),
// which is the form the bit-sliced sweep kernels consume.
__device__ __forceinline__ uint32_t byte_of(const uint4 &b, uint32_t pos)
{
    const uint32_t w[4] = {b.x, b.y, b.z, b.w};
    uint32_t byte = 0;
#pragma unroll
    for (uint32_t k = 0; k < 8; ++k) byte |= ((w[k >> 1] >> (16u * (k & 1u) + pos)) & 1u) << k;
    return byte;
}

// Bit 7 of byte_of(b, pos): the byte is < 128 iff this is 0.
__device__ __forceinline__ uint32_t top_bit_of(const uint4 &b, uint32_t pos)
{
    return (b.w >> (16u + pos)) & 1u;
}

// Plane k (k = 0..7) of the 32 items 32q .. 32q+31 from blocks A = block(2q)
// and B = block(2q+1): low half-word from A, high half-word from B.
__device__ __forceinline__ uint32_t plane_pair(const uint4 &A, const uint4 &B, int k)
{
    const uint32_t a = (k >> 1) == 0 ? A.x : (k >> 1) == 1 ? A.y : (k >> 1) == 2 ? A.z : A.w;
    const uint32_t b = (k >> 1) == 0 ? B.x : (k >> 1) == 1 ? B.y : (k >> 1) == 2 ? B.z : B.w;
    // bytes (little-endian) of the result: a.lo16 | b.lo16 << 16, or the hi16s
    return (k & 1) ? __builtin_amdgcn_perm(b, a, 0x07060302u) : __builtin_amdgcn_perm(b, a, 0x05040100u);
}

// A threshold T in [0, 2^32] split for the byte-lazy test r32 < T with
// r32 = byte << 24 | low24:  byte < top  => accept;  byte > top  => reject;
// byte == top => accept iff low24 < low.  T = 2^32 has top = 256.
struct Thr {
    uint32_t top;  // T >> 24, 0..256
    uint32_t low;  // T & 0xFFFFFF
};

__host__ __device__ __forceinline__ Thr split_thr(uint64_t T)
{
    Thr t;
    t.top = (uint32_t)(T >> 24);
    t.low = (uint32_t)(T & 0xFFFFFFu);
    return t;
}

// Bit masks of a threshold's top byte: tk[k] = all ones iff bit k of top is
// set (wave-uniform, lives in scalar registers); top = 256 (T = 2^32) is the
// "always" case.
struct TopMask {
    uint32_t tk[8];
    bool always;
};

__device__ __forceinline__ TopMask top_mask(uint32_t top)
{
    TopMask m;
#pragma unroll
    for (int k = 0; k < 8; ++k) m.tk[k] = ((top >> k) & 1u) ? ~0u : 0u;
    m.always = top >= 256u;
    return m;
}

// lt = (X < top), eq = (X == top) for 32 sites at once, X given as bit-planes
// X[0] (LSB) .. X[7].  lt is the borrow out of X - top, propagated from the
// least significant plane: borrow' = maj(~X_k, top_k, borrow); one bitop3 per
// plane for each of lt and eq.
__device__ __forceinline__ void compare_planes(const uint32_t (&X)[8], const TopMask &t, uint32_t &lt, uint32_t &eq)
{
    uint32_t b = 0u, e = ~0u;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        b = MCS_BOP3(X[k], t.tk[k], b, (~MCS_A & MCS_B) | (~MCS_A & MCS_C) | (MCS_B & MCS_C));
        e = MCS_BOP3(e, X[k], t.tk[k], MCS_A & ~(MCS_B ^ MCS_C));
    }
    lt = t.always ? ~0u : b;
    eq = t.always ? 0u : e;
}

// ---------------------------------------------------------------------------
// wave64 reductions
__device__ __forceinline__ long long wave_sum(long long v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

__device__ __forceinline__ int wave_sum_i(int v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Parameter blocks filled on the host.
struct Geom {
    int dims, Lx, Ly, Lz;
    int64_t N;      // sites per lattice
    int count;      // lattices (int8) or word lattices (msc64)
};

struct SweepTables {
    // Metropolis: index k = dE / 4 (k = 1..3); heat-bath: index h + z (0..12)
    Thr met[4];
    Thr hb[13];     // heat-bath, index h + 6 for every dimension
};

// most lattices one fused launch can carry with their own temperature
constexpr int kMaxTableLattices = 16;

struct SweepCall {
    Geom g;
    const int8_t *J;    // [dims][N] or nullptr
    int rule;           // 0 Metropolis, 1 heat-bath
    uint32_t seed_lo, seed_hi;
    uint32_t replica0;
    SweepTables tab;    // tables of the common temperature
    int per_lattice;    // 1: lattice l uses tabs[l] (host array, host code only)
    const SweepTables *tabs;
};

// Launchers (defined in the kernel files).  They only enqueue work.
hipError_t launch_fill_i64(int64_t *p, int64_t n, int64_t value, hipStream_t s);
hipError_t launch_init_int8(const Geom &g, int8_t *spins, int start, uint64_t seed, uint32_t replica0,
                            hipStream_t s);
hipError_t launch_init_msc64(const Geom &g, uint64_t *words, int start, uint64_t seed, uint32_t replica0,
                             hipStream_t s);
hipError_t launch_couplings(const Geom &g, int8_t *J, uint64_t seed, hipStream_t s);

hipError_t launch_measure_int8(const Geom &g, const int8_t *spins, const int8_t *J, int64_t *EM,
                               hipStream_t s);
hipError_t launch_measure_msc64(const Geom &g, const uint64_t *words, const int8_t *J, int64_t *EM,
                                hipStream_t s);

// generic in-place half-sweep, any even geometry, int8
hipError_t launch_phase_int8(const SweepCall &c, int8_t *spins, uint64_t sweep, int phase, hipStream_t s);
// generic in-place half-sweep, msc64
hipError_t launch_phase_msc64(const SweepCall &c, uint64_t *words, uint64_t sweep, int phase, hipStream_t s);

}  // namespace mcs
