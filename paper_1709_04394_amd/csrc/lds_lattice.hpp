// lds_lattice.hpp -- whole 2D L x L ferromagnets (J = 1) held bit-packed in
// one workgroup's LDS, swept there for several checkerboard Metropolis sweeps
// (Sec. "Checkerboard scheme", Eq. metropolis-canonical).  Shared by the
// population-annealing step (every lattice at the step's temperature) and by
// parallel tempering (each lattice at the temperature it currently holds).
//
// LDS image of lattice g: word (g, r, par, w) holds the sites x = 64 w + 2 b +
// par (b < Wb) of row r, bit set <=> s = -1, with Wb = min(32, L/2) bits per
// word and nwr = L / 64 words per row and parity for L >= 64 (one word
// otherwise).  The lattice is periodic inside the image, so no halo is needed.
#pragma once

#include "common.hpp"

namespace mcs {

constexpr int kLdsTieQueue = 256;

struct LdsLattices {
    int L, N, Wb, nwr;
    int ng;                 // lattices in this workgroup (at most 64)
    uint32_t rep0;          // replica id of lattice g is rep0 + g
    uint64_t sweep0;        // global number of the first sweep
    int theta;              // sweeps
    uint32_t seed_lo, seed_hi;
    __device__ int per_lat() const { return 2 * L * nwr; }
    __device__ int widx(int g, int r, int par, int w) const { return g * per_lat() + (r * 2 + par) * nwr + w; }
};

// Queue storage of the deferred ties of one half-sweep.
struct LdsTieQueue {
    uint32_t j[kLdsTieQueue], meta[kLdsTieQueue], rep[kLdsTieQueue];
    uint32_t cnt[4];
};

// int8 rows of one lattice -> its packed LDS image (row r at src + r L).
__device__ __forceinline__ void pack_lattice_rows(uint32_t *lds, const LdsLattices &a, int g, const int8_t *src,
                                                  int r, int w)
{
    const int8_t *row = src + (int64_t)r * a.L;
    uint32_t ev = 0, od = 0;
    if (a.Wb == 32) {
        const uint4 *q4 = (const uint4 *)(row + 64 * w);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint4 v = q4[q];
            const uint32_t dw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // sign bits at 7, 15, 23, 31 -> m + (m << 15) puts the two even-x
                // bits at 22..23 and the two odd-x bits at 30..31
                const uint32_t m = dw[i] & 0x80808080u;
                const uint32_t Pm = m + (m << 15);
                const int sh = 2 * (4 * q + i);
                ev |= ((Pm >> 22) & 3u) << sh;
                od |= (Pm >> 30) << sh;
            }
        }
    } else {
        for (int b = 0; b < a.Wb; ++b) {
            ev |= (uint32_t)(row[2 * b] < 0) << b;
            od |= (uint32_t)(row[2 * b + 1] < 0) << b;
        }
    }
    lds[a.widx(g, r, 0, w)] = ev;
    lds[a.widx(g, r, 1, w)] = od;
}

// packed LDS image -> int8 rows (row r at dst + r L)
__device__ __forceinline__ void unpack_lattice_rows(const uint32_t *lds, const LdsLattices &a, int g, int8_t *dst,
                                                    int r, int w)
{
    const uint32_t ev = lds[a.widx(g, r, 0, w)], od = lds[a.widx(g, r, 1, w)];
    int8_t *row = dst + (int64_t)r * a.L;
    if (a.Wb == 32) {
        uint4 *q4 = (uint4 *)(row + 64 * w);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            uint32_t dw[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int sh = 2 * (4 * q + i);
                const uint32_t bits = ((ev >> sh) & 1u) | (((od >> sh) & 1u) << 8) | (((ev >> (sh + 1)) & 1u) << 16) |
                                      (((od >> (sh + 1)) & 1u) << 24);
                // bit 0 -> byte 0x01 (+1), bit 1 -> byte 0xFF (-1)
                dw[i] = __builtin_amdgcn_perm(0u, 0x0000FF01u, bits);
            }
            q4[q] = make_uint4(dw[0], dw[1], dw[2], dw[3]);
        }
    } else {
        for (int b = 0; b < a.Wb; ++b) {
            row[2 * b] = ((ev >> b) & 1u) ? (int8_t)-1 : (int8_t)1;
            row[2 * b + 1] = ((od >> b) & 1u) ? (int8_t)-1 : (int8_t)1;
        }
    }
}

// Neighbour word along x of the active parity word of row r: the other
// parity's sites shifted by one site towards the active ones.
__device__ __forceinline__ uint32_t x_neighbour(const uint32_t *lds, const LdsLattices &a, int g, int r, int q, int w,
                                                uint32_t O, uint32_t wmask)
{
    if (a.nwr > 1) {
        const int wl = w == 0 ? a.nwr - 1 : w - 1, wr = w + 1 == a.nwr ? 0 : w + 1;
        return q == 0 ? __builtin_amdgcn_alignbit(O, lds[a.widx(g, r, 1, wl)], 31)
                      : __builtin_amdgcn_alignbit(lds[a.widx(g, r, 0, wr)], O, 1);
    }
    // one word per row: rotate inside the Wb used bits
    return q == 0 ? (((O << 1) | (O >> (a.Wb - 1))) & wmask) : (((O >> 1) | (O << (a.Wb - 1))) & wmask);
}

// theta checkerboard Metropolis sweeps of the ng lattices in LDS; the
// thresholds of lattice g are t4[g], t8[g] (dE = 4, 8) when PER_LAT, else
// u4, u8 for every lattice.  Then the energy of each lattice into e_lat[g].
// Every thread of the workgroup must call this (barriers inside).
template <bool PER_LAT>
__device__ void sweep_lds_lattices(uint32_t *lds, const LdsLattices &a, Thr u4, Thr u8, const Thr *t4,
                                   const Thr *t8, LdsTieQueue &tq, int *e_lat)
{
    const int L = a.L, Wb = a.Wb, nwr = a.nwr;
    const int tid = threadIdx.x, nt = blockDim.x;
    const uint32_t wmask = Wb == 32 ? ~0u : ((1u << Wb) - 1u);
    const int wave = tid >> 6, nwaves = nt >> 6;
    const uint32_t wq_cap = (uint32_t)(kLdsTieQueue / nwaves), wq_base = (uint32_t)wave * wq_cap;
    const int tasks = a.ng * L * nwr;
    const TopMask um4 = top_mask(u4.top), um8 = top_mask(u8.top);
    uint32_t wq_n = 0;
    for (int sw = 0; sw < a.theta; ++sw) {
        const uint64_t sweep = a.sweep0 + (uint64_t)sw;
        for (int c = 0; c < 2; ++c) {
            const uint32_t w3 = ctr_w3(kTagSweep, (uint32_t)c, sweep);
            const uint32_t w3lo = ctr_w3(kTagSweepLo, (uint32_t)c, sweep);
            for (int t = tid; t < tasks; t += nt) {
                const int g = t / (L * nwr), rem = t - g * L * nwr, r = rem / nwr, w = rem - r * nwr;
                const int q = (c + r) & 1;
                const int rm = r == 0 ? L - 1 : r - 1, rp = r + 1 == L ? 0 : r + 1;
                const int ws = a.widx(g, r, q, w);
                const uint32_t S = lds[ws];
                const uint32_t U = lds[a.widx(g, rm, q, w)], D = lds[a.widx(g, rp, q, w)];
                const uint32_t O = lds[a.widx(g, r, 1 - q, w)];
                const uint32_t Sh = x_neighbour(lds, a, g, r, q, w, O, wmask);
                const uint32_t u1 = S ^ U, u2 = S ^ D, u3 = S ^ O, u4b = S ^ Sh;
                const uint32_t t1 = u1 | u2, t2 = u3 | u4b;
                const uint32_t ge2 = MCS_BOP3(u1, u2, MCS_BOP3(u3, u4b, t1 & t2, (MCS_A & MCS_B) | MCS_C),
                                              (MCS_A & MCS_B) | MCS_C);
                const uint32_t c8 = ~(t1 | t2) & wmask;
                const uint32_t c4 = MCS_BOP3(t1, t2, ge2, (MCS_A | MCS_B) & ~MCS_C);
                // random planes of sites j0 .. j0 + Wb - 1, j0 = 32 w + (L/2) r
                const uint32_t j0 = 32u * (uint32_t)w + (uint32_t)(L >> 1) * (uint32_t)r;
                const uint32_t rep = a.rep0 + (uint32_t)g;
                uint32_t X[8];
                const uint4 A = philox(make_uint4(j0 >> 4, rep, (uint32_t)sweep, w3), a.seed_lo, a.seed_hi);
                if (Wb == 32) {
                    const uint4 B = philox(make_uint4((j0 >> 4) + 1u, rep, (uint32_t)sweep, w3), a.seed_lo, a.seed_hi);
#pragma unroll
                    for (int k = 0; k < 8; ++k) X[k] = plane_pair(A, B, k);
                } else {
                    const uint32_t off = j0 & 15u;
                    const uint32_t aw[4] = {A.x, A.y, A.z, A.w};
#pragma unroll
                    for (int k = 0; k < 8; ++k) X[k] = ((aw[k >> 1] >> (16u * (k & 1u))) >> off) & wmask;
                }
                uint32_t lt8, eq8, lt4, eq4;
                if (PER_LAT) {
                    compare_planes(X, top_mask(t8[g].top), lt8, eq8);
                    compare_planes(X, top_mask(t4[g].top), lt4, eq4);
                } else {
                    compare_planes(X, um8, lt8, eq8);
                    compare_planes(X, um4, lt4, eq4);
                }
                uint32_t acc = (MCS_BOP3(ge2, c8, lt8, MCS_A | (MCS_B & MCS_C)) | (c4 & lt4)) & wmask;
                uint32_t pend = ((c8 & eq8) | (c4 & eq4)) & wmask;
                uint64_t m = __ballot(pend != 0u);
                while (m) {
                    const uint32_t off = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                    if (pend) {
                        const int b = __builtin_ctz(pend);
                        pend &= pend - 1u;
                        const uint32_t cls8 = (c8 >> b) & 1u;
                        const uint32_t pos = wq_n + off;
                        if (pos < wq_cap) {
                            tq.j[wq_base + pos] = j0 + (uint32_t)b;
                            tq.rep[wq_base + pos] = rep;
                            tq.meta[wq_base + pos] = (uint32_t)ws | ((uint32_t)b << 16) | (cls8 << 21);
                        } else {
                            const uint4 lo = philox(make_uint4(j0 + (uint32_t)b, rep, (uint32_t)sweep, w3lo),
                                                    a.seed_lo, a.seed_hi);
                            const Thr tt = PER_LAT ? (cls8 ? t8[g] : t4[g]) : (cls8 ? u8 : u4);
                            if ((lo.x & 0xFFFFFFu) < tt.low) acc |= 1u << b;
                        }
                    }
                    wq_n = min(wq_cap, wq_n + (uint32_t)__popcll(m));
                    m = __ballot(pend != 0u);
                }
                lds[ws] = S ^ acc;
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) wq_n = max(wq_n, (uint32_t)__shfl_xor((int)wq_n, off, 64));
            if ((tid & 63) == 0) tq.cnt[wave] = wq_n;
            __syncthreads();
            uint32_t total = 0;
            for (int sg = 0; sg < nwaves; ++sg) total += tq.cnt[sg];
            for (uint32_t i = tid; i < total; i += nt) {
                uint32_t sg = 0, k = i;
                while (k >= tq.cnt[sg]) k -= tq.cnt[sg++];
                const uint32_t item = sg * wq_cap + k, meta = tq.meta[item];
                const uint4 lo = philox(make_uint4(tq.j[item], tq.rep[item], (uint32_t)sweep, w3lo), a.seed_lo,
                                        a.seed_hi);
                const bool cls8 = (meta >> 21) & 1u;
                Thr tt;
                if (PER_LAT) {
                    const int g = (int)(meta & 0xFFFFu) / a.per_lat();
                    tt = cls8 ? t8[g] : t4[g];
                } else {
                    tt = cls8 ? u8 : u4;
                }
                if ((lo.x & 0xFFFFFFu) < tt.low) atomicXor(&lds[meta & 0xFFFFu], 1u << ((meta >> 16) & 31u));
            }
            __syncthreads();
            wq_n = 0;
        }
    }

    // ---- energy over the odd sites' words (every bond has one odd end)
    for (int t = tid; t < tasks; t += nt) {
        const int g = t / (L * nwr), rem = t - g * L * nwr, r = rem / nwr, w = rem - r * nwr;
        const int q = (1 + r) & 1;
        const int rm = r == 0 ? L - 1 : r - 1, rp = r + 1 == L ? 0 : r + 1;
        const uint32_t S = lds[a.widx(g, r, q, w)];
        const uint32_t U = lds[a.widx(g, rm, q, w)], D = lds[a.widx(g, rp, q, w)];
        const uint32_t O = lds[a.widx(g, r, 1 - q, w)];
        const uint32_t Sh = x_neighbour(lds, a, g, r, q, w, O, wmask);
        const int n = __builtin_popcount(S ^ U) + __builtin_popcount(S ^ D) + __builtin_popcount(S ^ O) +
                      __builtin_popcount(S ^ Sh);
        atomicAdd(&e_lat[g], 2 * n - 4 * Wb);
    }
    __syncthreads();
}

}  // namespace mcs
