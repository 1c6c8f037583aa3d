// k_dcb.hip -- double-checkerboard Metropolis sweeps with k hits per tile
// (Sec. "Checkerboard scheme": tiles in a coarse checkerboard, each tile
// loaded once and updated k times; multi-hit updates) of the 2D ferromagnet
// (J = 1), on lattices kept bit-packed in global scratch between launches.
//
// One launch updates every tile of one coarse colour: a workgroup loads its
// T x T tile with a one-site halo (one row above and below, one 64-site word
// column left and right, of which only the edge sites are read) from the
// packed lattice into LDS, runs k rounds of the tile's own checkerboard (even
// sites, then odd), and writes the tile back in place.  The halo belongs to
// tiles of the other coarse colour, which no workgroup of this launch writes,
// so the launch has no race and no redone halo: every update is done once.
// A sweep is two launches (coarse colour 0, then 1).  The per-word update
// (four neighbour words, Metropolis classes from 3-input bit operations, the
// random top bytes as eight bit-planes from two Philox blocks, a bit-serial
// compare, ties settled after the half-step) follows the 2D band kernel.
//
// Energy and magnetisation of a sweep: every bond lies inside one tile or
// joins a tile of colour 0 to one of colour 1.  Colour-0 tiles are final
// after their launch and record their internal bonds and spins; colour-1
// tiles record theirs plus all bonds across their edges (the other ends are
// final).  Each tile writes its share to a slot of its own; the first
// workgroup of each lattice in the next sweep's colour-0 launch adds up the
// previous sweep's slots while it loads its tile (em_slots.hpp), and a small
// kernel adds up those of a call's last sweep.
#include <algorithm>

#include "internal.hpp"

namespace mcs {

constexpr int kDcbTieQueue = 512;
constexpr int kDcbMaxWaves = 4;  // at most 256 threads per workgroup

struct DcbArgs {
    uint32_t *lat;              // packed lattices, rows of 2 L/64 words (even-x array first)
    int L, T;                   // extent, tile side (multiples of 64)
    int coarse;                 // colour of the tiles of this launch
    int hits;
    uint32_t replica0;
    uint64_t sweep;             // global sweep number; hit h draws as plain sweep sweep * hits + h
    uint32_t seed_lo, seed_hi;
    Thr t4, t8;                 // Metropolis thresholds dE = 4, 8
    int64_t *part;              // [count][tiles][2] (E, M) shares of the tiles, or nullptr
    EmSlots prev;               // the previous sweep's slots (red_K = 1) to add up, or none
};

// Workgroup -> tile: tiles of one coarse colour, (L/T)^2 / 2 of them, row by
// row of tiles.
__device__ __forceinline__ void dcb_tile(const DcbArgs &a, int b, int &tx, int &ty)
{
    const int nt = a.L / a.T, half = nt / 2;
    ty = b / half;
    tx = 2 * (b - ty * half) + ((ty + a.coarse) & 1);
}

__global__ __launch_bounds__(256) void k_dcb(DcbArgs a)
{
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t q_ws[kDcbTieQueue], q_blk[kDcbTieQueue], q_p8[kDcbTieQueue], q_p4[kDcbTieQueue];
    __shared__ uint32_t q_cnt[kDcbMaxWaves];
    __shared__ long long red[2][kDcbMaxWaves];
    __shared__ long long red_prev[2][16];
    const int l = blockIdx.y;
    int tx, ty;
    dcb_tile(a, blockIdx.x, tx, ty);
    const int Wl = a.L >> 6;             // words per row and parity in the lattice
    const int Wt = a.T >> 6;             // words per row and parity in the tile
    const int Ww = Wt + 2;               // with the halo columns
    const int rows = a.T + 2;
    const int tid = threadIdx.x, nt = blockDim.x;
    const int wave = tid >> 6, nwaves = nt >> 6;
    const uint32_t rep = a.replica0 + (uint32_t)l;
    const int y0 = ty * a.T, wc0 = tx * Wt;
    uint32_t *lat = a.lat + (size_t)l * a.L * 2 * Wl;
    // LDS word (r, par, c): tile row r - 1 (r = 0 and T + 1 are halo rows),
    // word column c - 1 of the tile (c = 0 and Wt + 1 are halo columns)
    auto widx = [&](int r, int par, int c) { return (r * 2 + par) * Ww + c; };
    auto gy = [&](int r) {
        int y = y0 + r - 1;
        if (y < 0) y += a.L;
        if (y >= a.L) y -= a.L;
        return y;
    };
    auto gw = [&](int c) {
        int w = wc0 + c - 1;
        if (w < 0) w += Wl;
        if (w >= Wl) w -= Wl;
        return w;
    };
    const TopMask m4 = top_mask(a.t4.top), m8 = top_mask(a.t8.top);
    const uint32_t wq_cap = (uint32_t)(kDcbTieQueue / nwaves), wq_base = (uint32_t)wave * wq_cap;
    const int slots_per_lattice = (a.L / a.T) * (a.L / a.T);
    long long pre_e, pre_m;
    em_prefetch(a.prev, blockIdx.x, slots_per_lattice, l, gridDim.y, tid, pre_e, pre_m);

    // ---- load the tile and its halo (corner words are not needed), a batch
    // of words per thread in flight at once
    const int ld = rows * 2 * Ww;
    constexpr int kLoadBatch = 8;
    for (int i0 = tid; i0 < ld; i0 += kLoadBatch * nt) {
        uint32_t v[kLoadBatch];
#pragma unroll
        for (int j = 0; j < kLoadBatch; ++j) {
            const int i = i0 + j * nt;
            v[j] = 0u;
            if (i < ld) {
                const int r = i / (2 * Ww), rem = i - r * 2 * Ww, par = rem / Ww, c = rem - par * Ww;
                const bool corner = (r == 0 || r == rows - 1) && (c == 0 || c == Ww - 1);
                if (!corner) v[j] = lat[((size_t)gy(r) * 2 + par) * Wl + gw(c)];
            }
        }
#pragma unroll
        for (int j = 0; j < kLoadBatch; ++j)
            if (i0 + j * nt < ld) lds[i0 + j * nt] = v[j];
    }
    __syncthreads();
    em_reduce(a.prev, blockIdx.x, slots_per_lattice, l, gridDim.y, tid, nt, pre_e, pre_m, red_prev);

    const int tasks = a.T * Wt;  // words of one colour: one per (row, column)
    uint32_t wq_n = 0;
    for (int h = 0; h < a.hits; ++h) {
        const uint64_t dsweep = a.sweep * (uint64_t)a.hits + (uint64_t)h;
        for (int col = 0; col < 2; ++col) {
            const uint32_t w3 = ctr_w3(kTagSweep, (uint32_t)col, dsweep);
            const uint32_t w3lo = ctr_w3(kTagSweepLo, (uint32_t)col, dsweep);
            for (int t = tid; t < tasks; t += nt) {
                const int r = 1 + t / Wt, c = 1 + (t - (r - 1) * Wt);
                const int y = y0 + r - 1;
                const int q = (col + y) & 1;
                const int ws = widx(r, q, c);
                const uint32_t S = lds[ws];
                const uint32_t U = lds[widx(r - 1, q, c)], D = lds[widx(r + 1, q, c)];
                const uint32_t O = lds[widx(r, 1 - q, c)];
                // even-x sites: left neighbours are the odd sites one to the
                // left; odd-x sites: right neighbours are the even sites one
                // to the right (halo columns at the tile's edges)
                const uint32_t Sh = q == 0 ? __builtin_amdgcn_alignbit(O, lds[widx(r, 1, c - 1)], 31)
                                           : __builtin_amdgcn_alignbit(lds[widx(r, 0, c + 1)], O, 1);
                const uint32_t u1 = S ^ U, u2 = S ^ D, u3 = S ^ O, u4 = S ^ Sh;
                const uint32_t t1 = u1 | u2, t2 = u3 | u4;
                const uint32_t ge2 = MCS_BOP3(u1, u2, MCS_BOP3(u3, u4, t1 & t2, (MCS_A & MCS_B) | MCS_C),
                                              (MCS_A & MCS_B) | MCS_C);
                const uint32_t c8 = ~(t1 | t2);
                const uint32_t c4 = MCS_BOP3(t1, t2, ge2, (MCS_A | MCS_B) & ~MCS_C);
                // random planes of the 32 same-colour sites j0 .. j0+31,
                // j0 = 32 w + (L/2) y, w the lattice word column
                const uint32_t blk = 2u * (uint32_t)(wc0 + c - 1) + (uint32_t)(a.L >> 5) * (uint32_t)y;
                const uint4 A = philox(make_uint4(blk, rep, (uint32_t)dsweep, w3), a.seed_lo, a.seed_hi);
                const uint4 B = philox(make_uint4(blk + 1u, rep, (uint32_t)dsweep, w3), a.seed_lo, a.seed_hi);
                uint32_t X[8];
#pragma unroll
                for (int k = 0; k < 8; ++k) X[k] = plane_pair(A, B, k);
                uint32_t lt8, eq8, lt4, eq4;
                compare_planes(X, m8, lt8, eq8);
                compare_planes(X, m4, lt4, eq4);
                uint32_t acc = MCS_BOP3(ge2, c8, lt8, MCS_A | (MCS_B & MCS_C)) | (c4 & lt4);
                const uint32_t p8 = c8 & eq8, p4 = c4 & eq4;
                const uint64_t m = __ballot((p8 | p4) != 0u);
                if (m) {
                    if (p8 | p4) {
                        const uint32_t pos =
                            wq_n + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                        if (pos < wq_cap) {
                            q_ws[wq_base + pos] = (uint32_t)ws;
                            q_blk[wq_base + pos] = blk;
                            q_p8[wq_base + pos] = p8;
                            q_p4[wq_base + pos] = p4;
                        } else {
                            uint32_t pend = p8 | p4;
                            while (pend) {
                                const int b = __builtin_ctz(pend);
                                pend &= pend - 1u;
                                const uint4 lo = philox(make_uint4(16u * blk + (uint32_t)b, rep, (uint32_t)dsweep, w3lo),
                                                        a.seed_lo, a.seed_hi);
                                if ((lo.x & 0xFFFFFFu) < (((p8 >> b) & 1u) ? a.t8.low : a.t4.low)) acc |= 1u << b;
                            }
                        }
                    }
                    wq_n = min(wq_cap, wq_n + (uint32_t)__popcll(m));
                }
                lds[ws] = S ^ acc;
            }
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) wq_n = max(wq_n, (uint32_t)__shfl_xor((int)wq_n, off, 64));
            if ((tid & 63) == 0) q_cnt[wave] = wq_n;
            __syncthreads();
            uint32_t total = 0;
            for (int sg = 0; sg < nwaves; ++sg) total += q_cnt[sg];
            for (uint32_t i = tid; i < total; i += nt) {
                uint32_t sg = 0, k = i;
                while (k >= q_cnt[sg]) k -= q_cnt[sg++];
                const uint32_t item = sg * wq_cap + k;
                const uint32_t p8 = q_p8[item], p4 = q_p4[item], blk = q_blk[item];
                uint32_t pend = p8 | p4, acc = 0u;
                while (pend) {
                    const int b = __builtin_ctz(pend);
                    pend &= pend - 1u;
                    const uint4 lo = philox(make_uint4(16u * blk + (uint32_t)b, rep, (uint32_t)dsweep, w3lo),
                                            a.seed_lo, a.seed_hi);
                    if ((lo.x & 0xFFFFFFu) < (((p8 >> b) & 1u) ? a.t8.low : a.t4.low)) acc |= 1u << b;
                }
                if (acc) lds[q_ws[item]] ^= acc;
            }
            __syncthreads();
            wq_n = 0;
        }
    }

    // ---- store the tile in place
    for (int i = tid; i < a.T * 2 * Wt; i += nt) {
        const int r = 1 + i / (2 * Wt), rem = i - (r - 1) * 2 * Wt, par = rem / Wt, c = 1 + rem - par * Wt;
        lat[((size_t)(y0 + r - 1) * 2 + par) * Wl + wc0 + c - 1] = lds[widx(r, par, c)];
    }

    // ---- energy and magnetisation of this tile's share
    if (!a.part) return;
    long long e_acc = 0, m_acc = 0;
    const bool edges = a.coarse == 1;
    for (int t = tid; t < tasks; t += nt) {
        const int r = 1 + t / Wt, c = 1 + (t - (r - 1) * Wt);
        const int y = y0 + r - 1;
        // the odd-colour word of row r (x parity q) and its four neighbours
        const int q = (1 + y) & 1;
        const uint32_t S = lds[widx(r, q, c)];
        const uint32_t U = lds[widx(r - 1, q, c)], D = lds[widx(r + 1, q, c)];
        const uint32_t O = lds[widx(r, 1 - q, c)];
        const uint32_t Sh = q == 0 ? __builtin_amdgcn_alignbit(O, lds[widx(r, 1, c - 1)], 31)
                                   : __builtin_amdgcn_alignbit(lds[widx(r, 0, c + 1)], O, 1);
        // bonds inside the tile seen from their odd end: up and down unless
        // the neighbour row is a halo row, the same-column partner always,
        // the shifted partner but for the one bit across the tile's edge
        uint32_t shm = ~0u;
        if (q == 0 && c == 1) shm = ~1u;          // x - 1 of the tile's first site
        if (q == 1 && c == Wt) shm = 0x7FFFFFFFu; // x + 1 of the tile's last site
        int anti = __builtin_popcount(S ^ O) + __builtin_popcount((S ^ Sh) & shm);
        int nb = 32 + __builtin_popcount(shm);
        if (r > 1) anti += __builtin_popcount(S ^ U), nb += 32;
        if (r < a.T) anti += __builtin_popcount(S ^ D), nb += 32;
        e_acc += 2 * anti - nb;
        m_acc += 64 - 2 * (int)(__builtin_popcount(S) + __builtin_popcount(O));
    }
    if (edges) {
        // every bond across the tile's edges: top and bottom rows against the
        // halo rows (both parity arrays), first and last column against the
        // halo columns
        for (int t = tid; t < 2 * 2 * Wt; t += nt) {
            const int side = t / (2 * Wt), rem = t - side * 2 * Wt, par = rem / Wt, c = 1 + rem - par * Wt;
            const int r = side == 0 ? 1 : a.T, rh = side == 0 ? 0 : a.T + 1;
            e_acc += 2 * __builtin_popcount(lds[widx(r, par, c)] ^ lds[widx(rh, par, c)]) - 32;
        }
        for (int r = 1 + tid; r <= a.T; r += nt) {
            // x0 (even, bit 0 of the first even word) and x0 - 1 (bit 31 of the
            // left halo's odd word); x0 + T - 1 (odd, bit 31 of the last odd
            // word) and x0 + T (bit 0 of the right halo's even word)
            const uint32_t l0 = lds[widx(r, 0, 1)] & 1u, l1 = lds[widx(r, 1, 0)] >> 31;
            const uint32_t r1 = lds[widx(r, 1, Wt)] >> 31, r0 = lds[widx(r, 0, Wt + 1)] & 1u;
            e_acc += 2 * (int)((l0 ^ l1) + (r1 ^ r0)) - 2;
        }
    }
    e_acc = wave_sum(e_acc);
    m_acc = wave_sum(m_acc);
    if ((tid & 63) == 0) {
        red[0][wave] = e_acc;
        red[1][wave] = m_acc;
    }
    __syncthreads();
    if (tid == 0) {
        // one slot per tile (a plain store: thousands of workgroups adding
        // into the same two words would queue behind each other)
        long long te = 0, tm = 0;
        for (int i = 0; i < nwaves; ++i) te += red[0][i], tm += red[1][i];
        const int nt2 = a.L / a.T;
        int64_t *slot = a.part + 2 * ((int64_t)l * nt2 * nt2 + (int64_t)ty * nt2 + tx);
        slot[0] = te;
        slot[1] = tm;
    }
}

size_t dcb_lds_bytes(int T) { return (size_t)(T + 2) * 2 * (size_t)(T / 64 + 2) * 4; }

hipError_t launch_dcb_phase(uint32_t *packed, int L, int T, int count, int coarse, int hits, uint32_t replica0,
                            uint64_t sweep, uint32_t seed_lo, uint32_t seed_hi, const SweepTables &tab, int64_t *part,
                            const EmSlots &prev, hipStream_t s)
{
    DcbArgs a;
    a.lat = packed;
    a.L = L;
    a.T = T;
    a.coarse = coarse;
    a.hits = hits;
    a.replica0 = replica0;
    a.sweep = sweep;
    a.seed_lo = seed_lo;
    a.seed_hi = seed_hi;
    a.t4 = tab.met[1];
    a.t8 = tab.met[2];
    a.part = part;
    a.prev = prev;
    if (!prev.red_in) a.prev.red_K = 0;
    const int tiles = (L / T) * (L / T) / 2;
    // one thread per word of a colour (T^2 / 64 of them), at most 256
    const int threads = std::min(256, T * T / 64);
    hipLaunchKernelGGL(k_dcb, dim3((unsigned)tiles, (unsigned)count), dim3(threads), dcb_lds_bytes(T), s, a);
    return hipGetLastError();
}

}  // namespace mcs
