// k_tile2d.hip -- fused multi-sweep kernel for the 2D ferromagnet (J = 1),
// checkerboard Metropolis, int8 lattices with Lx a multiple of 64.
//
// Design (gfx950):
//  * One workgroup owns a band of H full-width rows of one lattice and runs K
//    complete sweeps on it per launch.  Counter-based randomness lets it redo
//    the updates of a halo of 2K rows above and below itself exactly as their
//    owners do (each half-sweep shrinks the valid region by one row), so no
//    workgroup ever waits for another; bands read one buffer and write the
//    other.
//  * In LDS the band is bit-packed and split by x parity: word w of the even
//    (odd) array of a row holds sites x = 64 w + 2 b (+1), b = 0..31, bit set
//    <=> s = -1.  In a half-sweep one parity array per row is active and all 32
//    sites of a word share one colour, so the four neighbours of 32 sites are
//    four words (up, down, other parity, other parity shifted by one site) and
//    the Metropolis classes (dE = 8, 4, <= 0) are a few 3-input bit operations
//    (v_bitop3_b32).
//  * Between the launches of one call the lattice stays in exactly that packed
//    form in global scratch (one bit per spin, rows of 2 Lx/64 words), so only
//    the first launch reads int8 and only the last writes int8: the traffic of
//    the intermediate launches is an eighth of the int8 lattice's.
//  * The random top bytes of those 32 sites are eight bit-planes taken straight
//    from two Philox blocks; r32 < T becomes a bit-serial comparison of the
//    planes with the threshold's top byte.  Words with ties (a site whose top
//    byte equals the threshold's, probability 1/256 per site) go to a
//    workgroup queue in LDS, one item per word, and are settled together at
//    the end of the half-sweep with one low-24-bit draw per tied site, so a tie
//    in one lane does not stall the other 63.
//  * Energy and magnetisation of each sweep come from the odd half-sweep:
//    every bond has exactly one odd end, and when the odd sites of a row are
//    updated its even sites are already final, so the band's own rows give E
//    from the odd sites' four bonds and M from both parity words, with no
//    extra pass.  Each band stores its (E, M) share of every sweep in a slot
//    of its own; the first workgroups of the next launch add them up
//    (em_slots.hpp).
//  * Several lattices (each with its own inverse temperature) can share one
//    launch, which gives taller bands and so less redone halo.
#include "em_slots.hpp"
#include "internal.hpp"

namespace mcs {

// Tie-queue items per workgroup (split evenly over its waves).  One item is a
// word with at least one tied site; a wave expects about
// 1 - (1 - 0.6/256)^32 ~ 7% of its 32-site words to have one.  A full segment
// falls back to drawing the ties in place.
constexpr int kTieQueue = 512;

struct Tile2DArgs {
    const void *src;                // int8 lattices, or packed rows if in_packed
    void *dst;                      // int8 lattices, or packed rows if out_packed
    int in_packed, out_packed;
    int Lx, Ly, H;
    int64_t N;
    uint32_t seed_lo, seed_hi, replica0;
    uint64_t sweep0;
    int per_lattice;                // thresholds indexed by lattice (else entry 0)
    Thr t4[kMaxTableLattices];      // dE = 4
    Thr t8[kMaxTableLattices];      // dE = 8
    EmSlots em;                     // band sums of this launch and the previous one
};

// Draw the low 24 bits of every tied site of one word (bits of p8 | p4) and
// return the mask of those that are accepted.
__device__ __forceinline__ uint32_t settle_ties(uint32_t p8, uint32_t p4, uint32_t blk, uint32_t rep,
                                                uint32_t sweep_lo, uint32_t w3lo, uint32_t k0, uint32_t k1,
                                                const Thr &t4, const Thr &t8)
{
    uint32_t pend = p8 | p4, acc = 0u;
    while (pend) {
        const int b = __builtin_ctz(pend);
        pend &= pend - 1u;
        const uint4 lo = philox(make_uint4(16u * blk + (uint32_t)b, rep, sweep_lo, w3lo), k0, k1);
        if ((lo.x & 0xFFFFFFu) < (((p8 >> b) & 1u) ? t8.low : t4.low)) acc |= 1u << b;
    }
    return acc;
}

template <int K, bool MEASURE>
__global__ __launch_bounds__(1024) void k_tile2d(Tile2DArgs a)
{
    extern __shared__ uint32_t lds[];
    __shared__ int red[2][16];
    __shared__ long long red64[2][16];
    __shared__ uint32_t q_ws[kTieQueue], q_blk[kTieQueue], q_p8[kTieQueue], q_p4[kTieQueue];
    __shared__ uint32_t q_cnt[16];  // items queued by each wave in this half-sweep
    const int l = blockIdx.y;
    const int y0 = blockIdx.x * a.H;
    const int Hh = min(a.H, a.Ly - y0);
    constexpr int R = 2 * K;
    const int rows = Hh + 2 * R;
    const int Wd = a.Lx >> 6;
    const int nt = blockDim.x;
    const int tid = threadIdx.x;
    const uint32_t rep = a.replica0 + (uint32_t)l;
    const Thr t4 = a.t4[a.per_lattice ? l : 0];
    const Thr t8 = a.t8[a.per_lattice ? l : 0];
    const TopMask m4 = top_mask(t4.top), m8 = top_mask(t8.top);
    // thread -> (word column, first row, row stride); no division in the loops
    int P, Q, w0, r0;
    if (Wd <= nt) {
        P = Wd;
        Q = nt / Wd;
        w0 = tid % Wd;
        r0 = tid / Wd;
        if (r0 >= Q) r0 = 1 << 30;  // surplus threads idle
    } else {
        P = nt;
        Q = 1;
        w0 = tid;
        r0 = 0;
    }
    auto widx = [&](int r, int par, int w) { return (r * 2 + par) * Wd + w; };
    auto lat_row = [&](int r) {
        int y = y0 - R + r;
        while (y < 0) y += a.Ly;
        while (y >= a.Ly) y -= a.Ly;
        return y;
    };
    // tie queue: wave w owns items [w * wq_cap, (w + 1) * wq_cap); its fill
    // level wq_n is wave-uniform
    const int wave = tid >> 6, nwaves = nt >> 6;
    const uint32_t wq_cap = (uint32_t)(kTieQueue / nwaves), wq_base = (uint32_t)wave * wq_cap;
    uint32_t wq_n = 0;
    const int ntile = gridDim.x, nlat = gridDim.y;
    long long pre_e, pre_m;
    em_prefetch(a.em, blockIdx.x, ntile, l, nlat, tid, pre_e, pre_m);

    // ---- load rows y0-R .. y0+Hh+R-1
    if (a.in_packed) {
        // packed row y of lattice l: 2 Wd words at (l Ly + y) 2 Wd, even array first
        const uint2 *src = (const uint2 *)a.src + (int64_t)l * a.Ly * Wd;
        for (int r = r0; r < rows; r += Q) {
            const uint2 *row = src + (int64_t)lat_row(r) * Wd;
            for (int w = w0; w < Wd; w += P) ((uint2 *)lds)[r * Wd + w] = row[w];
        }
    } else {
        // int8: sign bit of each byte, even-x sites to array 0, odd-x to array 1
        const int8_t *src = (const int8_t *)a.src + (int64_t)l * a.N;
        for (int r = r0; r < rows; r += Q) {
            const int8_t *row = src + (int64_t)lat_row(r) * a.Lx;
            for (int w = w0; w < Wd; w += P) {
                const uint4 *p = (const uint4 *)(row + 64 * w);
                uint32_t ev = 0, od = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const uint4 v = p[q];
                    const uint32_t dw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        // sign bits at 7, 15, 23, 31 -> m + (m << 15) puts the two
                        // even-x bits at 22..23 and the two odd-x bits at 30..31
                        const uint32_t m = dw[i] & 0x80808080u;
                        const uint32_t Pm = m + (m << 15);
                        const int sh = 2 * (4 * q + i);
                        ev |= ((Pm >> 22) & 3u) << sh;
                        od |= (Pm >> 30) << sh;
                    }
                }
                lds[widx(r, 0, w)] = ev;
                lds[widx(r, 1, w)] = od;
            }
        }
    }
    __syncthreads();
    em_reduce(a.em, blockIdx.x, ntile, l, nlat, tid, nt, pre_e, pre_m, red64);

    for (int s = 0; s < K; ++s) {
        const uint64_t sweep = a.sweep0 + (uint64_t)s;
        int e_acc = 0, m_acc = 0;  // this thread's share of the band's E and M
        for (int c = 0; c < 2; ++c) {
            const int p = 2 * s + c;
            const int r_lo = p + 1, r_hi = rows - p - 1;
            const uint32_t w3 = ctr_w3(kTagSweep, (uint32_t)c, sweep);
            const uint32_t w3lo = ctr_w3(kTagSweepLo, (uint32_t)c, sweep);
            for (int r = r_lo + r0; r < r_hi; r += Q) {
                const int y = lat_row(r);
                const int q = (c + y) & 1;
                const bool interior = MEASURE && c == 1 && r >= R && r < R + Hh;
                const uint32_t rowblk = (uint32_t)(a.Lx >> 5) * (uint32_t)y;
                for (int w = w0; w < Wd; w += P) {
                    const int ws = widx(r, q, w);
                    const uint32_t S = lds[ws];
                    const uint32_t U = lds[widx(r - 1, q, w)], D = lds[widx(r + 1, q, w)];
                    const uint32_t O = lds[widx(r, 1 - q, w)];
                    // even sites: left neighbours are the odd sites one to the
                    // left (carry from the previous odd word); odd sites: right
                    // neighbours are the even sites one to the right
                    const int wl = w == 0 ? Wd - 1 : w - 1, wr = w + 1 == Wd ? 0 : w + 1;
                    const uint32_t Ol = lds[widx(r, 1, wl)], Er = lds[widx(r, 0, wr)];
                    const uint32_t Sh = q == 0 ? __builtin_amdgcn_alignbit(O, Ol, 31) : __builtin_amdgcn_alignbit(Er, O, 1);
                    const uint32_t u1 = S ^ U, u2 = S ^ D, u3 = S ^ O, u4 = S ^ Sh;
                    const uint32_t t1 = u1 | u2, t2 = u3 | u4;
                    // at least two of four anti-aligned neighbours: dE <= 0
                    const uint32_t ge2 = MCS_BOP3(u1, u2, MCS_BOP3(u3, u4, t1 & t2, (MCS_A & MCS_B) | MCS_C),
                                                  (MCS_A & MCS_B) | MCS_C);
                    const uint32_t c8 = ~(t1 | t2);                      // none: dE = 8
                    const uint32_t c4 = MCS_BOP3(t1, t2, ge2, (MCS_A | MCS_B) & ~MCS_C);  // one: dE = 4
                    // random planes of the 32 sites j0 .. j0+31, j0 = 32 w + (Lx/2) y
                    const uint32_t blk = 2u * (uint32_t)w + rowblk;
                    const uint4 A = philox(make_uint4(blk, rep, (uint32_t)sweep, w3), a.seed_lo, a.seed_hi);
                    const uint4 B = philox(make_uint4(blk + 1u, rep, (uint32_t)sweep, w3), a.seed_lo, a.seed_hi);
                    uint32_t X[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) X[k] = plane_pair(A, B, k);
                    uint32_t lt8, eq8, lt4, eq4;
                    compare_planes(X, m8, lt8, eq8);
                    compare_planes(X, m4, lt4, eq4);
                    uint32_t acc = MCS_BOP3(ge2, c8, lt8, MCS_A | (MCS_B & MCS_C)) | (c4 & lt4);
                    const uint32_t p8 = c8 & eq8, p4 = c4 & eq4;
                    // words with ties join this wave's queue segment, one item
                    // per word, offsets from ballot + mbcnt
                    const uint64_t m = __ballot((p8 | p4) != 0u);
                    if (m) {
                        if (p8 | p4) {
                            const uint32_t pos = wq_n + __builtin_amdgcn_mbcnt_hi(
                                                            (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                            if (pos < wq_cap) {
                                q_ws[wq_base + pos] = (uint32_t)ws | ((uint32_t)interior << 31);
                                q_blk[wq_base + pos] = blk;
                                q_p8[wq_base + pos] = p8;
                                q_p4[wq_base + pos] = p4;
                            } else {
                                acc |= settle_ties(p8, p4, blk, rep, (uint32_t)sweep, w3lo, a.seed_lo, a.seed_hi, t4,
                                                   t8);
                            }
                        }
                        wq_n = min(wq_cap, wq_n + (uint32_t)__popcll(m));
                    }
                    const uint32_t Sn = S ^ acc;
                    lds[ws] = Sn;
                    if (interior) {
                        // bonds of the odd sites after their update: 2 (#anti-aligned) - 4 each
                        e_acc += 2 * (int)(__builtin_popcount(u1 ^ acc) + __builtin_popcount(u2 ^ acc) +
                                           __builtin_popcount(u3 ^ acc) + __builtin_popcount(u4 ^ acc)) -
                                 128;
                        m_acc += 64 - 2 * (int)(__builtin_popcount(Sn) + __builtin_popcount(O));
                    }
                }
            }
            // lanes that left the row loop early hold an older (smaller) fill
            // level; the lanes that ran longest hold the final one
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) wq_n = max(wq_n, (uint32_t)__shfl_xor((int)wq_n, off, 64));
            if ((tid & 63) == 0) q_cnt[wave] = wq_n;
            __syncthreads();
            // settle the queued words: item i of the concatenated segments goes
            // to thread i (mod nt); every item is a different word
            uint32_t total = 0;
            for (int sg = 0; sg < nwaves; ++sg) total += q_cnt[sg];
            for (uint32_t i = tid; i < total; i += nt) {
                uint32_t sg = 0, k = i;
                while (k >= q_cnt[sg]) k -= q_cnt[sg++];
                const uint32_t item = sg * wq_cap + k;
                const uint32_t p8 = q_p8[item], p4 = q_p4[item], wsm = q_ws[item];
                const uint32_t acc =
                    settle_ties(p8, p4, q_blk[item], rep, (uint32_t)sweep, w3lo, a.seed_lo, a.seed_hi, t4, t8);
                if (acc) {
                    const uint32_t ws = wsm & 0x7FFFFFFFu, old = lds[ws];
                    lds[ws] = old ^ acc;
                    if (MEASURE && (wsm >> 31)) {
                        e_acc += 8 * __builtin_popcount(acc & p8) + 4 * __builtin_popcount(acc & p4);
                        m_acc += 2 * (2 * __builtin_popcount(old & acc) - __builtin_popcount(acc));
                    }
                }
            }
            if (MEASURE && c == 1) {
                e_acc = wave_sum_i(e_acc);
                m_acc = wave_sum_i(m_acc);
                if ((tid & 63) == 0) {
                    red[0][wave] = e_acc;
                    red[1][wave] = m_acc;
                }
            }
            __syncthreads();
            wq_n = 0;
        }
        if (MEASURE && tid == 0) {
            long long te = 0, tm = 0;
            for (int i = 0; i < nwaves; ++i) {
                te += red[0][i];
                tm += red[1][i];
            }
            *em_slot(a.em.slots, s, l, nlat, blockIdx.x, ntile) = make_longlong2(te, tm);
        }
    }

    // ---- store the band's own rows
    if (a.out_packed) {
        uint2 *dst = (uint2 *)a.dst + (int64_t)l * a.Ly * Wd;
        for (int r = R + r0; r < R + Hh; r += Q) {
            uint2 *row = dst + (int64_t)(y0 + r - R) * Wd;
            for (int w = w0; w < Wd; w += P) row[w] = ((const uint2 *)lds)[r * Wd + w];
        }
        return;
    }
    int8_t *dst = (int8_t *)a.dst + (int64_t)l * a.N;
    for (int r = R + r0; r < R + Hh; r += Q) {
        int8_t *row = dst + (int64_t)(y0 + r - R) * a.Lx;
        for (int w = w0; w < Wd; w += P) {
            const uint32_t ev = lds[widx(r, 0, w)], od = lds[widx(r, 1, w)];
            uint4 *p = (uint4 *)(row + 64 * w);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t dw[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int sh = 2 * (4 * q + i);
                    // bytes: x = 16q+4i (even bit sh), +1 (odd bit sh), +2 (even sh+1), +3 (odd sh+1)
                    const uint32_t bits = ((ev >> sh) & 1u) | (((od >> sh) & 1u) << 8) |
                                          (((ev >> (sh + 1)) & 1u) << 16) | (((od >> (sh + 1)) & 1u) << 24);
                    // bit 0 -> byte 0x01 (+1), bit 1 -> byte 0xFF (-1)
                    dw[i] = __builtin_amdgcn_perm(0u, 0x0000FF01u, bits);
                }
                p[q] = make_uint4(dw[0], dw[1], dw[2], dw[3]);
            }
        }
    }
}

// ---------------------------------------------------------------------------
bool tile2d_supported(const SweepCall &c, int layout)
{
    return layout == MC_INT8 && c.g.dims == 2 && c.J == nullptr && c.rule == 0 && (c.g.Lx % 64) == 0 &&
           c.g.Lx <= 16384 && c.g.Ly >= 4 && (!c.per_lattice || c.g.count <= kMaxTableLattices);
}

size_t tile2d_lds_bytes(int Lx, int H, int K) { return (size_t)(H + 4 * K) * 2 * (size_t)(Lx / 64) * 4; }

template <int K>
static hipError_t launch_k(const Tile2DArgs &a, int count, int threads, hipStream_t s)
{
    const int tiles = (a.Ly + a.H - 1) / a.H;
    const size_t lds = tile2d_lds_bytes(a.Lx, a.H, K);
    dim3 grid((unsigned)tiles, (unsigned)count);
    // allow the largest dynamic LDS a plan may ask for (64 KB) next to the
    // static tie queue, once per device and kernel instance
    static LdsLimit lim[2];
    const bool measure = a.em.slots != nullptr;
    const void *f = measure ? (const void *)k_tile2d<K, true> : (const void *)k_tile2d<K, false>;
    const hipError_t e = lim[measure ? 1 : 0].ensure(f, 65536);
    if (e != hipSuccess) return e;
    if (measure) hipLaunchKernelGGL((k_tile2d<K, true>), grid, dim3(threads), lds, s, a);
    else hipLaunchKernelGGL((k_tile2d<K, false>), grid, dim3(threads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_tile2d(const SweepCall &c, const void *src, int in_packed, void *dst, int out_packed,
                         uint64_t sweep0, int k, int H, int threads, const EmSlots &em, hipStream_t s)
{
    Tile2DArgs a;
    a.src = src;
    a.dst = dst;
    a.in_packed = in_packed;
    a.out_packed = out_packed;
    a.Lx = c.g.Lx;
    a.Ly = c.g.Ly;
    a.H = H;
    a.N = c.g.N;
    a.seed_lo = c.seed_lo;
    a.seed_hi = c.seed_hi;
    a.replica0 = c.replica0;
    a.sweep0 = sweep0;
    a.per_lattice = c.per_lattice;
    for (int i = 0; i < kMaxTableLattices; ++i) {
        const SweepTables &t = (c.per_lattice && i < c.g.count) ? c.tabs[i] : c.tab;
        a.t4[i] = t.met[1];
        a.t8[i] = t.met[2];
    }
    a.em = em;
    if (k == 0) a.em.slots = nullptr;
    if (!em.red_in) a.em.red_K = 0;
    switch (k) {
    case 0: return launch_k<0>(a, c.g.count, threads, s);
    case 1: return launch_k<1>(a, c.g.count, threads, s);
    case 2: return launch_k<2>(a, c.g.count, threads, s);
    case 3: return launch_k<3>(a, c.g.count, threads, s);
    case 4: return launch_k<4>(a, c.g.count, threads, s);
    case 5: return launch_k<5>(a, c.g.count, threads, s);
    case 6: return launch_k<6>(a, c.g.count, threads, s);
    case 7: return launch_k<7>(a, c.g.count, threads, s);
    case 8: return launch_k<8>(a, c.g.count, threads, s);
    default: return hipErrorInvalidValue;
    }
}

// Adds up the workgroup sums of the last launch of a call: workgroup (j, l)
// writes EM of sweep j of that launch for lattice l.
__global__ __launch_bounds__(256) void k_em_slots(const int64_t *slots, int tiles, int64_t *EM, int64_t em_stride,
                                                  int64_t sweep0)
{
    __shared__ long long part[2][4];
    const int j = blockIdx.x, l = blockIdx.y, count = gridDim.y, tid = threadIdx.x;
    const longlong2 *src = em_slot((int64_t *)slots, j, l, count, 0, tiles);
    long long se = 0, sm = 0;
    for (int t = tid; t < tiles; t += 256) {
        const longlong2 v = src[t];
        se += v.x;
        sm += v.y;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        se += __shfl_xor(se, off, 64);
        sm += __shfl_xor(sm, off, 64);
    }
    if ((tid & 63) == 0) {
        part[0][tid >> 6] = se;
        part[1][tid >> 6] = sm;
    }
    __syncthreads();
    if (tid == 0) {
        int64_t *em = EM + (sweep0 + j) * em_stride + 2 * l;
        em[0] = part[0][0] + part[0][1] + part[0][2] + part[0][3];
        em[1] = part[1][0] + part[1][1] + part[1][2] + part[1][3];
    }
}

hipError_t launch_em_slots(const int64_t *slots, int tiles, int count, int K, int64_t *EM, int64_t em_stride,
                           int64_t sweep0, hipStream_t s)
{
    if (K <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_em_slots, dim3((unsigned)K, (unsigned)count), dim3(256), 0, s, slots, tiles, EM, em_stride,
                       sweep0);
    return hipGetLastError();
}

// Per-band (E, M) slots of one launch: K <= 8 sweeps x count lattices x
// ceil(Ly / 4) bands (a plan's band height is at least 4) x 16 bytes.
size_t tile2d_slot_bytes(const Geom &g)
{
    const size_t b = (size_t)8 * (size_t)g.count * (size_t)((g.Ly + 3) / 4) * 16;
    return (b + 255) / 256 * 256;
}

}  // namespace mcs
