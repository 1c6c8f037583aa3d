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
//  * The random top bytes of those 32 sites are eight bit-planes taken straight
//    from two Philox blocks; r32 < T becomes a bit-serial comparison of the
//    planes with the threshold's top byte.  Ties (probability 1/256 per site)
//    go to a workgroup queue in LDS and are settled together at the end of the
//    half-sweep, one low-24-bit draw per tie, so a tie in one lane does not
//    stall the other 63.
//  * The energy of each sweep is summed over odd sites while they are updated
//    (every bond has exactly one odd end), the magnetisation from popcounts of
//    the band after the sweep; one int64 atomic per band and sweep.
//  * Several lattices (each with its own inverse temperature) can share one
//    launch, which gives taller bands and so less redone halo.
#include "internal.hpp"

namespace mcs {

// Tie-queue items per workgroup (split evenly over its waves).  A wave expects
// about 0.6 * 32 / 256 ~ 0.075 ties per 32-site task; a full segment falls
// back to drawing the tie in place.
constexpr int kTieQueue = 512;

struct Tile2DArgs {
    const int8_t *src;
    int8_t *dst;
    int Lx, Ly, H;
    int64_t N;
    uint32_t seed_lo, seed_hi, replica0;
    uint64_t sweep0;
    int per_lattice;                // thresholds indexed by lattice (else entry 0)
    Thr t4[kMaxTableLattices];      // dE = 4
    Thr t8[kMaxTableLattices];      // dE = 8
    int64_t *EM;                    // [sweep][count][2] of this call, or nullptr
    int64_t em_stride;              // 2 * count
    int64_t em_sweep0;              // index of this launch's first sweep within EM
};

template <int K, bool MEASURE>
__global__ __launch_bounds__(1024) void k_tile2d(Tile2DArgs a)
{
    extern __shared__ uint32_t lds[];
    __shared__ long long red[2][16];
    __shared__ uint32_t q_j[kTieQueue], q_meta[kTieQueue];
    __shared__ uint32_t q_cnt[16];  // items queued by each wave in this half-sweep
    const int l = blockIdx.y;
    const int y0 = blockIdx.x * a.H;
    const int Hh = min(a.H, a.Ly - y0);
    constexpr int R = 2 * K;
    const int rows = Hh + 2 * R;
    const int Wd = a.Lx >> 6;
    const int nt = blockDim.x;
    const int tid = threadIdx.x;
    const int8_t *src = a.src + (int64_t)l * a.N;
    int8_t *dst = a.dst + (int64_t)l * a.N;
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

    // ---- load rows y0-R .. y0+Hh+R-1 and pack: sign bit of each byte,
    // even-x sites to array 0, odd-x sites to array 1.
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
    __syncthreads();

    for (int s = 0; s < K; ++s) {
        const uint64_t sweep = a.sweep0 + (uint64_t)s;
        long long e_acc = 0;
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
                    uint32_t pend = (c8 & eq8) | (c4 & eq4);
                    // append ties to this wave's queue segment: one item per
                    // pending lane per round, offsets from ballot + mbcnt
                    uint64_t m = __ballot(pend != 0u);
                    while (m) {
                        const uint32_t off = __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                        if (pend) {
                            const int b = __builtin_ctz(pend);
                            pend &= pend - 1u;
                            const uint32_t cls8 = (c8 >> b) & 1u;
                            const uint32_t pos = wq_n + off;
                            if (pos < wq_cap) {
                                q_j[wq_base + pos] = 16u * blk + (uint32_t)b;
                                q_meta[wq_base + pos] =
                                    (uint32_t)ws | ((uint32_t)b << 16) | (cls8 << 21) | ((uint32_t)interior << 22);
                            } else {
                                const uint4 lo = philox(
                                    make_uint4(16u * blk + (uint32_t)b, rep, (uint32_t)sweep, w3lo), a.seed_lo,
                                    a.seed_hi);
                                if ((lo.x & 0xFFFFFFu) < (cls8 ? t8.low : t4.low)) acc |= 1u << b;
                            }
                        }
                        wq_n = min(wq_cap, wq_n + (uint32_t)__popcll(m));
                        m = __ballot(pend != 0u);
                    }
                    lds[ws] = S ^ acc;
                    if (interior)
                        e_acc += 2 * (long long)(__builtin_popcount(u1 ^ acc) + __builtin_popcount(u2 ^ acc) +
                                                 __builtin_popcount(u3 ^ acc) + __builtin_popcount(u4 ^ acc)) -
                                 128;
                }
            }
            // lanes that left the row loop early hold an older (smaller) fill
            // level; the lanes that ran longest hold the final one
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) wq_n = max(wq_n, (uint32_t)__shfl_xor((int)wq_n, off, 64));
            if ((tid & 63) == 0) q_cnt[wave] = wq_n;
            __syncthreads();
            // settle the queued ties: low 24 bits of r32 against the threshold;
            // item i of the concatenated segments goes to thread i (mod nt)
            uint32_t total = 0;
            for (int sg = 0; sg < nwaves; ++sg) total += q_cnt[sg];
            for (uint32_t i = tid; i < total; i += nt) {
                uint32_t sg = 0, k = i;
                while (k >= q_cnt[sg]) k -= q_cnt[sg++];
                const uint32_t item = sg * wq_cap + k;
                const uint32_t meta = q_meta[item];
                const uint4 lo = philox(make_uint4(q_j[item], rep, (uint32_t)sweep, w3lo), a.seed_lo, a.seed_hi);
                const bool cls8 = (meta >> 21) & 1u;
                if ((lo.x & 0xFFFFFFu) < (cls8 ? t8.low : t4.low)) {
                    atomicXor(&lds[meta & 0xFFFFu], 1u << ((meta >> 16) & 31u));
                    if (MEASURE && ((meta >> 22) & 1u)) e_acc += cls8 ? 8 : 4;
                }
            }
            __syncthreads();
            wq_n = 0;
        }
        if (MEASURE) {
            long long m_acc = 0;
            for (int r = R + r0; r < R + Hh; r += Q)
                for (int w = w0; w < Wd; w += P)
                    m_acc += 64 - 2 * (__builtin_popcount(lds[widx(r, 0, w)]) + __builtin_popcount(lds[widx(r, 1, w)]));
            e_acc = wave_sum(e_acc);
            m_acc = wave_sum(m_acc);
            if ((tid & 63) == 0) {
                red[0][tid >> 6] = e_acc;
                red[1][tid >> 6] = m_acc;
            }
            __syncthreads();
            if (tid == 0) {
                long long te = 0, tm = 0;
                for (int i = 0; i < (nt >> 6); ++i) {
                    te += red[0][i];
                    tm += red[1][i];
                }
                int64_t *em = a.EM + (a.em_sweep0 + s) * a.em_stride + 2 * l;
                atomicAdd((unsigned long long *)&em[0], (unsigned long long)te);
                atomicAdd((unsigned long long *)&em[1], (unsigned long long)tm);
            }
            __syncthreads();
        }
    }

    // ---- unpack the band's own rows and store them
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
    if (a.EM) hipLaunchKernelGGL((k_tile2d<K, true>), grid, dim3(threads), lds, s, a);
    else hipLaunchKernelGGL((k_tile2d<K, false>), grid, dim3(threads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_tile2d(const SweepCall &c, const int8_t *src, int8_t *dst, uint64_t sweep0, int k, int H,
                         int threads, int64_t *EM, int64_t em_stride, int64_t em_sweep0, hipStream_t s)
{
    Tile2DArgs a;
    a.src = src;
    a.dst = dst;
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
    a.EM = EM;
    a.em_stride = em_stride;
    a.em_sweep0 = em_sweep0;
    switch (k) {
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

}  // namespace mcs
