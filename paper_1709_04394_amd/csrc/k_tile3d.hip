// k_tile3d.hip -- fused multi-sweep kernel for 3D simple-cubic lattices:
// Ising (J = 1) or +-J couplings, checkerboard Metropolis or heat-bath, int8
// lattices with Lx a multiple of 64 (Sec. "Checkerboard scheme": the
// checkerboard decomposition holds for any bipartite lattice).
//
// Design (gfx950):
//  * One workgroup owns a tile of hy x hz full-width rows (y, z) of one
//    lattice and runs K sweeps on it per launch, redoing a halo of 2K rows on
//    each side in y and z (each half-sweep shrinks the valid region by one row
//    per side), so no workgroup waits for another.
//  * Rows are bit-packed in LDS and split by x parity exactly as in the 2D
//    kernel: the six neighbours of 32 same-colour sites are six words, and
//    with couplings (bit set <=> J < 0, packed the same way) a bond is
//    unsatisfied where spin ^ neighbour ^ coupling is set.
//  * A site's class is a 3-bit count kept bit-sliced (carry-save adders over
//    the six bond words): Metropolis counts unsatisfied bonds a (dE = 12 - 4a,
//    a >= 3 always accepts); heat-bath counts neighbours with J s_j = -1, d
//    (h = 6 - 2d).  Each class has its own threshold; per random bit-plane the
//    threshold bit of every site comes from a multiplexer over the class bits,
//    and r32 < T is one bit-serial comparison.  Ties (top byte equal) are
//    queued per word and settled after the half-sweep.
//  * Per-sweep E and M are summed from the odd half-sweep, as in 2D, and
//    stored per tile in slots that the next launch adds up (em_slots.hpp).
//  * Between the launches of one call the lattice stays packed in global
//    scratch.
#include "internal.hpp"

namespace mcs {

constexpr int kTieQ3 = 256;  // queued words per workgroup (split over its waves)

struct Tile3DArgs {
    const void *src;
    void *dst;
    int in_packed, out_packed;
    const uint32_t *Jp;  // packed couplings [3][Lz][Ly][2 Wd] (bit set <=> J < 0), or nullptr
    int Lx, Ly, Lz, nty, ntz;
    int64_t N;
    uint32_t seed_lo, seed_hi, replica0;
    uint64_t sweep0;
    int per_lattice;
    // class thresholds (top byte 0..255 and low 24 bits, low = 2^24 encodes
    // T = 2^32 as 255 * 2^24 + 2^24); Metropolis: class a, T of dE = 12 - 4a
    // (a <= 2); heat-bath: class d, T of h = 6 - 2d
    uint32_t top[kMaxTableLattices][8];
    uint32_t low[kMaxTableLattices][8];
    EmSlots em;  // tile sums of this launch and the previous one
};

// floor(t / n) and t mod n for small non-negative t (below 2^20) through a
// float reciprocal with one correction step
__device__ __forceinline__ void divmod_small(int t, int n, float inv, int &q, int &r)
{
    q = (int)((float)t * inv);
    r = t - q * n;
    if (r < 0) {
        --q;
        r += n;
    } else if (r >= n) {
        ++q;
        r -= n;
    }
}

template <int K, bool MEASURE, bool HB, bool HASJ>
__global__ __launch_bounds__(1024) void k_tile3d(Tile3DArgs a)
{
    extern __shared__ uint32_t lds[];
    __shared__ int red[2][16];
    __shared__ long long red64[2][16];
    __shared__ uint32_t q_ws[kTieQ3], q_blk[kTieQ3], q_p[kTieQ3], q_c0[kTieQ3], q_c1[kTieQ3], q_c2[kTieQ3];
    __shared__ uint32_t q_cnt[16];
    __shared__ uint32_t tlow[8];
    const int l = blockIdx.y;
    const int ty = blockIdx.x % a.nty, tz = blockIdx.x / a.nty;
    const int y0 = (int)((int64_t)ty * a.Ly / a.nty), y1 = (int)((int64_t)(ty + 1) * a.Ly / a.nty);
    const int z0 = (int)((int64_t)tz * a.Lz / a.ntz), z1 = (int)((int64_t)(tz + 1) * a.Lz / a.ntz);
    const int hy = y1 - y0, hz = z1 - z0;
    constexpr int R = 2 * K;
    const int Ry = hy + 2 * R, Rz = hz + 2 * R, rows = Ry * Rz;
    const int Wd = a.Lx >> 6;
    const int nt = blockDim.x, tid = threadIdx.x;
    const uint32_t rep = a.replica0 + (uint32_t)l;
    const int li = a.per_lattice ? l : 0;
    if (tid < 8) tlow[tid] = a.low[li][tid];
    uint32_t *Jl = lds + (size_t)rows * 2 * Wd;  // 3 coupling planes of rows
    // per random plane k and class c the threshold bit as a full mask, kept
    // in the dynamic LDS array the sweep also writes, so the per-plane reads
    // stay in the loop (broadcast ds_read_b128) instead of occupying registers
    uint32_t *tm = lds + (((size_t)rows * 2 * Wd * (HASJ ? 4 : 1) + 3) & ~(size_t)3);
    if (tid < 64) tm[tid] = ((a.top[li][tid & 7] >> (tid >> 3)) & 1u) ? ~0u : 0u;
    // thread -> (word column, first row, row stride)
    int P, Q, w0, r0;
    if (Wd <= nt) {
        P = Wd;
        Q = nt / Wd;
        w0 = tid % Wd;
        r0 = tid / Wd;
        if (r0 >= Q) r0 = 1 << 28;
    } else {
        P = nt;
        Q = 1;
        w0 = tid;
        r0 = 0;
    }
    auto widx = [&](int row, int par, int w) { return (row * 2 + par) * Wd + w; };
    auto wrap = [](int v, int n) {
        while (v < 0) v += n;
        while (v >= n) v -= n;
        return v;
    };
    const int wave = tid >> 6, nwaves = nt >> 6;
    const uint32_t wq_cap = (uint32_t)(kTieQ3 / nwaves), wq_base = (uint32_t)wave * wq_cap;
    uint32_t wq_n = 0;
    const int64_t plane_rows = (int64_t)a.Ly * a.Lz;
    const int ntile = gridDim.x, nlat = gridDim.y;
    long long pre_e, pre_m;
    em_prefetch(a.em, blockIdx.x, ntile, l, nlat, tid, pre_e, pre_m);

    // ---- load rows (z0-R .. z1+R-1) x (y0-R .. y1+R-1), row id = rz Ry + ry
    const float invRy = 1.0f / (float)Ry;
    for (int rr = r0; rr < rows; rr += Q) {
        int rz, ry;
        divmod_small(rr, Ry, invRy, rz, ry);
        const int y = wrap(y0 - R + ry, a.Ly), z = wrap(z0 - R + rz, a.Lz);
        const int64_t grow = (int64_t)z * a.Ly + y;
        if (a.in_packed) {
            const uint2 *src = (const uint2 *)a.src + ((int64_t)l * plane_rows + grow) * Wd;
            for (int w = w0; w < Wd; w += P) ((uint2 *)lds)[rr * Wd + w] = src[w];
        } else {
            const int8_t *row = (const int8_t *)a.src + (int64_t)l * a.N + grow * a.Lx;
            for (int w = w0; w < Wd; w += P) {
                const uint4 *p = (const uint4 *)(row + 64 * w);
                uint32_t ev = 0, od = 0;
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) {
                    const uint4 v = p[qq];
                    const uint32_t dw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const uint32_t m = dw[i] & 0x80808080u;
                        const uint32_t Pm = m + (m << 15);
                        const int sh = 2 * (4 * qq + i);
                        ev |= ((Pm >> 22) & 3u) << sh;
                        od |= (Pm >> 30) << sh;
                    }
                }
                lds[widx(rr, 0, w)] = ev;
                lds[widx(rr, 1, w)] = od;
            }
        }
        if (HASJ) {
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const uint2 *src = (const uint2 *)a.Jp + ((int64_t)d * plane_rows + grow) * Wd;
                for (int w = w0; w < Wd; w += P) ((uint2 *)Jl)[((size_t)d * rows + rr) * Wd + w] = src[w];
            }
        }
    }
    __syncthreads();
    em_reduce(a.em, blockIdx.x, ntile, l, nlat, tid, nt, pre_e, pre_m, red64);

    for (int s = 0; s < K; ++s) {
        const uint64_t sweep = a.sweep0 + (uint64_t)s;
        int e_acc = 0, m_acc = 0;
        for (int c = 0; c < 2; ++c) {
            const int p = 2 * s + c;
            const int ny = Ry - 2 * p - 2, nz = Rz - 2 * p - 2;
            const int nrow = ny * nz;
            const float invny = 1.0f / (float)ny;
            const uint32_t w3 = ctr_w3(kTagSweep, (uint32_t)c, sweep);
            const uint32_t w3lo = ctr_w3(kTagSweepLo, (uint32_t)c, sweep);
            for (int rr = r0; rr < nrow; rr += Q) {
                int iz, iy;
                divmod_small(rr, ny, invny, iz, iy);
                const int ry = p + 1 + iy, rz = p + 1 + iz;
                const int row = rz * Ry + ry;
                const int y = wrap(y0 - R + ry, a.Ly), z = wrap(z0 - R + rz, a.Lz);
                const int q = (c + y + z) & 1;
                const bool interior = MEASURE && c == 1 && ry >= R && ry < R + hy && rz >= R && rz < R + hz;
                const uint32_t rowblk = (uint32_t)(a.Lx >> 5) * (uint32_t)((int64_t)z * a.Ly + y);
                for (int w = w0; w < Wd; w += P) {
                    const int ws = widx(row, q, w);
                    const uint32_t S = lds[ws];
                    const uint32_t O = lds[widx(row, 1 - q, w)];
                    const int wl = w == 0 ? Wd - 1 : w - 1, wr = w + 1 == Wd ? 0 : w + 1;
                    // x neighbours: even sites (q = 0) have +x in O, -x one odd
                    // site to the left; odd sites the mirror image
                    const uint32_t Ol = lds[widx(row, 1, wl)], Er = lds[widx(row, 0, wr)];
                    const uint32_t nxp = q == 0 ? O : __builtin_amdgcn_alignbit(Er, O, 1);
                    const uint32_t nxm = q == 0 ? __builtin_amdgcn_alignbit(O, Ol, 31) : O;
                    uint32_t w1 = nxp, w2 = nxm;
                    uint32_t w3b = lds[widx(row + 1, q, w)], w4 = lds[widx(row - 1, q, w)];
                    uint32_t w5 = lds[widx(row + Ry, q, w)], w6 = lds[widx(row - Ry, q, w)];
                    if (HASJ) {
                        auto jidx = [&](int d, int rw, int par, int ww) { return ((d * rows + rw) * 2 + par) * Wd + ww; };
                        const uint32_t Jxp = Jl[jidx(0, row, q, w)];
                        const uint32_t Jxm = q == 0 ? __builtin_amdgcn_alignbit(Jl[jidx(0, row, 1, w)],
                                                                                  Jl[jidx(0, row, 1, wl)], 31)
                                                    : Jl[jidx(0, row, 0, w)];
                        w1 ^= Jxp;
                        w2 ^= Jxm;
                        w3b ^= Jl[jidx(1, row, q, w)];
                        w4 ^= Jl[jidx(1, row - 1, q, w)];
                        w5 ^= Jl[jidx(2, row, q, w)];
                        w6 ^= Jl[jidx(2, row - Ry, q, w)];
                    }
                    // bit set in wk <=> J s_j = -1 for that bond; Metropolis
                    // counts unsatisfied bonds S ^ wk, heat-bath counts wk
                    uint32_t x1 = w1, x2 = w2, x3 = w3b, x4 = w4, x5 = w5, x6 = w6;
                    if (!HB) {
                        x1 ^= S;
                        x2 ^= S;
                        x3 ^= S;
                        x4 ^= S;
                        x5 ^= S;
                        x6 ^= S;
                    }
                    const uint32_t s1 = MCS_BOP3(x1, x2, x3, MCS_A ^ MCS_B ^ MCS_C);
                    const uint32_t k1 = MCS_BOP3(x1, x2, x3, (MCS_A & MCS_B) | (MCS_A & MCS_C) | (MCS_B & MCS_C));
                    const uint32_t s2 = MCS_BOP3(x4, x5, x6, MCS_A ^ MCS_B ^ MCS_C);
                    const uint32_t k2 = MCS_BOP3(x4, x5, x6, (MCS_A & MCS_B) | (MCS_A & MCS_C) | (MCS_B & MCS_C));
                    const uint32_t c0 = s1 ^ s2, kk = s1 & s2;
                    const uint32_t c1 = MCS_BOP3(k1, k2, kk, MCS_A ^ MCS_B ^ MCS_C);
                    const uint32_t c2 = MCS_BOP3(k1, k2, kk, (MCS_A & MCS_B) | (MCS_A & MCS_C) | (MCS_B & MCS_C));
                    // Metropolis: a >= 3 accepts without a random number
                    const uint32_t ge3 = HB ? 0u : (c2 | (c1 & c0));
                    // random planes of the 32 sites
                    const uint32_t blk = 2u * (uint32_t)w + rowblk;
                    const uint4 A = philox(make_uint4(blk, rep, (uint32_t)sweep, w3), a.seed_lo, a.seed_hi);
                    const uint4 B = philox(make_uint4(blk + 1u, rep, (uint32_t)sweep, w3), a.seed_lo, a.seed_hi);
                    // bit-serial r < T(class) from the least significant plane;
                    // the threshold bit of each site is chosen by its class
                    uint32_t lt = 0u, eq = ~0u;
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const uint32_t X = plane_pair(A, B, k);
                        const uint4 ml = *(const uint4 *)&tm[8 * k];
                        uint32_t T;
                        if (HB) {
                            const uint4 mh = *(const uint4 *)&tm[8 * k + 4];
                            const uint32_t m01 = (c0 & ml.y) | (~c0 & ml.x);
                            const uint32_t m23 = (c0 & ml.w) | (~c0 & ml.z);
                            const uint32_t m45 = (c0 & mh.y) | (~c0 & mh.x);
                            const uint32_t lo4 = (c1 & m23) | (~c1 & m01);
                            const uint32_t hi4 = (c1 & mh.z) | (~c1 & m45);
                            T = (c2 & hi4) | (~c2 & lo4);
                        } else {
                            const uint32_t m01 = (c0 & ml.y) | (~c0 & ml.x);
                            T = (c1 & ml.z) | (~c1 & m01);
                        }
                        lt = MCS_BOP3(X, T, lt, (~MCS_A & MCS_B) | (~MCS_A & MCS_C) | (MCS_B & MCS_C));
                        eq = MCS_BOP3(eq, X, T, MCS_A & ~(MCS_B ^ MCS_C));
                    }
                    // Metropolis: accept mask (flip); heat-bath: new spin
                    // word, +1 (bit 0) where r < T; ties provisionally -1
                    uint32_t acc = HB ? ~lt : (ge3 | lt);
                    const uint32_t pend = HB ? eq : (eq & ~ge3);
                    const uint64_t m = __ballot(pend != 0u);
                    if (m) {
                        if (pend) {
                            const uint32_t pos = wq_n + __builtin_amdgcn_mbcnt_hi(
                                                            (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                            if (pos < wq_cap) {
                                const uint32_t it = wq_base + pos;
                                q_ws[it] = (uint32_t)ws | ((uint32_t)interior << 31);
                                q_blk[it] = blk;
                                q_p[it] = pend;
                                q_c0[it] = c0 & pend;
                                q_c1[it] = c1 & pend;
                                q_c2[it] = c2 & pend;
                            } else {
                                uint32_t pp = pend, f = 0u;
                                while (pp) {
                                    const int b = __builtin_ctz(pp);
                                    pp &= pp - 1u;
                                    const uint32_t cls = ((c0 >> b) & 1u) | (((c1 >> b) & 1u) << 1) | (((c2 >> b) & 1u) << 2);
                                    const uint4 lo = philox(make_uint4(16u * blk + (uint32_t)b, rep, (uint32_t)sweep, w3lo),
                                                            a.seed_lo, a.seed_hi);
                                    if ((lo.x & 0xFFFFFFu) < tlow[cls]) f |= 1u << b;
                                }
                                acc ^= HB ? f : 0u;
                                acc |= HB ? 0u : f;
                            }
                        }
                        wq_n = min(wq_cap, wq_n + (uint32_t)__popcll(m));
                    }
                    const uint32_t Sn = HB ? acc : (S ^ acc);
                    lds[ws] = Sn;
                    if (interior) {
                        // bonds of the odd sites after their update
                        const uint32_t b1 = Sn ^ w1, b2 = Sn ^ w2, b3 = Sn ^ w3b, b4 = Sn ^ w4, b5 = Sn ^ w5,
                                       b6 = Sn ^ w6;
                        e_acc += 2 * (int)(__builtin_popcount(b1) + __builtin_popcount(b2) + __builtin_popcount(b3) +
                                           __builtin_popcount(b4) + __builtin_popcount(b5) + __builtin_popcount(b6)) -
                                 192;
                        m_acc += 64 - 2 * (int)(__builtin_popcount(Sn) + __builtin_popcount(O));
                    }
                }
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
                const uint32_t it = sg * wq_cap + k;
                const uint32_t wsm = q_ws[it], blk = q_blk[it], pend = q_p[it];
                const uint32_t c0 = q_c0[it], c1 = q_c1[it], c2 = q_c2[it];
                uint32_t pp = pend, f = 0u;
                int de = 0;
                while (pp) {
                    const int b = __builtin_ctz(pp);
                    pp &= pp - 1u;
                    const uint32_t cls = ((c0 >> b) & 1u) | (((c1 >> b) & 1u) << 1) | (((c2 >> b) & 1u) << 2);
                    const uint4 lo = philox(make_uint4(16u * blk + (uint32_t)b, rep, (uint32_t)sweep, w3lo), a.seed_lo,
                                            a.seed_hi);
                    if ((lo.x & 0xFFFFFFu) < tlow[cls]) {
                        f |= 1u << b;
                        // energy change of the flip: Metropolis 12 - 4a,
                        // heat-bath (-1 -> +1) 4d - 12
                        de += HB ? 4 * (int)cls - 12 : 12 - 4 * (int)cls;
                    }
                }
                if (f) {
                    const uint32_t ws = wsm & 0x7FFFFFFFu, old = lds[ws];
                    lds[ws] = old ^ f;
                    if (MEASURE && (wsm >> 31)) {
                        e_acc += de;
                        m_acc += 2 * (2 * __builtin_popcount(old & f) - __builtin_popcount(f));
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

    // ---- store the tile's own rows
    const int own = hy * hz;
    const float invhy = 1.0f / (float)hy;
    for (int rr = r0; rr < own; rr += Q) {
        int iz, iy;
        divmod_small(rr, hy, invhy, iz, iy);
        const int row = (R + iz) * Ry + (R + iy);
        const int64_t grow = (int64_t)(z0 + iz) * a.Ly + (y0 + iy);
        if (a.out_packed) {
            uint2 *dst = (uint2 *)a.dst + ((int64_t)l * plane_rows + grow) * Wd;
            for (int w = w0; w < Wd; w += P) dst[w] = ((const uint2 *)lds)[row * Wd + w];
        } else {
            int8_t *rowp = (int8_t *)a.dst + (int64_t)l * a.N + grow * a.Lx;
            for (int w = w0; w < Wd; w += P) {
                const uint32_t ev = lds[widx(row, 0, w)], od = lds[widx(row, 1, w)];
                uint4 *pp = (uint4 *)(rowp + 64 * w);
#pragma unroll
                for (int qq = 0; qq < 4; ++qq) {
                    uint32_t dw[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int sh = 2 * (4 * qq + i);
                        const uint32_t bits = ((ev >> sh) & 1u) | (((od >> sh) & 1u) << 8) |
                                              (((ev >> (sh + 1)) & 1u) << 16) | (((od >> (sh + 1)) & 1u) << 24);
                        dw[i] = __builtin_amdgcn_perm(0u, 0x0000FF01u, bits);
                    }
                    pp[qq] = make_uint4(dw[0], dw[1], dw[2], dw[3]);
                }
            }
        }
    }
}

// Couplings to the packed row layout: bit b of word w of the even (odd) array
// of row (y, z) of direction d is set iff J[d][z][y][64 w + 2 b (+1)] < 0.
__global__ void k_pack_couplings(const int8_t *J, uint32_t *Jp, int Lx, int64_t rows3)
{
    const int Wd = Lx >> 6;
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= rows3 * Wd) return;
    const int64_t r = t / Wd;
    const int w = (int)(t % Wd);
    const int8_t *row = J + r * Lx + 64 * w;
    uint32_t ev = 0, od = 0;
    for (int b = 0; b < 32; ++b) {
        ev |= (uint32_t)(row[2 * b] < 0) << b;
        od |= (uint32_t)(row[2 * b + 1] < 0) << b;
    }
    Jp[(r * 2 + 0) * Wd + w] = ev;
    Jp[(r * 2 + 1) * Wd + w] = od;
}

// ---------------------------------------------------------------------------
bool tile3d_supported(const SweepCall &c, int layout)
{
    return layout == MC_INT8 && c.g.dims == 3 && (c.g.Lx % 64) == 0 && c.g.Lx <= 4096 && c.g.Ly >= 4 &&
           c.g.Lz >= 4 && (!c.per_lattice || c.g.count <= kMaxTableLattices);
}

size_t tile3d_lds_bytes(int Lx, int H, int K, bool hasJ)
{
    const size_t side = (size_t)H + 4 * (size_t)K;
    const size_t words = (side * side * 2 * (size_t)(Lx / 64) * (hasJ ? 4 : 1) + 3) & ~(size_t)3;
    return (words + 64) * 4;  // rows, then the 8 x 8 threshold masks
}

template <int K, bool HB, bool HASJ>
static hipError_t launch3(const Tile3DArgs &a, int H, int count, int threads, hipStream_t s)
{
    const size_t lds = tile3d_lds_bytes(a.Lx, H, K, HASJ);
    dim3 grid((unsigned)(a.nty * a.ntz), (unsigned)count);
    static LdsLimit lim[2];
    {
        const void *f =
            a.em.slots ? (const void *)k_tile3d<K, true, HB, HASJ> : (const void *)k_tile3d<K, false, HB, HASJ>;
        const hipError_t e = lim[a.em.slots ? 1 : 0].ensure(f, 98304);
        if (e != hipSuccess) return e;
    }
    if (a.em.slots) hipLaunchKernelGGL((k_tile3d<K, true, HB, HASJ>), grid, dim3(threads), lds, s, a);
    else hipLaunchKernelGGL((k_tile3d<K, false, HB, HASJ>), grid, dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <bool HB, bool HASJ>
static hipError_t launch3k(const Tile3DArgs &a, int k, int H, int count, int threads, hipStream_t s)
{
    switch (k) {
    case 0: return launch3<0, HB, HASJ>(a, H, count, threads, s);
    case 1: return launch3<1, HB, HASJ>(a, H, count, threads, s);
    case 2: return launch3<2, HB, HASJ>(a, H, count, threads, s);
    case 3: return launch3<3, HB, HASJ>(a, H, count, threads, s);
    case 4: return launch3<4, HB, HASJ>(a, H, count, threads, s);
    default: return hipErrorInvalidValue;
    }
}

static void class_thresholds(const SweepTables &t, int rule, uint32_t *top, uint32_t *low)
{
    for (int cl = 0; cl < 8; ++cl) {
        Thr th{0u, 0u};
        if (rule == 0) {
            if (cl <= 2) th = t.met[3 - cl];       // dE = 12 - 4a
        } else if (cl <= 6) {
            th = t.hb[12 - 2 * cl];                // h = 6 - 2d, index h + 6
        }
        if (th.top >= 256u) th = Thr{255u, 1u << 24};  // T = 2^32
        top[cl] = th.top;
        low[cl] = th.low;
    }
}

hipError_t launch_tile3d(const SweepCall &c, const void *src, int in_packed, void *dst, int out_packed,
                         const uint32_t *Jp, uint64_t sweep0, int k, int H, int threads, const EmSlots &em,
                         hipStream_t s)
{
    Tile3DArgs a;
    a.src = src;
    a.dst = dst;
    a.in_packed = in_packed;
    a.out_packed = out_packed;
    a.Jp = Jp;
    a.Lx = c.g.Lx;
    a.Ly = c.g.Ly;
    a.Lz = c.g.Lz;
    a.nty = (c.g.Ly + H - 1) / H;
    a.ntz = (c.g.Lz + H - 1) / H;
    a.N = c.g.N;
    a.seed_lo = c.seed_lo;
    a.seed_hi = c.seed_hi;
    a.replica0 = c.replica0;
    a.sweep0 = sweep0;
    a.per_lattice = c.per_lattice;
    for (int i = 0; i < kMaxTableLattices; ++i) {
        const SweepTables &t = (c.per_lattice && i < c.g.count) ? c.tabs[i] : c.tab;
        class_thresholds(t, c.rule, a.top[i], a.low[i]);
    }
    a.em = em;
    if (k == 0) a.em.slots = nullptr;
    if (!em.red_in) a.em.red_K = 0;
    const bool hb = c.rule == 1, hj = Jp != nullptr;
    if (hb && hj) return launch3k<true, true>(a, k, H, c.g.count, threads, s);
    if (hb) return launch3k<true, false>(a, k, H, c.g.count, threads, s);
    if (hj) return launch3k<false, true>(a, k, H, c.g.count, threads, s);
    return launch3k<false, false>(a, k, H, c.g.count, threads, s);
}

// Per-tile (E, M) slots of one launch: K <= 4 sweeps x count lattices x
// ceil(Ly / 2) ceil(Lz / 2) tiles (a plan's tile side is at least 2, the
// smallest that fits LDS at Lx = 4096) x 16 bytes.
size_t tile3d_slot_bytes(const Geom &g)
{
    const size_t b = (size_t)4 * (size_t)g.count * (size_t)((g.Ly + 1) / 2) * (size_t)((g.Lz + 1) / 2) * 16;
    return (b + 255) / 256 * 256;
}

hipError_t launch_pack_couplings(const Geom &g, const int8_t *J, uint32_t *Jp, hipStream_t s)
{
    const int64_t rows3 = 3 * (int64_t)g.Ly * g.Lz;
    const int64_t n = rows3 * (g.Lx / 64);
    hipLaunchKernelGGL(k_pack_couplings, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, J, Jp, g.Lx, rows3);
    return hipGetLastError();
}

}  // namespace mcs
