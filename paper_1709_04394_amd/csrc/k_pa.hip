// k_pa.hip -- population annealing (Sec. "Population annealing", Eq. Q) for
// populations of 2D L x L ferromagnets, several populations (of different L)
// per launch.
//
// One annealing step is four kernels:
//  k_pa_scan      one workgroup per population: weights w_j = exp(-dbeta (E_j +
//                 2N)) from the step's host table, the fixed-order FP64 prefix
//                 sum (64-wide doubling scans by wave shuffles, chunk totals
//                 scanned the same way, group totals in sequence), C_total, and
//                 the running maximum of C used by the parent search;
//  k_pa_resample  one thread per new slot: u from Philox, t = u C_total, parent =
//                 first j with Cmax_j > t (binary search), integer copy counts;
//  k_pa_place     one workgroup per population: exclusive integer scan of the
//                 copy counts, copies of parent j fill slots [P_j, P_j + n_j);
//  k_pa_sweep     gathers each slot's parent into LDS (bit-packed, split by x
//                 parity, periodic in both directions, so a whole lattice lives
//                 in one workgroup and needs no halo), runs theta checkerboard
//                 Metropolis sweeps, and writes the lattice, its energy and the
//                 energy histogram.
#include "internal.hpp"
#include "pa.hpp"

namespace mcs {

// ----------------------------------------------------------------------------
// Inclusive scan of one wave's 64 doubles in the doubling order
// x_i <- x_i + x_{i-d}, d = 1, 2, ..., 32, from the values before each step.
__device__ __forceinline__ double wave_scan_f64(double v, int lane)
{
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const double t = __shfl_up(v, (unsigned)d, 64);
        if (lane >= d) v = v + t;
    }
    return v;
}

__global__ __launch_bounds__(1024) void k_pa_scan(PaStep st)
{
    const PaPop &P = st.pop[blockIdx.x];
    const int R = P.R, N = P.N;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    const int nb = (R + 63) / 64, ng = (nb + 63) / 64;
    __shared__ double tch[kPaMaxChunks];  // chunk totals, then their level-1 scan
    __shared__ double G[64];              // level-2 exclusive group offsets
    __shared__ double tmax[1024];
    for (int i = tid; i < R; i += blockDim.x) P.n[i] = 0;
    // level 0: blocks of 64 in index order
    for (int b = wave; b < nb; b += nw) {
        const int i = 64 * b + lane;
        double v = 0.0;
        if (i < R) v = st.wtab[(P.E[i] + 2 * N) / 4];
        v = wave_scan_f64(v, lane);
        if (i < R) P.x[i] = v;
        if (lane == 63) tch[b] = v;
    }
    __syncthreads();
    // level 1: block totals, 64 at a time
    for (int q = wave; q < ng; q += nw) {
        const int b = 64 * q + lane;
        double v = b < nb ? tch[b] : 0.0;
        v = wave_scan_f64(v, lane);
        if (b < nb) tch[b] = v;
    }
    __syncthreads();
    // level 2: group totals one after the other
    if (tid == 0) {
        double g = 0.0;
        G[0] = 0.0;
        for (int q = 1; q < ng; ++q) {
            g = g + tch[64 * (q - 1) + 63];
            G[q] = g;
        }
    }
    __syncthreads();
    // C_i = x_i + (G_q + B_b); C_total = C_{R-1}; running maximum of C
    const int per = (R + blockDim.x - 1) / blockDim.x;
    const int i0 = tid * per, i1 = min(R, i0 + per);
    double run = -1.0;
    for (int i = i0; i < i1; ++i) {
        const int b = i / 64, q = b / 64;
        const double Bb = (b % 64 == 0) ? 0.0 : tch[b - 1];
        const double C = P.x[i] + (G[q] + Bb);
        if (i == R - 1) P.ctot[st.ctot_idx] = C;
        run = fmax(run, C);
        P.cmax[i] = run;
    }
    tmax[tid] = run;
    __syncthreads();
    // exclusive maximum over the threads before this one (exact in any order)
    double before = -1.0;
    for (int k = 0; k < tid; ++k) before = fmax(before, tmax[k]);
    for (int i = i0; i < i1; ++i) P.cmax[i] = fmax(P.cmax[i], before);
}

__global__ void k_pa_resample(PaStep st)
{
    const int p = blockIdx.y;
    const PaPop &P = st.pop[p];
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= P.R) return;
    const uint4 r = philox(make_uint4((uint32_t)k, (uint32_t)p, st.step, ctr_w3(kTagResample, 0, st.step)),
                           st.seed_lo, st.seed_hi);
    const uint64_t a = r.x >> 5, b = r.y >> 6;
    const double u = (double)(a * 67108864ull + b) * (1.0 / 9007199254740992.0);
    const double t = u * P.ctot[st.ctot_idx];
    int lo = 0, hi = P.R - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (P.cmax[mid] > t) hi = mid;
        else lo = mid + 1;
    }
    atomicAdd(&P.n[lo], 1);
}

__global__ __launch_bounds__(1024) void k_pa_place(PaStep st)
{
    const PaPop &P = st.pop[blockIdx.x];
    const int R = P.R, tid = threadIdx.x;
    __shared__ int tsum[1024];
    const int per = (R + blockDim.x - 1) / blockDim.x;
    const int i0 = tid * per, i1 = min(R, i0 + per);
    int s = 0;
    for (int i = i0; i < i1; ++i) s += P.n[i];
    tsum[tid] = s;
    __syncthreads();
    int base = 0;
    for (int k = 0; k < tid; ++k) base += tsum[k];
    for (int i = i0; i < i1; ++i) {
        const int c = P.n[i];
        for (int m = 0; m < c; ++m) P.newparent[base + m] = i;
        base += c;
    }
}

// ----------------------------------------------------------------------------
// Sweep kernel.  LDS image of lattice g: word (g, r, par, w) holds the sites
// x = 64 w + 2 b + par (b < Wb) of row r, bit set <=> s = -1; Wb = min(32, L/2)
// and nwr = L / 64 words per row and parity for L >= 64, one word otherwise.
constexpr int kPaTieQueue = 256;

__global__ __launch_bounds__(256) void k_pa_sweep(PaStep st)
{
    extern __shared__ uint32_t lds[];
    __shared__ int e_lat[64];
    __shared__ uint32_t q_j[kPaTieQueue], q_meta[kPaTieQueue], q_rep[kPaTieQueue];
    __shared__ uint32_t q_cnt[4];
    int p = 0;
    while (p + 1 < st.npop && (int)blockIdx.x >= st.pop[p + 1].blk0) ++p;
    const PaPop &P = st.pop[p];
    const int L = P.L, N = P.N, Wb = P.Wb, nwr = P.nwr, G = P.G;
    const int s0 = ((int)blockIdx.x - P.blk0) * G;
    const int ng = min(G, P.R - s0);
    const int tid = threadIdx.x, nt = blockDim.x;
    const uint32_t wmask = Wb == 32 ? ~0u : ((1u << Wb) - 1u);
    const int per_lat = 2 * L * nwr;  // words per lattice
    auto widx = [&](int g, int r, int par, int w) { return g * per_lat + (r * 2 + par) * nwr + w; };
    const TopMask m4 = top_mask(st.t4.top), m8 = top_mask(st.t8.top);
    const int wave = tid >> 6, nwaves = nt >> 6;
    const uint32_t wq_cap = (uint32_t)(kPaTieQueue / nwaves), wq_base = (uint32_t)wave * wq_cap;
    uint32_t wq_n = 0;
    if (tid < 64) e_lat[tid] = 0;

    // ---- gather the parents and pack
    const int tasks_ld = ng * L * nwr;
    for (int t = tid; t < tasks_ld; t += nt) {
        const int g = t / (L * nwr), rem = t - g * L * nwr, r = rem / nwr, w = rem - r * nwr;
        const int slot = s0 + g;
        const int parent = st.identity ? slot : P.newparent[slot];
        const int8_t *row = P.cur + (int64_t)parent * N + (int64_t)r * L;
        uint32_t ev = 0, od = 0;
        if (Wb == 32) {
            const uint4 *q4 = (const uint4 *)(row + 64 * w);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const uint4 v = q4[q];
                const uint32_t dw[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t m = dw[i] & 0x80808080u;
                    const uint32_t Pm = m + (m << 15);
                    const int sh = 2 * (4 * q + i);
                    ev |= ((Pm >> 22) & 3u) << sh;
                    od |= (Pm >> 30) << sh;
                }
            }
        } else {
            for (int b = 0; b < Wb; ++b) {
                ev |= (uint32_t)(row[2 * b] < 0) << b;
                od |= (uint32_t)(row[2 * b + 1] < 0) << b;
            }
        }
        lds[widx(g, r, 0, w)] = ev;
        lds[widx(g, r, 1, w)] = od;
    }
    __syncthreads();

    const int tasks = ng * L * nwr;
    for (int sw = 0; sw < st.theta; ++sw) {
        const uint64_t sweep = (uint64_t)(st.step - 1) * (uint64_t)st.theta + (uint64_t)sw;
        for (int c = 0; c < 2; ++c) {
            const uint32_t w3 = ctr_w3(kTagSweep, (uint32_t)c, sweep);
            const uint32_t w3lo = ctr_w3(kTagSweepLo, (uint32_t)c, sweep);
            for (int t = tid; t < tasks; t += nt) {
                const int g = t / (L * nwr), rem = t - g * L * nwr, r = rem / nwr, w = rem - r * nwr;
                const int q = (c + r) & 1;
                const int rm = r == 0 ? L - 1 : r - 1, rp = r + 1 == L ? 0 : r + 1;
                const int ws = widx(g, r, q, w);
                const uint32_t S = lds[ws];
                const uint32_t U = lds[widx(g, rm, q, w)], D = lds[widx(g, rp, q, w)];
                const uint32_t O = lds[widx(g, r, 1 - q, w)];
                uint32_t Sh;
                if (nwr > 1) {
                    const int wl = w == 0 ? nwr - 1 : w - 1, wr = w + 1 == nwr ? 0 : w + 1;
                    const uint32_t Ol = lds[widx(g, r, 1, wl)], Er = lds[widx(g, r, 0, wr)];
                    Sh = q == 0 ? __builtin_amdgcn_alignbit(O, Ol, 31) : __builtin_amdgcn_alignbit(Er, O, 1);
                } else {
                    // one word per row: rotate inside the Wb used bits
                    Sh = q == 0 ? (((O << 1) | (O >> (Wb - 1))) & wmask) : (((O >> 1) | (O << (Wb - 1))) & wmask);
                }
                const uint32_t u1 = S ^ U, u2 = S ^ D, u3 = S ^ O, u4 = S ^ Sh;
                const uint32_t t1 = u1 | u2, t2 = u3 | u4;
                const uint32_t ge2 = MCS_BOP3(u1, u2, MCS_BOP3(u3, u4, t1 & t2, (MCS_A & MCS_B) | MCS_C),
                                              (MCS_A & MCS_B) | MCS_C);
                const uint32_t c8 = ~(t1 | t2) & wmask;
                const uint32_t c4 = MCS_BOP3(t1, t2, ge2, (MCS_A | MCS_B) & ~MCS_C);
                // random planes of sites j0 .. j0 + Wb - 1, j0 = 32 w + (L/2) r
                const uint32_t j0 = 32u * (uint32_t)w + (uint32_t)(L >> 1) * (uint32_t)r;
                const uint32_t rep = (uint32_t)p * (uint32_t)P.R + (uint32_t)(s0 + g);
                uint32_t X[8];
                const uint4 A = philox(make_uint4(j0 >> 4, rep, (uint32_t)sweep, w3), st.seed_lo, st.seed_hi);
                if (Wb == 32) {
                    const uint4 B = philox(make_uint4((j0 >> 4) + 1u, rep, (uint32_t)sweep, w3), st.seed_lo,
                                           st.seed_hi);
#pragma unroll
                    for (int k = 0; k < 8; ++k) X[k] = plane_pair(A, B, k);
                } else {
                    const uint32_t off = j0 & 15u;
                    const uint32_t aw[4] = {A.x, A.y, A.z, A.w};
#pragma unroll
                    for (int k = 0; k < 8; ++k) X[k] = ((aw[k >> 1] >> (16u * (k & 1u))) >> off) & wmask;
                }
                uint32_t lt8, eq8, lt4, eq4;
                compare_planes(X, m8, lt8, eq8);
                compare_planes(X, m4, lt4, eq4);
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
                            q_j[wq_base + pos] = j0 + (uint32_t)b;
                            q_rep[wq_base + pos] = rep;
                            q_meta[wq_base + pos] = (uint32_t)ws | ((uint32_t)b << 16) | (cls8 << 21);
                        } else {
                            const uint4 lo = philox(make_uint4(j0 + (uint32_t)b, rep, (uint32_t)sweep, w3lo),
                                                    st.seed_lo, st.seed_hi);
                            if ((lo.x & 0xFFFFFFu) < (cls8 ? st.t8.low : st.t4.low)) acc |= 1u << b;
                        }
                    }
                    wq_n = min(wq_cap, wq_n + (uint32_t)__popcll(m));
                    m = __ballot(pend != 0u);
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
                const uint32_t item = sg * wq_cap + k, meta = q_meta[item];
                const uint4 lo = philox(make_uint4(q_j[item], q_rep[item], (uint32_t)sweep, w3lo), st.seed_lo,
                                        st.seed_hi);
                const bool cls8 = (meta >> 21) & 1u;
                if ((lo.x & 0xFFFFFFu) < (cls8 ? st.t8.low : st.t4.low))
                    atomicXor(&lds[meta & 0xFFFFu], 1u << ((meta >> 16) & 31u));
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
        const uint32_t S = lds[widx(g, r, q, w)];
        const uint32_t U = lds[widx(g, rm, q, w)], D = lds[widx(g, rp, q, w)];
        const uint32_t O = lds[widx(g, r, 1 - q, w)];
        uint32_t Sh;
        if (nwr > 1) {
            const int wl = w == 0 ? nwr - 1 : w - 1, wr = w + 1 == nwr ? 0 : w + 1;
            Sh = q == 0 ? __builtin_amdgcn_alignbit(O, lds[widx(g, r, 1, wl)], 31)
                        : __builtin_amdgcn_alignbit(lds[widx(g, r, 0, wr)], O, 1);
        } else {
            Sh = q == 0 ? (((O << 1) | (O >> (Wb - 1))) & wmask) : (((O >> 1) | (O << (Wb - 1))) & wmask);
        }
        const int a = __builtin_popcount(S ^ U) + __builtin_popcount(S ^ D) + __builtin_popcount(S ^ O) +
                      __builtin_popcount(S ^ Sh);
        atomicAdd(&e_lat[g], 2 * a - 4 * Wb);
    }
    __syncthreads();
    if (tid < ng) {
        const int slot = s0 + tid;
        const int e = e_lat[tid];
        P.Enew[slot] = e;
        atomicAdd((unsigned long long *)&P.hist[(int64_t)st.hist_idx * (N + 1) + (e + 2 * N) / 4], 1ull);
    }

    // ---- unpack and store the new population
    for (int t = tid; t < tasks_ld; t += nt) {
        const int g = t / (L * nwr), rem = t - g * L * nwr, r = rem / nwr, w = rem - r * nwr;
        const uint32_t ev = lds[widx(g, r, 0, w)], od = lds[widx(g, r, 1, w)];
        int8_t *row = P.nxt + (int64_t)(s0 + g) * N + (int64_t)r * L;
        if (Wb == 32) {
            uint4 *q4 = (uint4 *)(row + 64 * w);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t dw[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int sh = 2 * (4 * q + i);
                    const uint32_t bits = ((ev >> sh) & 1u) | (((od >> sh) & 1u) << 8) |
                                          (((ev >> (sh + 1)) & 1u) << 16) | (((od >> (sh + 1)) & 1u) << 24);
                    dw[i] = __builtin_amdgcn_perm(0u, 0x0000FF01u, bits);
                }
                q4[q] = make_uint4(dw[0], dw[1], dw[2], dw[3]);
            }
        } else {
            for (int b = 0; b < Wb; ++b) {
                row[2 * b] = ((ev >> b) & 1u) ? (int8_t)-1 : (int8_t)1;
                row[2 * b + 1] = ((od >> b) & 1u) ? (int8_t)-1 : (int8_t)1;
            }
        }
    }
}

// ----------------------------------------------------------------------------
hipError_t launch_pa_step(const PaStep &st, int rmax, int sweep_blocks, hipStream_t s)
{
    if (!st.identity) {
        hipLaunchKernelGGL(k_pa_scan, dim3(st.npop), dim3(1024), 0, s, st);
        hipLaunchKernelGGL(k_pa_resample, dim3((rmax + 255) / 256, st.npop), dim3(256), 0, s, st);
        hipLaunchKernelGGL(k_pa_place, dim3(st.npop), dim3(1024), 0, s, st);
    }
    size_t lds = 0;
    for (int p = 0; p < st.npop; ++p) {
        const size_t b = (size_t)st.pop[p].G * 2 * st.pop[p].L * st.pop[p].nwr * 4;
        if (b > lds) lds = b;
    }
    hipLaunchKernelGGL(k_pa_sweep, dim3(sweep_blocks), dim3(256), lds, s, st);
    return hipGetLastError();
}

}  // namespace mcs
