/*
 * mcoracle.c -- CPU oracle for the Monte Carlo hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may use it.  It shares no code, header or table
 * generator with the HIP library: every piece of arithmetic below is written
 * out again from the paper (M. Weigel, "Monte Carlo methods for massively
 * parallel computers", arXiv:1709.04394), with the reading of the paper taken
 * where it leaves a choice stated beside each routine, as plainly as possible,
 * in the order the paper states it.
 *
 * Contents
 *   Philox4x32-10 ............ Sec. "Random number generation", counter-based
 *                              generators (mulhi/mullo round, key schedule)
 *   random streams ........... keyed by (seed; tag, site, replica, sweep, phase)
 *   acceptance tables ........ Eq. (metropolis-canonical), Eq. (heatbath)
 *   lattice init, couplings .. Sec. "Checkerboard scheme" step 1; Sec.
 *                              "Disordered systems" (bimodal J_ij)
 *   energy / magnetisation ... Eq. (ising_model) with h_i = 0
 *   checkerboard sweeps ...... Sec. "Checkerboard scheme" (even sub-lattice,
 *                              then odd sub-lattice; Metropolis or heat-bath)
 *   double checkerboard ...... Sec. "Checkerboard scheme" (tiles in a coarse
 *                              checkerboard, k hits per tile)
 *   population annealing ..... Sec. "Population annealing", Eq. (Q)
 *   multicanonical sweeps .... Sec. "Multicanonical simulations", Eq. (muca),
 *                              sequential site order, count-again rule
 *   Wang-Landau in windows ... Sec. "Wang-Landau update" (g(E) <- f g(E) per
 *                              visit, acceptance min[1, g(E)/g(E')]); energy
 *                              windows with the count-again rule of Sec.
 *                              "Multicanonical simulations"
 *
 * Floating point: plain IEEE double, -O2 -ffp-contract=off, no fast-math.
 * Every exp/log that decides a trajectory goes through the C library's exp()
 * and log(), computed once per table entry.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (counter-based generator, Sec. "Random number generation").
 * One round takes the two word pairs (R,L) = (x0,x1) and (x2,x3):
 *   L' = mullo(R, M),  R' = mulhi(R, M) xor k xor L,
 * followed by the word permutation of the 4x32 variant; the key is advanced
 * by the Weyl increments between rounds.  Multipliers and increments are the
 * published Philox4x32 constants (the increments are the fractional parts of
 * the golden ratio and of sqrt(3), times 2^32).                               */
#define ORC_PHILOX_M0 0xD2511F53u
#define ORC_PHILOX_M1 0xCD9E8D57u
#define ORC_PHILOX_W0 0x9E3779B9u
#define ORC_PHILOX_W1 0xBB67AE85u

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += ORC_PHILOX_W0;
            k1 += ORC_PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)ORC_PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)ORC_PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ------------------------------------------------------------------------ */
/* Random streams.  The key is the 64-bit seed; the counter names the draw by
 * intrinsic variables of the simulation (the paper's point (a) on
 * counter-based generators), so a result never depends on how work is spread
 * over threads:
 *   ctr = (a, replica, sweep mod 2^32, tag<<24 | phase<<23 | (sweep>>32 & 0x7FFFFF))
 * A 32-bit uniform for item j is assembled from two Philox blocks:
 *   top byte  = bit k (k = 0..7) is bit (j mod 16) of 16-bit half-word k of
 *               Philox(tag, a = j div 16) (half-word k = bits 16(k mod 2) ..
 *               16(k mod 2)+15 of output word k div 2), so one block holds
 *               the top bytes of 16 consecutive items as 8 bit-planes;
 *   low 24 b  = word 0 of Philox(tag_lo, a = j), masked to 24 bits;
 * r = top << 24 | low is an exactly uniform 32-bit integer, and the uniform
 * variate of the paper is r / 2^32 in [0,1).                                  */
enum {
    ORC_TAG_INIT = 1, ORC_TAG_SWEEP = 2, ORC_TAG_COUPLING = 3, ORC_TAG_RESAMPLE = 4,
    ORC_TAG_MUCA = 5, ORC_TAG_MLP_INIT = 6, ORC_TAG_SWEEP_LO = 7, ORC_TAG_MUCA_LO = 8,
    ORC_TAG_WINDOW = 10
};

static void orc_block(uint64_t seed, uint32_t tag, uint32_t a, uint32_t replica,
                      uint64_t sweep, uint32_t phase, uint32_t out[4])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t ctr[4];
    ctr[0] = a;
    ctr[1] = replica;
    ctr[2] = (uint32_t)sweep;
    ctr[3] = (tag << 24) | ((phase & 1u) << 23) | ((uint32_t)(sweep >> 32) & 0x7FFFFFu);
    orc_philox4x32_10(ctr, key, out);
}

uint32_t orc_draw_byte(uint64_t seed, uint32_t tag, uint32_t j, uint32_t replica,
                       uint64_t sweep, uint32_t phase)
{
    uint32_t out[4];
    orc_block(seed, tag, j >> 4, replica, sweep, phase, out);
    uint32_t pos = j & 15u, byte = 0;
    for (uint32_t k = 0; k < 8; ++k) {
        uint32_t halfword = (out[k >> 1] >> (16u * (k & 1u))) & 0xFFFFu;
        byte |= ((halfword >> pos) & 1u) << k;
    }
    return byte;
}

uint32_t orc_draw32(uint64_t seed, uint32_t tag, uint32_t tag_lo, uint32_t j,
                    uint32_t replica, uint64_t sweep, uint32_t phase)
{
    uint32_t top = orc_draw_byte(seed, tag, j, replica, sweep, phase);
    uint32_t out[4];
    orc_block(seed, tag_lo, j, replica, sweep, phase, out);
    return (top << 24) | (out[0] & 0xFFFFFFu);
}

/* Whole 32-bit draw for item j of a sequential chain (the multicanonical
 * walkers): word (j mod 4) of Philox(tag, a = j div 4).                      */
uint32_t orc_draw_word(uint64_t seed, uint32_t tag, uint32_t j, uint32_t replica, uint64_t sweep)
{
    uint32_t out[4];
    orc_block(seed, tag, j >> 2, replica, sweep, 0, out);
    return out[j & 3u];
}

/* 53-bit uniform in [0,1) for resampling slot k of population pop at
 * annealing step: words 0 and 1 of one Philox block, 27 + 26 bits.           */
double orc_resample_u(uint64_t seed, uint32_t k, uint32_t pop, uint32_t step)
{
    uint32_t out[4];
    orc_block(seed, ORC_TAG_RESAMPLE, k, pop, (uint64_t)step, 0, out);
    uint64_t a = out[0] >> 5, b = out[1] >> 6;
    return (double)(a * 67108864ull + b) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------------ */
/* Acceptance tables.  The paper compares a uniform r in [0,1) with
 * exp(-beta dE) (Eq. metropolis-canonical) and notes that the exponentials are
 * tabulated.  With r = r32 / 2^32 the test r < p is exactly r32 < ceil(p 2^32),
 * so each entry is that ceiling, as an integer in [0, 2^32].
 *   Metropolis: T[k] for dE = 4k (k = 0 gives 2^32: always accept).
 *   Heat-bath (Eq. heatbath for two states): P(s' = +1 | h) =
 *     1 / (1 + exp(-2 beta h)), T[h + z] = ceil(P 2^32), h = -z..z.          */
void orc_metropolis_table(double beta, int kmax, uint64_t *T)
{
    for (int k = 0; k <= kmax; ++k) {
        double p = exp(-beta * (double)(4 * k));
        T[k] = (uint64_t)ceil(ldexp(p, 32));
    }
}

void orc_heatbath_table(double beta, int z, uint64_t *T)
{
    for (int h = -z; h <= z; ++h) {
        double e = exp(-2.0 * beta * (double)h);
        double p = 1.0 / (1.0 + e);
        T[h + z] = (uint64_t)ceil(ldexp(p, 32));
    }
}

/* ------------------------------------------------------------------------ */
/* Geometry: site i = x + Lx (y + Ly z); dims 2 has Lz = 1.  Periodic in every
 * direction.  Couplings J[d*N + i] belong to the bond (i, i + e_d); NULL means
 * the ferromagnet J = 1.                                                     */
typedef struct { int dims, Lx, Ly, Lz; int64_t N; } orc_geom;

static orc_geom mkgeom(int dims, int Lx, int Ly, int Lz)
{
    orc_geom g;
    g.dims = dims; g.Lx = Lx; g.Ly = Ly; g.Lz = dims == 3 ? Lz : 1;
    g.N = (int64_t)Lx * Ly * g.Lz;
    return g;
}

static int geom_ok(const orc_geom *g)
{
    if (g->dims != 2 && g->dims != 3) return 0;
    if (g->Lx < 2 || g->Ly < 2 || g->Lz < 1) return 0;
    if (g->dims == 3 && g->Lz < 2) return 0;
    return 1;
}

static inline int64_t site(const orc_geom *g, int x, int y, int z)
{
    return (int64_t)x + (int64_t)g->Lx * ((int64_t)y + (int64_t)g->Ly * z);
}

/* Local field h_i = sum over the 2*dims neighbours j of J_ij s_j. */
static int local_field(const orc_geom *g, const int8_t *s, const int8_t *J, int x, int y, int z)
{
    int xp = x + 1 == g->Lx ? 0 : x + 1, xm = x == 0 ? g->Lx - 1 : x - 1;
    int yp = y + 1 == g->Ly ? 0 : y + 1, ym = y == 0 ? g->Ly - 1 : y - 1;
    int64_t i = site(g, x, y, z);
    int64_t n[6], b[6];
    int nn = 4;
    n[0] = site(g, xp, y, z); b[0] = 0 * g->N + i;
    n[1] = site(g, xm, y, z); b[1] = 0 * g->N + n[1];
    n[2] = site(g, x, yp, z); b[2] = 1 * g->N + i;
    n[3] = site(g, x, ym, z); b[3] = 1 * g->N + n[3];
    if (g->dims == 3) {
        int zp = z + 1 == g->Lz ? 0 : z + 1, zm = z == 0 ? g->Lz - 1 : z - 1;
        n[4] = site(g, x, y, zp); b[4] = 2 * g->N + i;
        n[5] = site(g, x, y, zm); b[5] = 2 * g->N + n[5];
        nn = 6;
    }
    int h = 0;
    for (int k = 0; k < nn; ++k)
        h += (J ? (int)J[b[k]] : 1) * (int)s[n[k]];
    return h;
}

/* Hot start: s_i = +1 iff the top bit of its random byte is clear (p = 1/2).
 * Cold start: all +1.                                                        */
int orc_init(int dims, int Lx, int Ly, int Lz, int8_t *s, int start, uint64_t seed, uint32_t replica)
{
    orc_geom g = mkgeom(dims, Lx, Ly, Lz);
    if (!geom_ok(&g)) return -1;
    for (int64_t i = 0; i < g.N; ++i) {
        if (start == 0) s[i] = 1;
        else s[i] = orc_draw_byte(seed, ORC_TAG_INIT, (uint32_t)i, replica, 0, 0) < 128u ? 1 : -1;
    }
    return 0;
}

/* Bimodal couplings J = +-1 with p = 1/2, one per bond (site, direction), of
 * disorder realisation `realisation` (counter word 1; realisation 0 is the
 * single realisation of the plain spin-glass runs).                          */
int orc_couplings_of(int dims, int Lx, int Ly, int Lz, int8_t *J, uint64_t seed, uint32_t realisation)
{
    orc_geom g = mkgeom(dims, Lx, Ly, Lz);
    if (!geom_ok(&g)) return -1;
    for (int64_t b = 0; b < (int64_t)dims * g.N; ++b)
        J[b] = orc_draw_byte(seed, ORC_TAG_COUPLING, (uint32_t)b, realisation, 0, 0) < 128u ? 1 : -1;
    return 0;
}

int orc_couplings(int dims, int Lx, int Ly, int Lz, int8_t *J, uint64_t seed)
{
    return orc_couplings_of(dims, Lx, Ly, Lz, J, seed, 0);
}

/* E = -sum over bonds J_ij s_i s_j (each bond once), M = sum s_i. */
void orc_measure(int dims, int Lx, int Ly, int Lz, const int8_t *s, const int8_t *J,
                 int64_t *E, int64_t *M)
{
    orc_geom g = mkgeom(dims, Lx, Ly, Lz);
    int64_t e = 0, m = 0;
    for (int z = 0; z < g.Lz; ++z)
        for (int y = 0; y < g.Ly; ++y)
            for (int x = 0; x < g.Lx; ++x) {
                int64_t i = site(&g, x, y, z);
                int64_t nb[3];
                nb[0] = site(&g, x + 1 == g.Lx ? 0 : x + 1, y, z);
                nb[1] = site(&g, x, y + 1 == g.Ly ? 0 : y + 1, z);
                nb[2] = dims == 3 ? site(&g, x, y, z + 1 == g.Lz ? 0 : z + 1) : 0;
                for (int d = 0; d < dims; ++d)
                    e -= (int64_t)(J ? J[d * g.N + i] : 1) * s[i] * s[nb[d]];
                m += s[i];
            }
    *E = e;
    *M = m;
}

/* ------------------------------------------------------------------------ */
/* Checkerboard sweep (Sec. "Checkerboard scheme"): phase c = 0 updates all
 * sites with x+y(+z) even, phase 1 the odd ones.  Sites of one colour have no
 * common bond, so updating them one after the other in place is the same as
 * updating them simultaneously.  Same-colour index j = i >> 1 (a bijection
 * onto 0..N/2-1 for each colour when Lx is even) keys the random number.
 * rule 0: Metropolis, dE = 2 s_i h_i, flip iff dE <= 0 or r32 < T[dE/4].
 * rule 1: heat-bath,  s_i' = +1 iff r32 < T_hb[h_i + z].
 * EM (optional) receives (E, M) after every sweep.                          */
int orc_sweep(int dims, int Lx, int Ly, int Lz, int8_t *s, const int8_t *J, int rule, double beta,
              uint64_t seed, uint32_t replica, uint64_t sweep0, int nsweeps, int64_t *EM)
{
    orc_geom g = mkgeom(dims, Lx, Ly, Lz);
    if (!geom_ok(&g) || (Lx & 1) || (Ly & 1) || (dims == 3 && (g.Lz & 1))) return -1;
    if (rule != 0 && rule != 1) return -1;
    int z_coord = 2 * dims;
    uint64_t Tm[4], Thb[13];
    orc_metropolis_table(beta, 3, Tm);
    orc_heatbath_table(beta, z_coord, Thb);
    for (int t = 0; t < nsweeps; ++t) {
        uint64_t sweep = sweep0 + (uint64_t)t;
        for (int c = 0; c < 2; ++c) {
            #pragma omp parallel for collapse(2) schedule(static) if (g.N >= 8192)
            for (int z = 0; z < g.Lz; ++z)
                for (int y = 0; y < g.Ly; ++y)
                    for (int x = 0; x < g.Lx; ++x) {
                        if (((x + y + z) & 1) != c) continue;
                        int64_t i = site(&g, x, y, z);
                        int h = local_field(&g, s, J, x, y, z);
                        uint32_t r = orc_draw32(seed, ORC_TAG_SWEEP, ORC_TAG_SWEEP_LO,
                                                (uint32_t)(i >> 1), replica, sweep, (uint32_t)c);
                        if (rule == 0) {
                            int dE = 2 * s[i] * h;
                            if (dE <= 0 || (uint64_t)r < Tm[dE / 4]) s[i] = (int8_t)-s[i];
                        } else {
                            s[i] = (uint64_t)r < Thb[h + z_coord] ? 1 : -1;
                        }
                    }
        }
        if (EM) orc_measure(dims, Lx, Ly, Lz, s, J, &EM[2 * t], &EM[2 * t + 1]);
    }
    return 0;
}

/* Three-colour Metropolis sweep of a 2D L x L torus with 3 | L (used for the
 * odd 3x3 torus, which is not bipartite): colour (x + 2y) mod 3 is proper,
 * phases c = 0, 1, 2 in turn; the draw for site i in phase c uses item
 * j = c N + i.                                                                */
int orc_sweep_q3(int L, int8_t *s, double beta, uint64_t seed, uint32_t replica,
                 uint64_t sweep0, int nsweeps, int64_t *EM)
{
    if (L < 3 || L % 3) return -1;
    orc_geom g = mkgeom(2, L, L, 1);
    uint64_t Tm[4];
    orc_metropolis_table(beta, 3, Tm);
    for (int t = 0; t < nsweeps; ++t) {
        uint64_t sweep = sweep0 + (uint64_t)t;
        for (int c = 0; c < 3; ++c)
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    if ((x + 2 * y) % 3 != c) continue;
                    int64_t i = site(&g, x, y, 0);
                    int h = local_field(&g, s, NULL, x, y, 0);
                    uint32_t r = orc_draw32(seed, ORC_TAG_SWEEP, ORC_TAG_SWEEP_LO,
                                            (uint32_t)(c * g.N + i), replica, sweep, 0);
                    int dE = 2 * s[i] * h;
                    if (dE <= 0 || (uint64_t)r < Tm[dE / 4]) s[i] = (int8_t)-s[i];
                }
        if (EM) orc_measure(2, L, L, 1, s, NULL, &EM[2 * t], &EM[2 * t + 1]);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Double-checkerboard sweep with k hits per tile (Sec. "Checkerboard scheme":
 * the two-level decomposition of the right panel of Fig. checkerboard, and
 * multi-hit updates).  The L x L torus is cut into T x T tiles; the tile
 * holding site (x, y) has coarse colour (x/T + y/T) mod 2, and L/T is even so
 * that the tiles form a checkerboard on the torus.  One sweep first updates
 * every tile of coarse colour 0, then every tile of coarse colour 1.  Tiles
 * of one coarse colour share no bond, so they are updated independently
 * while the spins of the other colour's tiles stay fixed; each such tile
 * takes k rounds of its own checkerboard update (its sites with x + y even,
 * then those with x + y odd).  Every site is therefore updated k times per
 * sweep.  Readings where the paper leaves a choice: coarse colour 0 first,
 * even sites first within a round, and the random numbers: hit h (0..k-1) of
 * sweep t of a site draws exactly what the plain checkerboard sweep numbered
 * t k + h draws for it (same-colour index j = i >> 1, its colour c).  Sites of
 * one coarse and one fine colour have no common bond, so updating them one
 * after the other in place equals updating them simultaneously.
 * Metropolis, J = 1.  EM (optional) receives (E, M) after every sweep.      */
int orc_sweep_dcb(int L, int T, int k, int8_t *s, double beta, uint64_t seed, uint32_t replica,
                  uint64_t sweep0, int nsweeps, int64_t *EM)
{
    if (L < 4 || T < 2 || (T & 1) || L % T || ((L / T) & 1) || k < 1 || nsweeps < 0) return -1;
    orc_geom g = mkgeom(2, L, L, 1);
    uint64_t Tm[4];
    orc_metropolis_table(beta, 3, Tm);
    for (int t = 0; t < nsweeps; ++t) {
        uint64_t sweep = sweep0 + (uint64_t)t;
        for (int P = 0; P < 2; ++P)
            for (int h = 0; h < k; ++h) {
                uint64_t draw_sweep = sweep * (uint64_t)k + (uint64_t)h;
                for (int c = 0; c < 2; ++c) {
                    #pragma omp parallel for schedule(static) if (g.N >= 8192)
                    for (int y = 0; y < L; ++y)
                        for (int x = 0; x < L; ++x) {
                            if (((x / T + y / T) & 1) != P || ((x + y) & 1) != c) continue;
                            int64_t i = site(&g, x, y, 0);
                            int hf = local_field(&g, s, NULL, x, y, 0);
                            uint32_t r = orc_draw32(seed, ORC_TAG_SWEEP, ORC_TAG_SWEEP_LO,
                                                    (uint32_t)(i >> 1), replica, draw_sweep, (uint32_t)c);
                            int dE = 2 * s[i] * hf;
                            if (dE <= 0 || (uint64_t)r < Tm[dE / 4]) s[i] = (int8_t)-s[i];
                        }
                }
            }
        if (EM) orc_measure(2, L, L, 1, s, NULL, &EM[2 * t], &EM[2 * t + 1]);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Population annealing (Sec. "Population annealing", Eq. Q) for one
 * population of R replicas of the 2D L x L ferromagnet.  Replica slot k of
 * population pop draws its randomness as replica id pop*R + k.               */

/* Inclusive prefix sum in a fixed association order, so that any
 * implementation which follows it gets the same bits:
 *   level 0: blocks of 64 in index order, each scanned by doubling steps
 *            d = 1, 2, ..., 32: x_i <- x_i + x_{i-d} for i >= d, from the
 *            values before that step;
 *   level 1: the block totals, grouped 64 at a time, scanned the same way;
 *   level 2: the group totals accumulated one after the other;
 *   result:  C_i = x_i + (G_g + B_b), where B_b is the level-1 prefix of the
 *            blocks before block b inside its group and G_g the level-2
 *            prefix of the groups before group g.
 * Entries past R are zero.                                                  */
static void scan64(double *v)
{
    double tmp[64];
    for (int d = 1; d < 64; d *= 2) {
        memcpy(tmp, v, sizeof tmp);
        for (int i = d; i < 64; ++i) v[i] = tmp[i] + tmp[i - d];
    }
}

void orc_canonical_scan(const double *w, double *C, int64_t R)
{
    int64_t nb = (R + 63) / 64, ng = (nb + 63) / 64;
    double *x = calloc((size_t)nb * 64, sizeof(double));
    double *t = calloc((size_t)ng * 64, sizeof(double));
    double *G = calloc((size_t)ng, sizeof(double));
    memcpy(x, w, (size_t)R * sizeof(double));
    for (int64_t b = 0; b < nb; ++b) scan64(x + 64 * b);
    for (int64_t b = 0; b < nb; ++b) t[b] = x[64 * b + 63];
    for (int64_t q = 0; q < ng; ++q) scan64(t + 64 * q);
    G[0] = 0.0;
    for (int64_t q = 1; q < ng; ++q) G[q] = G[q - 1] + t[64 * (q - 1) + 63];
    for (int64_t i = 0; i < R; ++i) {
        int64_t b = i / 64, q = b / 64;
        double Bb = (b % 64 == 0) ? 0.0 : t[b - 1];
        C[i] = x[i] + (G[q] + Bb);
    }
    free(x); free(t); free(G);
}

static void energies_2d(int L, int64_t R, const int8_t *spins, int64_t *E)
{
    int64_t N = (int64_t)L * L;
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < R; ++k) {
        int64_t e, m;
        orc_measure(2, L, L, 1, spins + k * N, NULL, &e, &m);
        E[k] = e;
    }
}

/* Population at beta_0 = 0: R independent hot starts (exact equilibrium). */
int orc_pa_init(int L, int R, int pop, uint64_t seed, int8_t *spins, int64_t *E)
{
    if (L < 2 || (L & 1) || R < 1) return -1;
    int64_t N = (int64_t)L * L;
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < R; ++k)
        orc_init(2, L, L, 1, spins + k * N, 1, seed, (uint32_t)((int64_t)pop * R + k));
    energies_2d(L, R, spins, E);
    return 0;
}

/* Annealing steps i = step_first .. step_first + nsteps - 1 (step_first >= 1),
 * with beta[] indexed by step number (beta[0] = beta_0).  Per step:
 *   1. w_j = exp(-(beta_i - beta_{i-1}) (E_j + 2N))  (shifted so w_j <= 1);
 *   2. C = canonical inclusive prefix sum of w; C_tot = C_{R-1};
 *      Q_i = exp(2N dbeta) C_tot / R, ln Q_i = log(C_tot / R) + 2N dbeta;
 *   3. multinomial resampling at fixed R: slot k draws u_k, t = u_k C_tot,
 *      parent = min{ j : Cmax_j > t } with Cmax the running maximum of C;
 *   4. copies of parent j fill slots [P_j, P_j + n_j), P = exclusive prefix
 *      sum of the integer copy numbers n_j;
 *   5. theta Metropolis sweeps at beta_i, sweep numbers (i-1) theta + t,
 *      replica id pop*R + slot;
 *   6. energies and the histogram of levels (E + 2N)/4.
 * Outputs per step s: Ctot[s], lnQ[s], hist[s*(N+1) ...].  counts (optional)
 * receives n_j of the last step.                                            */
int orc_pa_steps(int L, int R, int pop, int step_first, int nsteps, const double *beta, int theta,
                 uint64_t seed, int8_t *spins, int64_t *E, double *Ctot, double *lnQ,
                 int64_t *hist, int32_t *counts)
{
    if (L < 2 || (L & 1) || R < 1 || step_first < 1 || nsteps < 0 || theta < 0) return -1;
    int64_t N = (int64_t)L * L;
    double *w = malloc((size_t)R * sizeof(double));
    double *C = malloc((size_t)R * sizeof(double));
    double *wtab = malloc((size_t)(N + 1) * sizeof(double));
    int32_t *parent = malloc((size_t)R * sizeof(int32_t));
    int32_t *n = malloc((size_t)R * sizeof(int32_t));
    int64_t *P = malloc((size_t)R * sizeof(int64_t));
    int8_t *next = malloc((size_t)(R * N));
    for (int s = 0; s < nsteps; ++s) {
        int i = step_first + s;
        double dbeta = beta[i] - beta[i - 1];
        for (int64_t k = 0; k <= N; ++k) wtab[k] = exp(-dbeta * (double)(4 * k));
        for (int64_t j = 0; j < R; ++j) w[j] = wtab[(E[j] + 2 * N) / 4];
        orc_canonical_scan(w, C, R);
        double ct = C[R - 1];
        Ctot[s] = ct;
        lnQ[s] = log(ct / (double)R) + dbeta * (double)(2 * N);
        /* running maximum, then the first index whose value exceeds t */
        for (int64_t j = 1; j < R; ++j) if (C[j] < C[j - 1]) C[j] = C[j - 1];
        #pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < R; ++k) {
            double u = orc_resample_u(seed, (uint32_t)k, (uint32_t)pop, (uint32_t)i);
            double t = u * ct;
            int64_t j = 0;
            while (j < R - 1 && !(C[j] > t)) ++j;
            parent[k] = (int32_t)j;
        }
        memset(n, 0, (size_t)R * sizeof(int32_t));
        for (int64_t k = 0; k < R; ++k) n[parent[k]] += 1;
        P[0] = 0;
        for (int64_t j = 1; j < R; ++j) P[j] = P[j - 1] + n[j - 1];
        for (int64_t j = 0; j < R; ++j)
            for (int32_t c = 0; c < n[j]; ++c)
                memcpy(next + (P[j] + c) * N, spins + j * N, (size_t)N);
        memcpy(spins, next, (size_t)(R * N));
        if (counts) memcpy(counts, n, (size_t)R * sizeof(int32_t));
        #pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < R; ++k)
            orc_sweep(2, L, L, 1, spins + k * N, NULL, 0, beta[i], seed,
                      (uint32_t)((int64_t)pop * R + k), (uint64_t)(i - 1) * (uint64_t)theta, theta, NULL);
        energies_2d(L, R, spins, E);
        int64_t *hs = hist + (int64_t)s * (N + 1);
        memset(hs, 0, (size_t)(N + 1) * sizeof(int64_t));
        for (int64_t k = 0; k < R; ++k) hs[(E[k] + 2 * N) / 4] += 1;
    }
    free(w); free(C); free(wtab); free(parent); free(n); free(P); free(next);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Multicanonical walkers (Sec. "Multicanonical simulations").  Each walker is
 * its own 2D L x L ferromagnet restricted to the energy window [-2N, 0]
 * (levels k = (E + 2N)/4 = 0..N/2).  One sweep visits the sites in sequential
 * (typewriter) order i = 0..N-1, the same order for every walker; the move
 * s_i -> -s_i is accepted with min(1, W(E')/W(E)); a move that would leave the
 * window is rejected and the current energy is counted again.  The histogram
 * receives the level after every attempted move.
 * T[k*4 + d] for d = 0..3 <-> level change -2, -1, +1, +2:
 *   ceil(min(1, exp(lnW[k'] - lnW[k])) 2^32), at least 1.
 * The update of site i in sweep t of walker w draws the whole 32-bit word
 * (i mod 4) of Philox(TAG_MUCA, a = i div 4, replica = w, sweep = t).       */
void orc_muca_table(int L, const double *lnW, uint64_t *T)
{
    int64_t N = (int64_t)L * L, K = N / 2;
    static const int dk[4] = {-2, -1, 1, 2};
    for (int64_t k = 0; k <= K; ++k)
        for (int d = 0; d < 4; ++d) {
            int64_t k2 = k + dk[d];
            uint64_t v = 0;
            if (k2 >= 0 && k2 <= K) {
                double x = lnW[k2] - lnW[k];
                double p = x >= 0.0 ? 1.0 : exp(x);
                v = (uint64_t)ceil(ldexp(p, 32));
                if (v == 0) v = 1; /* p below 2^-32 (exp underflow) counts as 2^-32 */
            }
            T[k * 4 + d] = v;
        }
}

/* Walker start: hot start keyed by the walker index; if its energy lies above
 * the window, flip the spins of the odd sub-lattice, which maps E to -E.     */
/* Level of disorder of walker w of W in the stratified start: the largest
 * c in 0..128 with (257 - 2c)^2 * 2W > 65536 (2W - 2w - 1), i.e.
 * c = 128 (1 - sqrt(1 - (w + 1/2)/W)) rounded to the nearest integer, in
 * integer arithmetic.  Flipping each spin of the ground state with
 * probability c/256 gives E ~ -2N (1 - c/128)^2, so the walkers' starting
 * energies spread evenly over the window [-2N, 0].                            */
int orc_muca_strat_level(int w, int W)
{
    int c = 0;
    for (int t = 1; t <= 128; ++t) {
        int64_t a = (int64_t)(257 - 2 * t) * (257 - 2 * t) * 2 * (int64_t)W;
        int64_t b = (int64_t)65536 * (2 * (int64_t)W - 2 * (int64_t)w - 1);
        if (a > b) c = t;
    }
    return c;
}

/* Walker starts.  start 0 (hot): walker w is the hot start of replica id w.
 * start 1 (stratified): site i of walker w is -1 iff byte (i mod 16) of
 * Philox(INIT, i/16, w) is at least 256 - c_w (c_w = 128 is the hot start).
 * Either way the odd sub-lattice is flipped when E > 0 (E -> -E), so every
 * walker starts inside the window.                                           */
int orc_muca_start(int L, int walkers, uint64_t seed, int start, int8_t *spins, int64_t *E)
{
    if (L < 4 || (L & 1) || walkers < 1 || start < 0 || start > 1) return -1;
    int64_t N = (int64_t)L * L;
    #pragma omp parallel for schedule(static)
    for (int64_t w = 0; w < walkers; ++w) {
        int8_t *s = spins + w * N;
        int64_t e, m;
        unsigned c = start ? (unsigned)orc_muca_strat_level((int)w, walkers) : 128u;
        for (int64_t i = 0; i < N; ++i)
            s[i] = orc_draw_byte(seed, ORC_TAG_INIT, (uint32_t)i, (uint32_t)w, 0, 0) >= 256u - c ? -1 : 1;
        orc_measure(2, L, L, 1, s, NULL, &e, &m);
        if (e > 0) {
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x)
                    if ((x + y) & 1) s[x + (int64_t)L * y] = (int8_t)-s[x + (int64_t)L * y];
            orc_measure(2, L, L, 1, s, NULL, &e, &m);
        }
        E[w] = e;
    }
    return 0;
}

/* Energies of given walker lattices; a walker above the window has its odd
 * sub-lattice flipped (E -> -E).                                            */
int orc_muca_settle(int L, int walkers, int8_t *spins, int64_t *E)
{
    if (L < 4 || (L & 1) || walkers < 1) return -1;
    int64_t N = (int64_t)L * L;
    #pragma omp parallel for schedule(static)
    for (int64_t w = 0; w < walkers; ++w) {
        int8_t *s = spins + w * N;
        int64_t e, m;
        orc_measure(2, L, L, 1, s, NULL, &e, &m);
        if (e > 0) {
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x)
                    if ((x + y) & 1) s[x + (int64_t)L * y] = (int8_t)-s[x + (int64_t)L * y];
            e = -e;
        }
        E[w] = e;
    }
    return 0;
}

int orc_muca_sweeps(int L, int walkers, int8_t *spins, int64_t *E, const double *lnW, uint64_t seed,
                    uint64_t sweep0, int nsweeps, int record, int64_t *H)
{
    if (L < 4 || (L & 1) || walkers < 1 || nsweeps < 0) return -1;
    int64_t N = (int64_t)L * L, K = N / 2;
    uint64_t *T = malloc((size_t)(K + 1) * 4 * sizeof(uint64_t));
    orc_muca_table(L, lnW, T);
    orc_geom g = mkgeom(2, L, L, 1);
    int64_t *Hw = calloc((size_t)walkers * (K + 1), sizeof(int64_t));
    #pragma omp parallel for schedule(dynamic)
    for (int64_t w = 0; w < walkers; ++w) {
        int8_t *s = spins + w * N;
        int64_t e = E[w];
        int64_t *hw = Hw + w * (K + 1);
        for (int t = 0; t < nsweeps; ++t) {
            uint64_t sweep = sweep0 + (uint64_t)t;
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    int64_t i = site(&g, x, y, 0);
                    int h = local_field(&g, s, NULL, x, y, 0);
                    int dE = 2 * s[i] * h;
                    int64_t e2 = e + dE;
                    if (e2 <= 0) {
                        uint32_t r = orc_draw_word(seed, ORC_TAG_MUCA, (uint32_t)i, (uint32_t)w, sweep);
                        int64_t k = (e + 2 * N) / 4;
                        int accept;
                        if (dE == 0) accept = 1;
                        else {
                            int d = dE / 4;              /* -2, -1, 1, 2 */
                            int col = d < 0 ? d + 2 : d + 1;
                            accept = (uint64_t)r < T[k * 4 + col];
                        }
                        if (accept) { s[i] = (int8_t)-s[i]; e = e2; }
                    }
                    if (record) hw[(e + 2 * N) / 4] += 1;
                }
        }
        E[w] = e;
    }
    if (record)
        for (int64_t w = 0; w < walkers; ++w)
            for (int64_t k = 0; k <= K; ++k) H[k] += Hw[w * (K + 1) + k];
    free(Hw);
    free(T);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Wang-Landau sampling in energy windows (Sec. "Wang-Landau update").  Energy
 * levels k = (E + 2N)/4 of the 2D L x L torus; window i holds the levels
 * [lo_i, hi_i] within [0, N/2] (E <= 0) and is sampled by M walkers, walker w
 * (of nwin M) in window w / M.  Each walker keeps its own estimate of ln g
 * over its window's levels, G_w[k - lo] in units of 2^-32 (int64), and its own
 * visit counts H_w[k - lo]; both arrays have wmax entries per walker.
 *
 * One update of a walker: the typewriter site order of the multicanonical
 * walkers; the level k2 after a flip; a move out of the window is rejected
 * and the current level counted again; otherwise the move is accepted with
 * min[1, g(E)/g(E')] = exp(-(G[k2] - G[k]) 2^-32) when G[k2] > G[k] (always
 * when G[k2] <= G[k]), by r32 < ceil(p 2^32) with r32 word (i mod 4) of
 * Philox(MUCA, i div 4, w, sweep).  After the update, G[k] += inc (ln f in
 * units of 2^-32) and H[k] += 1 at the level the walker is at.
 *
 * The exponential of an estimate difference x (units of 2^-32) is the product,
 * in this order, of exp(-n), exp(-a 2^-8), exp(-b 2^-16), exp(-c 2^-24) and
 * exp(-d 2^-32), x = n 2^32 + a 2^24 + b 2^16 + c 2^8 + d, each factor from
 * libm exp in FP64; n >= 23 gives p < 2^-32, i.e. the threshold 1.          */
#define ORC_WL_NEXP 23

static void orc_wl_exp_tables(double *en, double *t8, double *t16, double *t24, double *t32)
{
    for (int n = 0; n < ORC_WL_NEXP; ++n) en[n] = exp(-(double)n);
    for (int a = 0; a < 256; ++a) {
        t8[a] = exp(-(double)a / 256.0);
        t16[a] = exp(-(double)a / 65536.0);
        t24[a] = exp(-(double)a / 16777216.0);
        t32[a] = exp(-(double)a / 4294967296.0);
    }
}

/* ceil(exp(-x 2^-32) 2^32) for x > 0 (at least 1) */
uint64_t orc_wl_threshold(uint64_t x)
{
    static double en[ORC_WL_NEXP], t8[256], t16[256], t24[256], t32[256];
    static int ready = 0;
    if (!ready) {
        #pragma omp critical(orc_wl_tab)
        {
            if (!ready) { orc_wl_exp_tables(en, t8, t16, t24, t32); ready = 1; }
        }
    }
    uint64_t n = x >> 32;
    if (n >= ORC_WL_NEXP) return 1;
    uint32_t lo = (uint32_t)x;
    double p = en[n];
    p = p * t8[lo >> 24];
    p = p * t16[(lo >> 16) & 255u];
    p = p * t24[(lo >> 8) & 255u];
    p = p * t32[lo & 255u];
    uint64_t T = (uint64_t)ceil(ldexp(p, 32));
    return T < 1 ? 1 : T;
}

/* Walkers into their windows: every walker starts from the ground state (all
 * +1, level 0) and runs typewriter passes in which a flip is taken iff the
 * walker is still below its window, the flip raises its level, and the top
 * bit of word (i mod 4) of Philox(WINDOW, i div 4, w, pass) is set; it stops
 * at the first level >= lo.  A flip moves the level by at most 2 and a window
 * spans at least 2 levels, so the walker stops inside.  Below E = 0 some flip
 * always raises the energy, so the walk cannot stall.  Returns -1 unless
 * every window is within [0, N/2] with hi - lo >= 1 and every walker arrived
 * within max_pass passes.                                                    */
int orc_win_drive(int L, int nwin, int M, const int32_t *lo, const int32_t *hi, uint64_t seed, int max_pass,
                  int8_t *spins, int64_t *E)
{
    if (L < 4 || (L & 1) || nwin < 1 || M < 1) return -1;
    int64_t N = (int64_t)L * L, K = N / 2;
    for (int i = 0; i < nwin; ++i)
        if (lo[i] < 0 || hi[i] > K || hi[i] - lo[i] < 1) return -1;
    orc_geom g = mkgeom(2, L, L, 1);
    int bad = 0;
    #pragma omp parallel for schedule(dynamic) reduction(|:bad)
    for (int64_t w = 0; w < (int64_t)nwin * M; ++w) {
        int8_t *s = spins + w * N;
        int64_t klo = lo[w / M], k = 0;
        for (int64_t i = 0; i < N; ++i) s[i] = 1;
        for (int pass = 0; pass < max_pass && k < klo; ++pass)
            for (int y = 0; y < L && k < klo; ++y)
                for (int x = 0; x < L && k < klo; ++x) {
                    int64_t i = site(&g, x, y, 0);
                    int dl = 2 * s[i] * local_field(&g, s, NULL, x, y, 0) / 4;
                    if (dl <= 0) continue;
                    uint32_t r = orc_draw_word(seed, ORC_TAG_WINDOW, (uint32_t)i, (uint32_t)w, (uint64_t)pass);
                    if (r >> 31) { s[i] = (int8_t)-s[i]; k += dl; }
                }
        if (k < klo) bad = 1;
        E[w] = 4 * k - 2 * N;
    }
    return bad ? -1 : 0;
}

/* nsweeps Wang-Landau sweeps (above) of the walkers of every window i with
 * active[i] (others are left as they are); inc[i] is ln f of window i in
 * units of 2^-32 (0: fixed weights, i.e. multicanonical sweeps with ln W =
 * -G 2^-32 in the window).  Afterwards each swept walker's estimate is shifted
 * to a minimum of 0 over its window's levels with states.                   */
int orc_wl_sweeps(int L, int nwin, int M, const int32_t *lo, const int32_t *hi, int wmax, const int64_t *inc,
                  const uint8_t *active, uint64_t seed, uint64_t sweep0, int nsweeps, int8_t *spins, int64_t *E,
                  int64_t *G, uint32_t *H)
{
    if (L < 4 || (L & 1) || nwin < 1 || M < 1 || nsweeps < 0) return -1;
    int64_t N = (int64_t)L * L, K = N / 2;
    for (int i = 0; i < nwin; ++i)
        if (lo[i] < 0 || hi[i] > K || hi[i] - lo[i] < 1 || hi[i] - lo[i] + 1 > wmax) return -1;
    orc_geom g = mkgeom(2, L, L, 1);
    #pragma omp parallel for schedule(dynamic)
    for (int64_t w = 0; w < (int64_t)nwin * M; ++w) {
        int win = (int)(w / M);
        if (active && !active[win]) continue;
        int8_t *s = spins + w * N;
        int64_t *Gw = G + w * wmax;
        uint32_t *Hw = H + w * wmax;
        int64_t klo = lo[win], khi = hi[win], k = (E[w] + 2 * N) / 4;
        for (int t = 0; t < nsweeps; ++t) {
            uint64_t sweep = sweep0 + (uint64_t)t;
            for (int y = 0; y < L; ++y)
                for (int x = 0; x < L; ++x) {
                    int64_t i = site(&g, x, y, 0);
                    int dl = 2 * s[i] * local_field(&g, s, NULL, x, y, 0) / 4;
                    int64_t k2 = k + dl;
                    int accept;
                    if (dl == 0) accept = 1;
                    else if (k2 < klo || k2 > khi) accept = 0;       /* counted again */
                    else {
                        int64_t d = Gw[k2 - klo] - Gw[k - klo];
                        if (d <= 0) accept = 1;
                        else {
                            uint32_t r = orc_draw_word(seed, ORC_TAG_MUCA, (uint32_t)i, (uint32_t)w, sweep);
                            accept = (uint64_t)r < orc_wl_threshold((uint64_t)d);
                        }
                    }
                    if (accept) { s[i] = (int8_t)-s[i]; k = k2; }
                    Gw[k - klo] += inc[win];
                    Hw[k - klo] += 1u;
                }
        }
        E[w] = 4 * k - 2 * N;
        /* ln g is fixed up to a constant: the walker's estimate is shifted to a
         * minimum of 0 over its levels with states (level 1 has none), which
         * keeps it bounded and changes no decision */
        int64_t mn = INT64_MAX;
        for (int64_t kk = klo; kk <= khi; ++kk)
            if (kk != 1 && Gw[kk - klo] < mn) mn = Gw[kk - klo];
        for (int64_t kk = klo; kk <= khi; ++kk) Gw[kk - klo] -= mn;
    }
    return 0;
}
