/*
 * mcspin.h -- C ABI of libmcspin, a gfx950 (MI355X) Monte Carlo engine for
 * Ising-type lattice spin models.
 *
 * Method: M. Weigel, "Monte Carlo methods for massively parallel computers",
 * arXiv:1709.04394.  Section names below refer to that text.
 *
 * Conventions shared by every call
 *   - Plain C types only.  A `stream` argument is a hipStream_t passed as
 *     void* (NULL = the default stream).  Pointers documented as "device" must
 *     point to memory of the context's device; "host" pointers to host memory.
 *   - The caller owns every buffer.  The library never allocates or frees
 *     device memory inside a call; scratch space comes from caller workspaces
 *     whose size the matching *_workspace_bytes() call reports (or, for
 *     mc_sweep_noalloc, from a fixed device array of the library).
 *   - Return value: 0 on success, a negative mc_status otherwise.  Arguments
 *     are checked in full before any device work is enqueued, so a failing call
 *     has no side effect.  mc_strerror() names a code, mc_ctx_last_error() gives
 *     the detail of the last failure on a context.  No C++ exception crosses
 *     this boundary.  Use one context per host thread.
 *   - Stream-ordered calls (mc_init, mc_couplings, mc_sweep, mc_measure,
 *     mc_muca_sweeps, mc_mlp_*) return once their work is enqueued; device
 *     buffers must stay alive until the stream has passed the call.  Calls that
 *     return host results (mc_pa_anneal, mc_pt_run, mc_muca_run) synchronise
 *     the stream.
 *   - Determinism: every output is a pure function of the inputs, the seed and
 *     the sweep numbers.  It does not depend on launch shape, tile choice, the
 *     number of lattices per launch or the run (Sec. "Random number
 *     generation": counter-based generators keyed by intrinsic variables).
 *
 * Lattice layout (MC_INT8): spins[l][z][y][x], x fastest, one int8 per site,
 * values +1 / -1; l = 0..count-1 are independent lattices whose random
 * streams use replica ids replica0 + l.  MC_MSC64 (multi-spin coding, Sec.
 * "Checkerboard scheme"): words[l][z][y][x] of uint64, bit b of a word is the
 * spin of replica replica0 + 64 l + b at that site, bit set <=> s = -1.
 * Couplings (+-J model, Sec. "Disordered systems"): J[d][z][y][x] int8 +-1 is
 * the coupling of the bond (site, site + e_d), d = x, y(, z); NULL means J = 1.
 * Boundary conditions are periodic in every direction.
 *
 * Random numbers: Philox4x32-10 (key = seed as two 32-bit words, counter as
 * given per call) yields a block of four 32-bit words w0..w3.  "Byte p of a
 * block" (p = 0..15) below is not the p-th byte of those 16 bytes: it is the
 * 8-bit number whose bit k (k = 0..7) is bit p of 16-bit half-word k of the
 * block, half-word k being bits 16 (k mod 2) .. 16 (k mod 2) + 15 of word
 * k / 2.  One block thus gives 16 bytes as eight bit-planes, the form the
 * bit-sliced kernels consume.  "Word 0" is w0.  The tags in counter word 3
 * (bits 24..31) are TAG_INIT = 1, TAG_SWEEP = 2, TAG_COUPLING = 3,
 * TAG_RESAMPLE = 4, TAG_MUCA = 5, TAG_MLP_INIT = 6, TAG_SWEEP_LO = 7,
 * TAG_EXCHANGE = 9 (8 is reserved); bit 23 holds the half-sweep colour where
 * one is given, bits 0..22 the high bits of a 64-bit sweep number.
 */
#ifndef MCSPIN_H
#define MCSPIN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MC_ABI_VERSION 1

typedef struct mc_ctx mc_ctx;

typedef enum {
    MC_OK = 0,
    MC_E_INVAL = -1,     /* null pointer, unknown enum value                     */
    MC_E_SHAPE = -2,     /* odd or too small extent, unsupported shape             */
    MC_E_RANGE = -3,     /* beta < 0 or NaN, negative counts, sizes out of range   */
    MC_E_LAYOUT = -4,    /* layout / rule / coupling combination not supported     */
    MC_E_WORKSPACE = -5, /* workspace missing or smaller than required             */
    MC_E_DEVICE = -6,    /* HIP runtime error (detail in mc_ctx_last_error)        */
    MC_E_NOTCONV = -7,   /* a run stopped unconverged (outputs still valid)        */
    MC_E_IO = -8         /* a file could not be opened, read or written            */
} mc_status;

enum { MC_INT8 = 0, MC_MSC64 = 1 };
enum { MC_METROPOLIS = 0, MC_HEATBATH = 1 };
enum { MC_COLD = 0, MC_HOT = 1 };

/* dims = 2 or 3; Lz = 1 when dims == 2; count = number of int8 lattices or of
 * 64-lane word lattices, 1..65535 (MC_E_RANGE otherwise).  Every extent must
 * be even and >= 4.                                                        */
typedef struct {
    int32_t dims, Lx, Ly, Lz, layout, count;
} mc_geom;

typedef struct {
    int32_t rule;      /* MC_METROPOLIS or MC_HEATBATH                          */
    double beta;       /* inverse temperature, >= 0                             */
    uint64_t seed;     /* Philox key                                            */
    uint32_t replica0; /* replica id of lattice 0 (of lane 0 for MC_MSC64)      */
    uint64_t sweep0;   /* global number of the first sweep of this call         */
    int32_t nsweeps;   /* >= 0                                                  */
} mc_sweep_args;

int mc_abi_version(void);
const char *mc_strerror(int code);

/* Create a context bound to HIP device `device` (host state only; the device
 * is first used, and checked, by the first call that enqueues work). */
int mc_ctx_create(mc_ctx **out, int device);
void mc_ctx_destroy(mc_ctx *ctx);
const char *mc_ctx_last_error(const mc_ctx *ctx);

/* Lattice initialisation (Sec. "Checkerboard scheme", step 1).
 * MC_COLD: every spin +1.  MC_HOT: site i of replica r is +1 iff byte (i mod
 * 16) of Philox4x32-10(key = seed, ctr = (i/16, r, 0, TAG_INIT << 24)) is
 * below 128, i.e. an independent fair coin per site.
 * spins: device, layout per geom.  Stream-ordered.                         */
int mc_init(mc_ctx *ctx, const mc_geom *geom, void *spins, int32_t start, uint64_t seed,
            uint32_t replica0, void *stream);

/* Bimodal couplings J = +-1 with p = 1/2 (Sec. "Disordered systems"): the
 * coupling with flat index b = d N + i is +1 iff byte (b mod 16) of
 * Philox(ctr = (b/16, 0, 0, TAG_COUPLING << 24)) is below 128.
 * J: device int8 [dims][N] (geom->count is ignored).  Stream-ordered.       */
int mc_couplings(mc_ctx *ctx, const mc_geom *geom, int8_t *J, uint64_t seed, void *stream);

/* Bytes of scratch mc_sweep can use to run several sweeps per fused launch:
 * two bit-packed copies of the lattices (count * Lz * Ly * Lx / 8 bytes
 * each), between which the launches of one call ping-pong; in 3D the
 * couplings packed once per call (3 * Lz * Ly * Lx / 8 bytes), the total so
 * far rounded up to a multiple of 256; then two arrays of per-tile (E, M)
 * sums of one launch, each rounded up to a multiple of 256 bytes: 8 * count *
 * ceil(Ly / 4) * 16 bytes in 2D, 4 * count * ceil(Ly / 2) * ceil(Lz / 2) * 16
 * in 3D.  Only the first launch reads and
 * only the last writes the caller's int8 lattices.  Non-zero
 * for int8 geometries with Lx a multiple of 64: 2D with Lx <= 16384, 3D with
 * Lx <= 4096 and Ly, Lz >= 4.  With a smaller or NULL workspace mc_sweep uses
 * kernels that need none (a whole small lattice per workgroup, or per-half-
 * sweep launches); the results are identical either way.                   */
size_t mc_sweep_workspace_bytes(const mc_geom *geom);

/* nsweeps checkerboard sweeps (Sec. "Checkerboard scheme"): one sweep updates
 * every site with x+y(+z) even, then every odd site; within a half-sweep all
 * sites of that colour are updated from the same neighbour values.
 *   Metropolis (Eq. metropolis-canonical): dE = 2 s_i h_i with
 *     h_i = sum_j J_ij s_j; flip iff dE <= 0 or r32 < ceil(exp(-beta dE) 2^32).
 *   Heat-bath (Eq. heatbath): s_i' = +1 iff r32 < ceil(2^32 / (1 + exp(-2 beta h_i))).
 *   r32 for the site with same-colour index j = i >> 1 of colour c in sweep t
 *   of replica r: (byte (j mod 16) of Philox(ctr = (j/16, r, t, TAG_SWEEP<<24 |
 *   c<<23 | t>>32)) << 24) | (word 0 of Philox(ctr = (j, r, t, TAG_SWEEP_LO<<24
 *   | c<<23 | t>>32)) & 0xFFFFFF).  Tables are built once per call in FP64 on
 *   the host; the device compares integers only.
 * spins: device, in/out.  J: device int8 [dims][N] or NULL.
 * EM: device int64 [nsweeps][count * lanes][2] = (E, M) after each sweep,
 *     lanes = 1 (MC_INT8) or 64 (MC_MSC64), E = -sum_<ij> J_ij s_i s_j over
 *     bonds (Eq. ising_model, h = 0), M = sum_i s_i; or NULL.
 * ws: device scratch of ws_bytes (may be NULL, see above).  Stream-ordered.  */
int mc_sweep(mc_ctx *ctx, const mc_geom *geom, void *spins, const int8_t *J, const mc_sweep_args *args,
             int64_t *EM, void *ws, size_t ws_bytes, void *stream);

/* As mc_sweep for MC_INT8 lattices, but lattice l runs at inverse temperature
 * betas[l] (host array of geom->count entries; args->beta is ignored).  The
 * results of lattice l are exactly those of mc_sweep on that lattice alone
 * with replica0 + l at betas[l]; batching only lets one launch carry all of
 * them (taller bands, less redone halo).                                   */
int mc_sweep_betas(mc_ctx *ctx, const mc_geom *geom, void *spins, const int8_t *J, const mc_sweep_args *args,
                   const double *betas, int64_t *EM, void *ws, size_t ws_bytes, void *stream);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): mc_sweep without a
 * workspace argument.  The scratch the fused kernels need (the size
 * mc_sweep_workspace_bytes reports) comes from a device array of the library
 * of mc_static_scratch_bytes() bytes (20 MiB), one per device, held until
 * the process ends; its address is looked up once per device on the first
 * call.  The call allocates nothing: no hipMalloc, hipFree or allocating
 * library routine.  Results are those of mc_sweep with a large enough
 * workspace.  Every call on a device shares that device's array and leaves
 * it holding its own intermediate lattices, so calls that overlap in time on
 * one device (different streams or host threads) race and must not be made;
 * calls in one stream are fine.  Errors: those of mc_sweep; MC_E_RANGE,
 * before any device work, when the geometry's fused scratch is larger than
 * the array (e.g. more than four 4096^2 lattices, or a 2D lattice of 2^27
 * sites); geometries that need no scratch run as mc_sweep does without
 * a workspace.  Stream-ordered.                                            */
size_t mc_static_scratch_bytes(void);
int mc_sweep_noalloc(mc_ctx *ctx, const mc_geom *geom, void *spins, const int8_t *J, const mc_sweep_args *args,
                     int64_t *EM, void *stream);

/* Double-checkerboard Metropolis sweeps with `hits` updates per tile load
 * (Sec. "Checkerboard scheme": the two-level "double checkerboard" of the
 * right panel of Fig. checkerboard, and multi-hit updates) of 2D L x L
 * ferromagnets (J = 1), MC_INT8, L a multiple of 64 up to 16384.  The
 * lattice is cut into tile x tile tiles (tile in {64, 128, 256, 512}, L /
 * tile even) whose coarse colour is (x/tile + y/tile) mod 2.  One sweep
 * updates every tile of coarse colour 0, then every tile of colour 1; each
 * tile, with the other colour's spins fixed, takes `hits` rounds of its own
 * checkerboard (sites with x + y even, then odd), so every site is updated
 * `hits` times per sweep.  Hit h of sweep t of a site draws exactly the r32
 * that mc_sweep's sweep number t hits + h draws for it (replica r, same-
 * colour index, colour).  This is a different Markov chain from mc_sweep's
 * (with the same stationary distribution; no detailed balance).  EM: device
 * int64 [nsweeps][count][2], (E, M) after each sweep, or NULL.  ws: device
 * scratch of mc_dcb_workspace_bytes(geom) bytes: one bit-packed copy of the
 * lattices (count * L * L / 8 bytes, rounded up to a multiple of 256),
 * updated in place by the sweeps' launches, then two arrays of per-tile
 * (E, M) shares used by alternate sweeps (count * (L / 64)^2 * 16 bytes
 * each, rounded up likewise).  args->rule must be
 * MC_METROPOLIS (MC_E_LAYOUT otherwise); MC_E_SHAPE for an unsupported L or
 * tile; MC_E_RANGE for hits outside 1..1000 or (sweep0 + nsweeps) hits >=
 * 2^55.  Stream-ordered.                                                    */
size_t mc_dcb_workspace_bytes(const mc_geom *geom);
int mc_sweep_dcb(mc_ctx *ctx, const mc_geom *geom, void *spins, const mc_sweep_args *args, int32_t tile, int32_t hits,
                 int64_t *EM, void *ws, size_t ws_bytes, void *stream);

/* Spin glasses multi-spin coded across disorder realisations (Sec.
 * "Disordered systems": the bits of a word are 64 realisations, each with its
 * own couplings; the coded copies share one random number per site).
 * mc_couplings_msc64: bimodal couplings of realisation k = realisation0 +
 *   64 l + b in bit b of word (l, d, i) of J (device uint64 [count][dims][N],
 *   bond (i, i + e_d), bit set <=> J = -1): exactly the couplings
 *   mc_couplings gives, but with counter word 1 = k (realisation 0 is
 *   mc_couplings' own).  geom: layout MC_MSC64.  Stream-ordered.
 * mc_sweep_sg_msc64: nsweeps checkerboard sweeps (rules as mc_sweep) of
 *   every realisation of the word lattices spins (MC_MSC64, bit b of word
 *   lattice l = realisation 64 l + b, e.g. initialised by mc_init: lane b is
 *   then the hot start of replica replica0 + 64 l + b) with couplings J (as
 *   above).  All 64 realisations of word lattice l draw the random numbers of
 *   replica id args->replica0 + l (the draw of mc_sweep for that replica and
 *   site): lane b evolves exactly as the int8 lattice of realisation 64 l + b
 *   under mc_sweep with replica id replica0 + l.  EM: device int64
 *   [nsweeps][count * 64][2] or NULL.  MC_E_LAYOUT unless MC_MSC64;
 *   MC_E_SHAPE unless the sites of one colour are a multiple of 64.
 *   Stream-ordered.                                                         */
int mc_couplings_msc64(mc_ctx *ctx, const mc_geom *geom, uint64_t *J, uint64_t seed, uint32_t realisation0,
                       void *stream);
int mc_sweep_sg_msc64(mc_ctx *ctx, const mc_geom *geom, uint64_t *spins, const uint64_t *J, const mc_sweep_args *args,
                      int64_t *EM, void *stream);

/* E and M of every lattice (lane) as in mc_sweep; EM: device int64
 * [count * lanes][2].  Stream-ordered.                                      */
int mc_measure(mc_ctx *ctx, const mc_geom *geom, const void *spins, const int8_t *J, int64_t *EM,
               void *stream);

/* The kernel family mc_sweep (per_lattice = 0) or mc_sweep_betas
 * (per_lattice != 0) runs for a geometry, update rule, presence of couplings
 * and workspace size, in order of preference: MC_PATH_FUSED_2D / _3D (int8,
 * Lx a multiple of 64, bit-packed tiles in LDS, several sweeps per launch;
 * 2D only for Metropolis without couplings; needs mc_sweep_workspace_bytes
 * of workspace), MC_PATH_SMALL_BITS (int8 lattices of 32-site rows that fit
 * one workgroup's LDS bit-packed), MC_PATH_SMALL (int8 lattices that fit one
 * workgroup's LDS), MC_PATH_MSC64 (64-lane words, Lx a multiple of 128),
 * MC_PATH_GENERIC (one launch per half-sweep).  Results never depend on the
 * path.  Host only: no device work.  Errors as for mc_sweep's geometry and
 * rule; MC_E_LAYOUT for per_lattice with MC_MSC64; MC_E_INVAL for a NULL
 * path.                                                                    */
enum { MC_PATH_FUSED_2D = 1, MC_PATH_FUSED_3D = 2, MC_PATH_SMALL_BITS = 3, MC_PATH_SMALL = 4,
       MC_PATH_MSC64 = 5, MC_PATH_GENERIC = 6 };
int mc_sweep_path(mc_ctx *ctx, const mc_geom *geom, int32_t rule, int32_t has_couplings, int32_t per_lattice,
                  size_t ws_bytes, int32_t *path);

/* Launch shape of the fused sweeps (int8, Lx a multiple of 64; 2D: J = 1,
 * Metropolis; 3D: Metropolis or heat-bath, with or without couplings): band
 * height H (2D rows per workgroup) or tile side H (3D: H x H rows in y, z),
 * K sweeps per launch and threads per workgroup.  The shape changes speed
 * only, never results (the determinism contract above).  mc_set_tile_plan
 * fixes it for the geometry (dims, extents, count) on this context;
 * mc_get_tile_plan reports the shape in use (the tuned or set one, else a
 * default).  Host-only calls.  A plan needs H >= 1, K >= 1 and threads a
 * multiple of 64 in 64..1024; in 2D H >= 4, K <= 8, the Lx/64 words of a row either
 * at most threads or a multiple of it, and (H + 4K) rows of 2 Lx/64 words
 * in at most 64 KB of LDS; in 3D H >= 2, K <= 4, Lx/64 <= threads, H <= min(Ly, Lz)
 * and the tile with its couplings in at most 96 KB.  MC_E_RANGE otherwise,
 * the geometry's own errors as for mc_sweep.                               */
int mc_set_tile_plan(mc_ctx *ctx, const mc_geom *geom, int32_t H, int32_t K, int32_t threads);
int mc_get_tile_plan(mc_ctx *ctx, const mc_geom *geom, int32_t *H, int32_t *K, int32_t *threads);

/* Autotuner: times every admissible (H, K, threads) for this geometry with
 * `sweeps` measured sweeps (the launches that compute per-sweep E, M, as
 * mc_sweep with EM; their per-tile sums go to the second half of scratch_b
 * and are not added up) at inverse temperature beta, in the steady state of
 * a long call (packed rows in and out), on two caller-provided scratch
 * lattices (device, count * N bytes each; overwritten), and keeps the
 * fastest shape on the context.
 * Synchronises the stream.                                                 */
int mc_tune_sweep(mc_ctx *ctx, const mc_geom *geom, void *scratch_a, void *scratch_b, double beta,
                  int32_t sweeps, void *stream);
/* As mc_tune_sweep for the given update rule (MC_METROPOLIS or MC_HEATBATH);
 * 3D geometries (Lx a multiple of 64) are tuned for tiles of H x H rows.  */
int mc_tune_sweep_rule(mc_ctx *ctx, const mc_geom *geom, int32_t rule, void *scratch_a, void *scratch_b,
                       double beta, int32_t sweeps, void *stream);

/* ------------------------------------------------------------------------
 * Population annealing (Sec. "Population annealing", Eq. Q) of npop
 * populations of R replicas of the 2D L x L ferromagnet (J = 1), one
 * population per extent L[p], all advanced together.
 *   Step i (beta_{i-1} -> beta_i): weights w_j = exp(-(beta_i - beta_{i-1})
 *   (E_j + 2N)) (FP64 host table per step, shifted so w <= 1); C = inclusive
 *   prefix sum of w in the fixed order: blocks of 64 by doubling steps
 *   x_i += x_{i-d} (d = 1, 2, .., 32), block totals 64 at a time the same way,
 *   group totals in sequence, C_i = x_i + (G + B); C_total = C_{R-1};
 *   ln Q_i = log(C_total / R) + 2N dbeta; multinomial resampling at fixed R:
 *   slot k draws u_k (53 bits from Philox(ctr = (k, p, i, TAG_RESAMPLE<<24)),
 *   words 0 and 1), parent = first j whose running maximum of C exceeds
 *   u_k C_total; copies of parent j fill slots [P_j, P_j + n_j) (P = exclusive
 *   prefix sum of the copy numbers n); then theta Metropolis sweeps at beta_i
 *   with replica id p R + slot and sweep numbers (i-1) theta + t.
 * A fresh anneal (step_first = 1) starts from R independent hot starts
 * (replica ids p R + k, the exact beta_0 = 0 equilibrium); a later
 * step_first continues from the population in pop_spins.
 * L[p] in {4, 8, 16, 32, 64} or a multiple of 64 up to 512; R <= 65536;
 * npop <= 8.                                                                */
typedef struct {
    int32_t npop;
    const int32_t *L;     /* host [npop]                                       */
    int32_t R;            /* replicas per population                           */
    int32_t theta;        /* Metropolis sweeps per step                        */
    uint64_t seed;
    int32_t step_first;   /* number of the first step of this call (>= 1)      */
    int32_t nsteps;       /* steps in this call                                */
    const double *beta;   /* host [step_first + nsteps]: beta[0..] schedule    */
} mc_pa_args;

size_t mc_pa_workspace_bytes(const mc_pa_args *args);

/* pop_spins: host array of npop device pointers, each to 2 R L^2 int8: the
 *   current population in the first R L^2 bytes (input when step_first > 1,
 *   output always), the second half is scratch.
 * Ctot, lnQ: host [npop][nsteps].  lnZ: host [npop][nsteps + 1]; lnZ[p][0] =
 *   ln Z at beta[step_first - 1] (set to L^2 ln 2 on a fresh anneal, read as
 *   given otherwise), lnZ[p][s] = lnZ[p][s-1] + lnQ[p][s-1].
 * hist: host int64, per population [nsteps + 1][L^2 + 1] (populations one
 *   after the other): row 0 the population at beta[step_first - 1], row s
 *   after step step_first + s - 1; column k counts replicas with E = 4k - 2N.
 * ws: device workspace of mc_pa_workspace_bytes(args).  Blocking: the steps
 *   run as one captured hipGraph on `stream`, which is synchronised.       */
int mc_pa_anneal(mc_ctx *ctx, const mc_pa_args *args, void *const *pop_spins, double *Ctot, double *lnQ,
                 double *lnZ, int64_t *hist, void *ws, size_t ws_bytes, void *stream);

/* Launch shape of population annealing: replicas per workgroup G of the
 * sweep kernel for populations of extent L (a per-context setting).  It
 * changes speed only: every replica draws from its own Philox stream keyed
 * by its replica id, so results are identical for every G.
 * mc_set_pa_group: G in 1..64 with G * 2 L * max(1, L/64) * 4 bytes of LDS
 *   at most 48 KB, else MC_E_RANGE; G = 0 restores the built-in rule (about
 *   256 packed 32-bit words per workgroup).  MC_E_SHAPE for an L that
 *   mc_pa_anneal rejects.
 * mc_get_pa_group: the G in use for L (set, tuned or built-in).           */
int mc_set_pa_group(mc_ctx *ctx, int32_t L, int32_t G);
int mc_get_pa_group(mc_ctx *ctx, int32_t L, int32_t *G);

/* Autotuner for G: for each population of args (extents must differ) it
 * times, with a host clock around blocking calls, a fresh anneal of that
 * population alone over the first min(step_first - 1 + nsteps, 20) steps of
 * the schedule, for G in {G0/4, G0/2, G0, 2 G0, 4 G0} (G0 the built-in rule,
 * candidates outside the limits above or above R skipped), best of two runs
 * each, and keeps the fastest G in the context.  G_out: host [npop] or NULL.
 * pop_spins[p] and ws are scratch (contents overwritten); ws must hold
 * mc_pa_workspace_bytes of one population over those steps.  Synchronises
 * `stream`.  Errors (before any device work): those of mc_pa_anneal's
 * arguments; MC_E_INVAL if an extent appears twice or pop_spins is NULL;
 * MC_E_RANGE if the schedule has no step; MC_E_WORKSPACE if ws is too small.
 * A device error while timing leaves the populations tuned so far set and
 * the current one at its previous setting.                                */
int mc_tune_pa(mc_ctx *ctx, const mc_pa_args *args, void *const *pop_spins, void *ws, size_t ws_bytes,
               int32_t *G_out, void *stream);

/* Parallel tempering (Sec. "Parallel Tempering", Eq. pt): one round of
 * replica-exchange moves, on the host.  n_temps replicas are held at the
 * inverse temperatures beta[0] < beta[1] < ... (host, strictly increasing,
 * finite, >= 0); replica_at[i] is the replica at temperature i and
 * temp_of[a] the temperature of replica a (host int32 [n_temps], inverse
 * permutations of 0..n_temps-1); E[a] is replica a's energy (host int64,
 * |E| <= 2^52), e.g. the last row of the per-sweep E of mc_sweep_betas run
 * with betas[a] = beta[temp_of[a]].  Round t proposes the pairs (i, i + 1)
 * with i = t mod 2, t mod 2 + 2, ...; with a, b the replicas at i and i + 1 the
 * exchange is accepted with min(1, exp((beta_i - beta_{i+1}) (E_a - E_b))):
 * always if the exponent is >= 0, else iff r32 < ceil(exp(exponent) 2^32)
 * (host FP64 libm exp), r32 = word (i mod 4) of Philox(ctr = (i / 4, 0, t,
 * TAG_EXCHANGE << 24 | t >> 32)).  Accepted: the two replicas' temperatures
 * are swapped in both maps and accepted[i] (host int64 [n_temps - 1]) is
 * incremented.  Configurations never move.  Host only: no device work.
 * Errors: MC_E_INVAL for a NULL pointer or maps that are not inverse
 * permutations; MC_E_RANGE for n_temps outside 2..2^20, a beta out of range
 * or not increasing, |E| > 2^52 or t >= 2^55.  Nothing is changed on error. */
int mc_pt_exchange(mc_ctx *ctx, int32_t n_temps, const double *beta, const int64_t *E, int32_t *temp_of,
                   int32_t *replica_at, uint64_t seed, uint64_t round, int64_t *accepted);

/* Parallel tempering on the device (Sec. "Parallel Tempering", Eq. pt):
 * n_sets independent sets of n_temps replicas of the 2D L x L ferromagnet
 * (J = 1), replica r of set s is lattice l = s n_temps + r of spins and has
 * replica id l.  Round t (t = round0 .. round0 + rounds - 1): every replica
 * runs theta checkerboard Metropolis sweeps (numbers t theta ..) at the
 * inverse temperature beta[temp_of[l]] it holds; then in every set, with
 * E the replicas' energies after those sweeps, the pairs of temperatures
 * (i, i + 1), i = t mod 2, t mod 2 + 2, .., are proposed as in
 * mc_pt_exchange, the draw being word (i mod 4) of Philox(ctr = (i / 4, s,
 * t, TAG_EXCHANGE << 24 | t >> 32)) (so set 0 draws exactly as
 * mc_pt_exchange); acceptance thresholds ceil(exp((beta_i - beta_{i+1}) 4m)
 * 2^32) for every energy difference 4m are built on the host once per call
 * (FP64 libm exp).  Temperatures are exchanged, configurations never move.
 * L as for mc_pa_anneal; 2 <= n_temps <= 1024; n_sets * n_temps <= 65535;
 * beta strictly increasing, finite, >= 0; theta >= 1.                     */
typedef struct {
    int32_t L;
    int32_t n_temps;
    int32_t n_sets;
    const double *beta;   /* host [n_temps]                                    */
    int32_t theta;        /* sweeps per round                                  */
    uint64_t seed;
    uint64_t round0;      /* number of the first round of this call            */
    int32_t rounds;
} mc_pt_args;

size_t mc_pt_workspace_bytes(const mc_pt_args *args);

/* spins: device int8 [n_sets * n_temps][L^2], in/out (initialise with mc_init
 *   and replica0 = 0 for a fresh run).
 * temp_of, replica_at: host int32 [n_sets][n_temps], in/out: per set the
 *   replica -> temperature map and its inverse (identity for a fresh run).
 * accepted: host int64 [n_sets][n_temps - 1], accepted exchanges of each
 *   pair, added to.
 * E_at: host int64 [rounds][n_sets][n_temps] or NULL: the energy held at each
 *   temperature in each round, before that round's exchanges.
 * ws: device workspace of mc_pt_workspace_bytes(args).  Blocking: the rounds
 *   run as one captured hipGraph on `stream`, which is synchronised; the
 *   context keeps the graph, and a call with the same arguments, buffers and
 *   launch shape launches it again.  A run split over several calls (round0
 *   advancing, maps and accepted carried over) equals one call.  Errors
 *   before any device work: MC_E_SHAPE for L, MC_E_RANGE for the counts and
 *   temperatures, MC_E_INVAL for a NULL pointer or maps that are not inverse
 *   permutations, MC_E_WORKSPACE.                                          */
int mc_pt_run(mc_ctx *ctx, const mc_pt_args *args, int8_t *spins, int32_t *temp_of, int32_t *replica_at,
              int64_t *accepted, int64_t *E_at, void *ws, size_t ws_bytes, void *stream);

/* Launch-shape cache: the tile plans (mc_set_tile_plan) and population-
 * annealing groups (mc_set_pa_group) a context holds, tuned or set, saved to
 * a text file and loaded into another context, so that tuning outlives the
 * process.  Shapes change speed only, never results; a file belongs to one
 * kind of device (tuned shapes are that device's).  Host only: no device
 * work, no stream.
 * Format: the line "libmcspin-launch-shapes 1", then one entry per line,
 *   "tile dims Lx Ly Lz count H K threads" (Lz = 1 in 2D) or "pa L G";
 *   '#' starts a comment, blank lines are skipped.
 * mc_tuning_save writes path + ".tmp" and renames it to path.  MC_E_IO if
 *   the file cannot be written; MC_E_INVAL for a NULL or empty path.
 * mc_tuning_load checks every entry as the setters do, then applies them all
 *   (overriding the context's entries for the same keys), or, on any error,
 *   none: MC_E_IO if the file cannot be read; MC_E_INVAL for a missing
 *   header, an unknown entry or a line over 255 characters; the setter's code
 *   (MC_E_RANGE, MC_E_SHAPE) for an entry it rejects.  mc_ctx_last_error
 *   names the file and line.                                             */
int mc_tuning_save(mc_ctx *ctx, const char *path);
int mc_tuning_load(mc_ctx *ctx, const char *path);

/* ------------------------------------------------------------------------
 * Multicanonical simulation with parallel walkers (Sec. "Multicanonical
 * simulations": walkers share W(E); their histograms are added; Eq. muca,
 * Eq. weight_modification) of the 2D L x L ferromagnet, restricted to the
 * energy window [-2N, 0] (levels k = (E + 2N)/4 = 0..N/2; g(E) = g(-E)
 * gives the other half).  Sites are visited in sequential (typewriter) order,
 * the same order for every walker; a flip is accepted with min(1,
 * W(E')/W(E)), i.e. r32 < T[k][d] = max(1, ceil(min(1, exp(lnW[k+d] -
 * lnW[k])) 2^32)) with r32 = word (i mod 4) of Philox(ctr = (i/4, walker,
 * sweep, TAG_MUCA << 24)); a move out of the window is rejected and the
 * current level counted again; the histogram counts the level after every
 * attempted move.  L in {4, 8, 12, 16, 24, 32, 48, 64, 96, 128}.            */
size_t mc_muca_workspace_bytes(int32_t L, int32_t walkers);

/* Walker starts.  MC_MUCA_HOT: walker w is the hot start of replica id w.
 * MC_MUCA_STRATIFIED: site i of walker w of W is -1 iff byte (i mod 16) of
 * Philox(ctr = (i/16, w, 0, TAG_INIT << 24)) is >= 256 - c_w, where c_w is
 * the largest c in 0..128 with (257 - 2c)^2 2W > 65536 (2W - 2w - 1), i.e.
 * 128 (1 - sqrt(1 - (w + 1/2)/W)) rounded: the expected starting energies
 * -2N (1 - c_w/128)^2 spread evenly over the window (c_w = 128 is the hot
 * start).  The paper leaves the walkers' initial states open.  Either way,
 * a walker whose energy is above the window has its odd sub-lattice flipped
 * (E -> -E).  spins: device int8 [walkers][L^2]; E: device int64 [walkers].
 * Stream-ordered.                                                          */
enum { MC_MUCA_HOT = 0, MC_MUCA_STRATIFIED = 1 };
int mc_muca_start(mc_ctx *ctx, int32_t L, int32_t walkers, uint64_t seed, int32_t start, int8_t *spins, int64_t *E,
                  void *stream);

/* nsweeps multicanonical sweeps of every walker at weights lnW (host
 * [N/2 + 1], finite), sweep numbers sweep0.., updating spins and E in place;
 * when record is set the visited levels are added to H (device int64
 * [N/2 + 1]).  Blocking (the host table must outlive the upload).          */
int mc_muca_sweeps(mc_ctx *ctx, int32_t L, int32_t walkers, int8_t *spins, int64_t *E, const double *lnW,
                   uint64_t seed, uint64_t sweep0, int32_t nsweeps, int32_t record, int64_t *H, void *ws,
                   size_t ws_bytes, void *stream);

/* Progress of a long multicanonical run, called on the calling thread after
 * every weight iteration (iteration >= 1, its flatness, sweeps per walker so
 * far) and after every 1000 production sweeps (iteration 0, flatness -1,
 * production sweeps so far).  It must not call back into the library.      */
typedef void (*mc_progress_fn)(void *user, int32_t iteration, double flatness, int64_t sweeps);

typedef struct {
    int32_t L, walkers;
    int32_t eq_sweeps;    /* unrecorded sweeps at the start of each iteration   */
    int32_t rec_sweeps;   /* recorded sweeps per iteration                      */
    int32_t max_iter;     /* weight iterations allowed                          */
    int32_t prod_sweeps;  /* production sweeps at the final weights             */
    double flat;          /* flatness criterion min/max over reachable levels   */
    uint64_t seed;
    int32_t start;        /* MC_MUCA_HOT or MC_MUCA_STRATIFIED walker starts    */
    int32_t rec_max;      /* recorded sweeps double, up to this, after every
                             iteration whose histogram reached every window
                             level (<= rec_sweeps: fixed length)              */
    int32_t eq_scale;     /* unrecorded sweeps per iteration: eq_sweeps +
                             eq_scale * (recorded sweeps of that iteration)   */
    int32_t prep_sweeps;  /* > 0: after the start, walker group g of 16 runs
                             this many canonical Metropolis sweeps (replica id
                             = walker, sweeps 0..) at the initial weights'
                             inverse temperature -d lnW/dE (central difference
                             around level round((g + 1/2) N / 32), at least 0;
                             flat weights: 0); energies are then recomputed and
                             walkers above the window flipped (E -> -E);
                             needs walkers <= 16 * 65535                      */
    int32_t rec_rule;     /* 0: double the recorded sweeps after every
                             iteration that reached every window level; 1:
                             only when such an iteration's flatness did not
                             improve on the previous iteration's             */
    mc_progress_fn progress;  /* or NULL                                       */
    void *progress_user;
} mc_muca_args;

typedef struct {
    int32_t iterations, converged;
    int64_t sweeps_per_walker;  /* eq + rec sweeps of all iterations          */
    double min_over_max;        /* flatness of the last iteration             */
} mc_muca_stats;

/* The whole method: walker start, iterations of eq_sweeps + eq_scale R
 * unrecorded and R recorded sweeps (the paper lets walkers thermalise to the
 * updated weights before each iteration's statistics; R = rec_sweeps, doubled
 * up to rec_max after every iteration that
 * visited every window level but k = 1; the paper leaves iteration lengths
 * open) with the plain recursion ln W -= ln H (H > 0; then ln W at E = 0 set
 * to 0) until
 * min/max of H over all window levels but k = 1 reaches flat, then
 * prod_sweeps at fixed weights; ln g = ln H_prod - ln W (-inf where empty).
 * lnW_init: host [N/2 + 1] initial ln W, or NULL for flat weights.
 * Outputs on the host: lnW_out, H_out (production), lng_out [N/2 + 1];
 * flat_out [max_iter] (may be NULL); stats.  spins: device int8
 * [walkers][L^2] walker lattices on return.  Returns MC_E_NOTCONV (outputs
 * still written) if max_iter iterations did not give a flat histogram.
 * Blocking.                                                                 */
int mc_muca_run(mc_ctx *ctx, const mc_muca_args *args, const double *lnW_init, int8_t *spins, double *lnW_out,
                int64_t *H_out, double *lng_out, double *flat_out, mc_muca_stats *stats, void *ws, size_t ws_bytes,
                void *stream);

/* One step of the weight recursion of mc_muca_run (Eq. weight_modification),
 * for callers that run their own iterations with mc_muca_sweeps:
 * ln W'(k) = ln W(k) - ln H(k) where H(k) > 0 (host FP64 libm log), then
 * ln W' shifted so that ln W'(N/2) = 0 (E = 0).  lnW, lnW_out: host double
 * [N/2 + 1] (may be the same array); H: host int64 [N/2 + 1], the histogram
 * of the iteration.  flat_out (or NULL): min/max of H over the window levels
 * but k = 1, 0 when H is empty, the flatness mc_muca_run tests.  Host only.
 * Errors: MC_E_SHAPE for an unsupported L; MC_E_INVAL for a NULL pointer;
 * MC_E_RANGE for a non-finite ln W or a negative count.                    */
int mc_muca_update(mc_ctx *ctx, int32_t L, const double *lnW, const int64_t *H, double *lnW_out,
                   double *flat_out);

/* ------------------------------------------------------------------------
 * Wang-Landau sampling in energy windows (Sec. "Wang-Landau update": g(E)
 * starts at 1 and is multiplied by f at every visit, a move E -> E' is
 * accepted with min[1, g(E)/g(E')], f -> sqrt(f) once the histogram is flat,
 * i.e. its minimum is at least `flat` (0.8) times its mean; the windowed
 * parallel form of the same section and of Sec. "Multicanonical
 * simulations": the levels are split into overlapping windows sampled by
 * separate walkers, a move out of the window is rejected and the current
 * level counted again, the walkers' estimates are averaged before f is
 * reduced, and the pieces are matched on the overlaps).
 * Levels k = (E + 2N)/4 of the 2D L x L torus (J = 1), k = 0..N/2 (E <= 0;
 * level 1 has no states).  Window i holds [lo[i], hi[i]] (at least 2 and at
 * most 192 levels) and walkers 64-multiple walkers, walker w = i walkers + m.
 * Every walker keeps its own estimate G_w(k) of ln g in units of 2^-32
 * (int64; ln f = 2^-s is added exactly) and its own visit counts; the
 * acceptance exp(-(G(k') - G(k)) 2^-32) is a fixed-order product of FP64
 * factors exp(-n), exp(-a 2^-8), exp(-b 2^-16), exp(-c 2^-24), exp(-d 2^-32)
 * (host libm exp) for the integer and the four fraction bytes of the
 * difference, tested as r32 < ceil(p 2^32) (r32 as for the multicanonical
 * walkers: word (i mod 4) of Philox(MUCA, i div 4, w, sweep)).
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t L;                 /* as for the multicanonical walkers         */
    int32_t nwin;
    const int32_t *lo, *hi;    /* host [nwin]: window levels; lo[0] = 0,
                                  hi[nwin-1] = N/2, each window overlapping
                                  the next on a level with states           */
    int32_t walkers;           /* per window, a multiple of 64              */
    int32_t check_sweeps;      /* sweeps between flatness checks (>= 1)     */
    double flat;               /* min >= flat * mean (the paper: 0.8)       */
    double lnf_final;          /* a window stops once ln f < lnf_final
                                  (in [2^-32, 1]; the paper names 1e-8)     */
    int64_t max_sweeps;        /* bound on the sweeps of the whole run      */
    int32_t max_pass;          /* passes allowed to reach the windows       */
    uint64_t seed;
    /* optional, called on the host after every check (NULL: none)          */
    void (*progress)(void *user, int32_t windows_done, int32_t min_stage, int64_t sweeps);
    void *progress_user;
} mc_wl_args;

typedef struct {
    int32_t stages;            /* halvings of ln f done (ln f = 2^-stages)  */
    int32_t converged;         /* ln f went below lnf_final                 */
    int64_t sweeps;            /* sweeps the window's walkers ran           */
} mc_wl_window_stats;

/* Device workspace of mc_wl_run, mc_win_drive and mc_wl_sweeps for these
 * windows and walkers (0 for invalid arguments).                            */
size_t mc_wl_workspace_bytes(const mc_wl_args *args);

/* Walkers into their windows: every walker of window i starts from the
 * ground state (all +1) and runs typewriter passes in which a flip is taken
 * iff the walker is below lo[i], the flip raises its level, and the top bit
 * of word (i mod 4) of Philox(WINDOW = 10, site div 4, w, pass) is set; it
 * stops at the first level >= lo[i] (a flip moves at most two levels, so it
 * stops inside).  spins: device int8 [nwin walkers][N]; E: device int64
 * [nwin walkers].  MC_E_NOTCONV if a walker is not inside after max_pass
 * passes.  Blocking.                                                         */
int mc_win_drive(mc_ctx *ctx, int32_t L, int32_t nwin, const int32_t *lo, const int32_t *hi, int32_t walkers,
                 uint64_t seed, int32_t max_pass, int8_t *spins, int64_t *E, void *ws, size_t ws_bytes, void *stream);

/* nsweeps Wang-Landau sweeps of the walkers of every window i with
 * active[i] (host uint8 [nwin]); inc: host int64 [nwin], ln f of each window
 * in units of 2^-32 (0..2^32; 0 gives fixed weights, a multicanonical sweep
 * with ln W = -G 2^-32 inside the window).  G: device int64 [nwin walkers]
 * [wmax], H: device uint32 [nwin walkers][wmax], wmax = the widest window;
 * level k of walker w at [w][k - lo].  After the sweeps each swept walker's
 * estimate is shifted to a minimum of 0 over its window's levels with states
 * and flags[w] (device int32) is 1 iff its counts are flat.  Blocking for the
 * host arrays, stream-ordered for the device work.                          */
int mc_wl_sweeps(mc_ctx *ctx, int32_t L, int32_t nwin, const int32_t *lo, const int32_t *hi, int32_t walkers,
                 const int64_t *inc, const uint8_t *active, double flat, uint64_t seed, uint64_t sweep0,
                 int32_t nsweeps, int8_t *spins, int64_t *E, int64_t *G, uint32_t *H, int32_t *flags, void *ws,
                 size_t ws_bytes, void *stream);

/* The whole method: mc_win_drive, estimates and counts cleared, then rounds
 * of check_sweeps sweeps of the windows still running (stage s: ln f = 2^-s,
 * f = e at s = 0).  After a round, a window whose walkers all have flat
 * counts averages their estimates (floor of the integer mean per level,
 * shifted to a minimum of 0 over the levels with states, given to every
 * walker), clears the counts and halves ln f; it stops once ln f <
 * lnf_final.  The run ends when every window has stopped or after
 * max_sweeps (windows still running then report their current average and
 * MC_E_NOTCONV, with every output written).  MC_E_RANGE if a stage would run
 * so long that a walker's visits of one level could exceed 2^32 - 1 (N times
 * the stage's sweeps).  Outputs on the host: pieces
 * [nwin][wmax] (window i's ln g at [i][k - lo[i]], in units of 1), lng
 * [N/2 + 1] (the matched ln g: window i + 1 shifted by the mean difference to
 * window i, as matched, over their overlap levels with states; level k taken
 * from window i up to the middle level of each overlap; ln g(0) = ln 2, the
 * two ground states; ln g(1) = -inf), stats [nwin].  Blocking.             */
int mc_wl_run(mc_ctx *ctx, const mc_wl_args *args, int8_t *spins, int64_t *E, double *pieces, double *lng,
              mc_wl_window_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* The multicanonical recursion in the same windows (Sec. "Multicanonical
 * simulations": windows simulated separately from flat weights, the
 * count-again rule, Eq. weight_modification, pieces matched on overlaps).
 * Walkers are driven into their windows (mc_win_drive); each window's
 * weights ln W = -G 2^-32 (G integer, start 0) are held by all its walkers.
 * An iteration of every window still running: eq_sweeps unrecorded and
 * rec_sweeps recorded sweeps (mc_wl_sweeps with ln f = 0), the walkers'
 * counts pooled into H; the window stops once min H >= flat * max H over its
 * levels with states (its piece: ln g = ln H + G 2^-32, 0 where H = 0);
 * otherwise G += floor(ln H 2^32 + 1/2) where H > 0 (host libm log), shifted
 * to a minimum of 0 over the levels with states.  Windows not flat after
 * max_iter iterations give -ln W = G 2^-32 of their last weights, and the call
 * returns MC_E_NOTCONV with every output written.  pieces, lng, windows and
 * matching as for mc_wl_run; stats [nwin].  Blocking.                       */
typedef struct {
    int32_t L, nwin;
    const int32_t *lo, *hi;    /* host [nwin], as for mc_wl_run             */
    int32_t walkers;           /* per window, a multiple of 64              */
    int32_t eq_sweeps, rec_sweeps, max_iter;
    double flat;               /* min/max of the pooled counts (0.8)        */
    int32_t max_pass;
    uint64_t seed;
    void (*progress)(void *user, int32_t windows_done, int32_t iteration, int64_t sweeps);
    void *progress_user;
} mc_muca_win_args;

typedef struct { int32_t iterations, converged; } mc_muca_win_stats;

size_t mc_muca_windows_workspace_bytes(const mc_muca_win_args *args);
int mc_muca_windows_run(mc_ctx *ctx, const mc_muca_win_args *args, int8_t *spins, int64_t *E, double *pieces,
                        double *lng, mc_muca_win_stats *stats, void *ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * A small MLP that predicts initial multicanonical weights from what the
 * method itself produced at smaller L: x = (E/N + 1, 32/L - 1) -> tanh(64)
 * -> tanh(64) -> y, FP32, 4417 parameters flattened as W1 [64][2], b1 [64],
 * W2 [64][64], b2 [64], W3 [1][64], b3 [1]; loss = mean squared error;
 * full-batch Adam.  The initial ln W of an L x L lattice is -N y(E).
 * X: device float [n][2]; Y: device float [n]; params: device float [4417]. */
int32_t mc_mlp_param_count(void);
size_t mc_mlp_workspace_bytes(int32_t n);

/* Xavier-uniform weights, zero biases: parameter idx draws word (idx mod 4)
 * of Philox(ctr = (idx / 4, 0, 0, TAG_MLP_INIT << 24)); w = (2u - 1)
 * sqrt(6 / (fan_in + fan_out)), u = (r >> 8) 2^-24, in FP64 rounded to FP32.
 * Stream-ordered.                                                          */
int mc_mlp_init(mc_ctx *ctx, float *params, uint64_t seed, void *stream);

/* Gradient of the loss (device float [4417]) and the loss (device float [1])
 * at params, summed over 32-sample chunks in chunk order.  Stream-ordered.  */
int mc_mlp_grad(mc_ctx *ctx, const float *params, const float *X, const float *Y, int32_t n, float *grad, float *loss,
                void *ws, size_t ws_bytes, void *stream);

typedef struct {
    int32_t epochs;
    float lr, beta1, beta2, eps;  /* Adam; 1e-3, 0.9, 0.999, 1e-8 as usual */
} mc_mlp_args;

/* epochs full-batch Adam steps on params (in/out); loss_log: device float
 * [epochs], the loss before each step.  Epochs run as a captured hipGraph of
 * up to 500 epochs, replayed; blocking.                                    */
int mc_mlp_train(mc_ctx *ctx, const mc_mlp_args *args, const float *X, const float *Y, int32_t n, float *params,
                 float *loss_log, void *ws, size_t ws_bytes, void *stream);

/* Y = network(X) for n samples.  Stream-ordered.                           */
int mc_mlp_predict(mc_ctx *ctx, const float *params, const float *X, int32_t n, float *Y, void *stream);

/* Training set from converged multicanonical weights (Sec. "Multicanonical
 * simulations": the weights the recursion of Eq. weight_modification
 * produced at smaller L): for each lattice size Ls[i] (even, >= 4) and every
 * level k = 0 .. N/2 of the window E = 4k - 2N in [-2N, 0] except the empty
 * level k = 1, one sample x = (E/N + 1, 32/L - 1), y = -(lnW[k] - lnW[N/2]) / N
 * - b(k), b(k) = h(k / 2N) - h(1/4) with h(x) = -x ln x - (1 - x) ln(1 - x)
 * the entropy of independent flipped spins (it carries the ground-state
 * singularity of g(E), so the network fits a smooth remainder), computed in
 * FP64 and rounded to FP32.  lnW: host array of nL pointers to
 * N/2 + 1 doubles each (finite except at k = 1).  X: host float [cap][2],
 * Y: host float [cap]; *n_out = samples written.  MC_E_RANGE if they do not
 * fit in cap or a weight is not finite.  Host-only call.                   */
int mc_mlp_training_set(mc_ctx *ctx, int32_t nL, const int32_t *Ls, const double *const *lnW, float *X, float *Y,
                        int32_t cap, int32_t *n_out);

/* Initial log-weights of an L x L lattice from a trained network: the inputs
 * of every window level are formed on the device, the network runs as in
 * mc_mlp_predict, and lnW_out[k] = -N (y(k) + b(k)) (FP64, host array of N/2 + 1),
 * shifted so that lnW_out[N/2] = 0.  If any prediction is not finite the
 * plain method's flat start is returned instead (all zeros) and
 * *used_fallback = 1, else 0.  ws: device scratch of
 * mc_mlp_lnw_workspace_bytes(L).  Blocking.                                */
size_t mc_mlp_lnw_workspace_bytes(int32_t L);
int mc_mlp_lnw_init(mc_ctx *ctx, const float *params, int32_t L, double *lnW_out, int32_t *used_fallback, void *ws,
                    size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* MCSPIN_H */
