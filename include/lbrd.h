/*
 * lbrd.h — C ABI of the MI355X (gfx950) reacting-species D2Q9 lattice
 * Boltzmann library.
 *
 * The method (Ayodele, Varnik & Raabe, "Lattice Boltzmann study of pattern
 * formation in reaction-diffusion systems", Section II.A, second Eq. "relax";
 * Appendix, Eq. "app1"): for every species s = 1..N and velocity i = 0..8 of
 * the D2Q9 lattice (weights 4/9, 1/9, 1/36, Eq. "Weights"),
 *
 *   f_{i,s}(x + e_i, t + 1) = f_{i,s}(x, t)
 *                             + (w_i rho_s(x,t) - f_{i,s}(x,t)) / tau_s
 *                             + w_i R_s(rho_1..rho_N)(x, t),
 *
 * with rho_s = sum_i f_{i,s}, the zero-velocity equilibrium w_i rho_s
 * (Eq. "equili"), periodic boundaries in x and y (Section II.B, Section IV)
 * and D_s = (tau_s - 1/2) / 3 in lattice units (Section II.A, last sentence).
 *
 * Conventions shared by every entry point:
 *  - Every function returns an int status: LBRD_OK (0) or a negative
 *    LBRD_E* code; lbrd_strerror() names it.  No C++ exception and no abort
 *    crosses this boundary.
 *  - "Device pointer" means memory allocated on the GPU the handle was created
 *    on (e.g. a torch tensor's data_ptr()); "host pointer" means ordinary CPU
 *    memory.  The caller owns every buffer it passes; the library owns only
 *    its opaque host-side handles and never frees caller memory.
 *  - Work is enqueued on the HIP stream given at creation (NULL = the null
 *    stream) and is asynchronous unless a host output is requested, in which
 *    case the call synchronises that stream before returning.
 *  - A handle must be used by one host thread at a time.
 *  - Density fields are dense row-major arrays rho[s][y][x] (x fastest);
 *    population fields are dense f[s][i][y][x] in the velocity numbering
 *    e_0 = (0,0), e_1..e_4 = (1,0), (0,1), (-1,0), (0,-1),
 *    e_5..e_8 = (1,1), (-1,1), (-1,-1), (1,-1).
 *  - The state at time t is the post-streaming, pre-collision f_{i,s}(x, t);
 *    t counts the steps taken since the last init / set_populations.
 */
#ifndef LBRD_H
#define LBRD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBRD_MAX_SPECIES 4

/* Status codes. */
#define LBRD_OK 0
#define LBRD_EINVAL (-1)      /* bad argument (range, enum, null pointer, tau <= 1/2) */
#define LBRD_ENOMEM (-2)      /* workspace or arena too small                        */
#define LBRD_EDEVICE (-3)     /* a HIP runtime call failed                            */
#define LBRD_ENONFINITE (-4)  /* a reduction produced NaN or Inf                      */
#define LBRD_ESTATE (-5)      /* call out of order (e.g. step before init)           */
#define LBRD_ENOTFOUND (-6)   /* unknown request ticket                               */
#define LBRD_ETIMEOUT (-7)    /* wait timed out                                       */

/* Population storage forms. */
#define LBRD_F64 0            /* double populations, double arithmetic               */
#define LBRD_F32 1            /* float populations, float arithmetic                 */
#define LBRD_F16_SHIFTED 2    /* binary16 of f - c_i rho_ref_s, float arithmetic     */
#define LBRD_BF16_SHIFTED 3   /* bfloat16 of f - c_i rho_ref_s, float arithmetic     */
                              /* (c_i = w_i, or c_i(u) with an advection velocity)   */

/* Reaction terms R_s. */
#define LBRD_REACT_NONE 0        /* R_s = 0                                           */
#define LBRD_REACT_LINEAR 1      /* R_s = sum_j K[s][j] rho_j + c_s (Section II.B:    */
                                 /* the decay R_A = -kappa rho_A, Eq. "reac_diff3")   */
#define LBRD_REACT_GRAY_SCOTT 2  /* N = 2, u = species 0, v = species 1:              */
                                 /* R_u = -u v^2 + F (1 - u), R_v = u v^2 - (F + k) v */
                                 /* (Section III, Eqs. "reac_diff10", "reac_diff11"   */
                                 /* with A_0 = k_1 = 1, F = k_f, k = k_2)             */

/* Element types of density / population arrays crossing the boundary. */
#define LBRD_DTYPE_F64 0
#define LBRD_DTYPE_F32 1

typedef struct lbrd_config {
    int32_t nspecies;     /* N, 1..LBRD_MAX_SPECIES (2 for GRAY_SCOTT)               */
    int32_t nx, ny;       /* periodic lattice size, each >= 1                          */
    int32_t storage;      /* LBRD_F64 / LBRD_F32 / LBRD_F16_SHIFTED / LBRD_BF16_SHIFTED */
    int32_t reaction;     /* LBRD_REACT_*                                              */
    int32_t reserved;     /* must be 0                                                 */
    double tau[LBRD_MAX_SPECIES];      /* relaxation times, each > 1/2                 */
    double rho_ref[LBRD_MAX_SPECIES];  /* storage shift (16-bit forms only)            */
    double K[LBRD_MAX_SPECIES * LBRD_MAX_SPECIES]; /* LINEAR: K[s*N + j]              */
    double c[LBRD_MAX_SPECIES];        /* LINEAR: constant source                      */
    double F, k;                       /* GRAY_SCOTT: feed and kill rates              */
    double u[2];                       /* advection velocity (lattice units) of the    */
                                       /* equilibrium, the same for every species:     */
                                       /* f^eq_i = c_i rho with the low-Mach Maxwellian */
                                       /* c_i = w_i [1 + 3 e_i.u + 9/2 (e_i.u)^2       */
                                       /*            - 3/2 u.u] (Section II.A, Eq.     */
                                       /* "Maxwellian", c_s^2 = 1/3); (0, 0) is the    */
                                       /* paper's pure reaction-diffusion.  Non-zero u */
                                       /* needs u.u < 1/3 and GRAY_SCOTT, or N = 1 with */
                                       /* LINEAR or NONE; otherwise LBRD_EINVAL.  The  */
                                       /* source term keeps w_i R_s.                   */
    double shear[2];                   /* prescribed shear flow added to u: the site   */
                                       /* (x, y) sees u_x = u[0] + A sin(2 pi m y / ny) */
                                       /* and u_y = u[1], with A = shear[0] and m =     */
                                       /* shear[1] a whole number >= 1 of periods over */
                                       /* the lattice; (0, 0) = no shear.  A shear     */
                                       /* needs (|u[0]| + |A|)^2 + u[1]^2 < 1/3, the   */
                                       /* reactions allowed with u, FP64 or FP32       */
                                       /* storage and a single solver (batches and the */
                                       /* server refuse it); otherwise LBRD_EINVAL.    */
} lbrd_config;

/* Kernel launch shape.
 *  vec: sites per lane along x (2 for F64; 2 or 4 for F32; 4 or 8 for the
 *       16-bit forms).  Single solvers only.
 *  lanes_x: lanes per row segment, a power of two 1..64 (0 = choose from nx).
 *       Single solvers only.
 *  waves: waves (64 lanes) per workgroup, 1..16 except 3.  One-step
 *       launches use min(waves, 4); multi-step launches use all of them.
 *  nontemporal: 1 = streaming (non-temporal) accesses: loads and stores of
 *       one-step launches, the result stores of multi-step launches (FP64
 *       marching strips store cached either way).
 *  graph_steps: steps per captured HIP graph (0 = plain launches; else even;
 *       batches with T steps per launch: a multiple of 2T).  Single solvers
 *       default to 32 for one-step launches on lattices of at most 2^18
 *       sites, else 0.
 *  blocks_per_cu: persistent workgroups per compute unit.  Batches: 1..32
 *       (one-step) or 0..32 (multi-step, 0 = one workgroup per tile).
 *       Single solvers: 0 = one tile per wave / workgroup, else 1..64 looping
 *       over tiles.
 *  plain_order: single solvers; 0 = consecutive tiles on the same XCD, 1 = the
 *       hardware's round-robin order.
 *  fused_steps: 1 = one step per launch; T = 2 .. 8 (2 .. 12 on marching
 *       strips, see march_rows, except FP64) =
 *       T steps per launch on tile_cols x tile_rows tiles staged in LDS
 *       (temporal blocking; a remainder of 2 .. T-1 steps runs as one shorter
 *       launch on the same tiles, a single remaining step as a one-step
 *       launch).  Results are bitwise identical for every setting.  Multi-step
 *       launches need each plane (one population of one species, pitch x ny
 *       values plus padding) below 4 GiB and a row below 16 MiB; a buffer of
 *       4 GiB or more is then addressed plane by plane.  Otherwise only
 *       fused_steps = 1 is valid (64-bit offsets).
 *  tile_rows, tile_cols: multi-step tile, rows 1..64 and columns 32, 64 or 128
 *       (0 = 64; 128 only for buffers below 4 GiB).
 *       With h = T-1 and w = tile_cols + 2h, the LDS region of tile_rows + 2h
 *       rows of 9 N w populations (each row padded by fewer than 256 bytes)
 *       must fit in 160 KB.  Ignored when fused_steps = 1.
 *  tile_strip: order of the tiles of a multi-step launch (single solvers;
 *       batches set it to 0): 0 = row-major over the lattice, S = 1..65536 =
 *       strips of S tile columns, row-major inside each strip, so that the
 *       tiles above and below one in flight are in flight too and their
 *       shared halo rows are read once from L2.  lbrd_create sets half the
 *       workgroups that one XCD holds at once (from the LDS of the default
 *       shape) when the lattice is wider than twice that many tiles (16-bit
 *       forms: at least twice), else 0.
 *       Results are bitwise identical for every order.
 *  march_rows: single solvers with fused_steps = T >= 2: 0 = the LDS tiles
 *       above; R = 1..65536 = marching wave strips
 *       instead: each wave (min(waves, 4) waves per workgroup) owns 64
 *       columns, 2(T-1) of them recomputed halo, and marches down segments of
 *       R rows carrying the launch's intermediate rows in registers (no LDS,
 *       no barriers; only the x-halo is recomputed).  tile_cols, tile_rows and
 *       tile_strip are then ignored.  Ignored when fused_steps = 1 (one-step
 *       launches).  On buffers of 4 GiB or more (each plane addressed by a
 *       resource of its own) only Gray-Scott and one or two linear species
 *       with T = 8, or 10 outside FP64, are accepted (else LBRD_EINVAL); a
 *       shorter remainder of a run there runs on the strips of T.
 *       lbrd_create chooses it from measurements (marching strips
 *       where they measured faster: most forms beyond the Infinity Cache,
 *       most inside it from 1024^2 sites), with R sized so that the
 *       strips' segments make a fixed number of waves per SIMD (one round of
 *       the launch for the kernels with one wave per SIMD).  Up to 12 steps
 *       a launch in FP32 and the 16-bit forms; FP64 up to 8.
 *       Batches (FP32 Gray-Scott sets and serving mixes): R > 0 with T >= 2
 *       runs their multi-step launches on marching strips too (waves 1, 2
 *       or 4; blocks_per_cu 0 = one wave per strip segment, else a
 *       persistent grid of that many workgroups per CU); lbrd_batch_create
 *       chooses them when the batch's buffers exceed the Infinity Cache.
 *       Results are bitwise identical either way. */
typedef struct lbrd_tuning {
    int32_t vec;
    int32_t lanes_x;
    int32_t waves;
    int32_t nontemporal;
    int32_t graph_steps;
    int32_t blocks_per_cu;
    int32_t plain_order;
    int32_t fused_steps;
    int32_t tile_rows;
    int32_t tile_cols;
    int32_t tile_strip;
    int32_t march_rows;
} lbrd_tuning;

const char *lbrd_strerror(int status);

/* Library version string; never NULL. */
const char *lbrd_version(void);

/* Text of the last LBRD_EDEVICE failure on the calling thread ("" if none). */
const char *lbrd_last_error(void);

/* ---------------------------------------------------------------- solver -- */

typedef struct lbrd_solver lbrd_solver;

/* Check a configuration without touching the GPU.  LBRD_EINVAL names no field;
 * every rule is listed on lbrd_config. */
int lbrd_validate(const lbrd_config *cfg);

/* Bytes of device workspace a solver of this configuration needs (two
 * population buffers plus reduction scratch).  Host-only. */
int lbrd_workspace_size(const lbrd_config *cfg, size_t *bytes);

/* Create a solver on the current HIP device.  workspace: device pointer to at
 * least lbrd_workspace_size() bytes, 256-byte aligned, owned by the caller and
 * kept alive until lbrd_destroy.  stream: hipStream_t or NULL.
 * Errors: EINVAL (config, null out, misaligned workspace), ENOMEM (too
 * small), EDEVICE. */
int lbrd_create(const lbrd_config *cfg, void *workspace, size_t bytes, void *stream, lbrd_solver **out);

/* Release the handle (NULL is accepted).  Does not free the workspace. */
int lbrd_destroy(lbrd_solver *h);

/* Initial state f_{i,s}(x, 0) = w_i rho0_s(x) (Eq. "equili"; the paper does
 * not state the initial populations), t = 0.  rho0: dense [N][ny][nx] of
 * dtype LBRD_DTYPE_F64/F32, a device pointer if on_device != 0, else a host
 * pointer (copied before return). */
int lbrd_init(lbrd_solver *h, const void *rho0, int dtype, int on_device);

/* Set / read the full state as dense f[N][9][ny][nx] (the numbering above).
 * set: t = 0 afterwards; host or device source.  get: device destination. */
int lbrd_set_populations(lbrd_solver *h, const void *f, int dtype, int on_device);
int lbrd_get_populations(lbrd_solver *h, void *f_out, int dtype);

/* Advance nsteps >= 0 time steps, asynchronously on the stream.
 * ESTATE before init. */
int lbrd_step(lbrd_solver *h, int64_t nsteps);

/* Densities rho_s(x, t) = sum_i f_{i,s}(x, t) (Section II.A, after Eq.
 * "relax").  rho_out: device [N][ny][nx] of dtype, or NULL.  mass_out: host
 * double[N] receiving M_s = sum_x rho_s(x, t) accumulated in FP64 on the GPU
 * with a fixed reduction order, or NULL; if given, the call synchronises and
 * returns ENONFINITE when any M_s is NaN or Inf. */
int lbrd_moments(lbrd_solver *h, void *rho_out, int dtype, double *mass_out);

/* Relative L2 error per species E_s = sqrt(sum_x (ref - rho)^2 / sum_x ref^2)
 * (Section II.B, the definition of E_rho), FP64 on the GPU.  ref: device
 * [N][ny][nx] of dtype; err_out: host double[N].  Synchronises. */
int lbrd_rel_l2(lbrd_solver *h, const void *ref, int dtype, double *err_out);

int lbrd_time(const lbrd_solver *h, int64_t *t);

/* Power spectrum of one species' density fluctuation, for the Fourier
 * diagnostic of Section III.D (Eq. "reac_diff35": the excited wave numbers
 * (n_x, n_y) of a pattern): P[k_y][k_x] = |sum_{x,y} (rho_s(x,y) - mean)
 * exp(-2 pi i (k_x x / nx + k_y y / ny))|^2, computed in FP64 on the GPU by a
 * row transform followed by a column transform (a mixed-radix FFT in LDS
 * for lines of at most 5120 points whose length factors into 2, 3 and 5;
 * direct sums for other lines).
 * out: device double [ny][nx].  work: device scratch of
 * lbrd_spectrum_work_size() bytes.  Asynchronous. */
int lbrd_spectrum_work_size(int nx, int ny, size_t *bytes);
int lbrd_spectrum(lbrd_solver *h, int species, void *out, void *work, size_t work_bytes);

/* lbrd_spectrum for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and the same result, with the scratch taken from a fixed
 * array of LBRD_SPECTRUM_STATIC_BYTES that the library holds in each GPU's
 * memory from the first call on that GPU until the process ends; the call
 * itself allocates nothing (no hipMalloc, no library allocation).  Lattices
 * of more than LBRD_SPECTRUM_STATIC_MAX_SITES sites: LBRD_ENOMEM.  Every call
 * on one GPU shares that GPU's array, which keeps the last call's contents
 * (nothing in it needs to start at zero): calls that overlap on one GPU (on
 * several streams or threads) race and must be serialised by the caller.
 * out: device double [ny][nx].  Asynchronous on the solver's stream.
 * Errors: EINVAL (null, bad species, misaligned out), ENOMEM (lattice too
 * large), ESTATE (not initialised), EDEVICE. */
#define LBRD_SPECTRUM_STATIC_MAX_SITES (1 << 20)
#define LBRD_SPECTRUM_STATIC_BYTES ((size_t)LBRD_SPECTRUM_STATIC_MAX_SITES * 24 + 256)
int lbrd_spectrum_static(lbrd_solver *h, int species, void *out);

/* Launch shape in use / override it (validated against the storage form). */
int lbrd_get_tuning(const lbrd_solver *h, lbrd_tuning *out);
int lbrd_set_tuning(lbrd_solver *h, const lbrd_tuning *t);

/* Time every valid launch shape on this solver's buffers for about `steps`
 * steps each (whole launches, at least about 1 ms, compared per step; each
 * multi-step shape with the tile_strip lbrd_create would give it, plain
 * launches), then re-time with runs of about 10 ms the six fastest, the shape
 * in use and the three fastest multi-step shapes with the other XCD order and
 * with the other strip choice (strips or row-major), keep the fastest of
 * those, and finally keep or drop captured graphs of 32 steps on it, whichever
 * is faster; writes the choice to *chosen if not NULL.  The shapes are timed
 * on the solver's own state when it is initialised, else on a scrambled field
 * of densities in [0.5, 1); either way the state is overwritten: the solver
 * must be (re)initialised afterwards (ESTATE until then).  cache_path: text
 * file of earlier results keyed by (device, storage, reaction, N, nx, ny),
 * read and appended; NULL disables the cache. */
int lbrd_autotune(lbrd_solver *h, int steps, const char *cache_path, lbrd_tuning *chosen);

/* Device time in milliseconds of `nsteps` steps measured with HIP events on
 * the solver's stream (the state advances).  Synchronises. */
int lbrd_time_steps(lbrd_solver *h, int64_t nsteps, double *ms);

/* --------------------------------------------------------------- batched -- */

/* Many independent lattices (any sizes, parameters, storage forms and
 * reactions) advanced together: every step is one persistent launch over the
 * wave tiles of all instances, and lbrd_batch_step replays HIP graphs of
 * such launches. */
typedef struct lbrd_batch lbrd_batch;

int lbrd_batch_workspace_size(const lbrd_config *cfgs, int count, size_t *bytes);
int lbrd_batch_create(const lbrd_config *cfgs, int count, void *workspace, size_t bytes, void *stream,
                      lbrd_batch **out);
int lbrd_batch_destroy(lbrd_batch *b);
/* Same contracts as lbrd_init / lbrd_moments / lbrd_get_populations for
 * instance idx (0..count-1). */
int lbrd_batch_init(lbrd_batch *b, int idx, const void *rho0, int dtype, int on_device);
int lbrd_batch_moments(lbrd_batch *b, int idx, void *rho_out, int dtype, double *mass_out);
int lbrd_batch_get_populations(lbrd_batch *b, int idx, void *f_out, int dtype);
/* Advance every instance by nsteps (ESTATE unless all are initialised). */
int lbrd_batch_step(lbrd_batch *b, int64_t nsteps);
/* Advance instance i by nsteps[i] >= 0 (count entries, host array); all
 * instances still advance together, each stopping at its own count. */
int lbrd_batch_advance(lbrd_batch *b, const int64_t *nsteps);
/* Steps taken by instance idx since its init. */
int lbrd_batch_time(const lbrd_batch *b, int idx, int64_t *t);
/* Same contract as lbrd_rel_l2 for instance idx. */
int lbrd_batch_rel_l2(lbrd_batch *b, int idx, const void *ref, int dtype, double *err_out);
/* Same contract as lbrd_spectrum for instance idx. */
int lbrd_batch_spectrum(lbrd_batch *b, int idx, int species, void *out, void *work, size_t work_bytes);
/* Launch shape of a batch.  Batches whose instances are all Gray-Scott FP32,
 * or all from the serving mix (one-species linear or Gray-Scott without a
 * velocity, in FP32 / F16 / BF16 storage, each buffer below 4 GiB), take
 * fused_steps = T in 2..8 on tile_cols x tile_rows tiles, tile_cols 32 or 64,
 * or with march_rows > 0 on marching strips, T in 2..12 (default 5 steps on 32 x 10
 * tiles, 8 waves, while the buffers fit in the 256 MB Infinity Cache;
 * beyond it 9 steps on marching strips of 128 rows, 4 waves; blocks_per_cu 0
 * = one workgroup per tile or strip segments, graph_steps the multiple of 2T
 * nearest 32):
 * launch j advances each instance by min(T, its steps left in the chunk), and
 * graph_steps must be a multiple of 2T.  Other batches use persistent
 * one-step launches: fused_steps = 1, waves 1/2/4, blocks_per_cu 1..32,
 * nontemporal, even graph_steps (vec and lanes_x are chosen per instance).
 * Results are bitwise identical for every shape. */
int lbrd_batch_get_tuning(const lbrd_batch *b, lbrd_tuning *out);
int lbrd_batch_set_tuning(lbrd_batch *b, const lbrd_tuning *t);
/* Time the launch-shape candidates (one-step persistent shapes and, where
 * allowed, multi-step shapes) and keep the fastest (state is overwritten;
 * re-initialise afterwards). */
int lbrd_batch_autotune(lbrd_batch *b, int steps, lbrd_tuning *chosen);
int lbrd_batch_time_steps(lbrd_batch *b, int64_t nsteps, double *ms);

/* --------------------------------------------------------------- serving -- */

/* Continuous-batching solve server.  Requests (a config, a host initial
 * density, a step count) are queued on submit; a worker thread admits them
 * into a caller-owned device arena as footprint allows, advances all resident
 * requests together in chunks of persistent batched launches, retires
 * finished ones (densities and FP64 masses copied to host) and frees their
 * memory for queued requests. */
typedef struct lbrd_server lbrd_server;

typedef struct lbrd_server_config {
    int32_t chunk_steps;   /* steps per scheduling round (>= 1)                   */
    int32_t max_slots;     /* most requests resident at once (>= 1)               */
    int32_t max_queue;     /* most requests waiting (>= 1); submit returns ENOMEM beyond */
    int32_t reserved;
} lbrd_server_config;

typedef struct lbrd_request_info {
    int32_t state;         /* 0 queued, 1 resident, 2 done, 3 rejected             */
    int32_t reserved;
    double submit_s;       /* seconds on the server clock                          */
    double admit_s;
    double done_s;         /* result ready on the host                             */
    int64_t steps;
    int64_t footprint;     /* device bytes while resident                          */
} lbrd_request_info;

typedef struct lbrd_server_stats {
    int64_t submitted, admitted, completed, rejected;
    int64_t resident, queued;
    int64_t species_site_steps;   /* sum over completed requests of N * sites * steps */
    int64_t arena_bytes, arena_peak_used;
    double busy_s;                /* wall time with at least one resident request   */
    double clock_s;               /* server clock now                               */
    int64_t arena_used;           /* arena bytes held by resident requests now      */
    double arena_used_byte_s;     /* integral of arena_used over the server clock   */
                                  /* (byte-seconds): the mean occupancy over a      */
                                  /* period is its change / (period x arena_bytes)  */
} lbrd_server_stats;

/* arena: device pointer, 256-byte aligned, owned by the caller until destroy. */
int lbrd_server_create(const lbrd_server_config *sc, void *arena, size_t bytes, void *stream, lbrd_server **out);
/* Stops the worker after finishing resident requests; queued ones are dropped. */
int lbrd_server_destroy(lbrd_server *s);
/* rho0_host: host double [N][ny][nx], copied before return.  A request whose
 * footprint exceeds the whole arena is rejected (ENOMEM, no ticket). */
int lbrd_server_submit(lbrd_server *s, const lbrd_config *cfg, const double *rho0_host, int64_t nsteps,
                       int64_t *ticket);
int lbrd_server_info(lbrd_server *s, int64_t ticket, lbrd_request_info *info);
/* Block until the request is done or timeout_s passes (ETIMEOUT). */
int lbrd_server_wait(lbrd_server *s, int64_t ticket, double timeout_s);
/* Copy a finished request's densities (host double [N][ny][nx], or NULL) and
 * masses (host double[N], or NULL) and forget the ticket. */
int lbrd_server_take(lbrd_server *s, int64_t ticket, double *rho_out, double *mass_out, lbrd_request_info *info);
int lbrd_server_stats_get(lbrd_server *s, lbrd_server_stats *out);
/* Device bytes a request of this configuration occupies while resident. */
int lbrd_server_footprint(const lbrd_config *cfg, size_t *bytes);

#ifdef __cplusplus
}
#endif
#endif /* LBRD_H */
