/*
 * dartray.h -- C ABI of the MI355X (gfx950) ray-march library for the
 * purely ray-tracing dust radiative-transfer method of DART-Ray V2
 * (Natale et al. 2017, arXiv:1709.03802).
 *
 * The method (paper Sect. 2): every radiation source of an adaptive Cartesian
 * grid casts rays along HEALPix directions; each ray-cell crossing attenuates
 * the ray and adds to the crossed cell's radiation-field energy density U and
 * to its angular scattered-luminosity array (Henyey-Greenstein phase function,
 * Eq. 4, and the albedo).  A run is step 1 (lower-limit U, adaptive rays only),
 * the direct-light pass and a number of scattering iterations, each of which
 * re-emits the scattered luminosity left by the previous pass.
 *
 * Conventions for every entry point:
 *  - Return value: DARTRAY_OK or a negative status; the message of the last
 *    failure on the calling thread is returned by dartray_last_error().
 *  - Argument errors are detected before any output is written.
 *  - All device buffers in dartray_fields are owned by the caller; the library
 *    never frees them.  The library owns only what dartray_grid_create
 *    allocates (geometry, tables, work arrays) and frees it in
 *    dartray_grid_destroy.  No entry point other than dartray_grid_create
 *    and dartray_batch_create (three small argument arrays) allocates device
 *    memory.
 *  - Work is queued on the stream given to dartray_grid_create and is
 *    asynchronous, except where a host output is returned (dartray_scatter_iter's
 *    r_k, dartray_debug_ray_cells), in adaptive-ray passes (which read the
 *    source count, and the deposit-log fill between launches) and when a
 *    batch uploads its arguments: those synchronise that stream.
 *  - One grid handle must not be used by two threads or streams at once.
 *  - Precision: ray geometry (positions, directions, exit distances) in
 *    FP64; luminosities, attenuation and deposits in FP32, except that the
 *    adaptive direct and scattering passes carry each ray's luminosity in
 *    FP64 for their significance decisions; energy-density accumulators, the
 *    luminosity tallies, the escape by direction and the convergence ratio
 *    in FP64.
 *  - Non-finite results: every pass records in a device word whether all of
 *    its U and S values are finite; the calls that synchronise anyway (r_k
 *    requested, adaptive passes) and every call with DARTRAY_FLAG_CHECK read
 *    it and return DARTRAY_E_NUMERIC when one was not.
 */
#ifndef DARTRAY_H
#define DARTRAY_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define DARTRAY_OK 0
#define DARTRAY_E_INVALID (-1)      /* bad argument or grid description */
#define DARTRAY_E_OOM (-2)          /* device allocation failed (create only) */
#define DARTRAY_E_DEVICE (-3)       /* HIP runtime error; message has the HIP string */
#define DARTRAY_E_STATE (-4)        /* call out of sequence (e.g. scatter before direct) */
#define DARTRAY_E_UNSUPPORTED (-5)  /* valid request the library does not handle */
#define DARTRAY_E_NUMERIC (-6)      /* non-finite value produced by a pass */

/* pass modes */
#define DARTRAY_MODE_STEP1 0        /* lower-limit U within r_pre (Sect. 2, step 1) */
#define DARTRAY_MODE_DIRECT 1       /* direct light from the emitting cells (step 2) */

/* option flags */
#define DARTRAY_FLAG_COUNTERS 1u    /* fill fields->counters */
#define DARTRAY_FLAG_CHECK 2u       /* synchronise after the pass and return DARTRAY_E_NUMERIC
                                       if it produced a non-finite U or S value */
#define DARTRAY_FLAG_CONTINUE 4u    /* DIRECT adds S_next to S_total instead of replacing it: a
                                       run that continues an earlier one (Sect. 3.3) */
#define DARTRAY_FLAG_2D 8u          /* 2D mode (Sect. 3.6), see below */

/* tally slots, per wavelength, FP64, in luminosity units */
#define DARTRAY_T_EMITTED 0         /* luminosity launched by the pass's sources */
#define DARTRAY_T_ABSORBED 1        /* (1 - albedo) * extinguished, deposited crossings */
#define DARTRAY_T_SCATTERED 2       /* albedo * extinguished, deposited crossings */
#define DARTRAY_T_ESCAPED 3         /* left the root block */
#define DARTRAY_T_CUT 4             /* carried by rays blocked by Eq. 1 / beyond r_pre */
#define DARTRAY_T_SKIPPED 5         /* extinguished at crossings skipped at that wavelength */
#define DARTRAY_N_TALLY 8

/* counter slots (uint64) */
#define DARTRAY_C_CROSSINGS 0       /* traversed crossings (edge and corner grazes, zero
                                       length up to FP64 rounding, excluded) */
#define DARTRAY_C_RAYS 1            /* rays launched from sources */
#define DARTRAY_C_SPLITS 2          /* rays replaced by 4 children (Eq. 2) */
#define DARTRAY_C_CUTS 3            /* rays blocked */
#define DARTRAY_C_ESCAPES 4         /* rays that left the root block */
#define DARTRAY_C_DEPOSITS 5        /* crossing x wavelength deposits */
#define DARTRAY_C_SKIPS 6           /* crossing x wavelength skipped (Sect. 3.2) */
#define DARTRAY_C_MAXSTEP 7         /* rays stopped by max_steps */
#define DARTRAY_C_MERGES 8          /* groups of 4 rays merged into 1 (Eq. 3) */
#define DARTRAY_C_U_ROWS 9          /* rows of per-wavelength deposits written, one atomic row each:
                                       step 1 without merging (FP64 energy density) and fixed rays
                                       (FP32 direction bins), where the crossings of a quad's rays
                                       into one cell share a row; 0 in the other passes */
#define DARTRAY_N_COUNT 16          /* slots of the counters buffer (10 .. 15 stay zero) */

typedef struct dartray_grid dartray_grid;   /* opaque handle */

/*
 * Grid description (host memory; read during dartray_grid_create only).
 *
 * The model is a block of nroot[0] x nroot[1] x nroot[2] cubic root cells of
 * edge root_size with lower corner lo; each root cell is an octree.  Leaf i
 * sits at refinement level leaf_level[i] (0 = root cell) with integer
 * coordinates leaf_ijk[3i..3i+2] counted in level-sized cells over the whole
 * block, so it spans lo + ijk * root_size / 2^level ... + root_size / 2^level.
 * The leaves must tile the block exactly (no gap, no overlap).  This is the
 * adaptive 3D Cartesian grid of Sect. 2.
 *
 * Per leaf: dust density rho (so that kappa[l] * rho is the optical depth per
 * unit length, Sect. 2) and stellar volume emissivity emis[l * n + i]
 * (luminosity per unit volume and solid angle).  Per wavelength: kappa,
 * albedo, g (Henyey-Greenstein, Eq. 4) and nside_sca, the HEALPix Nside of
 * the scattered source function at that wavelength (a power of two, or 0 to
 * apply the resolution rule of Eq. 5-6 with n_fwhm and the cap k_max).
 * Values must be finite, rho and emis >= 0, 0 <= albedo <= 1, |g| < 1,
 * nside_sca <= 8; n_leaves * n_lambda < 2^32 (DARTRAY_E_UNSUPPORTED above).
 * The Eq. 5 rule is applied with k_max <= 3 (Nside_sca <= 8): a larger k_max
 * with some nside_sca = 0 gives DARTRAY_E_UNSUPPORTED.
 */
typedef struct {
    int32_t nroot[3];
    double lo[3];
    double root_size;
    int64_t n_leaves;
    const int32_t *leaf_level;   /* [n] */
    const int64_t *leaf_ijk;     /* [n][3] */
    const float *rho;            /* [n] */
    const float *emis;           /* [n_lambda][n] */
    int32_t n_lambda;
    const float *kappa;          /* [n_lambda] */
    const float *albedo;         /* [n_lambda] */
    const float *g;              /* [n_lambda] */
    const int32_t *nside_sca;    /* [n_lambda] */
    double n_fwhm;               /* Eq. 6; the paper uses 5 */
    int32_t k_max;               /* cap on k of Eq. 5 (the paper suggests 2-3) */
    double c_light;              /* speed of light in the grid's units */
    int32_t nside_max;           /* largest ray Nside any trace on this handle uses
                                    (power of two, <= 1024; 0 means 64); sizes the
                                    direction table (16 * 4 nside_max^2 bytes) and,
                                    for adaptive rays, the phase-normalisation
                                    table (4 * n_lambda * 4 nside_max^2 bytes) */
    /* Point sources (Sect. 3.6): n_point isotropic sources at arbitrary
     * positions strictly inside the root block (host point_pos[3k..3k+2], grid
     * coordinates) with luminosity point_lum[l * n_point + k] (finite, >= 0).
     * They emit in step 1 and the direct pass: rays start at the point and
     * carry L / N_ray; the leaf holding the point (a point on a face belongs
     * to the upper side) is the source's own cell, where no split or block
     * test applies.  A source_mask then covers n + n_point entries (cells,
     * then point sources).  n_point = 0 and null arrays: none. */
    int32_t n_point;
    const double *point_pos;     /* [n_point][3] */
    const float *point_lum;      /* [n_lambda][n_point] */
} dartray_grid_desc;

/*
 * Ray policy and pass options (Sect. 3.1.1, 3.5).
 *
 * adaptive = 0: every source casts the 12 nside^2 HEALPix rays, no cutoff.
 * adaptive = 1: sources start with 12 nside^2 rays; a ray is split into its 4
 *   nested children (nside doubled, up to nside_max) when its beam is larger
 *   than the solid angle of the crossed cell over n_rays_min (Eq. 2) and it
 *   still matters; it is blocked when the beam is too large and its estimated
 *   contribution (Eq. 8) is below f_U times U_LL at every wavelength (Eq. 1);
 *   wavelengths below the threshold skip their deposits (Sect. 3.2).  In step
 *   1 the significance test is "entry distance < r_pre" and rays are cut at
 *   r_pre.  f_U < 0 selects f_U = 4 a_RT / N_s (Eq. 11) with N_s the number
 *   of radiation sources of the pass in the whole model (cells that emit at
 *   some wavelength, whether or not source_mask selects them).  The
 *   significance decisions are taken in FP64 (the ray's FP64 launch
 *   luminosity attenuated by its FP64 column density).
 * frame: row-major rotation applied to every HEALPix direction (rays and
 *   scattered-light pixels alike); identity when all zero.
 * source_mask: optional device uint8[n]; sources with 0 are skipped, in
 *   step 1, the direct pass and the scattering iterations alike (the
 *   emitted tally counts the selected sources only).  The passes are
 *   additive over sources (Sect. 3.4), so complementary masks add up to the
 *   unmasked pass when the other inputs (U_LL, S_pending) are the same.
 * max_steps: per-ray crossing limit (0 = unlimited).  It counts crossings of
 *   positive length (a zero-length graze of an edge or corner is none); a
 *   ray that has made max_steps of them and has a next cell stops there, is
 *   counted in DARTRAY_C_MAXSTEP and its remaining luminosity enters no
 *   tally (it is neither escaped nor cut).
 * n_rays_max > 0 (adaptive rays; >= 4 n_rays_min, so that a merged beam is
 *   not at once too large): ray merging (Eq. 3).  A ray above the launch
 *   Nside, outside its source's cell, whose beam is smaller than the crossed
 *   cell's solid angle over n_rays_max pauses before that crossing; when
 *   the four children of one split all pause having crossed the same grid
 *   plane they merge into one ray in the parent pixel that carries the sum
 *   of their luminosities (their average intensity over the four times
 *   wider beam) from the mean of their distances, and the parent's walk
 *   continues with it; otherwise the paused children carry on from where
 *   they stopped and pause no more.  At most 3 split levels (nside_max <=
 *   8 nside) with merging: deeper trees give DARTRAY_E_UNSUPPORTED.
 * DARTRAY_FLAG_2D (Sect. 3.6): for a model symmetric under reflection
 *   across the three planes through the centre of the root block (an
 *   axisymmetric model on a Cartesian grid is), only the sources of the
 *   first octant (leaf centre above the block centre on every axis) cast
 *   rays, and U, S and the escape by direction of each cell, pixel and
 *   direction become the sum of what those rays left in its 8 mirror
 *   images; the luminosity tallies count all 8 images of every source, the
 *   counters the rays actually traced.  Requires: every leaf's mirror images
 *   are leaves of the same size, density and emission (checked on the
 *   device when the flag is first used after a change; DARTRAY_E_INVALID
 *   otherwise), no leaf crosses a mirror plane, no point sources, no
 *   source_mask, the unrotated frame; not in the adjoint, batches or the
 *   allocation-free entry point (DARTRAY_E_UNSUPPORTED).  The unrotated
 *   ray and pixel directions are mirror symmetric bit for bit.
 */
typedef struct {
    int32_t mode;                /* DARTRAY_MODE_*, for dartray_trace_direct */
    int32_t adaptive;
    int32_t nside;
    int32_t nside_max;
    double n_rays_min;
    double f_U;
    double a_RT;
    double r_pre;
    double frame[9];
    const uint8_t *source_mask;  /* device, nullable */
    uint32_t flags;              /* DARTRAY_FLAG_* */
    int64_t max_steps;
    double n_rays_max;           /* N_rays^max of Eq. 3: ray merging (adaptive rays), 0 = none */
} dartray_trace_opts;

/*
 * Field buffers (device memory, caller-owned, FP32 unless stated).
 *  U         [n_lambda][n]  total energy density; each pass adds its U_k
 *  U_LL      [n_lambda][n]  lower limit used by the block test (adaptive);
 *                           step 1 writes it, every later pass sets it to U
 *  U_pass    [n_lambda][n]  nullable; receives this pass's U_k
 *  S_total   [s_size]       total scattered luminosity, all orders (Sect. 3.1.2)
 *  S_pending [s_size]       scattered luminosity waiting for the next iteration
 *  S_next    [s_size]       work array of the pass (overwritten)
 *  tally     [n_lambda][8]  FP64, overwritten by each pass (DARTRAY_T_*)
 *  counters  [16]           uint64 (DARTRAY_N_COUNT), overwritten when DARTRAY_FLAG_COUNTERS
 *  escape    [n_lambda][12 nside^2]  nullable; fixed rays only: luminosity of
 *                           the pass leaving the root block, by ray direction
 *                           (summed over sources; FP64 sums, FP32 output),
 *                           overwritten by each pass
 * S arrays hold one block per wavelength, block l starting at
 * dartray_s_offset(grid, l), laid out [n][12 nside_sca(l)^2] with the HEALPix
 * nested pixel index fastest.  S[l][c][p] is the luminosity scattered by cell
 * c into pixel p; j_sca = S / (V_c * 4 pi / N_pix).
 */
typedef struct {
    float *U;
    float *U_LL;
    float *U_pass;
    float *S_total;
    float *S_pending;
    float *S_next;
    double *tally;
    uint64_t *counters;
    float *escape;
} dartray_fields;

/* Build the device-side grid: validate, copy to the GPU, build the leaf
 * locator and the direction / phase-function tables.  `stream` is a
 * hipStream_t (NULL = default stream); all later work of the handle runs on
 * it.  On failure *out is NULL. */
int dartray_grid_create(const dartray_grid_desc *desc, void *stream, dartray_grid **out);

/* Release everything dartray_grid_create allocated.  Accepts NULL. */
int dartray_grid_destroy(dartray_grid *grid);

/* Size queries. */
int dartray_grid_info(const dartray_grid *grid, int64_t *n_leaves, int32_t *n_lambda, int64_t *s_size);
int dartray_nside_sca(const dartray_grid *grid, int32_t l, int32_t *nside);
int64_t dartray_s_offset(const dartray_grid *grid, int32_t l);

/* Replace the dust density (device float[n]); used by gradient-based fits. */
int dartray_grid_set_rho(dartray_grid *grid, const float *rho_device);

/*
 * Step 1 or the direct-light pass (Sect. 2, steps 1-2), by opts->mode.
 * STEP1: U_LL <- U_k of rays traced within r_pre (adaptive only).
 * DIRECT: U <- U + U_k, S_total <- S_next (S_total + S_next with
 *   DARTRAY_FLAG_CONTINUE), S_pending <- S_next; U_LL <- U when adaptive.
 *   Records sum(S_next) as the reference of the convergence ratio.
 */
int dartray_trace_direct(dartray_grid *grid, const dartray_trace_opts *opts, dartray_fields *fields);

/*
 * One scattering iteration (Sect. 2, step 3): the luminosity in S_pending is
 * re-emitted from each dusty cell along the ray directions (the ray inside
 * j_sca pixel p carries S_pending[p] * N_pix / N_ray), then U <- U + U_k,
 * S_total <- S_total + S_next, S_pending <- S_next, U_LL <- U when adaptive.
 * *r_k (host) receives sum(S_next) / sum(S after the direct pass), the ratio
 * tested against f_L; this synchronises the stream.  Requires a prior DIRECT.
 */
int dartray_scatter_iter(dartray_grid *grid, const dartray_trace_opts *opts, dartray_fields *fields, double *r_k);

/*
 * The direct pass of dartray_trace_direct for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, with the pass's work arrays
 * (energy-density accumulators, direction bins, source list, scan sums,
 * error word) taken from a static device array of 64 MiB per GPU instead of
 * the handle's own.  It calls no hipMalloc, hipFree or other allocating
 * routine (the first call on a device looks up that device's array once).
 * Fixed rays only (opts->adaptive = 0, opts->nside <= 16); a grid whose work
 * arrays exceed the 64 MiB (n_leaves * n_lambda * 12 bytes plus one
 * direction of bins, n_leaves * n_lambda * 4 bytes, and small parts) gives
 * DARTRAY_E_UNSUPPORTED with the size in the message, before any output is
 * written.  Every call on a GPU shares that GPU's array: calls that overlap
 * on one GPU (on different streams or threads) race.  Outputs and state as
 * dartray_trace_direct.
 */
int dartray_trace_direct_noalloc(dartray_grid *grid, const dartray_trace_opts *opts, dartray_fields *fields);

/*
 * Gradient dJ/drho of a loss J of the energy density U and of the escaping
 * luminosity F (escape summed over the passes) with respect to the per-cell
 * dust density, by an adjoint march over the passes of a fixed-ray
 * run in reverse order (scattering iteration n_scatter down to the direct
 * pass).  Rays are recomputed, not stored: each ray is walked twice, first for
 * the total of its loss-weighted deposits, then for the derivative at every
 * crossing as a prefix difference (FP64); the result flows from each pass to
 * the scattered luminosity that fed it through the inverse launch rule.
 * Fixed rays only (opts->adaptive = 0, opts->nside <= 16) and at most 8
 * wavelengths; opts must be those of the forward run, and the grid's rho the
 * forward run's.  This extends the method (the paper has no gradients).
 *  n_scatter  scattering iterations of the forward run (>= 0)
 *  S_hist     host array of n_scatter device pointers; S_hist[k-1] is the
 *             pending scattered luminosity iteration k processed (S_pending
 *             before that dartray_scatter_iter call), S layout
 *  dJ_dU      device float [n_lambda][n], or NULL for a loss without U
 *  dJ_dS      device float, S layout, or NULL: the derivative with respect
 *             to S_total, the scattered luminosity of every order (for a loss
 *             on j_sca = S_total / (V 4 pi / N_pix), dJ/dS = dJ/dj_sca /
 *             (V 4 pi / N_pix)); every order's S receives it
 *  dJ_desc    device float [n_lambda][12 nside^2], or NULL for a loss
 *             without the escaping luminosity (it enters each ray as the
 *             terminal value of the reverse recursion)
 *  dJ_drho    device float [n], overwritten
 */
int dartray_trace_adjoint(dartray_grid *grid, const dartray_trace_opts *opts, int32_t n_scatter,
                          const float *const *S_hist, const float *dJ_dU, const float *dJ_dS,
                          const float *dJ_desc, float *dJ_drho);

/*
 * Test helper: the cells crossed by n_rays rays (host arrays: origin[3i],
 * dir[3i], in grid coordinates), computed by the marches' own FP64 traversal
 * (exit distances, face-neighbour steps and tie rules of Sect. 2 as the
 * passes walk rays).  Up to max_cross segments per ray are written to
 * cells[i * max_cross + m] (leaf id) and lengths[...] (FP64 path length, 0
 * for zero-length segments, which are listed); counts[i] gets the number
 * written.  Allocates and frees small device buffers; synchronises the
 * stream.
 */
int dartray_debug_ray_cells(dartray_grid *grid, int32_t n_rays, const double *origin, const double *dir,
                            int32_t max_cross, int64_t *cells, double *lengths, int32_t *counts);

/* Timing of the ray-march kernels with HIP events recorded on the grid's
 * stream around every march launch of the selected kinds.  kinds is a mask of
 * DARTRAY_PROF_* bits; a nonzero mask clears earlier records and starts
 * recording, 0 stops. */
#define DARTRAY_PROF_FIXED 1        /* fixed-Nside march launches */
#define DARTRAY_PROF_STEP1 2        /* adaptive step-1 march launches */
#define DARTRAY_PROF_SCATTERING 4   /* adaptive direct / scattering march launches */
#define DARTRAY_PROF_ADJOINT 8      /* adjoint march launches (dartray_trace_adjoint) */
#define DARTRAY_PROF_ALL 15
int dartray_profile_enable(dartray_grid *grid, int32_t kinds);

/* Sum of the recorded march-kernel durations (ms) and the number of launches
 * since recording started; synchronises the stream. */
int dartray_profile_read(dartray_grid *grid, double *march_ms, int64_t *launches);

/* Device memory: with opts NULL, every byte the handle holds; with opts, the
 * bytes of the handle's work arrays that a pass with these options uses
 * (accumulators, tables, direction bins or deposit log), beyond the caller's
 * fields.  All of it is allocated by dartray_grid_create. */
int dartray_workspace_bytes(const dartray_grid *grid, const dartray_trace_opts *opts, size_t *bytes);

/*
 * Launch parameters of the fixed-ray passes (the autotuner's search space).
 * A zero field takes the default.  They change speed only: any setting gives
 * the same deposits, up to the order of FP32 additions into the bins.
 *  lambda_tile  wavelengths one march launch carries (1, 4, 8, 16, 32, 64;
 *               default all): the ray geometry is recomputed once per tile,
 *               so a tile of all wavelengths is the batched form of Sect. 3.3
 *               and a tile of 1 is the plain per-wavelength form
 *  block_waves  64-lane waves per workgroup of the march (1, 2 or 4; default 4)
 *  grid_blocks  workgroups of the persistent march (1 .. 65536; default 2048)
 *  dir_batch    directions binned between two flushes (default: as many as
 *               the handle's bin array holds)
 *  item_order   0: a wave's next work item is the next direction of the same
 *               64-source tile; 1: the next source tile of the same direction
 *               (also the order of the adjoint march)
 */
typedef struct {
    int32_t lambda_tile;
    int32_t block_waves;
    int32_t grid_blocks;
    int32_t dir_batch;
    int32_t item_order;
} dartray_tuning;

/* Set / read the handle's fixed-ray launch parameters.  Invalid values give
 * DARTRAY_E_INVALID and leave the setting unchanged. */
int dartray_set_tuning(dartray_grid *grid, const dartray_tuning *tuning);
int dartray_get_tuning(const dartray_grid *grid, dartray_tuning *tuning);

/*
 * Batches of models (fixed rays).  The sources of independent models are
 * independent work (Sect. 3.4 parallelises over sources); a batch runs the
 * passes of several grid handles together: per pass and direction batch one
 * persistent march launch takes (model, 64-source tile, direction) items of
 * every model, models in descending order of size, and one flush launch
 * covers every model's cells.  The handles must share the stream and the
 * number of wavelengths, stay owned by the caller and outlive the batch; the
 * first handle's tuning applies to the whole batch.
 */
typedef struct dartray_batch dartray_batch;

/* Group n_models distinct handles.  Allocates three small device arrays. */
int dartray_batch_create(dartray_grid *const *grids, int32_t n_models, dartray_batch **out);

/* Release a batch (not its grids).  Accepts NULL. */
int dartray_batch_destroy(dartray_batch *batch);

/* Direct pass then n_scatter scattering iterations of every model: fields[m]
 * receives model m's results as dartray_trace_direct followed by
 * dartray_scatter_iter would (opts: fixed rays, DARTRAY_MODE_DIRECT, no
 * source mask).  Synchronises the stream once, before any pass, to upload
 * the per-model launch arguments; the passes are queued asynchronously. */
int dartray_batch_run(dartray_batch *batch, const dartray_trace_opts *opts, dartray_fields *const *fields,
                      int32_t n_scatter);

/* The same sequence recorded by stream capture into a HIP graph (the stream
 * must not be the legacy NULL stream).  The field buffers named here are
 * baked into the graph; every replay rewrites them. */
int dartray_batch_capture(dartray_batch *batch, const dartray_trace_opts *opts, dartray_fields *const *fields,
                          int32_t n_scatter);

/* Launch the captured graph on the batch's stream (DARTRAY_E_STATE if none). */
int dartray_batch_replay(dartray_batch *batch);

/*
 * Observer maps (Sect. 2: the intensity reaching an observer is I_0 e^{-tau};
 * Sect. 3.6: maps seen from inside the model as HEALPix all-sky maps).
 * Every cell is a source of luminosity per unit solid angle towards the
 * observer: j V (stellar emission) plus S_total[p] N_pix / (4 pi) for the
 * j_sca pixel p holding that direction (scattered light, when S_total is
 * given), emitted at the cell centre and attenuated by
 * exp(-kappa sum rho l) from the centre to the observer (the cell's own half
 * included; FP64 path sums).
 *  DISTANT: the observer is far away along the unit vector `dir` (from the
 *    model towards the observer); the image plane has axes e2 = `up` made
 *    orthogonal to dir and e1 = e2 x dir, nx x ny pixels of edge pixel_size
 *    centred on the model point `centre`; a cell falls in the pixel of its
 *    centre's projection; map[l][iy * nx + ix] is the surface brightness
 *    (sum over the pixel's cells over the pixel area).
 *  INTERNAL: the observer sits at `pos`; map[l][p] (HEALPix nested pixel p at
 *    nside_map, in the grid's frame) is the sum over the cells whose
 *    direction from the observer lies in p of the flux (luminosity per
 *    steradian over the distance squared), per the pixel's solid angle.  The
 *    leaf holding the observer is left out.
 * frame: the rotation of the run's j_sca pixel directions (as
 * dartray_trace_opts.frame; all zero = identity).
 * map: device double [n_lambda][npix], overwritten.  Asynchronous, except an
 * internal observer's set-up (it reads the leaf boxes back once).
 */
#define DARTRAY_OBS_DISTANT 0
#define DARTRAY_OBS_INTERNAL 1
typedef struct {
    int32_t kind;                /* DARTRAY_OBS_* */
    double dir[3];
    double up[3];
    double centre[3];
    double pixel_size;
    int32_t nx, ny;
    double pos[3];
    int32_t nside_map;
    double frame[9];
} dartray_observer;

int dartray_observe(dartray_grid *grid, const dartray_observer *obs, const float *S_total, double *map);

/*
 * Dust emission and the self-heating loop (Sect. 3.3).
 *
 * Every wavelength of a grid stands for a band: U, j and the luminosities
 * are band-integrated.  The dust of a cell absorbs (1 - albedo_l) kappa_l
 * rho V c U_l in band l (with the deposit rule U = ext / (alpha V c) this is
 * the absorbed part of what the band's rays extinguish there).  The grain
 * model is the caller's choice in the paper (equilibrium or stochastic
 * heating); the library offers an equilibrium grain whose emission in band i
 * of the emitting grid is 4 pi rho V kappa_i (1 - albedo_i) B(lambda_i, T)
 * dlambda_i, with B(lambda, T) = b0 lambda^-5 / (exp(x0 / (lambda T)) - 1) and
 * T the temperature at which the cell emits what it absorbs (found by
 * bisection of [0, t_max] to adjacent doubles, in FP64).
 */
typedef struct {
    double b0;                   /* scale of B */
    double x0;                   /* h c / k in the units of lambda times temperature */
    double t_max;                /* upper end of the temperature bracket */
    const double *lambda;        /* host [n_lambda of the emitting grid] band centres, > 0 */
    const double *dlambda;       /* host [n_lambda of the emitting grid] band widths, > 0 */
} dartray_dust_model;

/* A[c] += sum_l (1 - albedo_l) kappa_l rho_c V_c c U[l][c].  U: device float
 * [n_lambda][n]; A: device double [n].  Asynchronous. */
int dartray_absorbed(const dartray_grid *grid, const float *U, double *A);

/* Equilibrium temperature T (device double [n]) and band emission j (device
 * double [n_lambda][n], per unit volume and steradian) of the emitting grid's
 * cells for absorbed luminosities A (device double [n]).  Cells without dust
 * or without absorbed light: T = 0, j = 0.  Synchronises; a cell that would
 * need more than t_max gives DARTRAY_E_NUMERIC (T and j then hold 0 there). */
int dartray_dust_emission(dartray_grid *grid, const dartray_dust_model *dm, const double *A, double *T, double *j);

/* Replace the grid's emission j (device double [n_lambda][n], per unit volume
 * and steradian, finite and >= 0; checked before anything changes, which
 * synchronises).  Later passes launch from it. */
int dartray_grid_set_emis(dartray_grid *grid, const double *j);

/*
 * The self-heating procedure of Sect. 3.3 on the emitting ("dust") grid, in
 * the paper's order:
 *  1. emission from the absorbed stellar luminosity A_star alone;
 *  2. a dust RT calculation of it: step 1 (adaptive rays, when so->step1),
 *     the direct pass, up to so->n_scatter scattering iterations (stopping
 *     early once r_k < so->f_L, when f_L > 0);
 *  3. the emission recomputed from A_star plus the dust light absorbed;
 *  4. dj = j - j_prev (not negative in exact arithmetic: more absorbed light,
 *     a warmer grain; rounding residues below zero are dropped);
 *  5. a dust RT calculation of dj alone, U and S_total continuing from the
 *     previous calculation's and U_LL = U (no step 1);
 *  6. 3-5 repeated until dj / j_prev < so->conv at every cell and band (a
 *     cell and band with j_prev = 0 < dj is not converged), at most
 *     so->max_iter calculations.
 * opts: the ray policy of every calculation (mode and DARTRAY_FLAG_CONTINUE
 * are set by the loop).  A_star: device double [n], dartray_absorbed of the
 * stellar run on a grid with the same cells.  fields: the dust grid's
 * buffers; U, U_LL and S_total are overwritten by the loop's results.
 * T [n], j [n_lambda][n]: the last update (the converged emission);
 * j_traced [n_lambda][n]: the emission whose light U and S_total hold; work:
 * device double [n (1 + n_lambda)]; all device, caller-owned.  ratios (host
 * double [max_iter]) receives max dj / j_prev after each calculation and
 * *n_rt (host) the number of calculations.  Synchronises once per
 * calculation; returns DARTRAY_E_NUMERIC as dartray_dust_emission does.
 */
typedef struct {
    int32_t step1;               /* adaptive rays: step 1 before the first calculation */
    int32_t n_scatter;           /* scattering iterations per calculation */
    int32_t max_iter;            /* at most this many calculations (>= 1) */
    double f_L;                  /* 0, or the r_k below which a calculation's iterations stop */
    double conv;                 /* convergence threshold of dj / j_prev (Sect. 3.3: 0.01) */
} dartray_selfheat_opts;

int dartray_dust_selfheat(dartray_grid *grid, const dartray_trace_opts *opts, const dartray_selfheat_opts *so,
                          const dartray_dust_model *dm, const double *A_star, dartray_fields *fields, double *T,
                          double *j, double *j_traced, double *work, double *ratios, int32_t *n_rt);

/* Message of the last failure on this thread ("" if none). */
const char *dartray_last_error(void);

/* Library version string. */
const char *dartray_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DARTRAY_H */
