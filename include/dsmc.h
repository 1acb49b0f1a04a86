/*
 * dsmc.h -- C ABI of the MI355X (gfx950) library for the data-parallel inner
 * loop of unsteady Direct Simulation Monte Carlo.
 *
 * The operation is the sequential unsteady-DSMC algorithm of Sec. 1.1 of
 * Bogdanov, Bykov, Grishin, Khanlarov, Lukianov and Zakharov, "Algorithms of
 * Two-Level Parallelization for DSMC of Unsteady Flows in Molecular
 * Gasdynamics" (Fig. 1): an inner loop
 * over time steps dt of one run -- Generation, Motion, Enumeration/Indexing
 * (the readdressing array LCR), Interaction, and Sampling at given moments --
 * and an outer loop over n statistically independent runs whose random number
 * generator is shifted per run.  Every call below advances many runs at once
 * (the paper's parallel independent runs, Sec. 1.3, inside one launch) with
 * data parallelism over particles and cells inside each run (Sec. 1.4).
 *
 * Conventions
 *  - Units are reduced: Boltzmann constant = molecular mass = 1.
 *  - Memory: the caller owns ALL device memory.  dsmc_required_bytes gives the
 *    size of one device arena; the caller allocates it (e.g. a torch tensor)
 *    and passes it to dsmc_init_runs.  The arena must outlive the context.
 *    The library allocates no device memory; it owns only the opaque context
 *    (host heap) and copies the run specs and sample schedule.
 *  - Streams: the caller's HIP stream is borrowed and every launch goes to
 *    it, except (a) with dsmc_options.n_streams > 1, where run groups go to
 *    streams of the library's own forked from and joined back into it by
 *    events, and (b) graph replay when it is the null stream, which runs on a
 *    library stream ordered after it by events.
 *  - Asynchrony: dsmc_step and dsmc_sample only enqueue work.
 *    dsmc_read_moments, dsmc_read_accum, dsmc_sync and the dsmc_get_* /
 *    dsmc_set_state calls synchronise the stream.
 *  - Errors: every call returns a dsmc_status (0 = DSMC_OK).  Argument errors
 *    are detected before anything is enqueued.  Device-side conditions
 *    (capacity overflow during Generation, too many wall interactions, a
 *    failed inflow draw, non-finite state, a HIP launch failure) latch an
 *    error that the next synchronising call returns; when several occur, the
 *    lowest (most negative) status is the one latched, whatever their order.
 *    After that only dsmc_destroy and dsmc_last_error are valid.  No
 *    exception or abort crosses the ABI.
 *  - Threading: a context is not thread-safe; distinct contexts are
 *    independent.
 */
#ifndef DSMC_H
#define DSMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t dsmc_status;
#define DSMC_OK 0
#define DSMC_EINVAL (-1)       /* invalid argument */
#define DSMC_ESIZE (-2)        /* buffer or arena too small */
#define DSMC_ECAPACITY (-3)    /* a run ran out of particle slots */
#define DSMC_EDEVICE (-4)      /* HIP error */
#define DSMC_ESTATE (-5)       /* call not valid in the current state */
#define DSMC_EUNSUPPORTED (-6) /* feature not supported */
#define DSMC_EBOUNCE (-7)      /* more than 64 wall interactions of one particle in one step */
#define DSMC_EREJECT (-8)      /* inflow velocity sampler or the fill of a run with solid cells exceeded
                                  its attempt limit */
#define DSMC_ENUMERIC (-9)     /* a non-finite coordinate or velocity met by Motion's flight (in 2-D, w
                                  only through a pair selection), or >= 1e9 pair selections in one cell
                                  and step (e.g. an infinite relative speed) */

/* Boundary kind of a face; faces are ordered -x, +x, -y, +y, -z, +z. */
#define DSMC_BC_SPECULAR 0     /* mirror reflection */
#define DSMC_BC_DIFFUSE 1      /* full accommodation at face_T */
#define DSMC_BC_INFLOW 2       /* -x only: drifting-Maxwellian reservoir; leavers are removed */
#define DSMC_BC_OUTFLOW 3      /* vacuum: leavers are removed */

/* Sampled sums per cell (dsmc_read_accum) and moments (dsmc_read_moments). */
#define DSMC_NSUM 7            /* N, sum u, sum v, sum w, sum u^2, sum v^2, sum w^2 */
#define DSMC_NMOM 8            /* n (particles per cell per run), ux, uy, uz, T, Tx, Ty, Tz */

typedef struct dsmc_ctx dsmc_ctx; /* opaque, library-owned */

/* One independent run (one iteration of the outer loop of Sec. 1.1). */
typedef struct {
  int32_t dim;                  /* 2 or 3 (all runs of a context share it) */
  int32_t nx, ny, nz;           /* uniform cell grid; nz = 1 in 2-D */
  double lx, ly, lz;            /* box [0,lx] x [0,ly] x [0,lz]; lz = 1 in 2-D */
  double dt;                    /* time step */
  double fnum_sigma;            /* Fnum * sigma_ref (0 = collisionless) */
  double omega;                 /* VHS viscosity index; 0.5 = hard sphere */
  double c_ref;                 /* VHS reference relative speed */
  int32_t face_bc[6];           /* DSMC_BC_* per face */
  double face_T[6];             /* wall temperature of DIFFUSE faces */
  double inflow_n, inflow_U, inflow_T; /* inflow density (simulated particles per unit volume), drift, T */
  int64_t capacity;             /* particle slots reserved for this run */
  int64_t n_init;               /* initial uniform Maxwellian fill (0 = empty) */
  double init_U[3];             /* initial drift */
  double init_T;                /* initial temperature */
  uint32_t run_id, seed;        /* Philox key of the run: runs are independent and replayable */
  int32_t ensemble;             /* runs with the same id are averaged together; they share a grid */
  int32_t subcells;             /* collision partners from sub-cells, k per axis (0 or 1 = none, at most 4):
                                   each particle's Indexing bin is its sub-cell (cell * k^dim + the
                                   sub-cell within it, from the floor on the k-times finer grid), and
                                   the second partner of a selection is drawn from the first one's
                                   sub-cell when it holds two or more particles, else from the cell (a
                                   refinement of the collision-partner choice of the DSMC method of
                                   Sec. 1.1, after Bird); the NTC count stays the cell's.  Not with
                                   solid_mask (DSMC_EUNSUPPORTED). */
  const uint8_t *solid_mask;    /* host [nz][ny][nx] (cell (iz*ny + iy)*nx + ix), nonzero = solid cell, or
                                   NULL.  Solid cells are an obstacle with diffuse faces at solid_T: a
                                   path is followed cell by cell in the time order of its plane crossings
                                   (ties: x, then y, then z) and the first solid cell it enters is hit on
                                   the crossed face.  Copied by dsmc_init_runs.  With inflow, the first
                                   layer of cells (ix = 0) must be fluid. */
  double solid_T;               /* temperature of the solid faces (> 0 when solid_mask is given) */
  double ntc_nbar_alpha;        /* NTC selection count of a cell (Sec. 1.1's collision step, after Bird):
                                   0 = N(N-1)/2 pairs times Fnum sigma_ref dt / V_c (sigma c_r)_max plus
                                   the remainder; in (0, 1] = N Nbar / 2 pairs instead, Nbar a running
                                   mean of the cell's count moved by Nbar += alpha (N - Nbar) before each
                                   count and started at n_init / cells (1: Nbar = N) */
} dsmc_run_spec;

typedef struct {
  int32_t state_fp64;           /* 1: FP64 particle state and arithmetic; 0: FP32 */
  int32_t n_groups;             /* run groups per ensemble for batch-means errors (>= 1) */
  int32_t n_samples;            /* sample slots (>= 0) */
  const int32_t *sample_steps;  /* host [n_samples]: 1-based step after which dsmc_step samples into slot k
                                   (entry < 1: slot filled only by dsmc_sample); may be NULL */
  int32_t use_graph;            /* 1: replay each step from a HIP graph (captured on hip_stream, or on a
                                   stream of the library's own ordered after it by events when
                                   hip_stream is the null stream) */
  int32_t tile_chunks;          /* tuning: 64-slot rounds per indexing tile, a multiple of 4 up to
                                   4096 (0 = default 256) */
  int32_t collide_mode;         /* tuning: 0 auto, 1 one lane per cell (up to 64 cells per
                                   wavefront), 2 one 256-thread block per cell, 3 one 64-lane
                                   wavefront per cell; auto takes 3 when the expected particles
                                   per cell (initial fill or inflow fill) reach 112 and 2 when
                                   they reach 288.  Results do not depend on it: every mode
                                   runs a cell's selections in the sequential order and adds
                                   its sample sums in one shared order (chunks of 16
                                   particles, each in order, then the chunk sums in order). */
  int32_t n_streams;            /* tuning: run groups stepped concurrently, each on a HIP stream of the
                                   library's own (0 = auto = 1, 1..4; 1 = every launch on hip_stream).
                                   The runs are split into contiguous groups of about equal slot
                                   counts; one group's Indexing and Interaction overlap the next
                                   group's Motion.  Results do not depend on it. */
  int32_t window_steps;         /* sampling window (0 or 1 = one snapshot per slot): slot k accumulates
                                   the snapshots after steps sample_steps[k] - j * window_stride,
                                   j = 0 .. window_steps - 1 (those >= 1), so that its moments average
                                   over time as well as over the runs -- the steady-flow variant: an
                                   averaging time much longer than dt once the flow is steady (Sec.
                                   1.1), with ensemble averaging of runs of fewer particles on top
                                   (end of Sec. 3).  Windows of different slots may share no step
                                   (DSMC_EINVAL). */
  int32_t window_stride;        /* steps between the snapshots of a window (0 = 1) */
  int32_t sched;                /* tuning: how Interaction's workgroups get their items (cells or groups
                                   of cells, of every run): 0 = one per workgroup (or wavefront) of a
                                   grid covering all items, handed to CUs by the hardware; 1 = a
                                   persistent grid drawing items from a device queue shared by all runs
                                   (dynamic reallocation of workgroups between runs, Sec. 3); 2 = a
                                   persistent grid whose workgroups are tied to runs (the static two-level
                                   split of Sec. 2: of U workgroups, g serves run g mod runs when U is at
                                   least the number of runs, else runs g, g + U, ... in turn).
                                   Results do not depend on it. */
  int32_t sched_blocks;         /* tuning: workgroups of each persistent grid (0 = as many as fit on
                                   the GPU at once) */
} dsmc_options;

/* Arena size for these runs/options.  Pure host computation.
 * Returns DSMC_EINVAL for an invalid spec (same checks as dsmc_init_runs). */
dsmc_status dsmc_required_bytes(const dsmc_run_spec *runs, int32_t n_runs, const dsmc_options *opt,
                                size_t *bytes);

/* Create a context: lays the runs out in the arena (device memory of at
 * least dsmc_required_bytes bytes, 256-byte aligned), fills each run with its
 * initial state (Philox stream "INIT" of its key) and returns the context.
 * The runs are the n statistically independent runs of the outer loop of
 * Sec. 1.1 (Fig. 1), each with its own shift of the random number generator
 * (here its Philox key); their arrays P, LCR and C (Sec. 1.1) live in the
 * arena.  hip_stream is a hipStream_t (NULL = default stream).
 * Synchronises. */
dsmc_status dsmc_init_runs(const dsmc_run_spec *runs, int32_t n_runs, const dsmc_options *opt, void *arena,
                           size_t arena_bytes, void *hip_stream, dsmc_ctx **out);

/* Advance every run by n_steps time steps (Sec. 1.1: Generation, Motion,
 * Enumeration/Indexing, Interaction; Sampling at the scheduled steps).
 * Asynchronous. */
dsmc_status dsmc_step(dsmc_ctx *ctx, int32_t n_steps);

/* Sampling (Sec. 1.1, Fig. 1): add the per-cell sums of the current state of
 * every run into sample slot k -- the cross-run accumulation of the
 * statistical data at a given moment of the unsteady process -- and count one
 * more snapshot of slot k.  Valid after at least one step.  Asynchronous. */
dsmc_status dsmc_sample(dsmc_ctx *ctx, int32_t sample_index);

/* Cell moments of one ensemble at sample slot k, FP64: the macroparameters
 * averaged over the particles of each cell and over the runs (Sec. 1.1), the
 * final division of the cross-run sums.  out[cell][DSMC_NMOM] on the host:
 * n = particles per cell per run and snapshot, the mean velocity, T and the
 * directional temperatures (pooled over runs, no N/(N-1) correction); out_se
 * (may be NULL) the batch-means standard error over the ensemble's run groups
 * (NaN with one group).  capacity_doubles is the size of each host array.
 * Cells with no particles give NaN.  Synchronises. */
dsmc_status dsmc_read_moments(dsmc_ctx *ctx, int32_t sample_index, int32_t ensemble, double *out,
                              double *out_se, size_t capacity_doubles);

/* Raw FP64 sums of one ensemble at slot k: out[group][cell][DSMC_NSUM].  Synchronises. */
dsmc_status dsmc_read_accum(dsmc_ctx *ctx, int32_t sample_index, int32_t ensemble, double *out,
                            size_t capacity_doubles);

/* Wait for all enqueued work; returns the latched device error, if any. */
dsmc_status dsmc_sync(dsmc_ctx *ctx);

void dsmc_destroy(dsmc_ctx *ctx);

/* Message of the last failed call on this context; for NULL, of the last failed
 * call on this thread that had no context to hold it (dsmc_required_bytes,
 * dsmc_init_runs, dsmc_autotune).  The text stays valid until the next call on
 * the context (or, for NULL, on the thread). */
const char *dsmc_last_error(const dsmc_ctx *ctx);

/* ---- inspection (tests, diagnostics); all synchronise ---------------------- */

/* Context facts: info[0] steps done, [1] runs, [2] ensembles, [3] 1 if FP64,
 * [4] indexing passes, [5] tiles, [6] slots, [7] latched device error,
 * [8] stream lanes, [9] 1 if steps replay from HIP graphs (outside profiling). */
#define DSMC_NINFO 10
dsmc_status dsmc_get_info(dsmc_ctx *ctx, int64_t info[DSMC_NINFO]);

/* Particle state of one run in slot order (cell-sorted after a step):
 * out[6][n] = x, y, z, u, v, w (z = 0 in 2-D), FP64.  *n receives the count;
 * cap is the per-component capacity of out. */
dsmc_status dsmc_get_state(dsmc_ctx *ctx, int32_t run, double *out, int64_t cap, int64_t *n);

/* Replace the particle state of one run (in[6][n], FP64; converted to the
 * state precision).  Returns DSMC_EINVAL, with nothing changed, for a
 * non-finite coordinate or velocity, a position outside the box (x in
 * [0, lx], y in [0, ly], and z in [0, lz] in 3-D) or n above the run's
 * capacity. */
dsmc_status dsmc_set_state(dsmc_ctx *ctx, int32_t run, const double *in, int64_t n);

/* Indexing of the last step of one run: lcr[n] (run-local slots in stable
 * bin order, DEAD last) and cell[n] (bin of each slot: its cell, or with
 * sub-cells its sub-cell bin; nbin = nc * k^dim = DEAD) for the n particles
 * present before removal; start[nbin + 2] bin starts (may be NULL). */
dsmc_status dsmc_get_lcr(dsmc_ctx *ctx, int32_t run, int32_t *lcr, int32_t *cell, int64_t *start,
                         int64_t cap, int64_t *n);

/* Per-cell interaction state of one run: remainder, (sigma c_r)_max in units
 * of sigma_ref, cumulative accepted collisions and the running mean of the
 * count (ntc_nbar_alpha; its start value when the run does not use it)
 * (each array [nc], may be NULL). */
dsmc_status dsmc_get_cell_state(dsmc_ctx *ctx, int32_t run, double *rem, double *gmax, int64_t *ncoll,
                                double *nbar);

/* Per run: [r][0] particles now, [r][1] particles generated in the last step. */
dsmc_status dsmc_get_counts(dsmc_ctx *ctx, int64_t *out, int32_t n_runs);

/* Snapshots accumulated so far in each sample slot (scheduled and by
 * dsmc_sample): out[k] for k < n_samples (n_samples must equal the
 * context's).  Synchronises. */
dsmc_status dsmc_get_sample_counts(dsmc_ctx *ctx, int64_t *out, int32_t n_samples);

/* Per-run diagnostics computed on the device from the current state, FP64:
 * out[r][DSMC_NDIAG] = particles, particles generated in the last step,
 * accepted collisions since init (over the run's cells), sum u, sum v, sum w
 * (momentum per unit mass) and sum |c|^2 (twice the kinetic energy per unit
 * mass) over the run's particles.  n_runs must equal the context's.  The
 * sums are in a fixed order: repeated calls give the same bits.
 * Synchronises. */
#define DSMC_NDIAG 7
dsmc_status dsmc_get_diag(dsmc_ctx *ctx, double *out, int32_t n_runs);

/* ---- checkpoint / resume --------------------------------------------------- */

/* Size in bytes of a checkpoint of the current state (it grows with the
 * particles alive).  Synchronises. */
dsmc_status dsmc_checkpoint_bytes(dsmc_ctx *ctx, size_t *bytes);

/* Copy everything a later step reads into the host buffer `host` (at least
 * dsmc_checkpoint_bytes, 8-byte aligned): per run the particles (P in its
 * cell-sorted order, in the state precision, bit for bit) and their count, the
 * per-cell interaction state (remainder, (sigma c_r)_max, running mean of the
 * count, collision counter)
 * and bin starts, the inflow faces' carried remainders; the accumulators and
 * snapshot counts of every sample slot; the step counter.  The steps of the
 * runs are replayable from their Philox keys and the step counter (Sec. 1.1:
 * runs made independent by shifting the generator), so a context restored
 * from it continues bit-identically.  Synchronises. */
dsmc_status dsmc_checkpoint(dsmc_ctx *ctx, void *host, size_t bytes);

/* Put a checkpoint back into a context made by dsmc_init_runs from the same
 * run specs, precision, run groups, sample schedule and window (tuning
 * fields may differ: results do not depend on them).  Returns DSMC_EINVAL,
 * with nothing changed, when the buffer is not a checkpoint of such a
 * context (magic, version, fingerprint of the specs, sizes).  The next
 * dsmc_step continues exactly where the checkpointed context would have.
 * Synchronises. */
dsmc_status dsmc_restore(dsmc_ctx *ctx, const void *host, size_t bytes);

/* ---- per-kernel timing ----------------------------------------------------- */

#define DSMC_NKERNELS 19 /* kernel kinds; names from dsmc_kernel_name */

/* Turn per-kernel timing on or off (synchronises).  While on, every launch is
 * bracketed by two HIP events on the context's stream and steps are not
 * replayed from graphs. */
dsmc_status dsmc_set_profiling(dsmc_ctx *ctx, int32_t on);

/* Accumulated event time (ms) and launch count per kernel kind since the last
 * call, for the first n kinds (n <= DSMC_NKERNELS); resets the totals.
 * Synchronises. */
dsmc_status dsmc_kernel_times(dsmc_ctx *ctx, double *ms, int64_t *launches, int32_t n);

/* Name of kernel kind k (static string), NULL if out of range. */
const char *dsmc_kernel_name(int32_t kind);

/* ---- autotuning ------------------------------------------------------------ */

/* Arena size dsmc_autotune needs for these runs: the largest dsmc_required_bytes
 * over its candidate settings.  Pure host computation; DSMC_EINVAL as
 * dsmc_required_bytes. */
dsmc_status dsmc_autotune_bytes(const dsmc_run_spec *runs, int32_t n_runs, const dsmc_options *opt,
                                size_t *bytes);

/* Chooses the tuning fields of dsmc_options (tile_chunks, collide_mode,
 * n_streams, sched, sched_blocks) for these runs by measurement.  None of
 * them changes any result (every setting computes the same sequential order
 * bit for bit); they only change speed.  Candidates: tiles of 4096, 8192 and
 * 16384 slots; all three interaction modes when a run's expected particles
 * per cell lie in 28..576; one or two stream lanes when n_runs >= 8; the
 * default tile with Interaction on persistent grids drawing from one queue
 * for all runs (sched 1) at two occupancies (as many workgroups as fit, and
 * 1024).  Each candidate is initialised in the caller's arena (at least
 * dsmc_autotune_bytes, 256-byte aligned), restored from `start` when given,
 * stepped once to warm up (graph capture included when opt->use_graph), then
 * n_steps (>= 1) steps are timed with HIP events on hip_stream.  start (host
 * memory, start_bytes long; NULL and 0 for the initial fill) is a checkpoint
 * written by dsmc_checkpoint for the same run specs, precision, groups,
 * schedule and window: an unsteady problem that starts from vacuum is then
 * tuned at the state it will run in (DSMC_EINVAL if it is not a checkpoint
 * of this problem).  *best receives *opt with
 * the fastest tuning fields; *best_ms_per_step (may be NULL) its time per
 * step.  tune_cache (may be NULL) names a text file of earlier results: when
 * it holds a result for the same run specs, precision, groups, schedule,
 * window, graph replay, device and starting step, that result (the last
 * such line) is returned without timing (and without touching the arena);
 * otherwise, or when that line holds settings dsmc_init_runs would refuse,
 * the candidates are timed and the new result is appended to it.
 * Concurrent writers of one cache file are not supported.  The arena holds no usable context afterwards.  Synchronises. */
dsmc_status dsmc_autotune(const dsmc_run_spec *runs, int32_t n_runs, const dsmc_options *opt, void *arena,
                          size_t arena_bytes, void *hip_stream, int32_t n_steps, const void *start,
                          size_t start_bytes, const char *tune_cache, dsmc_options *best,
                          double *best_ms_per_step);

/* ---- Indexing alone ------------------------------------------------------ */

/* Workspace bytes for dsmc_counting_sort. */
dsmc_status dsmc_counting_sort_bytes(int64_t n, int32_t nbins, size_t *bytes);

/* Stable counting sort (the Indexing step, Sec. 1.1/1.4) of n device keys in
 * [0, nbins): lcr[n] receives the positions 0..n-1 in ascending key order,
 * equal keys in ascending position; start[nbins + 1] the bin starts.  All
 * pointers are device memory; work has dsmc_counting_sort_bytes bytes.
 * Asynchronous on hip_stream.  Keys outside [0, nbins) are undefined
 * behaviour and must be excluded by the caller. */
dsmc_status dsmc_counting_sort(const int32_t *keys, int64_t n, int32_t nbins, int32_t *lcr, uint32_t *start,
                               void *work, size_t work_bytes, void *hip_stream);

/* Largest workspace (dsmc_counting_sort_bytes) dsmc_counting_sort_noalloc
 * accepts: 32 MiB, e.g. up to 67M keys with at most 2048 bins, or 2.6M keys
 * with up to 2^22 bins. */
#define DSMC_SORT_SCRATCH_BYTES ((size_t)32 << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * stable counting sort as dsmc_counting_sort, with the same arguments except
 * the workspace, computing the same lcr and start bit for bit.  Its workspace
 * is a static device array of DSMC_SORT_SCRATCH_BYTES that the library holds
 * on every GPU it runs on until the process ends; the call allocates nothing
 * (no hipMalloc, no allocating library routine).  Returns DSMC_ESIZE, before
 * anything is enqueued, when dsmc_counting_sort_bytes(n, nbins) exceeds
 * DSMC_SORT_SCRATCH_BYTES, DSMC_EINVAL for the argument errors of
 * dsmc_counting_sort, DSMC_EDEVICE when the array's address cannot be found
 * on the current device.  hip_stream must belong to the current device.
 * Asynchronous.  Every call on one GPU shares that GPU's array: calls whose
 * work overlaps on one GPU (two streams, or two host threads) race and give
 * undefined results; calls queued on one stream are ordered and safe. */
dsmc_status dsmc_counting_sort_noalloc(const int32_t *keys, int64_t n, int32_t nbins, int32_t *lcr,
                                       uint32_t *start, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* DSMC_H */
