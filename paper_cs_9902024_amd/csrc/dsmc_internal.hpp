// Internal declarations shared by the kernels and the host side of the DSMC
// library (gfx950).  Not part of the public C ABI (include/dsmc.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dsmc {

constexpr int kWave = 64;
constexpr int kWavesPerBlock = 4;          // 256-thread blocks
constexpr int kMaxGridBlocks = 1 << 23;    // workgroups per launch over items (2^31 work-items at 256 each;
                                           // a dispatch holds fewer than 2^32)
constexpr int kCollideWaves = 2;           // waves per block of the collide kernel
constexpr int kCollideCapF32 = 1280;       // particles staged in LDS per collide wavefront
constexpr int kCollideCapF64 = 1024;
constexpr int kWaveCapF32 = 384;           // particles staged in LDS per wavefront-per-cell item (a larger
                                           // stage fits fewer blocks per CU)
constexpr int kWaveCapF64 = 256;
constexpr int kLaneCapF32 = 640;           // particles staged in LDS per lane-per-cell wavefront
constexpr int kLaneCapF64 = 512;
constexpr int kDigitBits = 11;             // indexing digit: 2048 bins per pass
constexpr int kDigits = 1 << kDigitBits;
constexpr int kMaxWallHits = 64;           // wall interactions per particle per step
constexpr int kMaxGenAttempts = 1000;      // inflow normal-velocity rejection
// Motion writes only the new cell of a particle in free flight: Interaction,
// which gathers every particle anyway, applies its flight (the same
// expression) as it permutes the particles.  A particle that met a face was
// moved in place by the wall queue: its cell, and so its LCR entry, carries
// kMovedBit; the low 31 bits are the cell and the run-local slot.
constexpr uint32_t kMovedBit = 0x80000000u;
constexpr int32_t kSlotMask = 0x7FFFFFFF;
// Interaction also runs the next step's free-flight test on each particle it
// writes to P' (final position and velocity) and stores the cell the flight
// ends in, or kQueueBit when the particle must take the full flight (a face,
// or near a body).  Motion then reads that cell instead of the particle,
// except for particles generated since, which it tests itself.
constexpr int32_t kQueueBit = 0x40000000;
// Each inflow particle draws from its own stretch of its face element's
// stream, from uniform k * kGenUniforms for particle k, so particles do not
// depend on one another's rejections and are generated in parallel.  The
// 32-bit block counter bounds k below 2^21: runs expecting kMaxGenPerFace or
// more entrants per face element per step are refused.
constexpr uint32_t kGenUniforms = 4096;
constexpr double kMaxGenPerFace = 1048576.0;
static_assert(4 * kMaxGenAttempts + 5 <= (int)kGenUniforms, "a particle's draws must fit its stretch");
constexpr int kMaxInitAttempts = 100;      // initial position draws that land in solid cells
constexpr int kFields = 7;                 // N, sum u, v, w, u^2, v^2, w^2
constexpr int kMoments = 8;                // n, ux, uy, uz, T, Tx, Ty, Tz
constexpr int kDiag = 7;                   // particles, generated, collisions, sum u, v, w, |c|^2

// Philox counter word 1: what the stream is for.
enum : uint32_t { kInit = 0, kGen = 1, kWall = 2, kColl = 3 };
enum : int { kSpecular = 0, kDiffuse = 1, kInflow = 2, kOutflow = 3 };

// Device error codes (same values as the public status codes).
enum : int { kErrCapacity = -3, kErrBounce = -7, kErrReject = -8, kErrNumeric = -9 };
constexpr double kMaxSelections = 1e9;  // per cell per step; more means non-finite state
constexpr int kMaxLanes = 4;            // run groups stepped concurrently on their own streams
constexpr int kItemPlanes = 4;          // z planes per block of the 3-D interaction item order
constexpr double kWavePpc = 112.0;      // expected particles per cell from which a cell gets a wavefront
constexpr double kCrowdedPpc = 288.0;   // ... and from which it gets a whole block

// Per-run constants and layout, read by every kernel (AoS in device memory).
struct RunDev {
  int64_t so;        // first particle slot of the run
  int64_t cap;       // slots reserved (multiple of the tile)
  int64_t cap_spec;  // particle capacity the caller asked for (<= cap)
  int64_t co;        // first cell of the run in the global cell arrays (64-aligned)
  int64_t bo;        // first entry of the run in the bin-start array (nc + 2 entries)
  int64_t mo;        // first entry of the run in the tile histogram matrix
  int64_t cbo;       // first entry of the run in the digit-total array
  int64_t io;        // two-level Indexing: first bucket-item slot of the run
  int32_t nb;        // two-level Indexing: buckets (bins >> 11) of the run
  int32_t icap;      // two-level Indexing: bucket-item slots of the run (tiles + buckets)
  int64_t fo;        // first inflow face of the run
  int64_t n_init;
  int32_t to;        // first tile of the run
  int32_t nt;        // tiles of the run
  int32_t nc, nx, ny, nz;
  int32_t sub, S;    // collision partners from sub-cells: sub per axis, S = sub^dim per cell (1, 1 = none)
  int32_t nbin;      // Indexing bins: nc * S (a cell's S sub-cells consecutive); the DEAD bin is nbin
  int32_t nface;     // inflow face elements (0 without inflow)
  int32_t ndig;      // digits of the first indexing pass
  int32_t hs;        // hard sphere (omega == 0.5)
  int32_t coll_mode; // interaction work item: 0 lane_cells cells (a lane each), 1 one cell per
                     // wavefront, 2 one cell per block
  int32_t lane_cells;
  int32_t ahead;     // 1: Interaction writes each particle's next flight cell (kQueueBit) and
                     // Motion reads it; 0: Motion tests every particle itself
  int32_t bc[6];
  uint32_t key0, key1;   // Philox key: run id, seed
  double L[3], inv_d[3];
  double dt, coef, vhs_exp, c_ref, gmax0;
  double nbar_alpha;     // NTC count from N * Nbar / 2 with this running-mean weight (0: N(N-1)/2)
  double nbar0;          // start of the running mean: the expected count of the initial fill
  double face_T[6], face_sqrtT[6];
  double mbar, beta, s_inf, p_branch, inflow_sqrtT, dy, dz;
  double init_U[3], init_sqrtT;
  // voxel obstacle
  int32_t has_solid;     // any solid cell
  int32_t sb_lo[3], sb_hi[3];  // bounding box (cell indices, inclusive) of the solid cells
  int64_t sdo;           // first byte of the run's solid mask in the mask array
  double d[3];           // cell size per axis
  double solid_T, solid_sqrtT;
  // Motion's constants in both precisions, rounded once on the host (so a
  // kernel keeps them in scalar registers): dt, domain size, cells per unit
  // length, and the solid cells' bounding box widened by two cells
  float dt_f, L_f[3], inv_f[3], slo_f[3], shi_f[3];
  double slo[3], shi[3];
  double inv_bin[3];     // Indexing bins per unit length along each axis: cells, or sub-cells with
  float inv_bin_f[3];    // sub-cells (equal to inv_d without them)
  // the run's cell mask in device memory (null without solid cells): bit 0
  // the cell is solid, bit 1 a solid cell lies within two cells of it
  // (Chebyshev distance, the solid cells included)
  const uint8_t *mask;
};

constexpr uint8_t kMaskSolid = 1;
constexpr uint8_t kMaskNearSolid = 2;

// How an Interaction kernel's workgroups get their items (see the kernels).
enum : int32_t { kSchedGrid = 0, kSchedQueue = 1, kSchedPerRun = 2 };

struct Sched {
  int32_t mode;           // kSchedGrid, kSchedQueue or kSchedPerRun
  int32_t pad0;
  uint32_t *ctr;          // kSchedQueue: one counter per XCD; kSchedPerRun: one per run of the list
  const int64_t *first;   // kSchedPerRun: first item of each run of the list (nr + 1 entries)
  int32_t nr;             // kSchedPerRun: runs with items in the list
  int32_t pad;
};

template <typename real> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };
template <typename real> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

template <typename real>
__host__ __device__ inline typename Vec4<real>::type make_vec4(real a, real b, real c, real d) {
  typename Vec4<real>::type t;
  t.x = a;
  t.y = b;
  t.z = c;
  t.w = d;
  return t;
}

// One component of interleaved records seen as an array (S components per
// record).
template <typename real, int S = 4>
struct Strided {
  real *p;
  __host__ __device__ real &operator[](int64_t i) const { return p[S * i]; }
  __host__ __device__ Strided operator+(int64_t k) const { return Strided{p + S * k}; }
};

// The particle array P: per slot a record (x, y, u, v) and the rest, w in 2-D
// or the pair (z, w) in 3-D.  A particle that changed cell is gathered by
// Interaction from its old place: with the records it costs two cache lines
// instead of one per component.
template <typename real>
struct Particles {
  typename Vec4<real>::type *q;
  real *w;                        // 2-D
  typename Vec2<real>::type *zw;  // 3-D
  __host__ __device__ Strided<real> x() const { return Strided<real>{reinterpret_cast<real *>(q)}; }
  __host__ __device__ Strided<real> y() const { return Strided<real>{reinterpret_cast<real *>(q) + 1}; }
  __host__ __device__ Strided<real> u() const { return Strided<real>{reinterpret_cast<real *>(q) + 2}; }
  __host__ __device__ Strided<real> v() const { return Strided<real>{reinterpret_cast<real *>(q) + 3}; }
};

// Device pointers of one context, carved out of the caller's arena.
template <typename real>
struct DevPtrs {
  const RunDev *runs;
  const int32_t *tile_run;     // [n_tiles]
  const int32_t *face_run;     // [n_faces]
  const int32_t *cgroup_run;   // [n_cells_aligned / 64]
  const int32_t *inflow_runs;  // [n_inflow_runs]
  const int32_t *gen_blk;      // [n_inflow_runs + 1] first emission block of each inflow run
  const int32_t *eg_start;     // [n_eg + 1] CSR of runs per (ensemble, group)
  const int32_t *eg_runs;
  const int64_t *eg_acc;       // [n_eg + 1] offset (doubles) of each (ensemble, group) block
  const int32_t *eg_nc;        // [n_eg]
  const int32_t *sample_steps; // [n_samples]
  const int2 *items;           // [n_items] lane-per-cell interaction items: (run, first cell)
  const int2 *cell_items;      // [n_cell_items] block-per-cell interaction items: (run, cell)
  const int2 *wave_items;      // [n_wave_items] wavefront-per-cell interaction items: (run, cell)
  const uint8_t *solid;        // solid masks of the runs with obstacles (1 byte per cell)
  Particles<real> P[2];
  int32_t *cell;               // [slots] cell (bin) of each slot after Motion
  int32_t *lcr;                // [slots] run-local slot in cell order
  int32_t *lcr_tmp;            // [slots] previous indexing pass (multi-pass only)
  int32_t *key_tmp;            // [slots] bins carried between indexing passes (multi-pass only)
  uint32_t *hist;              // tile histograms, tile-major
  uint32_t *digit_tot;         // per run digit totals / digit starts
  uint32_t *bin_start;         // per run nc + 2 entries, run-local
  real *rem_c, *gmax;          // [cells]
  real *nbar;                  // [cells] running mean of the count (runs with nbar_alpha > 0)
  uint32_t *ncoll;             // [cells] cumulative accepted collisions
  double *rem_f;               // [faces]
  int32_t *gen_count;          // [faces] this step's first entrant of each face element (run-local)
  double *stage;               // [cells][7] per-run sample sums of one sample
  double *acc;                 // [n_samples][acc_stride]
  double *mom;                 // [2][max_nc][8]
  uint32_t *nsnap;             // [n_samples] snapshots accumulated in each sample slot
  uint32_t *sched_ctr;         // work counters of the persistent Interaction grids, zeroed every step
  const int64_t *sched_first;  // per interaction mode, the first item of each run with items in it
  double *diag;                // [runs][kDiag] per-run diagnostics (dsmc_get_diag)
  int32_t *n_alive;            // [runs]
  int32_t *n_sorted;           // [runs]
  int32_t *n_gen;              // [runs]
  uint32_t *step;              // device step counter
  int32_t *sample_slot;        // sample slot of the current step or -1
  int32_t *err;                // first device error (0 = none)
  uint32_t *wallq;             // [slots] per tile: run-local slots of particles that reach a face
  uint32_t *wallq_n;           // [tiles] queue length per tile
  // two-level Indexing (runs with 2049 .. 2^22 bins)
  int2 *bitem;                 // [bucket-item slots] (bucket, chunk), bucket -1 = unused slot
  const int32_t *bitem_run;    // [bucket-item slots] run of the slot
  int32_t *bfirst;             // [runs][2049] first item (run-local) of each bucket; [nb] = items
};

// The contiguous share of one stream lane: runs [r0, r1) and everything laid
// out per run in run order (tiles, inflow faces, inflow runs, interaction
// items).
struct LaneRange {
  int32_t r0, r1;    // runs
  int32_t t0, t1;    // tiles
  int64_t f0, f1;    // inflow faces
  int32_t i0, i1;    // entries of the inflow-run list
  int32_t g0, g1;    // emission blocks
  int64_t it0, it1;  // lane-per-cell interaction items
  int64_t ci0, ci1;  // block-per-cell interaction items
  int64_t wi0, wi1;  // wavefront-per-cell interaction items
  int32_t b0, b1;    // bucket-item slots (two-level Indexing)
  int32_t sr0[3], sr1[3];  // per interaction mode (lane, wave, cell items): the lane's runs in the mode's
                           // list of runs with items (persistent per-run scheduling)
};

struct Geometry {
  int dim;
  int fp64;
  int tile_chunks;       // 64-slot chunks per indexing tile
  int64_t tile;          // slots per tile
  int n_runs;
  int32_t n_tiles;
  int64_t n_slots;
  int64_t n_cells;       // aligned total
  int64_t n_faces;
  int32_t n_inflow_runs;
  int npass;             // indexing passes (1: digit = bin)
  int bucketed;          // two passes: high digit first, then the low digit within each bucket
  int32_t n_bitems;      // bucket-item slots
  int dstride;           // LDS words per wave for one histogram
  int max_nc;
  int max_nbin;          // Indexing bins of the largest run (cells times sub-cells)
  int n_eg;
  int64_t acc_stride;
  int n_samples;
  int window_steps;      // snapshots per sample slot (time window of a steady flow; 1 = one)
  int window_stride;     // steps between the snapshots of a window
  int64_t n_items;      // lane-per-cell interaction items (up to 64 cells each)
  int64_t n_cell_items; // block-per-cell interaction items
  int64_t n_wave_items; // wavefront-per-cell interaction items
  int collide_mode;      // 0 auto, 1 lane per cell, 2 wave per cell
  int any_solid;         // some run has solid cells (Motion checks paths against them)
  int any_sub;           // some run has sub-cells
  int n_lanes;           // run groups per step (1: everything on the caller's stream)
  int sched;             // Interaction work distribution: kSchedGrid, kSchedQueue or kSchedPerRun
  int sched_blocks[3];   // persistent grid (workgroups) per interaction mode (lane, wave, cell kernels)
  int64_t sched_first_off[3];  // offset of each mode's list of run starts in sched_first
  int64_t sched_ctr_off[3];    // offset of each mode's per-run counters in sched_ctr
  int64_t n_sched_ctr;   // counters in sched_ctr: [mode][lane][XCD] queue counters, then the per-run ones
  LaneRange lane[kMaxLanes];
};

// Streams and events of a step split over lanes.  Lane L waits for the fork
// (step counter advanced) and for lane L-1 to finish Motion, so one lane's
// Indexing and Interaction overlap the next lane's Motion; the caller's
// stream joins every lane before Sampling's accumulation.
struct LaneStreams {
  hipStream_t s[kMaxLanes];
  hipEvent_t fork;
  hipEvent_t moved[kMaxLanes];
  hipEvent_t done[kMaxLanes];
};

// Kernel kinds for per-kernel event timing (order = dsmc_kernel_name).
enum KernelKind : int {
  kKStepBegin, kKGenCount, kKGenEmit, kKMotion, kKMotionWalls, kKDigCount, kKColScan, kKDigScan, kKScatter,
  kKBinBounds, kKBinFinalize, kKCollide, kKCollideCell, kKAccumulate, kKSample, kKMoments, kKBucketItems,
  kKBucketScan, kKCollideWave, kNumKinds
};

// Optional hook around every launch (event timing); null = no hook.
struct Prof {
  void *user;
  void (*mark)(void *user, int kind, int begin, hipStream_t s);
};

// ---------------------------------------------------------------------------
// Kernel launchers (dsmc_kernels.hip)
// ---------------------------------------------------------------------------
template <typename real>
void launch_init(const Geometry &g, const DevPtrs<real> &d, hipStream_t s);
// The flight cells (see kQueueBit) of the live particles in slots
// [so, so + n) of buffer buf: after the initial fill, or after a run's state
// is replaced.
template <typename real>
void launch_next_cells(const Geometry &g, const DevPtrs<real> &d, int buf, int64_t so, int64_t n, hipStream_t s);
template <typename real>
void launch_step(const Geometry &g, const DevPtrs<real> &d, int buf, hipStream_t s, const LaneStreams *lanes,
                 const Prof *prof);
template <typename real>
void launch_sample(const Geometry &g, const DevPtrs<real> &d, int buf, int slot, hipStream_t s,
                   const Prof *prof);
template <typename real>
void launch_moments(const Geometry &g, const DevPtrs<real> &d, int slot, int eg0, int n_groups,
                    int nc, int n_runs_ens, hipStream_t s);
// Resident workgroups per CU of each Interaction kernel of this geometry
// (lane, wave, cell items), from the occupancy calculator.
void collide_occupancy(const Geometry &g, int out[3]);
// Per-run diagnostics of the particles in buffer buf into d.diag.
template <typename real>
void launch_diag(const Geometry &g, const DevPtrs<real> &d, int buf, hipStream_t s);

// Stand-alone stable counting sort of keys[0..n) into lcr (device pointers).
size_t counting_sort_workspace(int64_t n, int32_t nbins, int tile_chunks);
void launch_counting_sort(const int32_t *keys, int64_t n, int32_t nbins, int32_t *lcr,
                          uint32_t *start, void *work, int tile_chunks, hipStream_t s);

}  // namespace dsmc
