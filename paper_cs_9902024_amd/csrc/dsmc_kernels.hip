// HIP kernels of the unsteady-DSMC inner loop for gfx950 (MI355X).
//
// One time step follows the order of the sequential algorithm of Sec. 1.1 of
// the paper: Generation -> Motion (+Enumeration) -> Indexing (the LCR
// readdressing array) -> Interaction -> Sampling.  The paper's data
// parallelisation (Sec. 1.4: processor m takes elements m, m+p, m+2p, ... of
// the particle array P and of the cell array C) becomes contiguous, coalesced
// per-lane ownership of particles and cells; its parallel independent runs
// (Sec. 1.3) become many runs advanced by every launch.  The one step the paper
// runs sequentially (filling LCR, Sec. 1.4) is a parallel, stable counting sort
// here: a per-tile LDS digit histogram (fused into Motion), a column scan over
// tiles, a per-run digit scan, and a scatter whose within-tile ranks come from
// wavefront ballots, so the result equals the sequential stable order exactly.
//
// Every kernel reads the step number and the sample slot from device memory,
// so a whole step can be replayed from a HIP graph without host involvement.
#include "dsmc_internal.hpp"

#include <algorithm>
#include <type_traits>

namespace dsmc {

// ---------------------------------------------------------------------------
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) and conversions
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    // one 32x32->64 multiply gives both halves of each product
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x, p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
  }
  return c;
}

// Uniform in (0,1).  FP64: 52 bits from a word pair, centred.  FP32: 23 bits
// of the first word of the pair, centred.
template <typename real> __device__ __forceinline__ real u01(uint32_t a, uint32_t b);
template <> __device__ __forceinline__ double u01<double>(uint32_t a, uint32_t b) {
  const uint64_t m = ((uint64_t)a << 20) | (uint64_t)(b >> 12);
  return ((double)m + 0.5) * 0x1p-52;
}
template <> __device__ __forceinline__ float u01<float>(uint32_t a, uint32_t) {
  return ((float)(a >> 9) + 0.5f) * 0x1p-23f;
}

template <typename real> __device__ __forceinline__ real two_pi();
template <> __device__ __forceinline__ double two_pi<double>() { return 6.283185307179586476925286766559; }
template <> __device__ __forceinline__ float two_pi<float>() { return 6.2831853071795864769f; }

template <typename real> __device__ __forceinline__ real infinity();
template <> __device__ __forceinline__ double infinity<double>() { return __builtin_inf(); }
template <> __device__ __forceinline__ float infinity<float>() { return __builtin_inff(); }

// Stream of uniforms for one (key, step, purpose, index): uniform k comes from
// Philox block k/2 (counter word 3), words 2(k%2) and 2(k%2)+1.
template <typename real>
struct UStream {
  uint32_t k0, k1, c0, c1, c2;
  uint32_t next;
  uint32_t blk_id;
  uint4 blk;
  __device__ UStream(uint32_t key0, uint32_t key1, uint32_t step, uint32_t purpose, uint32_t idx)
      : k0(key0), k1(key1), c0(step), c1(purpose), c2(idx), next(0), blk_id(0xFFFFFFFFu) {}
  __device__ __forceinline__ void seek(uint32_t k) { next = k; }
  __device__ __forceinline__ real operator()() {
    const uint32_t b = next >> 1;
    if (b != blk_id) {
      blk = philox(make_uint4(c0, c1, c2, b), k0, k1);
      blk_id = b;
    }
    const bool hi = next & 1u;
    next++;
    return hi ? u01<real>(blk.z, blk.w) : u01<real>(blk.x, blk.y);
  }
};

template <typename real>
__device__ __forceinline__ void box_muller(real u1, real u2, real &n0, real &n1) {
  const real r = sqrt((real)-2 * log(u1));
  const real th = two_pi<real>() * u2;
  n0 = r * cos(th);
  n1 = r * sin(th);
}

// Latches a device error: the lowest code wins (deterministic whatever the
// order of the failures); a non-returning atomic, so no register waits on it.
__device__ __forceinline__ void set_error(int32_t *err, int code) { (void)atomicMin(err, code); }

// The wavefront's index in its block, as a wave-uniform (scalar) value, so
// that what is indexed by it (a tile, its run's constants) is read with
// scalar loads: a vector load would make the next wait for vector memory
// also wait for it.
__device__ __forceinline__ int wave_index() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Block index remapped so that each XCD (blocks are dealt round-robin over
// the 8 XCDs) works on one contiguous range of items: neighbouring cells read
// overlapping source ranges of P, and neighbouring tiles write into each
// other's ranges of the LCR, which then meet in the same L2.
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nblk) {
  const int64_t q = nblk / 8, rmd = nblk % 8;
  const int64_t x = b % 8, pos = b / 8;
  return x < rmd ? x * (q + 1) + pos : rmd * (q + 1) + (x - rmd) * q + pos;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <typename real>
__device__ __forceinline__ int32_t axis_index(real x, real inv, int32_t n) {
  const real f = floor(x * inv);
  if (!(f > (real)0)) return 0;
  if (f >= (real)(n - 1)) return n - 1;
  return (int32_t)f;
}

// sigma(c_r)/sigma_ref * c_r: hard sphere or VHS.
template <typename real, typename RunT>
__device__ __forceinline__ real g_of(const RunT &R, real cr) {
  if (R.hs) return cr;
  if (!(cr > (real)0)) return (real)0;
  return cr * pow(cr / (real)R.c_ref, (real)R.vhs_exp);
}

__device__ __forceinline__ int32_t blocks_for(int64_t n, int per) { return (int32_t)((n + per - 1) / per); }

// Run-local cell of a position (floor per axis, clamped to the grid).
template <typename real, int DIM>
__device__ __forceinline__ int32_t cell_of(const RunDev &R, const real (&pos)[3]) {
  const int32_t ix = axis_index(pos[0], (real)R.inv_d[0], R.nx);
  const int32_t iy = axis_index(pos[1], (real)R.inv_d[1], R.ny);
  const int32_t iz = (DIM == 3) ? axis_index(pos[2], (real)R.inv_d[2], R.nz) : 0;
  return (iz * R.ny + iy) * R.nx + ix;
}

// The Indexing bin of a position on the sub-cell grid (sub per axis): cell *
// S + (sz * sub + sy) * sub + sx, the cell being the sub-cell index divided
// by sub along each axis.  inv: sub-cells per unit length; n: cells per axis.
template <typename real, int DIM>
__device__ __forceinline__ int32_t subcell_bin(const real (&pos)[3], const real (&inv)[3], const int32_t (&n)[3],
                                               int32_t sub, int32_t S) {
  const int32_t fx = axis_index(pos[0], inv[0], n[0] * sub);
  const int32_t fy = axis_index(pos[1], inv[1], n[1] * sub);
  const int32_t fz = (DIM == 3) ? axis_index(pos[2], inv[2], n[2] * sub) : 0;
  const int32_t c = ((fz / sub) * n[1] + fy / sub) * n[0] + fx / sub;
  return c * S + ((fz % sub) * sub + fy % sub) * sub + fx % sub;
}

// The bin of a position: its cell, or its sub-cell with sub-cells.
template <typename real, int DIM>
__device__ __forceinline__ int32_t bin_of(const RunDev &R, const real (&pos)[3]) {
  if (R.sub == 1) return cell_of<real, DIM>(R, pos);
  const real inv[3] = {(real)R.inv_bin[0], (real)R.inv_bin[1], (real)R.inv_bin[2]};
  const int32_t n[3] = {R.nx, R.ny, R.nz};
  return subcell_bin<real, DIM>(pos, inv, n, R.sub, R.S);
}

// ---------------------------------------------------------------------------
// Initialisation
// ---------------------------------------------------------------------------

template <typename real>
__global__ __launch_bounds__(256) void k_init_cells(DevPtrs<real> d, int64_t n_cells) {
  for (int64_t gc = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; gc < n_cells;
       gc += (int64_t)gridDim.x * blockDim.x) {
    const RunDev &R = d.runs[d.cgroup_run[gc >> 6]];
    if (gc - R.co >= R.nc) continue;
    d.rem_c[gc] = (real)0;
    d.gmax[gc] = (real)R.gmax0;
    d.nbar[gc] = (real)R.nbar0;
    d.ncoll[gc] = 0;
  }
}

__global__ __launch_bounds__(256) void k_fill_f64(double *p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename real>
__global__ __launch_bounds__(256) void k_init_runs(DevPtrs<real> d, int n_runs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n_runs) {
    d.n_alive[r] = (int32_t)d.runs[r].n_init;
    d.n_sorted[r] = 0;
    d.n_gen[r] = 0;
  }
  if (r == 0) {
    *d.step = 0;
    *d.sample_slot = -1;
    *d.err = 0;
  }
}

// Uniform Maxwellian fill: slot i draws from (step 0, INIT, i).  Uniforms 0..3
// are two Box-Muller pairs for the velocity (last output unused), 4..6 the
// position, drawn again (7..9, ...) while it lies in a solid cell.
// z and w of slot i (z = 0 in 2-D), and their store.
template <int DIM, typename real>
__device__ __forceinline__ void load_zw(const Particles<real> &P, int64_t i, real &z, real &w) {
  if constexpr (DIM == 3) {
    const typename Vec2<real>::type t = P.zw[i];
    z = t.x;
    w = t.y;
  } else {
    z = (real)0;
    w = P.w[i];
  }
}
template <int DIM, typename real>
__device__ __forceinline__ void store_zw(const Particles<real> &P, int64_t i, real z, real w) {
  if constexpr (DIM == 3) {
    typename Vec2<real>::type t;
    t.x = z;
    t.y = w;
    P.zw[i] = t;
  } else {
    P.w[i] = w;
  }
}
// The w components from slot o on, as an array.
template <int DIM, typename real>
__device__ __forceinline__ Strided<real, DIM == 3 ? 2 : 1> w_view(const Particles<real> &P, int64_t o) {
  if constexpr (DIM == 3) return Strided<real, 2>{reinterpret_cast<real *>(P.zw) + 1} + o;
  else return Strided<real, 1>{P.w} + o;
}

template <typename real, int DIM>
__global__ __launch_bounds__(256) void k_init_particles(DevPtrs<real> d, int64_t n_slots, int64_t tile) {
  Particles<real> P = d.P[0];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_slots;
       i += (int64_t)gridDim.x * blockDim.x) {
    const RunDev &R = d.runs[d.tile_run[i / tile]];
    const int64_t loc = i - R.so;
    if (loc >= R.n_init) continue;
    UStream<real> s(R.key0, R.key1, 0u, kInit, (uint32_t)loc);
    const real a0 = s(), a1 = s(), a2 = s(), a3 = s();
    real n0, n1, n2, n3;
    box_muller(a0, a1, n0, n1);
    box_muller(a2, a3, n2, n3);
    const real st = (real)R.init_sqrtT;
    const real u0 = (real)R.init_U[0] + st * n0;
    const real v0 = (real)R.init_U[1] + st * n1;
    const real w0 = (real)R.init_U[2] + st * n2;
    real pos[3];
    for (int att = 0;; ++att) {
      if (att == kMaxInitAttempts) {
        set_error(d.err, kErrReject);
        break;
      }
      const real ux = s(), uy = s(), uz = s();
      pos[0] = ux * (real)R.L[0];
      pos[1] = uy * (real)R.L[1];
      pos[2] = DIM == 3 ? uz * (real)R.L[2] : (real)0;
      if (!R.has_solid || !(d.solid[R.sdo + cell_of<real, DIM>(R, pos)] & kMaskSolid)) break;
    }
    P.q[i] = make_vec4<real>(pos[0], pos[1], u0, v0);
    store_zw<DIM>(P, i, pos[2], w0);
  }
}

// ---------------------------------------------------------------------------
// Step bookkeeping
// ---------------------------------------------------------------------------

// Advances the step counter and finds the sample slot of the new step: slot
// k takes the snapshots after steps sample_steps[k] - j * stride, j = 0 ..
// window - 1 (one snapshot when window = 1; a time window of a steady flow
// otherwise).  Windows of different slots share no step (checked on the host).
__global__ void k_step_begin(uint32_t *step, int32_t *slot, const int32_t *sample_steps, int n_samples, int window,
                             int stride) {
  const uint32_t s = *step + 1u;
  *step = s;
  int k = -1;
  for (int i = 0; i < n_samples; ++i) {
    const int64_t back = (int64_t)sample_steps[i] - (int64_t)s;  // steps before the window's last snapshot
    if (sample_steps[i] >= 1 && back >= 0 && back % stride == 0 && back / stride < window) {
      k = i;
      break;
    }
  }
  *slot = k;
}

// ---------------------------------------------------------------------------
// Generation: drifting-Maxwellian inflow through the -x face
// ---------------------------------------------------------------------------

// One block per run with inflow: the number entering through each face
// element this step (the mean plus the carried remainder, rounded down),
// turned in place into each element's first entrant in the run's emission
// order (face order); then the capacity check and the run's new live count.
template <typename real>
__global__ __launch_bounds__(256) void k_gen_count(DevPtrs<real> d, int32_t i0) {
  __shared__ int64_t s_part[256];
  const int r = d.inflow_runs[i0 + blockIdx.x];
  const RunDev &R = d.runs[r];
  const int tid = threadIdx.x;
  int64_t carry = 0;
  for (int base = 0; base < R.nface; base += 256) {
    const int j = base + tid;
    int32_t cnt = 0;
    if (j < R.nface) {
      const double M = R.mbar + d.rem_f[R.fo + j];
      const double fl = floor(M);
      d.rem_f[R.fo + j] = M - fl;
      cnt = (int32_t)fl;
    }
    s_part[tid] = cnt;
    __syncthreads();
    // inclusive Hillis-Steele scan of 256 counts
    for (int o = 1; o < 256; o <<= 1) {
      const int64_t add = (tid >= o) ? s_part[tid - o] : 0;
      __syncthreads();
      s_part[tid] += add;
      __syncthreads();
    }
    // a start beyond 2^31 only arises when the capacity check below fails,
    // and then nothing is emitted
    if (j < R.nface) d.gen_count[R.fo + j] = (int32_t)(carry + s_part[tid] - cnt);
    carry += s_part[255];
    __syncthreads();
  }
  if (tid == 0) {
    const int64_t n0 = d.n_alive[r];
    if (n0 + carry <= R.cap_spec) {
      d.n_alive[r] = (int32_t)(n0 + carry);
      d.n_gen[r] = (int32_t)carry;
    } else {
      set_error(d.err, kErrCapacity);
      d.n_gen[r] = 0;
    }
  }
}

// Entrant k of face element j (drawing from uniform k * kGenUniforms of the
// element's stream for this step), written to slot o.
template <typename real, int DIM>
__device__ __forceinline__ void emit_one(const RunDev &R, uint32_t step, int32_t j, int32_t k, int64_t o,
                                         Particles<real> P, int32_t *err) {
  UStream<real> s(R.key0, R.key1, step, kGen, (uint32_t)j);
  s.seek((uint32_t)k * kGenUniforms);
  const real s_inf = (real)R.s_inf, p_branch = (real)R.p_branch, beta = (real)R.beta;
  // normal velocity: z = beta*u has density ~ z exp(-(z-s)^2), z > 0
  real z = 0;
  int att;
  for (att = 0; att < kMaxGenAttempts; ++att) {
    const real ub = s(), up = s(), uq = s(), ua = s();
    const real r = sqrt(-log(up));
    const real x = (ub < p_branch) ? ((uq < (real)0.5) ? -r : r) : r * cos(two_pi<real>() * uq);
    z = s_inf + x;
    if (z > (real)0 && ua < z / (s_inf + fabs(x))) break;
  }
  if (att == kMaxGenAttempts) {
    set_error(err, kErrReject);
    return;
  }
  const real u = z / beta;
  const real v1 = s(), v2 = s();
  real t0, t1;
  box_muller(v1, v2, t0, t1);
  const int32_t iy = j % R.ny, iz = j / R.ny;
  const real y = ((real)iy + s()) * (real)R.dy;
  real zc = 0;
  if (DIM == 3) zc = ((real)iz + s()) * (real)R.dz;
  const real ut = s();
  const real x0 = -(u * (real)R.dt) * ((real)1 - ut);
  const real st = (real)R.inflow_sqrtT;
  P.q[o] = make_vec4<real>(x0, y, u, st * t0);
  store_zw<DIM>(P, o, zc, st * t1);
}

// The last index in [lo, hi] whose start is <= t (start[lo] <= t).
__device__ __forceinline__ int32_t last_start_le(const int32_t *start, int32_t lo, int32_t hi, int64_t t) {
  while (lo < hi) {
    const int32_t mid = (lo + hi + 1) >> 1;
    if (start[mid] <= t) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Particle-parallel emission: the inflow runs own consecutive ranges of
// blocks (gen_blk, sized from each run's largest possible entrant count).
// A thread takes one entrant t of its run, finds its face element among the
// starts and writes it behind the run's live particles, in face order.
template <typename real, int DIM>
__global__ __launch_bounds__(256) void k_gen_emit(DevPtrs<real> d, int buf, int32_t i0, int32_t i1) {
  const int32_t b = d.gen_blk[i0] + (int32_t)blockIdx.x;
  const int32_t i = last_start_le(d.gen_blk, i0, i1 - 1, b);
  const int r = d.inflow_runs[i];
  const RunDev &R = d.runs[r];
  const int32_t total = d.n_gen[r];
  const int64_t t0 = (int64_t)(b - d.gen_blk[i]) * 256;
  if (t0 >= total) return;
  const int32_t *start = d.gen_count + R.fo;
  // the face elements of the block's first and last entrants bound every
  // thread's search
  const int32_t ja = last_start_le(start, 0, R.nface - 1, t0);
  const int32_t jb = last_start_le(start, ja, R.nface - 1, min<int64_t>(t0 + 255, total - 1));
  const int64_t t = t0 + threadIdx.x;
  if (t >= total) return;
  const int32_t j = last_start_le(start, ja, jb, t);
  const int64_t n0 = (int64_t)d.n_alive[r] - total;
  emit_one<real, DIM>(R, *d.step, j, (int32_t)(t - start[j]), R.so + n0 + t, d.P[buf], d.err);
}

// ---------------------------------------------------------------------------
// Motion + Enumeration
// ---------------------------------------------------------------------------

// Voxel obstacle: follows the straight path from pos (in cell vox) with
// velocity vel for a time tlim, crossing cell planes (k * d, k = 0..n) in time
// order, ties to the lower axis.  Returns the axis of the face of the first
// solid cell entered and its time in th, or -1 if none; vox follows the path
// up to that face (or up to tlim).
template <typename real, int DIM>
__device__ __forceinline__ int solid_walk(const RunDev &R, const uint8_t *solid, const real (&pos)[3],
                                          const real (&vel)[3], real tlim, int32_t (&vox)[3], real &th) {
  const int32_t n[3] = {R.nx, R.ny, R.nz};
  for (;;) {
    real tn = infinity<real>();
    int ax = -1;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      real t;
      if (vel[a] > (real)0) t = ((real)(vox[a] + 1) * (real)R.d[a] - pos[a]) / vel[a];
      else if (vel[a] < (real)0) t = ((real)vox[a] * (real)R.d[a] - pos[a]) / vel[a];
      else continue;
      if (t < tn) {
        tn = t;
        ax = a;
      }
    }
    if (ax < 0 || !(tn < tlim)) return -1;
    int32_t nv[3] = {vox[0], vox[1], vox[2]};
#pragma unroll
    for (int a = 0; a < DIM; ++a)
      if (a == ax) nv[a] += vel[a] > (real)0 ? 1 : -1;
    int32_t na = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a)
      if (a == ax) na = nv[a];
    if (na < 0 || na >= n[ax]) return -1;  // a domain face: not the walk's
    if (solid[R.sdo + ((int64_t)nv[2] * R.ny + nv[1]) * R.nx + nv[0]] & kMaskSolid) {
      th = tn > (real)0 ? tn : (real)0;
      return ax;
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) vox[a] = nv[a];
  }
}

// Neighbouring representable values of a finite x (IEEE bit patterns are
// ordered like the magnitudes they encode).
__device__ __forceinline__ double next_toward(double x, bool up) {
  if (x == 0.0) return up ? 0x1p-1074 : -0x1p-1074;
  const int64_t b = __double_as_longlong(x);
  return __longlong_as_double(((x > 0.0) == up) ? b + 1 : b - 1);
}
__device__ __forceinline__ float next_toward(float x, bool up) {
  if (x == 0.0f) return up ? 0x1p-149f : -0x1p-149f;
  const int32_t b = __float_as_int(x);
  return __int_as_float(((x > 0.0f) == up) ? b + 1 : b - 1);
}

// Coordinate x moved by rounding steps into cell i along an axis (cell size
// d, n cells): used when an end point rounds across the face of a solid cell
// next to the fluid cell its path ended in.
template <typename real>
__device__ __forceinline__ real snap_into(real x, int32_t i, real d, real inv, int32_t n) {
  if (axis_index(x, inv, n) > i) {
    x = (real)(i + 1) * d;
    while (axis_index(x, inv, n) > i) x = next_toward(x, false);
  } else {
    x = (real)i * d;
    while (axis_index(x, inv, n) < i) x = next_toward(x, true);
  }
  return x;
}

// Diffuse re-emission at temperature Tw (sqrt stw) from a surface with normal
// axis ax; side 1: the particle arrived moving +, so it leaves moving -.
// Uniforms 4h .. 4h+2 of the slot's WALL stream for the h-th wall interaction.
template <typename real>
__device__ __forceinline__ void diffuse_emit(const RunDev &R, uint32_t step, uint32_t slot, int hits, real Tw,
                                             real stw, int ax, int side, real (&vel)[3]) {
  UStream<real> ws(R.key0, R.key1, step, kWall, slot);
  ws.seek(4u * (uint32_t)hits);
  const real w0 = ws(), w1 = ws(), w2 = ws();
  const real vn = sqrt((real)-2 * Tw * log(w0));
  real n0, n1;
  box_muller(w1, w2, n0, n1);
  const int t1 = (ax == 0) ? 1 : 0, t2 = (ax == 2) ? 1 : 2;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (a == ax) vel[a] = side ? -vn : vn;
    else if (a == t1) vel[a] = stw * n0;
    else if (a == t2) vel[a] = stw * n1;
  }
}

// Moves one particle for dt (specular / diffuse / open faces, solid cells);
// returns the new cell, or nc (DEAD) when it leaves.  hit reports a velocity
// change, reemit a diffuse re-emission (w changed in 2-D).
template <typename real, int DIM>
__device__ __forceinline__ int32_t move_one(const RunDev &R, const uint8_t *solid, uint32_t step, uint32_t slot,
                                            real (&pos)[3], real (&vel)[3], bool &hit, bool &reemit,
                                            int32_t *err) {
  real L[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) L[a] = (real)R.L[a];
  real trem = (real)R.dt;
  int hits = 0;
  hit = false;
  reemit = false;
  int32_t vox[3] = {axis_index(pos[0], (real)R.inv_d[0], R.nx), axis_index(pos[1], (real)R.inv_d[1], R.ny),
                    DIM == 3 ? axis_index(pos[2], (real)R.inv_d[2], R.nz) : 0};
  for (;;) {
    real tmin = infinity<real>();
    int ax = -1, side = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      real th;
      int sd;
      if (vel[a] > (real)0) {
        th = (L[a] - pos[a]) / vel[a];
        sd = 1;
      } else if (vel[a] < (real)0) {
        th = ((real)0 - pos[a]) / vel[a];
        sd = 0;
      } else {
        continue;
      }
      if (th < (real)0) th = (real)0;
      if (th < tmin) {
        tmin = th;
        ax = a;
        side = sd;
      }
    }
    if (R.has_solid) {
      // a solid cell entered before the domain face (or the end of the step)
      real ts;
      const int sa = solid_walk<real, DIM>(R, solid, pos, vel, (ax < 0 || tmin >= trem) ? trem : tmin, vox, ts);
      if (sa >= 0) {
        int up = 0;
        real plane = (real)0;
#pragma unroll
        for (int a = 0; a < DIM; ++a)
          if (a == sa) {
            up = vel[a] > (real)0;
            plane = (real)(up ? vox[a] + 1 : vox[a]) * (real)R.d[a];
          }
#pragma unroll
        for (int a = 0; a < DIM; ++a) pos[a] = (a == sa) ? plane : pos[a] + vel[a] * ts;
        trem = trem - ts;
        hit = true;
        reemit = true;
        diffuse_emit<real>(R, step, slot, hits, (real)R.solid_T, (real)R.solid_sqrtT, sa, up, vel);
        if (++hits == kMaxWallHits) {
          set_error(err, kErrBounce);
          break;
        }
        continue;
      }
    }
    if (ax < 0 || tmin >= trem) {
#pragma unroll
      for (int a = 0; a < DIM; ++a) pos[a] = pos[a] + vel[a] * trem;
      break;
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) pos[a] = (a == ax) ? (side ? L[a] : (real)0) : pos[a] + vel[a] * tmin;
    trem = trem - tmin;
    const int f = 2 * ax + side;
    const int bc = R.bc[f];
    hit = true;
    if (bc == kSpecular) {
#pragma unroll
      for (int a = 0; a < DIM; ++a)
        if (a == ax) vel[a] = -vel[a];
    } else if (bc == kDiffuse) {
      reemit = true;
      diffuse_emit<real>(R, step, slot, hits, (real)R.face_T[f], (real)R.face_sqrtT[f], ax, side, vel);
    } else {
      return R.nbin;  // inflow plane crossed outward, or outflow
    }
    if (++hits == kMaxWallHits) {
      set_error(err, kErrBounce);
      break;
    }
  }
  if (pos[0] < (real)0) return R.nbin;  // generated upstream and never entered
  if (R.sub > 1) return bin_of<real, DIM>(R, pos);  // (no solid cells with sub-cells)
  int32_t c = cell_of<real, DIM>(R, pos);
  if (R.has_solid && (solid[R.sdo + c] & kMaskSolid)) {
    // rounding put the end point across the face of a solid cell: it belongs
    // to the fluid cell the path ended in
    const int32_t n[3] = {R.nx, R.ny, R.nz};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
      const real inv = (real)R.inv_d[a];
      if (axis_index(pos[a], inv, n[a]) != vox[a]) pos[a] = snap_into<real>(pos[a], vox[a], (real)R.d[a], inv, n[a]);
    }
    c = cell_of<real, DIM>(R, pos);
  }
  return c;
}

// Fast-path check for runs with solid cells, on coordinates: whether the
// bounding box of the straight flight from pos to out meets the bounding box
// of the solid cells widened by two cells on each side (lo, hi).  A flight
// that does not cannot enter a solid cell or end in one (the widening also
// covers the rounding of positions to cells); Motion sends the others to the
// wall queue, whose full flight (move_one) walks their cells.
template <typename real, int DIM>
__device__ __forceinline__ bool near_solid(const real (&pos)[3], const real (&out)[3], const real (&lo)[3],
                                           const real (&hi)[3]) {
  bool near = true;
#pragma unroll
  for (int a = 0; a < DIM; ++a) near = near && fmax(pos[a], out[a]) >= lo[a] && fmin(pos[a], out[a]) <= hi[a];
  return near;
}

// Free flight with no face reached this step, decided without divisions:
// the end point lies inside the box by a margin far above the rounding of the
// full face-time test, so both tests agree and the result is identical.
// A run constant in the state precision (both roundings are made on the host).
template <typename real> __device__ __forceinline__ real in_precision(double d, float f);
template <> __device__ __forceinline__ double in_precision<double>(double d, float) { return d; }
template <> __device__ __forceinline__ float in_precision<float>(double, float f) { return f; }

template <typename real> __device__ __forceinline__ real flight_margin_eps();
template <> __device__ __forceinline__ double flight_margin_eps<double>() { return 64.0 * 0x1p-53; }
template <> __device__ __forceinline__ float flight_margin_eps<float>() { return 64.0f * 0x1p-24f; }

template <typename real, int DIM>
__device__ __forceinline__ bool free_flight(real dt, const real (&L)[3], const real (&pos)[3], const real (&vel)[3],
                                            real (&out)[3]) {
  bool inside = true;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    out[a] = pos[a] + vel[a] * dt;
    const real m = flight_margin_eps<real>() * (L[a] + fabs(vel[a]) * dt);
    inside = inside && (pos[a] >= (real)0) && (pos[a] <= L[a]) && (out[a] >= m) && (out[a] <= L[a] - m);
  }
  return inside;
}

// A run's constants for Motion's test, in the state precision (rounded on
// the host), copied to registers once per loop: read through the run table
// inside a loop that stores, they would be read again for every particle.
template <typename real>
struct Flight {
  real dt, L[3], inv[3], slo[3], shi[3];
  int32_t n[3];
  bool solid;
  const uint8_t *mask;  // the run's cell mask (runs with solid cells)
  int32_t sub, S;  // sub-cells per axis and per cell (1, 1 without)
  Flight() = default;
  __device__ __forceinline__ explicit Flight(const RunDev &R) {
    dt = in_precision<real>(R.dt, R.dt_f);
    sub = R.sub;
    S = R.S;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      L[a] = in_precision<real>(R.L[a], R.L_f[a]);
      // the grid the flight's end is placed on: the cells, or the sub-cells
      // (one load, independent of sub)
      inv[a] = in_precision<real>(R.inv_bin[a], R.inv_bin_f[a]);
      slo[a] = in_precision<real>(R.slo[a], R.slo_f[a]);
      shi[a] = in_precision<real>(R.shi[a], R.shi_f[a]);
    }
    n[0] = R.nx;
    n[1] = R.ny;
    n[2] = R.nz;
    solid = R.has_solid;
    mask = R.mask;
  }
};

// Motion's test for one particle: the cell its free flight ends in, or
// kQueueBit when it must take the full flight (it reaches a face, or passes
// near a body).  Motion and Interaction's look-ahead both call this, so they
// decide identically.  SUB = false: a kernel instantiated for batches
// without sub-cells (no sub-cell code in its write-back).
template <typename real, int DIM, bool SUB = true>
__device__ __forceinline__ int32_t flight_cell(const Flight<real> &F, const real (&pos)[3], const real (&vel)[3]) {
  real out[3];
  bool fast = free_flight<real, DIM>(F.dt, F.L, pos, vel, out);
  if (F.solid && fast && near_solid<real, DIM>(pos, out, F.slo, F.shi)) {
    // near the body's box: still free if the flight moves at most one cell
    // along each axis from a cell with no solid cell within two cells (every
    // cell it touches, or its end rounds into, is then at least one cell
    // away from a solid one; runs with solid cells have no sub-cells, so the
    // bins are the cells)
    bool short_flight = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) short_flight = short_flight && fabs(out[a] - pos[a]) * F.inv[a] <= (real)1;
    const int32_t ix = axis_index(pos[0], F.inv[0], F.n[0]);
    const int32_t iy = axis_index(pos[1], F.inv[1], F.n[1]);
    const int32_t iz = (DIM == 3) ? axis_index(pos[2], F.inv[2], F.n[2]) : 0;
    fast = short_flight && !(F.mask[((int64_t)iz * F.n[1] + iy) * F.n[0] + ix] & kMaskNearSolid);
  }
  if (!fast) return kQueueBit;
  if constexpr (SUB) {
    if (F.sub > 1) return subcell_bin<real, DIM>(out, F.inv, F.n, F.sub, F.S);
  }
  const int32_t ix = axis_index(out[0], F.inv[0], F.n[0]);
  const int32_t iy = axis_index(out[1], F.inv[1], F.n[1]);
  const int32_t iz = (DIM == 3) ? axis_index(out[2], F.inv[2], F.n[2]) : 0;
  return (iz * F.n[1] + iy) * F.n[0] + ix;
}

// Adds 1 per active lane to h[key]: one LDS atomic per run of equal keys in
// consecutive active lanes (an inactive lane ends a run).
__device__ __forceinline__ void histogram_add(uint32_t *h, uint32_t key, bool active) {
  const int lane = threadIdx.x & 63;
  const uint32_t k = active ? key : 0xFFFFFFFFu;  // never equal to a live key
  const uint32_t prev = __shfl_up(k, 1);
  const bool boundary = !active || lane == 0 || prev != k;
  const uint64_t bm = __ballot(boundary);
  const uint64_t after = lane == 63 ? 0ull : (bm & ~((2ull << lane) - 1ull));
  const int nxt = after ? __ffsll((unsigned long long)after) - 1 : 64;
  if (active && boundary) atomicAdd(&h[key], (uint32_t)(nxt - lane));
}


template <typename real>
__device__ __forceinline__ void load4(const real *p, int64_t i, real (&o)[4]) {
  const typename Vec4<real>::type t = *reinterpret_cast<const typename Vec4<real>::type *>(p + i);
  o[0] = t.x; o[1] = t.y; o[2] = t.z; o[3] = t.w;
}
template <typename real>
__device__ __forceinline__ void store4(real *p, int64_t i, const real (&o)[4]) {
  typename Vec4<real>::type t;
  t.x = o[0]; t.y = o[1]; t.z = o[2]; t.w = o[3];
  *reinterpret_cast<typename Vec4<real>::type *>(p + i) = t;
}

// Wall-queue entries a Motion wavefront stages in LDS before writing them to
// the tile's queue: stores to global memory inside the round loop would also
// hold back the waits for the loads issued before them (one counter for
// vector loads and stores), so they go out in coalesced batches instead.
constexpr int kMotionQueueStage = 384;

// Moves the wavefront's staged queue entries qb[0, ql) to the tile's queue
// wq[qn, ...).
__device__ __forceinline__ void motion_flush(uint32_t *qb, uint32_t &ql, uint32_t *wq, uint32_t &qn) {
  const int lane = threadIdx.x & 63;
  for (uint32_t k = lane; k < ql; k += kWave) wq[qn + k] = qb[k];
  qn += ql;
  ql = 0;
  wave_sync();
}

// One round of Motion's counting: the new cell of every free particle into
// the tile histogram, the others (those that reach a face) into the staged
// wall queue, in slot order within the round; the stage goes out when the
// next round might not fit it.
__device__ __forceinline__ void motion_count(uint32_t *h, uint32_t *qb, uint32_t &ql, uint32_t *wq, uint32_t &qn,
                                             int64_t i0, const uint32_t (&key)[4], const bool (&fast)[4],
                                             const bool (&act)[4]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int e = 0; e < 4; ++e) histogram_add(h, key[e], fast[e]);
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const bool mine = act[e] && !fast[e];
    const uint64_t m = __ballot(mine);
    if (m == 0ull) continue;
    if (mine) qb[ql + __popcll(m & ((1ull << lane) - 1ull))] = (uint32_t)(i0 + e);
    ql += (uint32_t)__popcll(m);
  }
  if (ql > (uint32_t)(kMotionQueueStage - 4 * kWave)) motion_flush(qb, ql, wq, qn);
}

// A round whose four cells per lane the last Interaction left in place.
template <bool SINGLE>
__device__ __forceinline__ void motion_pre_round(uint32_t *h, uint32_t *qb, uint32_t &ql, uint32_t *wq, uint32_t &qn,
                                                 int64_t i0, int4 c4, int shift0) {
  const int32_t oc[4] = {c4.x, c4.y, c4.z, c4.w};
  const bool act[4] = {true, true, true, true};
  uint32_t key[4];
  bool fast[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    fast[e] = !(oc[e] & kQueueBit);
    key[e] = SINGLE ? (uint32_t)oc[e] : (((uint32_t)oc[e] >> shift0) & (kDigits - 1));
  }
  motion_count(h, qb, ql, wq, qn, i0, key, fast, act);
}

// One wavefront per tile of tile_chunks*64 consecutive slots of one run.
// Each round covers 256 slots, four consecutive ones per lane, read with
// 128-bit loads (only a run's last, partial round goes slot by slot).  The
// particles written by the last Interaction already have their cell (or the
// queue mark) in place: for them Motion reads only that.  The others (those
// generated this step) are tested here and their cell written.  No position
// is written: Interaction applies the flight when it moves every particle to
// its sorted place anyway.  The rounds whose cells are all in place come
// first in a tile; they are read four rounds at a time, so that each
// wavefront keeps four loads in flight.  Particles that reach a face go to the tile's wall
// queue (k_motion_walls).  The new cell of every free particle is counted in
// the tile's histogram of the first indexing digit, kept in wave-private LDS.
template <typename real, int DIM, bool SINGLE, bool OBST>
__global__ __launch_bounds__(256) void k_motion(DevPtrs<real> d, int buf, int32_t t0, int32_t t1, int64_t tile,
                                                int dstride, int shift0) {
  extern __shared__ uint32_t lds[];
  const int wave = wave_index(), lane = threadIdx.x & 63;
  const int t = t0 + (int)blockIdx.x * kWavesPerBlock + wave;
  if (t >= t1) return;
  const int r = d.tile_run[t];
  const RunDev &R = d.runs[r];
  const int64_t tl = t - R.to;
  const int D = R.ndig;
  uint32_t *h = lds + wave * dstride;
  uint32_t *qb = lds + kWavesPerBlock * dstride + wave * kMotionQueueStage;  // staged queue entries
  uint32_t ql = 0;
  for (int q = lane; q < D; q += kWave) h[q] = 0;
  wave_sync();
  const int64_t n = d.n_alive[r];
  const int64_t npre = R.ahead ? n - d.n_gen[r] : 0;  // cells in place from the last Interaction
  const int64_t begin = tl * tile, end = min(begin + tile, n);
  const typename Vec4<real>::type *__restrict__ Q = d.P[buf].q + R.so;
  const Particles<real> PP = d.P[buf];
  int32_t *__restrict__ cell = d.cell + R.so;
  uint32_t *__restrict__ wq = d.wallq + (int64_t)t * tile;  // this tile's queue segment
  uint32_t qn = 0;
  Flight<real> F(R);
  F.solid = OBST && R.has_solid;
  // rounds [begin, pre_end) have every cell in place (a tile is whole rounds)
  const int64_t pre_n = min(end, npre) - begin;
  const int64_t pre_end = begin + (pre_n > 0 ? pre_n / (4 * kWave) * (4 * kWave) : 0);
  constexpr int PU = 4;
  int64_t b = begin;
  for (; b + PU * 4 * kWave <= pre_end; b += PU * 4 * kWave) {
    int4 c4[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) c4[u] = *reinterpret_cast<const int4 *>(cell + b + u * 4 * kWave + 4 * lane);
#pragma unroll
    for (int u = 0; u < PU; ++u)
      motion_pre_round<SINGLE>(h, qb, ql, wq, qn, b + u * 4 * kWave + 4 * lane, c4[u], shift0);
  }
  for (; b < pre_end; b += 4 * kWave)
    motion_pre_round<SINGLE>(h, qb, ql, wq, qn, b + 4 * lane, *reinterpret_cast<const int4 *>(cell + b + 4 * lane),
                             shift0);
  for (; b < end; b += 4 * kWave) {
    const int64_t i0 = b + 4 * lane;
    const bool full = b + 4 * kWave <= end;  // wave-uniform
    int32_t oc[4];
    uint32_t key[4];
    bool fast[4];
    bool act[4];
    real px[4], py[4], pz[4], vx[4], vy[4], vz[4];
    if (full) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const typename Vec4<real>::type r4 = Q[i0 + e];
        px[e] = r4.x;
        py[e] = r4.y;
        vx[e] = r4.z;
        vy[e] = r4.w;
        act[e] = true;
      }
      if (DIM == 3)
#pragma unroll
        for (int e = 0; e < 4; ++e) load_zw<DIM>(PP, R.so + i0 + e, pz[e], vz[e]);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        act[e] = i0 + e < end;
        if (act[e]) {
          const typename Vec4<real>::type r4 = Q[i0 + e];
          px[e] = r4.x;
          py[e] = r4.y;
          vx[e] = r4.z;
          vy[e] = r4.w;
          if (DIM == 3) load_zw<DIM>(PP, R.so + i0 + e, pz[e], vz[e]);
        }
      }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      // in 2-D Motion never reads w: only a diffuse re-emission sets it
      const real pos[3] = {px[e], py[e], DIM == 3 ? pz[e] : (real)0};
      const real vel[3] = {vx[e], vy[e], DIM == 3 ? vz[e] : (real)0};
      const int32_t c = act[e] ? flight_cell<real, DIM>(F, pos, vel) : kQueueBit;
      fast[e] = act[e] && !(c & kQueueBit);
      oc[e] = c;
      key[e] = SINGLE ? (uint32_t)c : (((uint32_t)c >> shift0) & (kDigits - 1));
    }
    // (a queued particle's cell is rewritten by k_motion_walls)
    if (full) {
      *reinterpret_cast<int4 *>(cell + i0) = make_int4(oc[0], oc[1], oc[2], oc[3]);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e)
        if (act[e]) cell[i0 + e] = oc[e];
    }
    motion_count(h, qb, ql, wq, qn, i0, key, fast, act);
  }
  if (ql) motion_flush(qb, ql, wq, qn);
  if (lane == 0) d.wallq_n[t] = qn;
  wave_sync();
  uint32_t *Mt = d.hist + R.mo + tl * D;
  for (int q = lane; q < D; q += kWave) Mt[q] = h[q];
}

// The particles Motion queued because they reach a face this step (one block
// per tile): the full face-by-face flight (specular, diffuse, open faces) and
// their cells added to the tile histogram of the first indexing digit.
template <typename real, int DIM, bool SINGLE>
__global__ __launch_bounds__(256) void k_motion_walls(DevPtrs<real> d, int buf, int32_t t0, int32_t t1,
                                                      int64_t tile, int shift0) {
  const int32_t t = t0 + (int32_t)blockIdx.x;
  if (t >= t1) return;
  const uint32_t nq = d.wallq_n[t];
  if (nq == 0) return;
  const RunDev &R = d.runs[d.tile_run[t]];
  const uint32_t step = *d.step;
  const int D = R.ndig;
  uint32_t *Mt = d.hist + R.mo + (int64_t)(t - R.to) * D;
  const uint32_t *wq = d.wallq + (int64_t)t * tile;
  const Particles<real> P = d.P[buf];
  // every lane takes part in each round (the histogram adds are aggregated
  // over runs of equal digits across the wavefront)
  for (uint32_t i0 = 0; i0 < nq; i0 += blockDim.x) {
    const uint32_t i = i0 + threadIdx.x;
    const bool active = i < nq;
    uint32_t key = 0;
    if (active) {
      const int64_t loc = wq[i];
      const int64_t gs = R.so + loc;
      const typename Vec4<real>::type r4 = P.q[gs];
      real z0, w0;
      load_zw<DIM>(P, gs, z0, w0);
      real p3[3] = {r4.x, r4.y, z0};
      real v3[3] = {r4.z, r4.w, DIM == 3 ? w0 : (real)0};
      bool hit = false, reemit = false;
      // a non-finite coordinate or velocity fails Motion's free-flight test
      // and so arrives here: report it and remove the particle
      const bool finite = isfinite(r4.x) && isfinite(r4.y) && isfinite(z0) && isfinite(r4.z) && isfinite(r4.w) &&
                          isfinite(w0);
      if (!finite) set_error(d.err, kErrNumeric);
      const int32_t c =
          finite ? move_one<real, DIM>(R, d.solid, step, (uint32_t)loc, p3, v3, hit, reemit, d.err) : R.nbin;
      // (the velocity is unchanged unless a face was hit)
      P.q[gs] = make_vec4<real>(p3[0], p3[1], v3[0], v3[1]);
      if (DIM == 3) store_zw<DIM>(P, gs, p3[2], v3[2]);
      else if (hit && reemit) P.w[gs] = v3[2];
      d.cell[gs] = (int32_t)((uint32_t)c | kMovedBit);  // moved here, not by Interaction
      key = SINGLE ? (uint32_t)c : (((uint32_t)c >> shift0) & (kDigits - 1));
    }
    histogram_add(Mt, key, active);
  }
}

// ---------------------------------------------------------------------------
// Indexing: stable counting sort (LSD over 11-bit digits when a run has more
// than 2048 bins)
// ---------------------------------------------------------------------------

struct IndexArgs {
  const RunDev *runs;
  const int32_t *tile_run;
  const int32_t *cell;     // bin of each slot (slot order)
  const int32_t *in;       // previous pass order (run-local slots) or null: identity
  int32_t *out;            // this pass' order
  const int32_t *kin;      // bins in the order of `in` (carried from the previous pass), or null:
                           // read cell[in[k]]
  int32_t *kout;           // bins in the order of `out`, or null
  uint32_t *hist;          // tile histograms, tile-major: [tile][digit]
  uint32_t *tot;           // per run digit totals -> digit starts
  uint32_t *bin_start;     // per run nbin + 2 bin starts (single pass / bounds)
  int32_t *n_sorted;
  int32_t *n_alive;
  int32_t t0, t1;          // tiles [t0, t1)
  int32_t r0;              // first run (grid y / x of the per-run scans)
  int64_t tile;
  int dstride;
  int shift;               // digit = (bin >> shift) & (kDigits - 1), unless single
  int single;
  // second pass of the two-level sort: work items = chunks of `tile`
  // positions of one bucket (the positions whose bins share bin >> 11)
  int2 *bitem;             // (bucket, chunk) per item slot, bucket -1 = unused
  const int32_t *bitem_run;
  int32_t *bfirst;         // per run kDigits + 1: first item (run-local) of each bucket
  int32_t b0, b1;          // item slots [b0, b1)
};

__device__ __forceinline__ uint32_t digit_of(int32_t bin, int shift, bool single) {
  return single ? (uint32_t)bin : (((uint32_t)bin >> shift) & (kDigits - 1));
}

// Tile histogram of one digit over an existing order (passes after the first,
// and the stand-alone sort).
__global__ __launch_bounds__(256) void k_digcount(IndexArgs a, int use_n_alive) {
  extern __shared__ uint32_t lds[];
  const int wave = wave_index(), lane = threadIdx.x & 63;
  const int t = a.t0 + (int)blockIdx.x * kWavesPerBlock + wave;
  if (t >= a.t1) return;
  const int r = a.tile_run[t];
  const RunDev &R = a.runs[r];
  const int64_t tl = t - R.to;
  const bool single = a.single;
  const int D = R.ndig;
  uint32_t *h = lds + wave * a.dstride;
  for (int q = lane; q < D; q += kWave) h[q] = 0;
  wave_sync();
  const int64_t n = use_n_alive ? a.n_alive[r] : a.n_sorted[r];
  const int64_t begin = tl * a.tile, end = min(begin + a.tile, n);
  if (a.kin) {
    // carried bins: a sequential read, 4 consecutive per lane
    const int32_t *__restrict__ kin = a.kin + R.so;
    for (int64_t b = begin; b < end; b += 4 * kWave) {
      const int64_t i0 = b + 4 * lane;
      if (b + 4 * kWave <= end) {
        const int4 k4 = *reinterpret_cast<const int4 *>(kin + i0);
        atomicAdd(&h[digit_of(k4.x, a.shift, single)], 1u);
        atomicAdd(&h[digit_of(k4.y, a.shift, single)], 1u);
        atomicAdd(&h[digit_of(k4.z, a.shift, single)], 1u);
        atomicAdd(&h[digit_of(k4.w, a.shift, single)], 1u);
      } else {
        for (int e = 0; e < 4; ++e)
          if (i0 + e < end) atomicAdd(&h[digit_of(kin[i0 + e], a.shift, single)], 1u);
      }
    }
  } else {
    for (int64_t b = begin; b < end; b += kWave) {
      const int64_t loc = b + lane;
      if (loc < end) {
        const int32_t v = (a.in ? a.in[R.so + loc] : (int32_t)loc) & kSlotMask;
        atomicAdd(&h[digit_of(a.cell[R.so + v] & kSlotMask, a.shift, single)], 1u);
      }
    }
  }
  wave_sync();
  uint32_t *Mt = a.hist + R.mo + tl * D;
  for (int q = lane; q < D; q += kWave) Mt[q] = h[q];
}

// Per (run, digit): exclusive scan of the digit's counts over the run's tiles
// (in place) and the digit total.  Coalesced across digits.
__global__ __launch_bounds__(256) void k_colscan(IndexArgs a) {
  const RunDev &R = a.runs[a.r0 + blockIdx.y];
  const int D = R.ndig;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= D) return;
  uint32_t *col = a.hist + R.mo + q;
  // one block per 256 digits of a run gives few wavefronts on a large grid,
  // so each lane keeps 32 rows' loads in flight where it can
  uint32_t sum = 0;
  int t = 0;
  for (; t + 32 <= R.nt; t += 32) {
    uint32_t v[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) v[k] = col[(int64_t)(t + k) * D];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      col[(int64_t)(t + k) * D] = sum;
      sum += v[k];
    }
  }
  for (; t + 8 <= R.nt; t += 8) {
    uint32_t v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = col[(int64_t)(t + k) * D];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      col[(int64_t)(t + k) * D] = sum;
      sum += v[k];
    }
  }
  for (; t < R.nt; ++t) {
    const uint32_t v = col[(int64_t)t * D];
    col[(int64_t)t * D] = sum;
    sum += v;
  }
  a.tot[R.cbo + q] = sum;
}

// One block per run: exclusive scan of the digit totals -> digit starts.  With
// a single pass the digits are the bins: also the run's bin starts and its
// live count (everything before the DEAD bin).
__global__ __launch_bounds__(256) void k_digscan(IndexArgs a) {
  __shared__ uint32_t s[256];
  const int r = a.r0 + (int)blockIdx.x;
  const RunDev &R = a.runs[r];
  const bool single = a.single;
  const int D = R.ndig;
  uint32_t *tot = a.tot + R.cbo;
  const int per = (D + 255) / 256;  // <= 8
  const int tid = threadIdx.x;
  const int q0 = tid * per;
  uint32_t v[8];
  uint32_t local = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    v[k] = (k < per && q0 + k < D) ? tot[q0 + k] : 0u;
    local += v[k];
  }
  s[tid] = local;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const uint32_t add = (tid >= o) ? s[tid - o] : 0u;
    __syncthreads();
    s[tid] += add;
    __syncthreads();
  }
  uint32_t run = s[tid] - local;
  const uint32_t total = s[255];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (k < per && q0 + k < D) {
      tot[q0 + k] = run;
      if (single) {
        a.bin_start[R.bo + q0 + k] = run;
        if (q0 + k == R.nbin) a.n_alive[r] = (int32_t)run;  // everything before the DEAD bin
      }
      run += v[k];
    }
  }
  if (tid == 0) {
    a.n_sorted[r] = (int32_t)total;
    if (single) a.bin_start[R.bo + R.nbin + 1] = total;
  }
}

// ---------------------------------------------------------------------------
// Two-level sort (2049 .. 2^22 bins): the first pass orders the positions by
// bucket (bin >> 11) with the tile machinery above; the second sorts every
// bucket by its low digit.  Its work items are chunks of `tile` positions of
// one bucket, listed per run by k_bucket_items.  Each bucket's digit starts
// are the bin starts of its 2048 cells, so no bin bounds pass is needed.
// ---------------------------------------------------------------------------

// End of bucket h's positions [A_h, A_{h+1}) in run r: A_h are the first
// pass' digit starts, the last bucket ends at the run's count.
__device__ __forceinline__ int64_t bucket_end(const IndexArgs &a, const RunDev &R, int r, int h) {
  return h + 1 < R.nb ? (int64_t)a.tot[R.cbo + h + 1] : (int64_t)a.n_sorted[r];
}

// Run, bucket and position range of bucket item slot i; false for an unused slot.
__device__ __forceinline__ bool bucket_item(const IndexArgs &a, int32_t i, int &r, int &h, int64_t &begin,
                                            int64_t &end) {
  const int2 hk = a.bitem[i];
  if (hk.x < 0) return false;
  r = a.bitem_run[i];
  const RunDev &R = a.runs[r];
  h = hk.x;
  begin = (int64_t)a.tot[R.cbo + h] + (int64_t)hk.y * a.tile;
  end = min(begin + a.tile, bucket_end(a, R, r, h));
  return true;
}

// Exclusive scan of one value per thread across a 256-thread block.
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t *part) {
  const int tid = threadIdx.x;
  part[tid] = v;
  __syncthreads();
  for (int o = 1; o < 256; o <<= 1) {
    const int64_t add = tid >= o ? part[tid - o] : 0;
    __syncthreads();
    part[tid] += add;
    __syncthreads();
  }
  const int64_t incl = part[tid];
  __syncthreads();
  return incl - v;
}

// One block per run: the bucket items (bucket, chunk) of the run in bucket
// order, each bucket's first item, and -1 in the run's unused item slots.
__global__ __launch_bounds__(256) void k_bucket_items(IndexArgs a) {
  __shared__ int64_t part[256];
  const int r = a.r0 + (int)blockIdx.x;
  const RunDev &R = a.runs[r];
  const int tid = threadIdx.x;
  const int per = (R.nb + 255) / 256;  // <= 8
  const int h0 = tid * per;
  int32_t nch[8];
  int64_t sum = 0;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int h = h0 + e;
    int32_t c = 0;
    if (e < per && h < R.nb) {
      const int64_t size = bucket_end(a, R, r, h) - (int64_t)a.tot[R.cbo + h];
      c = (int32_t)((size + a.tile - 1) / a.tile);
    }
    nch[e] = c;
    sum += c;
  }
  const int64_t excl = block_exclusive_scan(sum, part);
  int32_t first = (int32_t)excl;
  int32_t *bf = a.bfirst + (int64_t)r * (kDigits + 1);
  int2 *items = a.bitem + R.io;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int h = h0 + e;
    if (e < per && h < R.nb) {
      bf[h] = first;
      for (int32_t k = 0; k < nch[e]; ++k) items[first + k] = make_int2(h, k);
      first += nch[e];
    }
  }
  const int32_t total = (int32_t)(part[255]);  // inclusive sum of the last thread
  if (tid == 0) bf[R.nb] = total;
  for (int32_t i = total + tid; i < R.icap; i += 256) items[i] = make_int2(-1, 0);
}

// Low-digit histogram of one bucket item (one wavefront per item slot).
__global__ __launch_bounds__(256) void k_digcount_bucket(IndexArgs a) {
  extern __shared__ uint32_t lds[];
  constexpr int U = 8;
  const int wave = wave_index(), lane = threadIdx.x & 63;
  const int32_t i = a.b0 + (int)blockIdx.x * kWavesPerBlock + wave;
  if (i >= a.b1) return;
  int r, h;
  int64_t begin, end;
  if (!bucket_item(a, i, r, h, begin, end)) return;
  const RunDev &R = a.runs[r];
  uint32_t *hs = lds + wave * kDigits;
  for (int q = lane; q < kDigits; q += kWave) hs[q] = 0;
  wave_sync();
  const int32_t *__restrict__ kin = a.kin + R.so;
  for (int64_t b = begin; b < end; b += U * kWave) {
    int32_t k[U];
#pragma unroll
    for (int e = 0; e < U; ++e) k[e] = kin[min(b + e * kWave + lane, end - 1)];
#pragma unroll
    for (int e = 0; e < U; ++e) histogram_add(hs, (uint32_t)k[e] & (kDigits - 1), b + e * kWave + lane < end);
  }
  wave_sync();
  uint32_t *M = a.hist + (int64_t)i * kDigits;
  for (int q = lane; q < kDigits; q += kWave) M[q] = hs[q];
}

// One block per (bucket, run): for every low digit, the counts of the
// bucket's earlier items in place of its item counts (a scan down the
// column) and its total; the totals' exclusive scan over the digits, from the
// bucket's first position, gives the bin starts of the bucket's cells.
__global__ __launch_bounds__(256) void k_bucket_scan(IndexArgs a) {
  __shared__ uint32_t col[kDigits];
  __shared__ int64_t part[256];
  const int r = a.r0 + (int)blockIdx.y;
  const RunDev &R = a.runs[r];
  const int h = (int)blockIdx.x;
  if (h >= R.nb) return;
  const int tid = threadIdx.x;
  const int32_t *bf = a.bfirst + (int64_t)r * (kDigits + 1);
  const int64_t f0 = R.io + bf[h], f1 = R.io + bf[h + 1];
  uint32_t s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t it = f0; it < f1; ++it) {
    uint32_t *M = a.hist + it * kDigits;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int q = tid + 256 * e;
      const uint32_t v = M[q];
      M[q] = s[e];
      s[e] += v;
    }
  }
#pragma unroll
  for (int e = 0; e < 8; ++e) col[tid + 256 * e] = s[e];
  __syncthreads();
  // digits 8 tid .. 8 tid + 7 are this thread's in the scan
  uint32_t v[8];
  int64_t sum = 0;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    v[e] = col[8 * tid + e];
    sum += v[e];
  }
  int64_t run = block_exclusive_scan(sum, part) + (int64_t)a.tot[R.cbo + h];
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    col[8 * tid + e] = (uint32_t)run;
    run += v[e];
  }
  __syncthreads();
  const int64_t c0 = (int64_t)h << kDigitBits;
  uint32_t *bs = a.bin_start + R.bo + c0;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int q = tid + 256 * e;
    if (c0 + q <= R.nbin) bs[q] = col[q];
  }
}

// A wave's cursor table: cursor[q] = S[q] + M[q] for q < min(D, valid), 0 for
// the rest of [0, D).  Eight loads of each source per lane are issued before
// the first is stored, so the table's set-up is not one memory latency per
// 64 entries.
__device__ __forceinline__ void init_cursors(uint32_t *cursor, const uint32_t *S, const uint32_t *M, int D,
                                             int64_t valid) {
  constexpr int B = 8;
  const int lane = threadIdx.x & 63;
  // loads from an index clamped into [0, lim) and no condition around them:
  // a load inside a branch is waited for at the branch's join, which would
  // serialise the eight
  const int lim = (int)(valid < (int64_t)D ? valid : (int64_t)D);  // >= 1
  for (int q0 = 0; q0 < D; q0 += B * kWave) {
    uint32_t v[B];
#pragma unroll
    for (int e = 0; e < B; ++e) {
      const int q = q0 + e * kWave + lane;
      const int qc = q < lim ? q : lim - 1;
      v[e] = S[qc] + M[qc];
    }
#pragma unroll
    for (int e = 0; e < B; ++e) {
      const int q = q0 + e * kWave + lane;
      if (q >= lim) v[e] = 0u;
    }
#pragma unroll
    for (int e = 0; e < B; ++e) {
      const int q = q0 + e * kWave + lane;
      if (q < D) cursor[q] = v[e];
    }
  }
}

// Rank of each lane among the active lanes holding the same digit (lanes
// below it) and the size of that group, from one ballot per distinct digit
// present.  Inactive lanes hold kNoDigit.
constexpr uint32_t kNoDigit = 0xFFFFFFFFu;

__device__ __forceinline__ void rank_in_wave(uint32_t key, uint64_t rest, uint32_t &rank, uint32_t &cnt) {
  // each lane keeps the ballot of its digit (a select, no branch: the loop
  // costs a few scalar and vector instructions per distinct digit)
  uint64_t peers = 0;
  while (rest) {
    const int leader = (int)__builtin_ctzll(rest);
    const uint32_t dl = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
    const bool same = key == dl;
    const uint64_t pm = __builtin_amdgcn_ballot_w64(same);
    peers = same ? pm : peers;
    rest &= ~pm;
  }
  rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(peers >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
  cnt = (uint32_t)__popcll(peers);
}

// One wavefront per tile, 64 consecutive positions per round in order: the
// rank of a position among equal digits is (digit start) + (count in earlier
// tiles) + (count in earlier rounds of this tile) + (earlier lanes with the
// same digit, from ballots).  That is exactly the sequential stable order.
// The first two terms are summed into the wave's LDS cursor table up front.
// CARRIED: positions and bins come from the previous pass (a.in, a.kin);
// otherwise the positions are the slots and the bins are read from cell[].
// KOUT: the bins are also written to a.kout in the output order, so the next
// pass and the bin bounds read them sequentially.
// BUCKETED: the second pass of the two-level sort; the wave's work is a bucket
// item (a chunk of one bucket's positions) and its cursors are the bin starts
// of the bucket's cells plus the counts of earlier chunks of the bucket.
// The sources are read sequentially with no per-lane condition, and the next
// chunk's reads are issued before the current chunk is ranked, so their
// latency overlaps the ranking; the ragged last chunk is handled apart.
template <bool KOUT, bool CARRIED, bool BUCKETED>
__global__ __launch_bounds__(256) void k_scatter(IndexArgs a) {
  extern __shared__ uint32_t lds[];
  constexpr int U = 16;
  constexpr int CH = U * kWave;
  const int wave = wave_index(), lane = threadIdx.x & 63;
  const bool single = a.single;
  const int shift = a.shift;
  uint32_t *cursor = lds + wave * a.dstride;
  int r;
  int64_t begin, end;
  const int blk = (int)xcd_block(blockIdx.x, gridDim.x);
  if (BUCKETED) {
    const int32_t i = a.b0 + blk * kWavesPerBlock + wave;
    if (i >= a.b1) return;
    int h;
    if (!bucket_item(a, i, r, h, begin, end)) return;
    const RunDev &R = a.runs[r];
    const uint32_t *M = a.hist + (int64_t)i * kDigits;
    const int64_t c0 = (int64_t)h << kDigitBits;
    const uint32_t *S = a.bin_start + R.bo + c0;
    const int64_t last = R.nbin - c0;  // digits beyond are no bins of the run
    init_cursors(cursor, S, M, kDigits, last + 1);
  } else {
    const int t = a.t0 + blk * kWavesPerBlock + wave;
    if (t >= a.t1) return;
    r = a.tile_run[t];
    const RunDev &R = a.runs[r];
    const int64_t tl = t - R.to;
    const int D = R.ndig;
    const uint32_t *Mt = a.hist + R.mo + tl * D;
    const uint32_t *S = a.tot + R.cbo;
    init_cursors(cursor, S, Mt, D, D);
    begin = tl * a.tile;
    end = min(begin + a.tile, (int64_t)a.n_sorted[r]);
  }
  wave_sync();
  if (begin >= end) return;
  const RunDev &R = a.runs[r];
  const uint64_t all = ~0ull;
  const int32_t *__restrict__ src_v = CARRIED ? a.in + R.so : nullptr;
  const int32_t *__restrict__ src_b = CARRIED ? a.kin + R.so : a.cell + R.so;
  int32_t *__restrict__ out = a.out + R.so;
  int32_t *__restrict__ kout = KOUT ? a.kout + R.so : nullptr;
  const int64_t nfull = (end - begin) / CH;
  const int64_t full_end = begin + nfull * CH;
  int32_t nv[U], nb[U];
  // reads of the chunk at b, clamped into the tile so they never branch
#define SCATTER_LOAD(b)                                        \
  _Pragma("unroll") for (int q = 0; q < U; ++q) {              \
    const int64_t loc = min((b) + q * kWave + lane, end - 1);  \
    nb[q] = src_b[loc];                                        \
    if (CARRIED) nv[q] = src_v[loc];                           \
  }
  SCATTER_LOAD(begin);
  for (int64_t b = begin; b < full_end; b += CH) {
    int32_t v[U], bin[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      // a first pass reads Motion's cells: their moved bit goes with the slot
      v[q] = CARRIED ? nv[q] : (int32_t)(b + q * kWave + lane) | (nb[q] & ~kSlotMask);
      bin[q] = CARRIED ? nb[q] : nb[q] & kSlotMask;
    }
    SCATTER_LOAD(b + CH);
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const uint32_t key = digit_of(bin[q], shift, single);
      uint32_t rank, cnt;
      rank_in_wave(key, all, rank, cnt);
      const uint32_t prior = cursor[key];
      out[prior + rank] = v[q];
      if (KOUT) kout[prior + rank] = bin[q];
      if (rank == cnt - 1) cursor[key] = prior + cnt;
      wave_sync();
    }
  }
#undef SCATTER_LOAD
  if (full_end < end) {
    // the ragged last chunk: its reads were issued by the last full chunk
    // (or before the loop)
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int64_t loc = full_end + q * kWave + lane;
      const bool act = loc < end;
      const int32_t bn = CARRIED ? nb[q] : nb[q] & kSlotMask;
      const uint32_t key = act ? digit_of(bn, shift, single) : kNoDigit;
      uint32_t rank, cnt;
      rank_in_wave(key, __builtin_amdgcn_ballot_w64(act), rank, cnt);
      if (act) {
        const uint32_t prior = cursor[key];
        out[prior + rank] = CARRIED ? nv[q] : (int32_t)loc | (nb[q] & ~kSlotMask);
        if (KOUT) kout[prior + rank] = bn;
        if (rank == cnt - 1) cursor[key] = prior + cnt;
      }
      wave_sync();
    }
  }
}

// Bin starts from the final order (multi-pass): position p starts every bin in
// (bin(p-1), bin(p)].  sorted[] holds the bin at each sorted position (the
// keys the last pass carried).  One wavefront per tile of tiles [a.t0, a.t1),
// four consecutive positions per lane.
__global__ __launch_bounds__(256) void k_bin_bounds(IndexArgs a, const int32_t *sorted) {
  const int wave = wave_index(), lane = threadIdx.x & 63;
  const int t = a.t0 + (int)blockIdx.x * kWavesPerBlock + wave;
  if (t >= a.t1) return;
  const int r = a.tile_run[t];
  const RunDev &R = a.runs[r];
  const int64_t n = a.n_sorted[r];
  const int64_t begin = (int64_t)(t - R.to) * a.tile, end = min(begin + a.tile, n);
  const int32_t *__restrict__ key = sorted + R.so;
  uint32_t *__restrict__ bs = a.bin_start + R.bo;
  for (int64_t b = begin; b < end; b += 4 * kWave) {
    const int64_t i0 = b + 4 * lane;
    int32_t k[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) k[e] = i0 + e < end ? key[i0 + e] : 0;
    int32_t prev = __shfl_up(k[3], 1);
    if (lane == 0) prev = b > 0 ? key[b - 1] : -1;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t loc = i0 + e;
      if (loc >= end) break;
      for (int32_t q = prev + 1; q <= k[e]; ++q) bs[q] = (uint32_t)loc;
      if (loc == n - 1)
        for (int32_t q = k[e] + 1; q <= R.nbin + 1; ++q) bs[q] = (uint32_t)n;
      prev = k[e];
    }
  }
}

__global__ void k_bin_finalize(IndexArgs a, int r1, int set_alive) {
  const int r = a.r0 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (r >= r1) return;
  const RunDev &R = a.runs[r];
  if (a.n_sorted[r] == 0)
    for (int32_t q = 0; q <= R.nbin + 1; ++q) a.bin_start[R.bo + q] = 0;
  // (the two-level sort's bucket scans end at bin nc)
  a.bin_start[R.bo + R.nbin + 1] = (uint32_t)a.n_sorted[r];
  if (set_alive) a.n_alive[r] = (int32_t)a.bin_start[R.bo + R.nbin];
}

// ---------------------------------------------------------------------------
// Interaction (NTC) fused with the permutation P' = P[LCR] and Sampling
// ---------------------------------------------------------------------------
//
// Work items: up to 64 consecutive sparse cells of one run per wavefront (a
// lane per cell, k_collide), or one crowded cell per 256-thread block
// (k_collide_cell).  The item gathers its cells' particles through LCR (that
// is the permutation: positions go straight to P', velocities are staged in
// LDS), runs the collisions on LDS, writes the velocities back to P'
// coalesced and samples from LDS.  Results are those of the sequential
// per-cell order: the block mode runs 256 selections at a time in
// conflict-free levels and replays a window sequentially whenever
// (sigma c_r)_max grows inside it.

template <typename real> struct CollideCap;
template <> struct CollideCap<float> { static constexpr int value = kCollideCapF32; };
template <> struct CollideCap<double> { static constexpr int value = kCollideCapF64; };

// Lane-per-cell items: a smaller stage per wavefront (velocities only), so
// more wavefronts fit a CU for the gather.
template <typename real> struct LaneCap;
template <> struct LaneCap<float> { static constexpr int value = kLaneCapF32; };
template <> struct LaneCap<double> { static constexpr int value = kLaneCapF64; };

template <typename real>
constexpr int collide_wave_bytes() {
  return ((LaneCap<real>::value * 3 * (int)sizeof(real)) + 15) & ~15;
}

template <typename real>
struct Selection {
  uint32_t i, j;
  real ua, uc, ue;
};

// The sub-cells of one cell, for the choice of the second partner: the
// cell's S + 1 bin starts (run-local positions, in global memory) and its
// first position; no sub-cells when start is null.
struct SubCells {
  const uint32_t *start = nullptr;
  uint32_t base = 0;
};

// Selection k of cell c: pair (i, j != i) and the acceptance and scattering
// uniforms, from Philox blocks (step, COLL, c, 2k) and (step, COLL, c, 2k+1).
// The second partner comes from the first one's sub-cell when it holds two or
// more particles (with sub-cells), else from the cell.
template <typename real, typename RunT>
__device__ __forceinline__ Selection<real> draw_selection(const RunT &R, uint32_t step, uint32_t c, int64_t k,
                                                          uint32_t N, const SubCells &sub = SubCells{}) {
  const uint4 b0 = philox(make_uint4(step, kColl, c, (uint32_t)(2 * k)), R.key0, R.key1);
  const uint4 b1 = philox(make_uint4(step, kColl, c, (uint32_t)(2 * k + 1)), R.key0, R.key1);
  Selection<real> s;
  s.i = __umulhi(b0.x, N);
  uint32_t lo = 0, span = N;  // the second partner: one of [lo, lo + span) other than i
  if (sub.start) {
    uint32_t q = 0;
    while (sub.start[q + 1] - sub.base <= s.i) ++q;
    const uint32_t ns = sub.start[q + 1] - sub.start[q];
    if (ns >= 2) {
      lo = sub.start[q] - sub.base;
      span = ns;
    }
  }
  const uint32_t jp = lo + __umulhi(b0.y, span - 1u);
  s.j = jp + (jp >= s.i ? 1u : 0u);
  s.ua = u01<real>(b0.z, b0.w);
  s.uc = u01<real>(b1.x, b1.y);
  s.ue = u01<real>(b1.z, b1.w);
  return s;
}

// Isotropic scattering of one accepted pair.
template <typename real>
struct Angles {
  real cosx, sinx, ce, se;  // cos chi, sin chi, cos eps, sin eps
};

// sin and cos of one angle with one shared argument reduction.
__device__ __forceinline__ void sin_cos(float x, float &s, float &c) { sincosf(x, &s, &c); }
__device__ __forceinline__ void sin_cos(double x, double &s, double &c) { sincos(x, &s, &c); }

// Deflection angles of a selection from its two scattering uniforms.
template <typename real>
__device__ __forceinline__ Angles<real> angles_of(real uc, real ue) {
  Angles<real> a;
  a.cosx = (real)2 * uc - (real)1;
  a.sinx = sqrt((real)1 - a.cosx * a.cosx);
  const real eps = two_pi<real>() * ue;
  sin_cos(eps, a.se, a.ce);
  return a;
}

template <typename real>
__device__ __forceinline__ void scatter_pair(real cr, const Angles<real> &an, real &ui, real &vi, real &wi,
                                             real &uj, real &vj, real &wj) {
  const real rx = cr * an.cosx, ry = cr * an.sinx * an.ce, rz = cr * an.sinx * an.se;
  const real mx = (real)0.5 * (ui + uj), my = (real)0.5 * (vi + vj), mz = (real)0.5 * (wi + wj);
  ui = mx + (real)0.5 * rx;
  vi = my + (real)0.5 * ry;
  wi = mz + (real)0.5 * rz;
  uj = mx - (real)0.5 * rx;
  vj = my - (real)0.5 * ry;
  wj = mz - (real)0.5 * rz;
}

// Selections [k0, k1) of one cell in order, by one lane, on arrays u/v/w
// (LDS, or P' seen through Strided views).  Returns the accepted collisions;
// updates gm.
template <typename real, typename RunT, typename PU, typename PV, typename PW>
__device__ uint32_t chain_serial(const RunT &R, uint32_t step, uint32_t c, uint32_t N, int64_t k0, int64_t k1,
                                 PU u, PV v, PW w, real &gm, const SubCells &sub = SubCells{}) {
  uint32_t ncol = 0;
  for (int64_t k = k0; k < k1; ++k) {
    const Selection<real> s = draw_selection<real>(R, step, c, k, N, sub);
    const real du = u[s.i] - u[s.j], dv = v[s.i] - v[s.j], dw = w[s.i] - w[s.j];
    const real cr = sqrt(du * du + dv * dv + dw * dw);
    const real g = g_of<real>(R, cr);
    if (g > gm) gm = g;
    if (!(s.ua < g / gm)) continue;
    real ui = u[s.i], vi = v[s.i], wi = w[s.i], uj = u[s.j], vj = v[s.j], wj = w[s.j];
    scatter_pair(cr, angles_of(s.uc, s.ue), ui, vi, wi, uj, vj, wj);
    u[s.i] = ui; v[s.i] = vi; w[s.i] = wi;
    u[s.j] = uj; v[s.j] = vj; w[s.j] = wj;
    ncol++;
  }
  return ncol;
}

// NTC bookkeeping: number of selections this step and the new remainder.
// The pairs are N(N-1)/2, or with a running mean of the count (nbar_alpha >
// 0, Bird's variant) N * Nbar / 2 after Nbar has moved towards N.
template <typename real, typename RunT>
__device__ __forceinline__ int64_t ntc_selections(const RunT &R, int64_t N, real gm, real &rem, real &nb,
                                                  int32_t *err) {
  real npairs;
  if (R.nbar_alpha > 0.0) {
    nb = nb + (real)R.nbar_alpha * ((real)N - nb);
    npairs = (real)0.5 * (real)N * nb;
  } else {
    npairs = (real)0.5 * (real)(N * (N - 1));
  }
  const real M = npairs * (real)R.coef * gm + rem;
  int64_t nsel = 0;
  if (M >= (real)0 && M < (real)kMaxSelections) {
    const real fl = floor(M);
    nsel = (int64_t)fl;
    rem = M - fl;
  } else {  // non-finite velocities or an absurd rate: stop, report
    set_error(err, kErrNumeric);
    rem = (real)0;
  }
  return N < 2 ? 0 : nsel;
}

// Per-cell sample sums (count, sum u, v, w, sum u^2, v^2, w^2), taken by one
// whole wavefront in every Interaction mode, so the sums do not depend on the
// mode: lane l adds the cell's particles l, l + 64, ... (P' order) in order,
// then the 64 partial sums are added by the xor butterfly (offsets 32, 16,
// ..., 1); lane 0 writes.
template <typename PU, typename PV, typename PW>
__device__ __forceinline__ void sample_cell_wave(PU u, PV v, PW w, int64_t N, double *out) {
  const int lane = threadIdx.x & 63;
  double s[kFields] = {0, 0, 0, 0, 0, 0, 0};
  for (int64_t k = lane; k < N; k += kWave) {
    const double a = (double)u[k], b = (double)v[k], c = (double)w[k];
    s[0] += 1.0;
    s[1] += a;
    s[2] += b;
    s[3] += c;
    s[4] += a * a;
    s[5] += b * b;
    s[6] += c * c;
  }
#pragma unroll
  for (int f = 0; f < kFields; ++f) {
    double x = s[f];
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    s[f] = x;
  }
  if (lane == 0)
#pragma unroll
    for (int f = 0; f < kFields; ++f) out[f] = s[f];
}

// A gathered coordinate at the end of the step's flight: Motion left a free
// particle where it began (its entry lacks kMovedBit), and its flight is the
// same expression as Motion's test used.
template <typename real>
__device__ __forceinline__ real flown(real p, real v, real dt, int32_t entry) {
  return entry < 0 ? p : p + v * dt;
}

// Gather particles [b, b+n) of a run (sorted positions) through LCR into P',
// whole records, moving the free ones (an item beyond its LDS stage).
template <typename real, int DIM>
__device__ __forceinline__ void gather_to_p(const RunDev &R, const int32_t *lcr, const Particles<real> &A,
                                            const Particles<real> &B, int64_t b, int64_t n) {
  const int lane = threadIdx.x & 63;
  constexpr int U = 4;
  // reads clamped into [0, n) instead of masked: no branch whose join would
  // make the compiler wait for each load before issuing the next
  const int32_t *__restrict__ lp = lcr + R.so + b;
  const real dt = in_precision<real>(R.dt, R.dt_f);
  for (int64_t k0 = 0; k0 < n; k0 += U * kWave) {
    int32_t l[U];
#pragma unroll
    for (int q = 0; q < U; ++q) l[q] = lp[min(k0 + q * kWave + lane, n - 1)];
    typename Vec4<real>::type r4[U];
    real z[U], ww[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int64_t src = R.so + (l[q] & kSlotMask);
      r4[q] = A.q[src];
      load_zw<DIM>(A, src, z[q], ww[q]);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int64_t k = k0 + q * kWave + lane;
      if (k >= n) continue;
      const int64_t dst = R.so + b + k;
      B.q[dst] = make_vec4<real>(flown(r4[q].x, r4[q].z, dt, l[q]), flown(r4[q].y, r4[q].w, dt, l[q]), r4[q].z,
                                 r4[q].w);
      store_zw<DIM>(B, dst, DIM == 3 ? flown(z[q], ww[q], dt, l[q]) : (real)0, ww[q]);
    }
  }
}

// Gather into the LDS stage (at most NH*64 particles): velocities to su/sv/sw,
// and each lane's final positions kept in registers (particle j*64 + lane at
// index j, constant indices: the chunk loop is unrolled) until the
// write-back stores the whole record.
template <typename real, int DIM, int NH>
__device__ __forceinline__ void gather_hold(const RunDev &R, const int32_t *lcr, const Particles<real> &A, int64_t b,
                                            int64_t n, real *su, real *sv, real *sw, real (&hx)[NH], real (&hy)[NH],
                                            real (&hz)[NH]) {
  const int lane = threadIdx.x & 63;
  constexpr int U = 4;
  static_assert(NH % U == 0, "whole chunks");
  const int32_t *__restrict__ lp = lcr + R.so + b;
  const real dt = in_precision<real>(R.dt, R.dt_f);
#pragma unroll
  for (int ch = 0; ch < NH / U; ++ch) {
    const int64_t k0 = (int64_t)ch * U * kWave;
    if (k0 >= n) break;
    int32_t l[U];
#pragma unroll
    for (int q = 0; q < U; ++q) l[q] = lp[min(k0 + q * kWave + lane, n - 1)];
    typename Vec4<real>::type r4[U];
    real z[U], ww[U];
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int64_t src = R.so + (l[q] & kSlotMask);
      r4[q] = A.q[src];
      load_zw<DIM>(A, src, z[q], ww[q]);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const int64_t k = k0 + q * kWave + lane;
      const int j = ch * U + q;
      hx[j] = flown(r4[q].x, r4[q].z, dt, l[q]);
      hy[j] = flown(r4[q].y, r4[q].w, dt, l[q]);
      hz[j] = DIM == 3 ? flown(z[q], ww[q], dt, l[q]) : (real)0;
      if (k >= n) continue;
      su[k] = r4[q].z;
      sv[k] = r4[q].w;
      sw[k] = ww[q];
    }
  }
}

// Write-back of an item gathered by gather_hold: whole records to P' (held
// positions, final velocities) and, with the look-ahead, each particle's
// next flight cell.
template <typename real, int DIM, int NH, bool SUB = true>
__device__ __forceinline__ void write_back_held(const RunDev &R, const Particles<real> &B, int32_t *cell, int64_t b,
                                                int64_t n, const real *u, const real *v, const real *w,
                                                const real (&hx)[NH], const real (&hy)[NH], const real (&hz)[NH]) {
  const int lane = threadIdx.x & 63;
  const Flight<real> F(R);
  const bool ahead = R.ahead;
  const int64_t base = R.so + b;
#pragma unroll
  for (int j = 0; j < NH; ++j) {
    const int64_t k = (int64_t)j * kWave + lane;
    if (k < n) {
      B.q[base + k] = make_vec4<real>(hx[j], hy[j], u[k], v[k]);
      store_zw<DIM>(B, base + k, hz[j], w[k]);
      if (ahead) {
        const real pos[3] = {hx[j], hy[j], hz[j]};
        const real vel[3] = {u[k], v[k], DIM == 3 ? w[k] : (real)0};
        cell[base + k] = flight_cell<real, DIM, SUB>(F, pos, vel);
      }
    }
  }
}

// Look-ahead for the next step's Motion over P' positions [b, b+n) of a run
// whose particles are complete in P' (this thread's share: t, t + nt, ...,
// the same thread that wrote them): the cell each particle's next free
// flight ends in, or the queue mark.
template <typename real, int DIM, bool SUB = true>
__device__ __forceinline__ void next_cells(const RunDev &R, const Particles<real> &B, int32_t *cell, int64_t b,
                                           int64_t n, int t, int nt) {
  const Flight<real> F(R);
  const int64_t base = R.so + b;
  for (int64_t k = t; k < n; k += nt) {
    const int64_t dst = base + k;
    const typename Vec4<real>::type r4 = B.q[dst];
    real z, w;
    load_zw<DIM>(B, dst, z, w);
    const real pos[3] = {r4.x, r4.y, z};
    const real vel[3] = {r4.z, r4.w, DIM == 3 ? w : (real)0};
    cell[dst] = flight_cell<real, DIM, SUB>(F, pos, vel);
  }
}

__device__ __forceinline__ void global_sync_wave() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// Work distribution of an Interaction kernel over its items [i0, i1)
// ---------------------------------------------------------------------------
//
// kSchedGrid: one item per workgroup (or wavefront) from the grid index, the
// hardware dispatcher handing workgroups to CUs as they free up.
// kSchedQueue: a persistent grid whose workgroups draw items from a device
// queue shared by all runs (the GPU form of dynamic processor reallocation:
// a workgroup done with one run's work takes any run's next item).  The list
// is split into eight contiguous shares with a counter each, one per XCD
// (neighbouring cells stay on one L2); a workgroup draws from its own XCD's
// share, then from the others'.
// kSchedPerRun: a persistent grid whose workgroups are tied to runs (the
// static two-level split): of U units (workgroups, or wavefronts), unit g
// serves run g mod nr when U >= nr (p2 = U / nr units per run), else runs g,
// g + U, g + 2U, ... one after the other.
// The item a workgroup draws never changes what is computed for it.
constexpr int kXcds = 8;

// A draw takes kSchedBatch consecutive items of one share: [first, end) with
// end - first <= kSchedBatch; first = i1 when the queue is used up.
constexpr int kSchedBatch = 4;

struct Draw {
  int64_t first, end;
};

// The draw state x of unit `unit`: its XCD (kSchedQueue), its first run
// (kSchedPerRun).
__device__ __forceinline__ int sched_start(const Sched &s, int unit) {
  if (s.mode == kSchedPerRun) return s.nr > 0 ? unit % s.nr : 0;
  return (int)(blockIdx.x % kXcds);
}

// `units`: U, the persistent grid's units (kSchedPerRun).
__device__ __forceinline__ Draw sched_draw(const Sched &s, int64_t i0, int64_t i1, int units, int &x, int &tries) {
  if (s.mode == kSchedPerRun) {
    while (x < s.nr) {
      const int64_t item = s.first[x] + (int64_t)atomicAdd(&s.ctr[x], 1u) * kSchedBatch;
      const int64_t lim = s.first[x + 1];
      if (item < lim) return Draw{item, min(item + kSchedBatch, lim)};
      x += units;  // this run's items are all taken: the unit's next run
    }
    return Draw{i1, i1};
  }
  const int64_t N = i1 - i0;
  while (tries < kXcds) {
    // XCD x's share: a contiguous 1/8 of the list (as the grid's block order
    // gives it), so neighbouring cells, whose gathers share lines, meet in
    // one L2
    const int64_t q = N / kXcds, rmd = N % kXcds;
    const int64_t lo = x < rmd ? x * (q + 1) : rmd * (q + 1) + (x - rmd) * q;
    const int64_t hi = lo + (x < rmd ? q + 1 : q);
    const int64_t item = lo + (int64_t)atomicAdd(&s.ctr[x], 1u) * kSchedBatch;
    if (item < hi) return Draw{i0 + item, i0 + min(item + kSchedBatch, hi)};
    // this XCD's share is used up: take from the next one's
    x = (x + 1) % kXcds;
    ++tries;
  }
  return Draw{i1, i1};
}

__device__ __forceinline__ int64_t first_lane_i64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A wavefront's next draw (lane 0 draws, every lane gets it).
__device__ __forceinline__ Draw sched_next_wave(const Sched &s, int64_t i0, int64_t i1, int units, int &x,
                                                int &tries) {
  Draw d{0, 0};
  if ((threadIdx.x & 63) == 0) d = sched_draw(s, i0, i1, units, x, tries);
  x = __builtin_amdgcn_readfirstlane(x);
  tries = __builtin_amdgcn_readfirstlane(tries);
  return Draw{first_lane_i64(d.first), first_lane_i64(d.end)};
}

// SUB = false: instantiated for batches without sub-cells.
template <typename real, int DIM, bool SUB>
__device__ __forceinline__ void collide_lanes_item(const DevPtrs<real> &d, int src, int64_t item,
                                                   unsigned char *lds_bytes) {
  constexpr int CAP = LaneCap<real>::value;
  const int wave = wave_index(), lane = threadIdx.x & 63;
  const int2 it = d.items[item];
  const RunDev &R = d.runs[it.x];
  const int32_t c0 = it.y;
  const int32_t ncell = min(R.lane_cells, R.nc - c0);
  real *su = (real *)(lds_bytes + wave * collide_wave_bytes<real>());
  real *sv = su + CAP, *sw = sv + CAP;
  const Particles<real> A = d.P[src], B = d.P[1 - src];
  const int S = R.S;  // a cell's bins: S consecutive sub-cells (1 without sub-cells)
  const int64_t b0 = d.bin_start[R.bo + (int64_t)c0 * S];
  const int64_t n = (int64_t)d.bin_start[R.bo + (int64_t)(c0 + ncell) * S] - b0;
  const bool in_lds = n <= CAP;
  constexpr int NH = (CAP + 4 * kWave - 1) / (4 * kWave) * 4;
  real hx[NH], hy[NH], hz[NH];
  if (in_lds) gather_hold<real, DIM, NH>(R, d.lcr, A, b0, n, su, sv, sw, hx, hy, hz);
  else gather_to_p<real, DIM>(R, d.lcr, A, B, b0, n);
  if (in_lds) wave_sync();
  else global_sync_wave();
  const uint32_t step = *d.step;
  const bool sample = *d.sample_slot >= 0;
  // one lane per cell
  if (lane < ncell) {
    const int32_t c = c0 + lane;
    const int64_t gc = R.co + c;
    const int64_t cs = (int64_t)d.bin_start[R.bo + (int64_t)c * S];
    const int64_t cb = cs - b0;
    const int64_t N = (int64_t)d.bin_start[R.bo + (int64_t)(c + 1) * S] - cs;
    SubCells sub;
    if (SUB && S > 1) {
      sub.start = d.bin_start + R.bo + (int64_t)c * S;
      sub.base = (uint32_t)cs;
    }
    real gm = d.gmax[gc], rem = d.rem_c[gc];
    real nb = R.nbar_alpha > 0.0 ? d.nbar[gc] : (real)0;
    const int64_t nsel = ntc_selections<real>(R, N, gm, rem, nb, d.err);
    if (R.nbar_alpha > 0.0) d.nbar[gc] = nb;
    uint32_t ncol;
    if (in_lds) {
      ncol = chain_serial<real>(R, step, (uint32_t)c, (uint32_t)N, 0, nsel, su + cb, sv + cb, sw + cb, gm, sub);
    } else {
      const int64_t o = R.so + b0 + cb;
      ncol = chain_serial<real>(R, step, (uint32_t)c, (uint32_t)N, 0, nsel, B.u() + o, B.v() + o, w_view<DIM>(B, o),
                                gm, sub);
    }
    d.gmax[gc] = gm;
    d.rem_c[gc] = rem;
    d.ncoll[gc] += ncol;
  }
  if (sample) {
    // the whole wavefront samples the item's cells one after the other
    if (in_lds) wave_sync();
    else global_sync_wave();
    for (int32_t j = 0; j < ncell; ++j) {
      const int32_t c = c0 + j;
      const int64_t cs = (int64_t)d.bin_start[R.bo + (int64_t)c * S];
      const int64_t N = (int64_t)d.bin_start[R.bo + (int64_t)(c + 1) * S] - cs;
      double *out = d.stage + (R.co + c) * kFields;
      if (in_lds) {
        sample_cell_wave(su + (cs - b0), sv + (cs - b0), sw + (cs - b0), N, out);
      } else {
        const int64_t o = R.so + cs;
        sample_cell_wave(B.u() + o, B.v() + o, w_view<DIM>(B, o), N, out);
      }
    }
  }
  if (in_lds) {
    wave_sync();
    write_back_held<real, DIM, NH, SUB>(R, B, d.cell, b0, n, su, sv, sw, hx, hy, hz);
  } else if (R.ahead) {
    global_sync_wave();  // every lane's chain on P' is visible
    next_cells<real, DIM, SUB>(R, B, d.cell, b0, n, lane, kWave);
  }
}

// PERSIST: the persistent grid (Sched); otherwise one item per wavefront of
// the grid.  Separate instantiations: the loop's state would cost the grid
// kernel registers.
template <typename real, int DIM, bool PERSIST, bool SUB>
__global__ __launch_bounds__(kCollideWaves * 64) void k_collide(DevPtrs<real> d, int src, int64_t it0, int64_t it1,
                                                                Sched sc) {
  extern __shared__ __align__(16) unsigned char lds_bytes[];
  const int wave = wave_index();
  if constexpr (!PERSIST) {
    const int64_t item = it0 + xcd_block(blockIdx.x, gridDim.x) * kCollideWaves + wave;
    if (item < it1) collide_lanes_item<real, DIM, SUB>(d, src, item, lds_bytes);
    return;
  }
  const int units = (int)gridDim.x * kCollideWaves;
  int x = sched_start(sc, (int)blockIdx.x * kCollideWaves + wave), tries = 0;
  Draw cur = sched_next_wave(sc, it0, it1, units, x, tries);
  while (cur.first < it1) {
    // the next draw goes out before this one's items, so its latency overlaps them
    const Draw nxt = sched_next_wave(sc, it0, it1, units, x, tries);
    for (int64_t item = cur.first; item < cur.end; ++item) {
      collide_lanes_item<real, DIM, SUB>(d, src, item, lds_bytes);
      wave_sync();  // the stage is free again
    }
    cur = nxt;
  }
}

// One cell per 256-thread block (crowded cells): the gather, the write-back
// and the sampling use all 256 threads.  Selections run 256 at a time: thread
// k draws selection w0 + k; among the pending selections touching a
// particle, the lowest-numbered one owns it (LDS atomicMin), and a selection
// owning both its particles runs now.  So every selection runs after all
// earlier ones sharing a particle with it and sees exactly the velocities of
// the sequential order.  The window assumes (sigma c_r)_max stays put; if
// some g exceeds it, the selections from the first such one (ks) on are undone
// in reverse order of execution, ks is applied with the raised maximum, and
// the window restarts at ks + 1.
template <typename real>
struct BlockScratch {
  int32_t vote[2][kWavesPerBlock];  // per-wavefront partial results of LdsSync::any / count
  int32_t ks;
  uint32_t ncol;
  real gm;
};

// Block synchronisation of the collision chain.  FullSync: __syncthreads
// (which also waits for the thread's outstanding global loads).  LdsSync:
// orders LDS only -- it waits for the wavefront's LDS operations, not for its
// global loads, so a gather into another LDS buffer (global_load_lds) stays in
// flight across it; the empty asm statements keep the compiler from moving
// memory accesses across the barrier.
struct FullSync {
  static constexpr int kSize = 256;  // threads sharing one chain
  __device__ static int tid() { return (int)threadIdx.x; }
  __device__ static void bar() { __syncthreads(); }
  __device__ static int any(int p, int32_t (&)[2][kWavesPerBlock], int) { return __syncthreads_or(p); }
  __device__ static int count(int p, int32_t (&)[2][kWavesPerBlock], int) { return __syncthreads_count(p); }
};
struct LdsSync {
  static constexpr int kSize = 256;
  __device__ static int tid() { return (int)threadIdx.x; }
  __device__ static void bar() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0); vmcnt, expcnt left open
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
  }
  // `slot` alternates between calls; every use is followed by another bar()
  // before the same slot is written again
  __device__ static int any(int p, int32_t (&v)[2][kWavesPerBlock], int slot) {
    const uint64_t m = __ballot(p);
    if ((threadIdx.x & 63) == 0) v[slot][threadIdx.x >> 6] = m != 0ull;
    bar();
    int r = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) r |= v[slot][w];
    return r;
  }
  __device__ static int count(int p, int32_t (&v)[2][kWavesPerBlock], int slot) {
    const uint64_t m = __ballot(p);
    if ((threadIdx.x & 63) == 0) v[slot][threadIdx.x >> 6] = __popcll(m);
    bar();
    int r = 0;
#pragma unroll
    for (int w = 0; w < kWavesPerBlock; ++w) r += v[slot][w];
    return r;
  }
};

// One wavefront per chain: its lanes run in lockstep and its LDS operations
// complete in order, so a barrier is only a compiler fence and a wait for
// the wavefront's own LDS operations; votes are ballots.
struct WaveSync {
  static constexpr int kSize = kWave;
  __device__ static int tid() { return (int)(threadIdx.x & (kWave - 1)); }
  __device__ static void bar() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
  }
  __device__ static int any(int p, int32_t (&)[2][kWavesPerBlock], int) {
    bar();
    return __builtin_amdgcn_ballot_w64(p != 0) != 0ull;
  }
  __device__ static int count(int p, int32_t (&)[2][kWavesPerBlock], int) {
    bar();
    return (int)__popcll(__builtin_amdgcn_ballot_w64(p != 0));
  }
};

template <typename real>
constexpr int collide_cell_bytes() {
  return ((CollideCap<real>::value * (3 * (int)sizeof(real) + 4)) + 15) & ~15;
}

template <typename real, typename Sync = FullSync, typename RunT = RunDev>
__device__ uint32_t chain_block(const RunT &R, uint32_t step, uint32_t c, uint32_t N, int64_t nsel, real *u,
                                real *v, real *w, int32_t *own, BlockScratch<real> &sh, real &gm,
                                const SubCells &sub = SubCells{}) {
  const int tid = Sync::tid();
  uint32_t ncol = 0;
  int64_t w0 = 0;
  int slot = 0;
  while (w0 < nsel) {
    const bool act = w0 + tid < nsel;
    Selection<real> s{0u, 0u, (real)0, (real)0, (real)0};
    Angles<real> an{(real)1, (real)0, (real)1, (real)0};
    if (act) {
      s = draw_selection<real>(R, step, c, w0 + tid, N, sub);
      // deflection angles once per selection, not once per conflict round
      an = angles_of(s.uc, s.ue);
    }
    bool pending = act, accepted = false;
    int my_round = -1;
    real g = (real)0;
    real bu_i = 0, bv_i = 0, bw_i = 0, bu_j = 0, bv_j = 0, bw_j = 0;
    int rounds = 0;
    while (Sync::any(pending, sh.vote, slot ^= 1)) {
      if (pending) {
        own[s.i] = 0x7fffffff;
        own[s.j] = 0x7fffffff;
      }
      Sync::bar();
      if (pending) {
        atomicMin(&own[s.i], tid);
        atomicMin(&own[s.j], tid);
      }
      Sync::bar();
      const bool ready = pending && own[s.i] == tid && own[s.j] == tid;
      Sync::bar();
      if (ready) {
        real ui = u[s.i], vi = v[s.i], wi = w[s.i], uj = u[s.j], vj = v[s.j], wj = w[s.j];
        bu_i = ui; bv_i = vi; bw_i = wi; bu_j = uj; bv_j = vj; bw_j = wj;
        const real du = ui - uj, dv = vi - vj, dw = wi - wj;
        const real cr = sqrt(du * du + dv * dv + dw * dw);
        g = g_of<real>(R, cr);
        accepted = s.ua < g / gm;
        if (accepted) {
          scatter_pair(cr, an, ui, vi, wi, uj, vj, wj);
          u[s.i] = ui; v[s.i] = vi; w[s.i] = wi;
          u[s.j] = uj; v[s.j] = vj; w[s.j] = wj;
        }
        my_round = rounds;
        pending = false;
      }
      ++rounds;
    }
    if (tid == 0) sh.ks = 0x7fffffff;
    Sync::bar();
    if (act && g > gm) atomicMin(&sh.ks, tid);
    Sync::bar();
    const int ks = sh.ks;
    if (ks == 0x7fffffff) {
      ncol += Sync::count(accepted, sh.vote, slot ^= 1);
      w0 += Sync::kSize;
      continue;
    }
    // undo selections ks.. in reverse order of execution
    for (int r = rounds - 1; r >= 0; --r) {
      if (act && tid >= ks && my_round == r && accepted) {
        u[s.i] = bu_i; v[s.i] = bv_i; w[s.i] = bw_i;
        u[s.j] = bu_j; v[s.j] = bv_j; w[s.j] = bw_j;
      }
      Sync::bar();
    }
    ncol += Sync::count(accepted && tid < ks, sh.vote, slot ^= 1);
    // selection ks raises (sigma c_r)_max to its own g, so it is accepted
    // (U < g/g = 1); it ran on exactly its sequential inputs, so apply it again
    // from the restored state and restart the window right after it
    if (tid == ks) {
      real ui = u[s.i], vi = v[s.i], wi = w[s.i], uj = u[s.j], vj = v[s.j], wj = w[s.j];
      const real du = ui - uj, dv = vi - vj, dw = wi - wj;
      const real cr = sqrt(du * du + dv * dv + dw * dw);
      const real gg = g_of<real>(R, cr);
      const real gnew = gg > gm ? gg : gm;
      const bool acc = s.ua < gg / gnew;
      if (acc) {
        scatter_pair(cr, an, ui, vi, wi, uj, vj, wj);
        u[s.i] = ui; v[s.i] = vi; w[s.i] = wi;
        u[s.j] = uj; v[s.j] = vj; w[s.j] = wj;
      }
      sh.gm = gnew;
      sh.ncol = acc ? 1u : 0u;
    }
    Sync::bar();
    gm = sh.gm;
    ncol += sh.ncol;
    w0 += ks + 1;
    Sync::bar();
  }
  return ncol;
}

template <typename real, int DIM>
__device__ __forceinline__ void collide_cell_item(const DevPtrs<real> &d, int src, int64_t item,
                                                  unsigned char *lds_bytes, BlockScratch<real> &sh) {
  constexpr int CAP = CollideCap<real>::value;
  const int tid = threadIdx.x;
  const int2 it = d.cell_items[item];
  const RunDev &R = d.runs[it.x];
  const int32_t c = it.y;
  const int64_t gc = R.co + c;
  real *su = (real *)lds_bytes;
  real *sv = su + CAP, *sw = sv + CAP;
  int32_t *own = (int32_t *)(sw + CAP);
  const Particles<real> A = d.P[src], B = d.P[1 - src];
  const int64_t b0 = d.bin_start[R.bo + (int64_t)c * R.S];
  const int64_t n = (int64_t)d.bin_start[R.bo + (int64_t)(c + 1) * R.S] - b0;
  const bool in_lds = n <= CAP;
  SubCells sub;
  if (R.S > 1) {
    sub.start = d.bin_start + R.bo + (int64_t)c * R.S;
    sub.base = (uint32_t)b0;
  }
  // cell state and step facts are loaded up front, their latency hidden
  // behind the gather
  const uint32_t step = *d.step;
  const bool sample = *d.sample_slot >= 0;
  real gm = d.gmax[gc], rem = d.rem_c[gc];
  real nb = R.nbar_alpha > 0.0 ? d.nbar[gc] : (real)0;
  // gather through LCR: whole records to P' (their velocities are replaced at
  // the write-back of an LDS item), velocities to LDS
  {
    constexpr int U = 4;
    const real dt = in_precision<real>(R.dt, R.dt_f);
    for (int64_t k0 = 0; k0 < n; k0 += U * 256) {
      int64_t sidx[U];
      int32_t ent[U];
      bool ok[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const int64_t k = k0 + q * 256 + tid;
        ok[q] = k < n;
        ent[q] = ok[q] ? d.lcr[R.so + b0 + k] : 0;
        sidx[q] = R.so + (ent[q] & kSlotMask);
      }
      typename Vec4<real>::type r4[U];
      real z[U], ww[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        if (ok[q]) {
          r4[q] = A.q[sidx[q]];
          load_zw<DIM>(A, sidx[q], z[q], ww[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < U; ++q) {
        if (!ok[q]) continue;
        const int64_t k = k0 + q * 256 + tid;
        const int64_t dst = R.so + b0 + k;
        B.q[dst] = make_vec4<real>(flown(r4[q].x, r4[q].z, dt, ent[q]), flown(r4[q].y, r4[q].w, dt, ent[q]),
                                   r4[q].z, r4[q].w);
        // w goes to P' now, and again at the write-back of an LDS item
        store_zw<DIM>(B, dst, DIM == 3 ? flown(z[q], ww[q], dt, ent[q]) : (real)0, ww[q]);
        if (in_lds) {
          su[k] = r4[q].z;
          sv[k] = r4[q].w;
          sw[k] = ww[q];
        }
      }
    }
  }
  __syncthreads();
  const int64_t nsel = ntc_selections<real>(R, n, gm, rem, nb, d.err);
  if (tid == 0 && R.nbar_alpha > 0.0) d.nbar[gc] = nb;
  const Strided<real> gu = B.u() + (R.so + b0), gv = B.v() + (R.so + b0);
  const auto gw = w_view<DIM>(B, R.so + b0);
  uint32_t ncol = 0;
  if (in_lds) {
    ncol = chain_block<real>(R, step, (uint32_t)c, (uint32_t)n, nsel, su, sv, sw, own, sh, gm, sub);
  } else {
    if (tid == 0) {
      ncol = chain_serial<real>(R, step, (uint32_t)c, (uint32_t)n, 0, nsel, gu, gv, gw, gm, sub);
      sh.gm = gm;
    }
    __syncthreads();
    gm = sh.gm;
  }
  __syncthreads();
  if (in_lds)
    for (int64_t k = tid; k < n; k += 256) {
      gu[k] = su[k];
      gv[k] = sv[k];
      gw[k] = sw[k];
    }
  if (R.ahead) next_cells<real, DIM>(R, B, d.cell, b0, n, tid, 256);  // this thread's own records
  if (sample && tid < kWave) {  // the first wavefront, in the order all modes share
    if (in_lds) sample_cell_wave(su, sv, sw, n, d.stage + gc * kFields);
    else sample_cell_wave(gu, gv, gw, n, d.stage + gc * kFields);
  }
  if (tid == 0) {
    d.gmax[gc] = gm;
    d.rem_c[gc] = rem;
    d.ncoll[gc] += ncol;
  }
}

// A workgroup's next draw: thread 0 issues it (into a register) and, after
// the current draw's items, publishes it; the block reads it.
__device__ __forceinline__ Draw sched_publish(const Draw &mine, Draw *slot) {
  if (threadIdx.x == 0) *slot = mine;
  __syncthreads();
  const Draw d = *slot;
  __syncthreads();  // every thread has it before thread 0 publishes again
  return d;
}

template <typename real, int DIM, bool PERSIST>
__global__ __launch_bounds__(256) void k_collide_cell(DevPtrs<real> d, int src, int64_t ci0, int64_t ci1, Sched sc) {
  extern __shared__ __align__(16) unsigned char lds_bytes[];
  __shared__ BlockScratch<real> sh;
  __shared__ Draw next;
  if constexpr (!PERSIST) {
    const int64_t item = ci0 + xcd_block(blockIdx.x, gridDim.x);
    if (item < ci1) collide_cell_item<real, DIM>(d, src, item, lds_bytes, sh);
    return;
  }
  int x = sched_start(sc, (int)blockIdx.x), tries = 0;
  Draw mine{ci1, ci1};
  if (threadIdx.x == 0) mine = sched_draw(sc, ci0, ci1, (int)gridDim.x, x, tries);
  Draw cur = sched_publish(mine, &next);
  while (cur.first < ci1) {
    // the next draw goes out before this one's items, so its latency overlaps them
    if (threadIdx.x == 0) mine = sched_draw(sc, ci0, ci1, (int)gridDim.x, x, tries);
    for (int64_t item = cur.first; item < cur.end; ++item) {
      collide_cell_item<real, DIM>(d, src, item, lds_bytes, sh);
      __syncthreads();  // LDS and the scratch are free again
    }
    cur = sched_publish(mine, &next);
  }
}

// Cells of a few hundred particles: one wavefront per cell, four cells per
// block.  The wavefront gathers its cell through LCR (positions to P',
// velocities to its LDS stage), runs the same collision chain as the block
// mode, 64 selections per window, synchronised within the wavefront only,
// writes the velocities back and samples.  A cell beyond the stage runs the
// sequential chain on P' in one lane.
template <typename real> struct WaveCap;
template <> struct WaveCap<float> { static constexpr int value = kWaveCapF32; };
template <> struct WaveCap<double> { static constexpr int value = kWaveCapF64; };

template <typename real> struct WaveStage {
  real vel[kWavesPerBlock][3 * WaveCap<real>::value];
  int32_t own[kWavesPerBlock][WaveCap<real>::value];
  BlockScratch<real> shs[kWavesPerBlock];
};

template <typename real, int DIM, bool SUB>
__device__ __forceinline__ void collide_wave_item(const DevPtrs<real> &d, int src, int64_t item,
                                                  WaveStage<real> &st) {
  constexpr int CAP = WaveCap<real>::value;
  auto &own = st.own;
  auto &shs = st.shs;
  const int wave = wave_index(), lane = threadIdx.x & 63;
  const int2 it = d.wave_items[item];
  const RunDev &R = d.runs[it.x];
  const int32_t c = it.y;
  const int64_t gc = R.co + c;
  const int64_t b0 = d.bin_start[R.bo + (int64_t)c * R.S];
  const int64_t n = (int64_t)d.bin_start[R.bo + (int64_t)(c + 1) * R.S] - b0;
  const bool in_lds = n <= CAP;
  SubCells sub;
  if (SUB && R.S > 1) {
    sub.start = d.bin_start + R.bo + (int64_t)c * R.S;
    sub.base = (uint32_t)b0;
  }
  real *su = st.vel[wave], *sv = su + CAP, *sw = sv + CAP;
  const Particles<real> A = d.P[src], B = d.P[1 - src];
  constexpr int NH = (CAP + 4 * kWave - 1) / (4 * kWave) * 4;
  real hx[NH], hy[NH], hz[NH];
  if (in_lds) gather_hold<real, DIM, NH>(R, d.lcr, A, b0, n, su, sv, sw, hx, hy, hz);
  else gather_to_p<real, DIM>(R, d.lcr, A, B, b0, n);
  if (in_lds) WaveSync::bar();
  else global_sync_wave();
  const uint32_t step = *d.step;
  const bool sample = *d.sample_slot >= 0;
  real gm = d.gmax[gc], rem = d.rem_c[gc];
  real nb = R.nbar_alpha > 0.0 ? d.nbar[gc] : (real)0;
  const int64_t nsel = ntc_selections<real>(R, n, gm, rem, nb, d.err);
  if (lane == 0 && R.nbar_alpha > 0.0) d.nbar[gc] = nb;
  uint32_t ncol = 0;
  if (in_lds) {
    ncol = chain_block<real, WaveSync>(R, step, (uint32_t)c, (uint32_t)n, nsel, su, sv, sw, own[wave], shs[wave],
                                       gm, sub);
    WaveSync::bar();
    write_back_held<real, DIM, NH, SUB>(R, B, d.cell, b0, n, su, sv, sw, hx, hy, hz);
    if (sample) sample_cell_wave(su, sv, sw, n, d.stage + gc * kFields);
  } else {
    const int64_t o = R.so + b0;
    if (lane == 0)
      ncol = chain_serial<real>(R, step, (uint32_t)c, (uint32_t)n, 0, nsel, B.u() + o, B.v() + o, w_view<DIM>(B, o), gm,
                                sub);
    global_sync_wave();
    if (R.ahead) next_cells<real, DIM, SUB>(R, B, d.cell, b0, n, lane, kWave);
    if (sample) sample_cell_wave(B.u() + o, B.v() + o, w_view<DIM>(B, o), n, d.stage + gc * kFields);
  }
  if (lane == 0) {
    d.gmax[gc] = gm;
    d.rem_c[gc] = rem;
    d.ncoll[gc] += ncol;
  }
}

template <typename real, int DIM, bool PERSIST, bool SUB>
__global__ __launch_bounds__(256) void k_collide_wave(DevPtrs<real> d, int src, int64_t wi0, int64_t wi1, Sched sc) {
  __shared__ __align__(16) WaveStage<real> st;
  const int wave = wave_index();
  if constexpr (!PERSIST) {
    const int64_t item = wi0 + xcd_block(blockIdx.x, gridDim.x) * kWavesPerBlock + wave;
    if (item < wi1) collide_wave_item<real, DIM, SUB>(d, src, item, st);
    return;
  }
  const int units = (int)gridDim.x * kWavesPerBlock;
  int x = sched_start(sc, (int)blockIdx.x * kWavesPerBlock + wave), tries = 0;
  Draw cur = sched_next_wave(sc, wi0, wi1, units, x, tries);
  while (cur.first < wi1) {
    // the next draw goes out before this one's items, so its latency overlaps them
    const Draw nxt = sched_next_wave(sc, wi0, wi1, units, x, tries);
    for (int64_t item = cur.first; item < cur.end; ++item) {
      collide_wave_item<real, DIM, SUB>(d, src, item, st);
      wave_sync();  // the wavefront's stage is free again
    }
    cur = nxt;
  }
}

// Crowded cells in FP32: one 256-thread block per cell.  The cell's
// bookkeeping (slots, bin range, NTC state, the run's constants) is read once
// into LDS, so the collisions read no global memory; the gather through LCR
// goes to registers with clamped, never masked, reads issued back to back,
// then positions to P' and velocities to LDS, and the collision chain
// synchronises with LDS-only barriers.  Each cell is processed exactly as
// k_collide_cell does (same selections, order and arithmetic).
// One cell per block measured fastest: a cell's gather also reads its
// neighbours' source ranges, and the blocks of consecutive cells, running at
// once on one XCD, then find those lines in its L2.  A block that walked its
// own consecutive cells (pipelining the next cell's gather under the current
// cell's collisions) read each range again a cell's time later, after the L2
// had turned over (16 cells per block: 7.2 ms and 3x the bytes read from
// memory on the 512 x 1M box, against 6.3 ms and 1x with one).
constexpr int kPipeChunks = kCollideCapF32 / 256;

// The run constants the collisions need.
struct RunView {
  uint32_t key0, key1;
  int32_t hs;
  double c_ref, vhs_exp, coef, nbar_alpha;
};

struct PipeMeta {
  int64_t so, b0, n, gc;
  const uint32_t *sub_start;  // the cell's sub-cell bin starts, null without sub-cells
  int32_t c;
  uint32_t ncoll;
  float gm, rem, dt, nb;
  int32_t ahead;
  RunView rv;
  const RunDev *run;
};

// The particles of the cell in flight, kPipeChunks per thread (k = q*256 + tid).
struct PipeRegs {
  int32_t l[kPipeChunks];
  float x[kPipeChunks], y[kPipeChunks], z[kPipeChunks], u[kPipeChunks], v[kPipeChunks], w[kPipeChunks];
};

// Final positions of the particles this thread placed (k = q*256 + tid), kept
// for the look-ahead at the write-back.
struct PipePos {
  float x[kPipeChunks], y[kPipeChunks], z[kPipeChunks];
};

// LCR entries (run-local slots) of the particles this thread handles in an
// item that fits in LDS; beyond n an entry of the item (unused), and slot 0
// of the run for an empty or unused item.  Unconditional loads: no branch
// whose join would make the compiler wait for them.
__device__ __forceinline__ void pipe_lcr(const int32_t *lcr, const PipeMeta &m, bool valid,
                                         int32_t (&l)[kPipeChunks]) {
  const bool use = valid && m.n > 0 && m.n <= kCollideCapF32;
  const int32_t *lp = use ? lcr + m.so + m.b0 : lcr;
  const int64_t lim = use ? m.n - 1 : 0;
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < kPipeChunks; ++q) {
    const int64_t k = q * 256 + tid;
    const int32_t e = lp[k < lim ? k : lim];
    l[q] = use ? e : 0;
  }
}

// Starts the gather of an item into registers (LDS items), or moves an item
// beyond the LDS capacity straight to P' (synchronously).
template <int DIM>
__device__ __forceinline__ void pipe_gather(const int32_t *lcr, const Particles<float> &A, const Particles<float> &B,
                                            const PipeMeta &m, bool valid, PipeRegs &pr) {
  if (!valid) return;
  const int tid = threadIdx.x;
  if (m.n <= kCollideCapF32) {
#pragma unroll
    for (int q = 0; q < kPipeChunks; ++q) {
      const int64_t sidx = m.so + (pr.l[q] & kSlotMask);  // a valid slot beyond n (unused)
      const float4 r4 = A.q[sidx];
      pr.x[q] = r4.x;
      pr.y[q] = r4.y;
      pr.u[q] = r4.z;
      pr.v[q] = r4.w;
      load_zw<DIM>(A, sidx, pr.z[q], pr.w[q]);
    }
  } else {
    for (int64_t k = tid; k < m.n; k += 256) {
      const int32_t e = lcr[m.so + m.b0 + k];
      const int64_t sidx = m.so + (e & kSlotMask);
      const int64_t dst = m.so + m.b0 + k;
      const float4 r4 = A.q[sidx];
      float z, w;
      load_zw<DIM>(A, sidx, z, w);
      B.q[dst] = make_vec4<float>(flown(r4.x, r4.z, m.dt, e), flown(r4.y, r4.w, m.dt, e), r4.z, r4.w);
      store_zw<DIM>(B, dst, DIM == 3 ? flown(z, w, m.dt, e) : 0.0f, w);
    }
  }
}

// An LDS item's gathered particles: positions to P', velocities to LDS.
template <int DIM>
__device__ __forceinline__ void pipe_place(const PipeMeta &m, const PipeRegs &pr, float *su, float *sv, float *sw,
                                           PipePos &pp) {
  if (m.n > kCollideCapF32) return;
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < kPipeChunks; ++q) {
    const int64_t k = q * 256 + tid;
    pp.x[q] = flown(pr.x[q], pr.u[q], m.dt, pr.l[q]);
    pp.y[q] = flown(pr.y[q], pr.v[q], m.dt, pr.l[q]);
    pp.z[q] = DIM == 3 ? flown(pr.z[q], pr.w[q], m.dt, pr.l[q]) : 0.0f;
    if (k < m.n) {
      su[k] = pr.u[q];
      sv[k] = pr.v[q];
      sw[k] = pr.w[q];
    }
  }
}

// Collisions, write-back (with the next step's flight cells), sampling and
// cell state of one item whose data is in place (LDS su/sv/sw, or P' for an
// item beyond the LDS capacity).
// SUB: some run of the batch has sub-cells (a separate instantiation: the
// sub-cell search would cost the plain kernel registers).
template <int DIM, bool SUB>
__device__ __forceinline__ void pipe_collide(const DevPtrs<float> &d, const Particles<float> &B, const PipeMeta &m,
                                             const Flight<float> &fl, const PipePos &pp, float *su, float *sv,
                                             float *sw, int32_t *own, BlockScratch<float> &sh, uint32_t step,
                                             bool sample) {
  const int tid = threadIdx.x;
  const int64_t n = m.n;
  const bool lds = n <= kCollideCapF32;
  float gm = m.gm, rem = m.rem, nb = m.nb;
  const int64_t nsel = ntc_selections<float>(m.rv, n, gm, rem, nb, d.err);
  if (tid == 0 && m.rv.nbar_alpha > 0.0) d.nbar[m.gc] = nb;  // final now: not held through the chain
  uint32_t ncol = 0;
  const Strided<float> gu = B.u() + (m.so + m.b0), gv = B.v() + (m.so + m.b0);
  const auto gw = w_view<DIM>(B, m.so + m.b0);
  if (lds) {
    ncol = chain_block<float, LdsSync>(m.rv, step, (uint32_t)m.c, (uint32_t)n, nsel, su, sv, sw, own, sh, gm,
                                       SUB ? SubCells{m.sub_start, (uint32_t)m.b0} : SubCells{});
  } else {
    __syncthreads();  // every thread's stores to P' are visible
    if (tid == 0) {
      ncol = chain_serial<float>(m.rv, step, (uint32_t)m.c, (uint32_t)n, 0, nsel, gu, gv, gw, gm,
                                 SUB ? SubCells{m.sub_start, (uint32_t)m.b0} : SubCells{});
      sh.gm = gm;
    }
    __syncthreads();
    gm = sh.gm;
  }
  LdsSync::bar();
  if (lds) {
    // whole records from the positions this thread placed (still in its
    // registers) and the final velocities, and the look-ahead (the run's
    // flight constants from LDS, where the item's bookkeeping put them)
    const Flight<float> F = fl;
    const int64_t base = m.so + m.b0;
#pragma unroll
    for (int q = 0; q < kPipeChunks; ++q) {
      const int64_t k = q * 256 + tid;
      if (k < n) {
        B.q[base + k] = make_vec4<float>(pp.x[q], pp.y[q], su[k], sv[k]);
        store_zw<DIM>(B, base + k, pp.z[q], sw[k]);
        if (m.ahead) {
          const float pos[3] = {pp.x[q], pp.y[q], pp.z[q]};
          const float vel[3] = {su[k], sv[k], sw[k]};
          d.cell[base + k] = flight_cell<float, DIM, SUB>(F, pos, vel);
        }
      }
    }
  } else if (m.ahead) {
    next_cells<float, DIM, SUB>(*m.run, B, d.cell, m.b0, n, tid, 256);
  }
  if (sample && tid < kWave) {
    // the first wavefront, in the order all modes share; LDS and global are
    // summed by separate calls: a pointer to either would be a flat access
    // the compiler must also wait for as a global one
    if (lds) sample_cell_wave(su, sv, sw, n, d.stage + m.gc * kFields);
    else sample_cell_wave(gu, gv, gw, n, d.stage + m.gc * kFields);
  }
  if (tid == 0) {
    d.gmax[m.gc] = gm;
    d.rem_c[m.gc] = rem;
    d.ncoll[m.gc] = m.ncoll + ncol;
  }
  LdsSync::bar();  // LDS, own[] and sh are free again
}

template <int DIM, bool SUB>
__device__ __forceinline__ void collide_pipe_body(const DevPtrs<float> &d, int src, int64_t item) {
  constexpr int CAP = kCollideCapF32;
  __shared__ __align__(16) float vel[3 * CAP];
  __shared__ int32_t own[CAP];
  __shared__ PipeMeta meta;
  __shared__ Flight<float> flight;
  __shared__ BlockScratch<float> sh;
  const int tid = threadIdx.x;
  const Particles<float> A = d.P[src], B = d.P[1 - src];
  const uint32_t step = *d.step;
  const bool sample = *d.sample_slot >= 0;
  // the item's bookkeeping, once
  if (tid == 0) {
    const int2 it = d.cell_items[item];
    const RunDev &R = d.runs[it.x];
    PipeMeta m;
    m.so = R.so;
    m.c = it.y;
    m.b0 = d.bin_start[R.bo + (int64_t)it.y * R.S];
    m.n = (int64_t)d.bin_start[R.bo + (int64_t)(it.y + 1) * R.S] - m.b0;
    m.sub_start = R.S > 1 ? d.bin_start + R.bo + (int64_t)it.y * R.S : nullptr;
    m.gc = R.co + it.y;
    m.ncoll = d.ncoll[m.gc];
    m.gm = d.gmax[m.gc];
    m.rem = d.rem_c[m.gc];
    m.nb = R.nbar_alpha > 0.0 ? d.nbar[m.gc] : 0.f;
    m.dt = R.dt_f;
    m.ahead = R.ahead;
    m.run = &R;
    m.rv.key0 = R.key0;
    m.rv.key1 = R.key1;
    m.rv.hs = R.hs;
    m.rv.c_ref = R.c_ref;
    m.rv.vhs_exp = R.vhs_exp;
    m.rv.coef = R.coef;
    m.rv.nbar_alpha = R.nbar_alpha;
    meta = m;
    flight = Flight<float>(R);
  }
  __syncthreads();
  const PipeMeta m = meta;
  PipeRegs pr;
  pipe_lcr(d.lcr, m, true, pr.l);
  pipe_gather<DIM>(d.lcr, A, B, m, true, pr);
  // positions to P', velocities to LDS (the gathers return here)
  PipePos pp;
  pipe_place<DIM>(m, pr, vel, vel + CAP, vel + 2 * CAP, pp);
  if (m.n > CAP) __threadfence_block();
  LdsSync::bar();
  pipe_collide<DIM, SUB>(d, B, m, flight, pp, vel, vel + CAP, vel + 2 * CAP, own, sh, step, sample);
}

// The kernel per dimension.  The 2-D one asks for six wavefronts per SIMD
// (80 VGPRs): the compiler fits that with no scratch, and with the gather
// bound by requests in flight it runs 10 % faster than at five (86 VGPRs).
// The 3-D one would spill at six and keeps the compiler's choice.
template <int DIM, bool PERSIST, bool SUB>
__device__ __forceinline__ void collide_pipe_sched(const DevPtrs<float> &d, int src, int64_t ci0, int64_t ci1,
                                                   const Sched &sc) {
  __shared__ Draw next;
  if constexpr (!PERSIST) {
    const int64_t item = ci0 + xcd_block(blockIdx.x, gridDim.x);
    if (item < ci1) collide_pipe_body<DIM, SUB>(d, src, item);
    return;
  }
  int x = sched_start(sc, (int)blockIdx.x), tries = 0;
  Draw mine{ci1, ci1};
  if (threadIdx.x == 0) mine = sched_draw(sc, ci0, ci1, (int)gridDim.x, x, tries);
  Draw cur = sched_publish(mine, &next);
  while (cur.first < ci1) {
    // the next draw goes out before this one's items, so its latency overlaps them
    if (threadIdx.x == 0) mine = sched_draw(sc, ci0, ci1, (int)gridDim.x, x, tries);
    for (int64_t item = cur.first; item < cur.end; ++item)
      collide_pipe_body<DIM, SUB>(d, src, item);  // ends with a barrier: LDS is free again
    cur = sched_publish(mine, &next);
  }
}

template <int DIM, bool PERSIST, bool SUB>
__global__ void k_collide_pipe(DevPtrs<float> d, int src, int64_t ci0, int64_t ci1, Sched sc);
template <>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(6, 8))) void k_collide_pipe<2, false, false>(
    DevPtrs<float> d, int src, int64_t ci0, int64_t ci1, Sched sc) {
  collide_pipe_sched<2, false, false>(d, src, ci0, ci1, sc);
}
template <>
__global__ __launch_bounds__(256) void k_collide_pipe<3, false, false>(DevPtrs<float> d, int src, int64_t ci0,
                                                                       int64_t ci1, Sched sc) {
  collide_pipe_sched<3, false, false>(d, src, ci0, ci1, sc);
}
// the persistent loop's state, or the sub-cell search, does not fit six
// wavefronts per SIMD without spilling: the compiler's choice
#define DSMC_PIPE_KERNEL(D, P, S)                                                                              \
  template <>                                                                                                  \
  __global__ __launch_bounds__(256) void k_collide_pipe<D, P, S>(DevPtrs<float> d, int src, int64_t ci0,      \
                                                                 int64_t ci1, Sched sc) {                      \
    collide_pipe_sched<D, P, S>(d, src, ci0, ci1, sc);                                                         \
  }
DSMC_PIPE_KERNEL(2, true, false)
DSMC_PIPE_KERNEL(3, true, false)
DSMC_PIPE_KERNEL(2, false, true)
DSMC_PIPE_KERNEL(3, false, true)
DSMC_PIPE_KERNEL(2, true, true)
DSMC_PIPE_KERNEL(3, true, true)
#undef DSMC_PIPE_KERNEL

template <typename real>
__global__ __launch_bounds__(256) void k_sample_cells(DevPtrs<real> d, int buf, int64_t gc0, int64_t n_cells) {
  // one wavefront per cell, as in the Interaction kernels
  const int64_t gc = gc0 + (int64_t)blockIdx.x * (256 / kWave) + wave_index();
  if (gc >= n_cells) return;
  const RunDev &R = d.runs[d.cgroup_run[gc >> 6]];
  const int32_t c = (int32_t)(gc - R.co);
  if (c >= R.nc) return;
  const int64_t b = d.bin_start[R.bo + (int64_t)c * R.S];
  const int64_t N = (int64_t)d.bin_start[R.bo + (int64_t)(c + 1) * R.S] - b;
  const Particles<real> P = d.P[buf];
  if (P.zw)
    sample_cell_wave(P.u() + (R.so + b), P.v() + (R.so + b), w_view<3>(P, R.so + b), N, d.stage + gc * kFields);
  else
    sample_cell_wave(P.u() + (R.so + b), P.v() + (R.so + b), w_view<2>(P, R.so + b), N, d.stage + gc * kFields);
}

// acc[slot][eg][c][f] += sum over the runs of (ensemble, group) eg, in run order.
template <typename real>
__global__ __launch_bounds__(256) void k_accumulate(DevPtrs<real> d, int slot_arg, int64_t stride, int n_eg) {
  const int slot = slot_arg >= 0 ? slot_arg : *d.sample_slot;
  if (slot < 0) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) d.nsnap[slot] += 1u;  // one more snapshot of every run
  double *acc = d.acc + (int64_t)slot * stride;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < stride;
       i += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = n_eg;  // eg_acc[lo] <= i < eg_acc[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (d.eg_acc[mid] <= i) lo = mid;
      else hi = mid;
    }
    const int64_t local = i - d.eg_acc[lo];
    const int64_t c = local / kFields;
    const int f = (int)(local - c * kFields);
    double a = acc[i];
    for (int k = d.eg_start[lo]; k < d.eg_start[lo + 1]; ++k) {
      const RunDev &R = d.runs[d.eg_runs[k]];
      a += d.stage[(R.co + c) * kFields + f];
    }
    acc[i] = a;
  }
}

// FP64 division of sums into n (per run and snapshot), mean velocity and
// temperatures.  `samples` = runs x snapshots of each run in the sums.
__device__ __forceinline__ void moments_of(const double *S, double samples, double *m) {
  const double N = S[0];
  const double inv = N > 0.0 ? 1.0 / N : __builtin_nan("");
  const double ux = S[1] * inv, uy = S[2] * inv, uz = S[3] * inv;
  const double Tx = S[4] * inv - ux * ux;
  const double Ty = S[5] * inv - uy * uy;
  const double Tz = S[6] * inv - uz * uz;
  m[0] = samples > 0.0 ? N / samples : __builtin_nan("");
  m[1] = ux;
  m[2] = uy;
  m[3] = uz;
  m[4] = (Tx + Ty + Tz) / 3.0;
  m[5] = Tx;
  m[6] = Ty;
  m[7] = Tz;
}

template <typename real>
__global__ __launch_bounds__(256) void k_moments(DevPtrs<real> d, int slot, int64_t stride, int eg0, int G,
                                                 int nc, int n_runs_ens, int max_nc) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const double *acc = d.acc + (int64_t)slot * stride;
  const double snaps = (double)d.nsnap[slot];
  double S[kFields] = {0, 0, 0, 0, 0, 0, 0};
  for (int g = 0; g < G; ++g) {
    const double *e = acc + d.eg_acc[eg0 + g] + (int64_t)c * kFields;
#pragma unroll
    for (int f = 0; f < kFields; ++f) S[f] += e[f];
  }
  double m[kMoments];
  moments_of(S, (double)n_runs_ens * snaps, m);
  double *out = d.mom + (int64_t)c * kMoments;
  double *se = d.mom + (int64_t)max_nc * kMoments + (int64_t)c * kMoments;
#pragma unroll
  for (int f = 0; f < kMoments; ++f) out[f] = m[f];
  // batch means over the run groups
  double mean[kMoments] = {0, 0, 0, 0, 0, 0, 0, 0}, m2[kMoments] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int g = 0; g < G; ++g) {
    const double *e = acc + d.eg_acc[eg0 + g] + (int64_t)c * kFields;
    double mg[kMoments];
    moments_of(e, (double)(d.eg_start[eg0 + g + 1] - d.eg_start[eg0 + g]) * snaps, mg);
#pragma unroll
    for (int f = 0; f < kMoments; ++f) {
      const double delta = mg[f] - mean[f];
      mean[f] += delta / (double)(g + 1);
      m2[f] += delta * (mg[f] - mean[f]);
    }
  }
#pragma unroll
  for (int f = 0; f < kMoments; ++f)
    se[f] = G > 1 ? sqrt(m2[f] / (double)(G - 1) / (double)G) : __builtin_nan("");
}

// Per-run diagnostics, one block per run: particles, particles generated in
// the last step, accepted collisions so far (over the run's cells), and the
// sums of u, v, w and |c|^2 over its particles in FP64 (each thread a fixed
// stride, then a fixed-order tree: the same bits on every call).
template <typename real, int DIM>
__global__ __launch_bounds__(256) void k_diag(DevPtrs<real> d, int buf) {
  __shared__ double red[5][256];
  const int r = blockIdx.x, tid = threadIdx.x;
  const RunDev &R = d.runs[r];
  const Particles<real> P = d.P[buf];
  const int64_t n = d.n_alive[r];
  double su = 0.0, sv = 0.0, sw = 0.0, se = 0.0, sc = 0.0;
  for (int64_t i = tid; i < n; i += 256) {
    const typename Vec4<real>::type r4 = P.q[R.so + i];
    real z, w;
    load_zw<DIM>(P, R.so + i, z, w);
    const double u = (double)r4.z, v = (double)r4.w, ww = (double)w;
    su += u;
    sv += v;
    sw += ww;
    se += u * u + v * v + ww * ww;
  }
  for (int64_t c = tid; c < R.nc; c += 256) sc += (double)d.ncoll[R.co + c];
  red[0][tid] = su;
  red[1][tid] = sv;
  red[2][tid] = sw;
  red[3][tid] = se;
  red[4][tid] = sc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (tid < o)
      for (int f = 0; f < 5; ++f) red[f][tid] += red[f][tid + o];
    __syncthreads();
  }
  if (tid == 0) {
    double *out = d.diag + (int64_t)r * kDiag;
    out[0] = (double)n;
    out[1] = (double)d.n_gen[r];
    out[2] = red[4][0];
    out[3] = red[0][0];
    out[4] = red[1][0];
    out[5] = red[2][0];
    out[6] = red[3][0];
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

static inline int grid_for(int64_t n, int cap_blocks = 65536) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > cap_blocks) b = cap_blocks;
  return (int)b;
}

template <typename real>
static IndexArgs index_args(const Geometry &g, const DevPtrs<real> &d) {
  IndexArgs a;
  a.runs = d.runs;
  a.tile_run = d.tile_run;
  a.cell = d.cell;
  a.in = nullptr;
  a.out = d.lcr;
  a.kin = nullptr;
  a.kout = nullptr;
  a.hist = d.hist;
  a.tot = d.digit_tot;
  a.bin_start = d.bin_start;
  a.n_sorted = d.n_sorted;
  a.n_alive = d.n_alive;
  a.t0 = 0;
  a.t1 = g.n_tiles;
  a.r0 = 0;
  a.tile = g.tile;
  a.dstride = g.dstride;
  a.shift = 0;
  a.single = g.npass == 1;
  a.bitem = d.bitem;
  a.bitem_run = d.bitem_run;
  a.bfirst = d.bfirst;
  a.b0 = 0;
  a.b1 = g.n_bitems;
  return a;
}

static int digit_bits(int D) {
  int b = 0;
  while ((1 << b) < D) ++b;
  return b;
}

// Brackets a launch on stream `s` (in scope) with the profiling hook.
#define TIMED(kind, ...)                              \
  do {                                                \
    if (prof) prof->mark(prof->user, (kind), 1, s);   \
    __VA_ARGS__;                                      \
    if (prof) prof->mark(prof->user, (kind), 0, s);   \
  } while (0)

// Scans and scatter of the digit at bit `shift` over the runs [a.r0, a.r0 +
// n_runs) and tiles [a.t0, a.t1); the tile histograms are already in place.
static void index_pass(IndexArgs a, int max_digits, int n_runs, int shift, const int32_t *in, int32_t *out,
                       hipStream_t s, const Prof *prof = nullptr) {
  a.shift = shift;
  a.in = in;
  a.out = out;
  const size_t lds = (size_t)kWavesPerBlock * a.dstride * sizeof(uint32_t);
  const int wblocks = (a.t1 - a.t0 + kWavesPerBlock - 1) / kWavesPerBlock;
  TIMED(kKColScan, hipLaunchKernelGGL(k_colscan, dim3((max_digits + 255) / 256, n_runs), dim3(256), 0, s, a));
  TIMED(kKDigScan, hipLaunchKernelGGL(k_digscan, dim3(n_runs), dim3(256), 0, s, a));
  // positions come either from the slots (first pass) or, with their bins
  // (a.kin, always set together with a.in), from the previous pass
  // at most four blocks per CU (LDS beyond the cursor tables is unused):
  // measured faster than more, on the 32x32-cell box (1.24 -> 1.16 ms per
  // pass) and neutral on a 2M-cell grid's bucket pass
  constexpr size_t kTilePassLds = 40 * 1024;
  const size_t slds = lds < kTilePassLds ? kTilePassLds : lds;
  if (a.kout && a.in)
    TIMED(kKScatter, hipLaunchKernelGGL((k_scatter<true, true, false>), dim3(wblocks), dim3(256), slds, s, a));
  else if (a.kout)
    TIMED(kKScatter, hipLaunchKernelGGL((k_scatter<true, false, false>), dim3(wblocks), dim3(256), slds, s, a));
  else if (a.in)
    TIMED(kKScatter, hipLaunchKernelGGL((k_scatter<false, true, false>), dim3(wblocks), dim3(256), slds, s, a));
  else
    TIMED(kKScatter, hipLaunchKernelGGL((k_scatter<false, false, false>), dim3(wblocks), dim3(256), slds, s, a));
}

// The flight cells of the live particles in slots [s0, s1) (their run's
// first n_alive slots) of buffer buf, as Interaction leaves them after a step:
// after the initial fill and after a run's state is replaced.
template <typename real, int DIM>
__global__ __launch_bounds__(256) void k_next_cells(DevPtrs<real> d, int buf, int64_t s0, int64_t s1, int64_t tile) {
  const Particles<real> P = d.P[buf];
  for (int64_t i = s0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < s1;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int r = d.tile_run[i / tile];
    const RunDev &R = d.runs[r];
    if (i - R.so >= d.n_alive[r]) continue;
    const typename Vec4<real>::type r4 = P.q[i];
    real z, w;
    load_zw<DIM>(P, i, z, w);
    const real pos[3] = {r4.x, r4.y, z};
    const real vel[3] = {r4.z, r4.w, DIM == 3 ? w : (real)0};
    d.cell[i] = flight_cell<real, DIM>(Flight<real>(R), pos, vel);
  }
}

template <typename real>
void launch_next_cells(const Geometry &g, const DevPtrs<real> &d, int buf, int64_t so, int64_t n, hipStream_t s) {
  if (n <= 0) return;
  if (g.dim == 3)
    hipLaunchKernelGGL((k_next_cells<real, 3>), dim3(grid_for(n)), dim3(256), 0, s, d, buf, so, so + n, g.tile);
  else
    hipLaunchKernelGGL((k_next_cells<real, 2>), dim3(grid_for(n)), dim3(256), 0, s, d, buf, so, so + n, g.tile);
}

template <typename real>
void launch_init(const Geometry &g, const DevPtrs<real> &d, hipStream_t s) {
  hipLaunchKernelGGL(k_init_runs<real>, dim3((g.n_runs + 255) / 256), dim3(256), 0, s, d, g.n_runs);
  hipLaunchKernelGGL(k_init_cells<real>, dim3(grid_for(g.n_cells)), dim3(256), 0, s, d, g.n_cells);
  if (g.n_faces > 0)
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(g.n_faces)), dim3(256), 0, s, d.rem_f, g.n_faces, 0.0);
  if (g.n_samples > 0) {
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(g.acc_stride * g.n_samples)), dim3(256), 0, s, d.acc,
                       g.acc_stride * g.n_samples, 0.0);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, s, d.nsnap, (int64_t)g.n_samples, 0u);
  }
  if (g.dim == 3)
    hipLaunchKernelGGL((k_init_particles<real, 3>), dim3(grid_for(g.n_slots)), dim3(256), 0, s, d, g.n_slots,
                       g.tile);
  else
    hipLaunchKernelGGL((k_init_particles<real, 2>), dim3(grid_for(g.n_slots)), dim3(256), 0, s, d, g.n_slots,
                       g.tile);
  launch_next_cells<real>(g, d, 0, 0, g.n_slots, s);
}

// The work distribution of interaction mode m (0 lane, 1 wave, 2 cell items)
// in lane L.
template <typename real>
static Sched sched_of(const Geometry &g, const DevPtrs<real> &d, int m, const LaneRange &L, int lane_id) {
  Sched sc{};
  sc.mode = g.sched;
  if (g.sched == kSchedQueue) {
    sc.ctr = d.sched_ctr + ((int64_t)m * kMaxLanes + lane_id) * kXcds;
  } else if (g.sched == kSchedPerRun) {
    sc.ctr = d.sched_ctr + g.sched_ctr_off[m] + L.sr0[m];
    sc.first = d.sched_first + g.sched_first_off[m] + L.sr0[m];
    sc.nr = L.sr1[m] - L.sr0[m];
  }
  return sc;
}

// Workgroups of a launch: one per `per` items on the grid; the persistent
// grid of mode m otherwise (per-run scheduling: at least one workgroup, or
// wavefront, per run).
static int64_t sched_grid(const Geometry &g, const Sched &sc, int m, int64_t grid_blocks, int per) {
  if (sc.mode == kSchedGrid) return grid_blocks;
  const int64_t b = std::max<int64_t>(1, g.sched_blocks[m]);
  if (sc.mode == kSchedPerRun) return std::max<int64_t>(b, (sc.nr + per - 1) / per);
  return std::min<int64_t>(b, grid_blocks);  // never more workgroups than items
}

// One lane's share of a step: Generation, Motion, Indexing and Interaction of
// the runs [L.r0, L.r1) on stream s.  `moved` (may be null) is recorded once
// Motion is complete.
template <typename real, int DIM>
static void lane_step(const Geometry &g, const LaneRange &L, int lane_id, const DevPtrs<real> &d, int buf, hipStream_t s,
                      hipEvent_t moved, const Prof *prof) {
  const int n_runs = L.r1 - L.r0;
  const int32_t n_tiles = L.t1 - L.t0;
  if (L.i1 > L.i0) {
    TIMED(kKGenCount, hipLaunchKernelGGL(k_gen_count<real>, dim3(L.i1 - L.i0), dim3(256), 0, s, d, L.i0));
    TIMED(kKGenEmit, hipLaunchKernelGGL((k_gen_emit<real, DIM>), dim3(L.g1 - L.g0), dim3(256), 0, s, d, buf, L.i0,
                                        L.i1));
  }
  const size_t lds = (size_t)kWavesPerBlock * g.dstride * sizeof(uint32_t);
  const size_t mlds = lds + (size_t)kWavesPerBlock * kMotionQueueStage * sizeof(uint32_t);
  const int wblocks = (n_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
  IndexArgs a = index_args(g, d);
  a.t0 = L.t0;
  a.t1 = L.t1;
  a.r0 = L.r0;
  if (g.npass == 1) {
    if (g.any_solid)
      TIMED(kKMotion, hipLaunchKernelGGL((k_motion<real, DIM, true, true>), dim3(wblocks), dim3(256), mlds, s, d, buf,
                                         L.t0, L.t1, g.tile, g.dstride, 0));
    else
      TIMED(kKMotion, hipLaunchKernelGGL((k_motion<real, DIM, true, false>), dim3(wblocks), dim3(256), mlds, s, d,
                                         buf, L.t0, L.t1, g.tile, g.dstride, 0));
    TIMED(kKMotionWalls, hipLaunchKernelGGL((k_motion_walls<real, DIM, true>), dim3(n_tiles), dim3(256), 0, s, d,
                                            buf, L.t0, L.t1, g.tile, 0));
    if (moved) (void)hipEventRecord(moved, s);
    index_pass(a, g.max_nbin + 1, n_runs, 0, nullptr, d.lcr, s, prof);
  } else {
    // the first digit: the bucket (two-level sort) or the lowest 11 bits
    const int shift0 = g.bucketed ? kDigitBits : 0;
    if (g.any_solid)
      TIMED(kKMotion, hipLaunchKernelGGL((k_motion<real, DIM, false, true>), dim3(wblocks), dim3(256), mlds, s, d,
                                         buf, L.t0, L.t1, g.tile, g.dstride, shift0));
    else
      TIMED(kKMotion, hipLaunchKernelGGL((k_motion<real, DIM, false, false>), dim3(wblocks), dim3(256), mlds, s, d,
                                         buf, L.t0, L.t1, g.tile, g.dstride, shift0));
    TIMED(kKMotionWalls, hipLaunchKernelGGL((k_motion_walls<real, DIM, false>), dim3(n_tiles), dim3(256), 0, s, d,
                                            buf, L.t0, L.t1, g.tile, shift0));
    if (moved) (void)hipEventRecord(moved, s);
    if (g.bucketed) {
      // pass 1: positions by bucket, bins carried; pass 2: each bucket by its
      // low digit, straight into LCR and the bin starts
      a.kout = d.key_tmp;
      index_pass(a, kDigits, n_runs, kDigitBits, nullptr, d.lcr_tmp, s, prof);
      a.b0 = L.b0;
      a.b1 = L.b1;
      a.in = d.lcr_tmp;
      a.kin = d.key_tmp;
      a.kout = nullptr;
      a.out = d.lcr;
      a.shift = 0;
      const int iblocks = (L.b1 - L.b0 + kWavesPerBlock - 1) / kWavesPerBlock;
      TIMED(kKBucketItems, hipLaunchKernelGGL(k_bucket_items, dim3(n_runs), dim3(256), 0, s, a));
      if (iblocks > 0) {
        TIMED(kKDigCount, hipLaunchKernelGGL(k_digcount_bucket, dim3(iblocks), dim3(256), lds, s, a));
        const int max_nb = (g.max_nbin >> kDigitBits) + 1;
        TIMED(kKBucketScan, hipLaunchKernelGGL(k_bucket_scan, dim3(max_nb, n_runs), dim3(256), 0, s, a));
        // at most three blocks per CU (LDS beyond the cursor tables is
        // unused): with fewer wavefronts writing scattered stretches of the
        // LCR at once the pass runs faster on large grids, at the same HBM
        // traffic
        constexpr size_t kBucketPassLds = 52 * 1024;
        TIMED(kKScatter, hipLaunchKernelGGL((k_scatter<false, true, true>), dim3(iblocks), dim3(256),
                                            lds < kBucketPassLds ? kBucketPassLds : lds, s, a));
      }
    } else {
      // bins are carried through the passes: key_tmp and (free after Motion)
      // the wall queue alternate as key buffers
      int32_t *kbuf[2] = {d.key_tmp, (int32_t *)d.wallq};
      const int32_t *in = nullptr, *kin = nullptr;
      for (int p = 0; p < g.npass; ++p) {
        int32_t *out = ((g.npass - 1 - p) % 2 == 0) ? d.lcr : d.lcr_tmp;
        int32_t *kout = kbuf[p % 2];
        if (p > 0) {
          a.shift = kDigitBits * p;
          a.in = in;
          a.kin = kin;
          TIMED(kKDigCount, hipLaunchKernelGGL(k_digcount, dim3(wblocks), dim3(256), lds, s, a, 0));
        }
        a.kin = kin;
        a.kout = kout;
        index_pass(a, kDigits, n_runs, kDigitBits * p, in, out, s, prof);
        in = out;
        kin = kout;
      }
      TIMED(kKBinBounds, hipLaunchKernelGGL(k_bin_bounds, dim3(wblocks), dim3(256), 0, s, a, kin));
    }
    TIMED(kKBinFinalize,
          hipLaunchKernelGGL(k_bin_finalize, dim3((n_runs + 255) / 256), dim3(256), 0, s, a, L.r1, 1));
  }
  // Interaction.  A grid-mode launch has one workgroup per `per` items; more
  // than kMaxGridBlocks workgroups are split into launches over consecutive
  // item ranges (a dispatch holds fewer than 2^32 work-items).
  auto for_chunks = [](int64_t i0, int64_t i1, int per, auto &&launch) {
    const int64_t span = (int64_t)kMaxGridBlocks * per;
    for (int64_t c0 = i0; c0 < i1; c0 += span) {
      const int64_t c1 = std::min(c0 + span, i1);
      launch(c0, c1, dim3((unsigned)((c1 - c0 + per - 1) / per)));
    }
  };
  if (L.it1 > L.it0) {
    const int64_t nblk = (L.it1 - L.it0 + kCollideWaves - 1) / kCollideWaves;
    const Sched sc = sched_of(g, d, 0, L, lane_id);
    const size_t lb = (size_t)kCollideWaves * collide_wave_bytes<real>();
    const dim3 bl(kCollideWaves * 64);
    if (sc.mode == kSchedGrid) {
      for_chunks(L.it0, L.it1, kCollideWaves, [&](int64_t c0, int64_t c1, dim3 gr) {
        if (!g.any_sub)
          TIMED(kKCollide, hipLaunchKernelGGL((k_collide<real, DIM, false, false>), gr, bl, lb, s, d, buf, c0, c1, sc));
        else
          TIMED(kKCollide, hipLaunchKernelGGL((k_collide<real, DIM, false, true>), gr, bl, lb, s, d, buf, c0, c1, sc));
      });
    } else {
      const dim3 gr((unsigned)sched_grid(g, sc, 0, nblk, kCollideWaves));
      if (!g.any_sub)
        TIMED(kKCollide, hipLaunchKernelGGL((k_collide<real, DIM, true, false>), gr, bl, lb, s, d, buf, L.it0, L.it1,
                                            sc));
      else
        TIMED(kKCollide, hipLaunchKernelGGL((k_collide<real, DIM, true, true>), gr, bl, lb, s, d, buf, L.it0, L.it1,
                                            sc));
    }
  }
  if (L.wi1 > L.wi0) {
    const int64_t nblk = (L.wi1 - L.wi0 + kWavesPerBlock - 1) / kWavesPerBlock;
    const Sched sc = sched_of(g, d, 1, L, lane_id);
    const dim3 bl(256);
    if (sc.mode == kSchedGrid) {
      for_chunks(L.wi0, L.wi1, kWavesPerBlock, [&](int64_t c0, int64_t c1, dim3 gr) {
        if (!g.any_sub)
          TIMED(kKCollideWave, hipLaunchKernelGGL((k_collide_wave<real, DIM, false, false>), gr, bl, 0, s, d, buf, c0,
                                                  c1, sc));
        else
          TIMED(kKCollideWave, hipLaunchKernelGGL((k_collide_wave<real, DIM, false, true>), gr, bl, 0, s, d, buf, c0,
                                                  c1, sc));
      });
    } else {
      const dim3 gr((unsigned)sched_grid(g, sc, 1, nblk, kWavesPerBlock));
      if (!g.any_sub)
        TIMED(kKCollideWave, hipLaunchKernelGGL((k_collide_wave<real, DIM, true, false>), gr, bl, 0, s, d, buf, L.wi0,
                                                L.wi1, sc));
      else
        TIMED(kKCollideWave, hipLaunchKernelGGL((k_collide_wave<real, DIM, true, true>), gr, bl, 0, s, d, buf, L.wi0,
                                                L.wi1, sc));
    }
  }
  if (L.ci1 > L.ci0) {
    const int64_t nblk = L.ci1 - L.ci0;
    const Sched sc = sched_of(g, d, 2, L, lane_id);
    const bool grid_mode = sc.mode == kSchedGrid;
    const dim3 bl(256);
    if constexpr (std::is_same<real, float>::value) {
      if (grid_mode) {
        for_chunks(L.ci0, L.ci1, 1, [&](int64_t c0, int64_t c1, dim3 gr) {
          if (!g.any_sub)
            TIMED(kKCollideCell, hipLaunchKernelGGL((k_collide_pipe<DIM, false, false>), gr, bl, 0, s, d, buf, c0, c1,
                                                    sc));
          else
            TIMED(kKCollideCell, hipLaunchKernelGGL((k_collide_pipe<DIM, false, true>), gr, bl, 0, s, d, buf, c0, c1,
                                                    sc));
        });
      } else {
        const dim3 gr((unsigned)sched_grid(g, sc, 2, nblk, 1));
        if (!g.any_sub)
          TIMED(kKCollideCell, hipLaunchKernelGGL((k_collide_pipe<DIM, true, false>), gr, bl, 0, s, d, buf, L.ci0,
                                                  L.ci1, sc));
        else
          TIMED(kKCollideCell, hipLaunchKernelGGL((k_collide_pipe<DIM, true, true>), gr, bl, 0, s, d, buf, L.ci0,
                                                  L.ci1, sc));
      }
    } else {
      const size_t cb = (size_t)collide_cell_bytes<real>();
      if (grid_mode)
        for_chunks(L.ci0, L.ci1, 1, [&](int64_t c0, int64_t c1, dim3 gr) {
          TIMED(kKCollideCell, hipLaunchKernelGGL((k_collide_cell<real, DIM, false>), gr, bl, cb, s, d, buf, c0, c1,
                                                  sc));
        });
      else
        TIMED(kKCollideCell, hipLaunchKernelGGL((k_collide_cell<real, DIM, true>),
                                                dim3((unsigned)sched_grid(g, sc, 2, nblk, 1)), bl, cb, s, d, buf,
                                                L.ci0, L.ci1, sc));
    }
  }
}

template <typename real, int DIM>
static void step_dim(const Geometry &g, const DevPtrs<real> &d, int buf, hipStream_t s, const LaneStreams *ls,
                     const Prof *prof) {
  TIMED(kKStepBegin, hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(1), 0, s, d.step, d.sample_slot,
                                        d.sample_steps, g.n_samples, g.window_steps, g.window_stride));
  if (g.sched != kSchedGrid)  // the persistent grids' work counters start at zero every step
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(g.n_sched_ctr)), dim3(256), 0, s, d.sched_ctr, g.n_sched_ctr, 0u);
  if (g.n_lanes <= 1 || !ls) {
    LaneRange all = g.lane[0];
    if (g.n_lanes > 1) {
      all.r1 = g.lane[g.n_lanes - 1].r1;
      all.t1 = g.lane[g.n_lanes - 1].t1;
      all.f1 = g.lane[g.n_lanes - 1].f1;
      all.i1 = g.lane[g.n_lanes - 1].i1;
      all.g1 = g.lane[g.n_lanes - 1].g1;
      all.it1 = g.lane[g.n_lanes - 1].it1;
      all.ci1 = g.lane[g.n_lanes - 1].ci1;
      all.wi1 = g.lane[g.n_lanes - 1].wi1;
      all.b1 = g.lane[g.n_lanes - 1].b1;
      for (int m = 0; m < 3; ++m) all.sr1[m] = g.lane[g.n_lanes - 1].sr1[m];
    }
    lane_step<real, DIM>(g, all, 0, d, buf, s, nullptr, prof);
  } else {
    (void)hipEventRecord(ls->fork, s);
    for (int l = 0; l < g.n_lanes; ++l) {
      hipStream_t q = ls->s[l];
      (void)hipStreamWaitEvent(q, ls->fork, 0);
      if (l > 0) (void)hipStreamWaitEvent(q, ls->moved[l - 1], 0);
      lane_step<real, DIM>(g, g.lane[l], l, d, buf, q, ls->moved[l], prof);
      (void)hipEventRecord(ls->done[l], q);
    }
    for (int l = 0; l < g.n_lanes; ++l) (void)hipStreamWaitEvent(s, ls->done[l], 0);
  }
  if (g.n_samples > 0)
    TIMED(kKAccumulate, hipLaunchKernelGGL(k_accumulate<real>, dim3(grid_for(g.acc_stride)), dim3(256), 0, s, d,
                                           -1, g.acc_stride, g.n_eg));
}

template <typename real>
void launch_step(const Geometry &g, const DevPtrs<real> &d, int buf, hipStream_t s, const LaneStreams *ls,
                 const Prof *prof) {
  if (g.dim == 3) step_dim<real, 3>(g, d, buf, s, ls, prof);
  else step_dim<real, 2>(g, d, buf, s, ls, prof);
}

template <typename real>
void launch_sample(const Geometry &g, const DevPtrs<real> &d, int buf, int slot, hipStream_t s, const Prof *prof) {
  // (a dispatch holds fewer than 2^32 work-items: kMaxGridBlocks workgroups
  // of four cells at a time)
  for (int64_t c0 = 0; c0 < g.n_cells; c0 += (int64_t)kMaxGridBlocks * 4) {
    const int64_t nb = std::min<int64_t>((g.n_cells - c0 + 3) / 4, kMaxGridBlocks);
    TIMED(kKSample, hipLaunchKernelGGL(k_sample_cells<real>, dim3((unsigned)nb), dim3(256), 0, s, d, buf, c0,
                                       g.n_cells));
  }
  TIMED(kKAccumulate, hipLaunchKernelGGL(k_accumulate<real>, dim3(grid_for(g.acc_stride)), dim3(256), 0, s, d, slot,
                                         g.acc_stride, g.n_eg));
}

template <typename real>
void launch_moments(const Geometry &g, const DevPtrs<real> &d, int slot, int eg0, int n_groups, int nc,
                    int n_runs_ens, hipStream_t s) {
  hipLaunchKernelGGL(k_moments<real>, dim3((nc + 255) / 256), dim3(256), 0, s, d, slot, g.acc_stride, eg0,
                     n_groups, nc, n_runs_ens, g.max_nc);
}

template <typename real>
void launch_diag(const Geometry &g, const DevPtrs<real> &d, int buf, hipStream_t s) {
  if (g.dim == 3) hipLaunchKernelGGL((k_diag<real, 3>), dim3(g.n_runs), dim3(256), 0, s, d, buf);
  else hipLaunchKernelGGL((k_diag<real, 2>), dim3(g.n_runs), dim3(256), 0, s, d, buf);
}

template <typename real, int DIM, bool SUB>
static void occupancy_dim(int out[3]) {
  auto occ = [](const void *k, int threads, size_t lds) {
    int b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k, threads, lds) != hipSuccess) b = 1;
    return b > 0 ? b : 1;
  };
  out[0] = occ(reinterpret_cast<const void *>(&k_collide<real, DIM, true, SUB>), kCollideWaves * 64,
               (size_t)kCollideWaves * collide_wave_bytes<real>());
  out[1] = occ(reinterpret_cast<const void *>(&k_collide_wave<real, DIM, true, SUB>), 256, 0);
  if constexpr (std::is_same<real, float>::value)
    out[2] = occ(reinterpret_cast<const void *>(&k_collide_pipe<DIM, true, SUB>), 256, 0);
  else
    out[2] = occ(reinterpret_cast<const void *>(&k_collide_cell<real, DIM, true>), 256,
                 (size_t)collide_cell_bytes<real>());
}

// Workgroups per CU of the persistent Interaction kernels the batch launches.
void collide_occupancy(const Geometry &g, int out[3]) {
  if (g.fp64) {
    if (g.dim == 3) g.any_sub ? occupancy_dim<double, 3, true>(out) : occupancy_dim<double, 3, false>(out);
    else g.any_sub ? occupancy_dim<double, 2, true>(out) : occupancy_dim<double, 2, false>(out);
  } else {
    if (g.dim == 3) g.any_sub ? occupancy_dim<float, 3, true>(out) : occupancy_dim<float, 3, false>(out);
    else g.any_sub ? occupancy_dim<float, 2, true>(out) : occupancy_dim<float, 2, false>(out);
  }
}

template void launch_init<float>(const Geometry &, const DevPtrs<float> &, hipStream_t);
template void launch_diag<float>(const Geometry &, const DevPtrs<float> &, int, hipStream_t);
template void launch_diag<double>(const Geometry &, const DevPtrs<double> &, int, hipStream_t);
template void launch_init<double>(const Geometry &, const DevPtrs<double> &, hipStream_t);
template void launch_next_cells<float>(const Geometry &, const DevPtrs<float> &, int, int64_t, int64_t, hipStream_t);
template void launch_next_cells<double>(const Geometry &, const DevPtrs<double> &, int, int64_t, int64_t,
                                        hipStream_t);
template void launch_step<float>(const Geometry &, const DevPtrs<float> &, int, hipStream_t, const LaneStreams *,
                                 const Prof *);
template void launch_step<double>(const Geometry &, const DevPtrs<double> &, int, hipStream_t, const LaneStreams *,
                                  const Prof *);
template void launch_sample<float>(const Geometry &, const DevPtrs<float> &, int, int, hipStream_t,
                                   const Prof *);
template void launch_sample<double>(const Geometry &, const DevPtrs<double> &, int, int, hipStream_t,
                                    const Prof *);
template void launch_moments<float>(const Geometry &, const DevPtrs<float> &, int, int, int, int, int, hipStream_t);
template void launch_moments<double>(const Geometry &, const DevPtrs<double> &, int, int, int, int, int,
                                     hipStream_t);

// ---------------------------------------------------------------------------
// Stand-alone stable counting sort (same kernels as the step's Indexing)
// ---------------------------------------------------------------------------

namespace {
struct SortLayout {
  int64_t tile;
  int32_t nt;
  int npass;
  int D;
  size_t off_run, off_tile_run, off_hist, off_tot, off_ns, off_na, off_tmp, off_k0, off_k1, total;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

SortLayout sort_layout(int64_t n, int32_t nbins, int tile_chunks) {
  SortLayout L;
  L.tile = (int64_t)tile_chunks * kWave;
  L.nt = (int32_t)std::max<int64_t>(1, (n + L.tile - 1) / L.tile);
  L.npass = 1;
  if (nbins > kDigits) {
    int bits = digit_bits(nbins);
    L.npass = (bits + kDigitBits - 1) / kDigitBits;
  }
  L.D = L.npass == 1 ? nbins : kDigits;
  size_t o = 0;
  L.off_run = o;
  o = align256(o + sizeof(RunDev));
  L.off_tile_run = o;
  o = align256(o + (size_t)L.nt * 4);
  L.off_hist = o;
  o = align256(o + (size_t)L.nt * L.D * 4);
  L.off_tot = o;
  o = align256(o + (size_t)L.D * 4);
  L.off_ns = o;
  o = align256(o + 4);
  L.off_na = o;
  o = align256(o + 4);
  L.off_tmp = o;
  o = align256(o + (L.npass > 1 ? (size_t)n * 4 : 0));
  L.off_k0 = o;
  o = align256(o + (L.npass > 1 ? (size_t)n * 4 : 0));
  L.off_k1 = o;
  o = align256(o + (L.npass > 1 ? (size_t)n * 4 : 0));
  L.total = o;
  return L;
}

__global__ void k_sort_setup(RunDev rd, RunDev *dst, int32_t *tile_run, int32_t nt, int32_t *ns, int32_t n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    *dst = rd;
    *ns = n;
  }
  for (int t = i; t < nt; t += gridDim.x * blockDim.x) tile_run[t] = 0;
}
}  // namespace

size_t counting_sort_workspace(int64_t n, int32_t nbins, int tile_chunks) {
  return sort_layout(n, nbins, tile_chunks).total;
}

void launch_counting_sort(const int32_t *keys, int64_t n, int32_t nbins, int32_t *lcr, uint32_t *start,
                          void *work, int tile_chunks, hipStream_t s) {
  SortLayout L = sort_layout(n, nbins, tile_chunks);
  char *w = (char *)work;
  RunDev rd = {};
  rd.so = 0;
  rd.cap = (int64_t)L.nt * L.tile;
  rd.nc = nbins - 1;
  rd.nbin = nbins - 1;
  rd.sub = 1;
  rd.S = 1;
  rd.nt = L.nt;
  rd.ndig = L.D;
  RunDev *runs = (RunDev *)(w + L.off_run);
  int32_t *tile_run = (int32_t *)(w + L.off_tile_run);
  int32_t *ns = (int32_t *)(w + L.off_ns);
  hipLaunchKernelGGL(k_sort_setup, dim3(grid_for(L.nt, 1024)), dim3(256), 0, s, rd, runs, tile_run, L.nt, ns,
                     (int32_t)n);
  IndexArgs a;
  a.runs = runs;
  a.tile_run = tile_run;
  a.cell = keys;
  a.in = nullptr;
  a.out = lcr;
  a.kin = nullptr;
  a.kout = nullptr;
  a.hist = (uint32_t *)(w + L.off_hist);
  a.tot = (uint32_t *)(w + L.off_tot);
  a.bin_start = start;
  a.n_sorted = ns;
  a.n_alive = (int32_t *)(w + L.off_na);
  a.t0 = 0;
  a.t1 = L.nt;
  a.r0 = 0;
  a.tile = L.tile;
  a.dstride = L.D;
  a.shift = 0;
  a.single = L.npass == 1;
  a.bitem = nullptr;
  a.bitem_run = nullptr;
  a.bfirst = nullptr;
  a.b0 = a.b1 = 0;
  const size_t lds = (size_t)kWavesPerBlock * a.dstride * sizeof(uint32_t);
  const int wblocks = (L.nt + kWavesPerBlock - 1) / kWavesPerBlock;
  int32_t *tmp = (int32_t *)(w + L.off_tmp);
  int32_t *kbuf[2] = {(int32_t *)(w + L.off_k0), (int32_t *)(w + L.off_k1)};
  const int32_t *in = nullptr, *kin = nullptr;
  for (int p = 0; p < L.npass; ++p) {
    int32_t *out = ((L.npass - 1 - p) % 2 == 0) ? lcr : tmp;
    int32_t *kout = L.npass > 1 ? kbuf[p % 2] : nullptr;
    a.shift = kDigitBits * p;
    a.in = in;
    a.kin = kin;
    hipLaunchKernelGGL(k_digcount, dim3(wblocks), dim3(256), lds, s, a, 0);
    a.kout = kout;
    index_pass(a, L.D, 1, kDigitBits * p, in, out, s);
    in = out;
    kin = kout;
  }
  if (L.npass > 1) {
    hipLaunchKernelGGL(k_bin_bounds, dim3(wblocks), dim3(256), 0, s, a, kin);
    hipLaunchKernelGGL(k_bin_finalize, dim3(1), dim3(256), 0, s, a, 1, 0);
  }
}

}  // namespace dsmc
