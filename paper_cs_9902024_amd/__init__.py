"""MI355X-native unsteady-DSMC inner loop: Python binding of ``libdsmc.so``.

The functions below carry the names of the C ABI in ``include/dsmc.h`` and do
argument marshalling only: every step of the method runs in the HIP kernels
of the library.  PyTorch supplies the device arena (one uint8 tensor) and the
stream.  If the library is not built, importing works but every call raises
``DsmcError`` -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdsmc.so")

DSMC_OK = 0
STATUS_NAMES = {0: "DSMC_OK", -1: "DSMC_EINVAL", -2: "DSMC_ESIZE", -3: "DSMC_ECAPACITY",
                -4: "DSMC_EDEVICE", -5: "DSMC_ESTATE", -6: "DSMC_EUNSUPPORTED",
                -7: "DSMC_EBOUNCE", -8: "DSMC_EREJECT", -9: "DSMC_ENUMERIC"}
BC = {"specular": 0, "diffuse": 1, "inflow": 2, "outflow": 3}
NSUM = 7
NMOM = 8
MOMENT_NAMES = ("n", "ux", "uy", "uz", "T", "Tx", "Ty", "Tz")

# Every symbol declared in include/dsmc.h.
EXPORTS = ("dsmc_required_bytes", "dsmc_init_runs", "dsmc_step", "dsmc_sample", "dsmc_read_moments",
           "dsmc_read_accum", "dsmc_sync", "dsmc_destroy", "dsmc_last_error", "dsmc_get_info",
           "dsmc_get_state", "dsmc_set_state", "dsmc_get_lcr", "dsmc_get_cell_state",
           "dsmc_get_counts", "dsmc_counting_sort_bytes", "dsmc_counting_sort",
           "dsmc_set_profiling", "dsmc_kernel_times", "dsmc_kernel_name", "dsmc_autotune_bytes",
           "dsmc_autotune", "dsmc_counting_sort_noalloc", "dsmc_get_sample_counts", "dsmc_get_diag",
           "dsmc_checkpoint_bytes", "dsmc_checkpoint", "dsmc_restore")
NKERNELS = 19
NINFO = 10
NDIAG = 7
DIAG_NAMES = ("particles", "generated", "collisions", "sum_u", "sum_v", "sum_w", "sum_c2")


class DsmcError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str = ""):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)} {msg}".strip())


class dsmc_run_spec(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("dt", C.c_double), ("fnum_sigma", C.c_double), ("omega", C.c_double),
                ("c_ref", C.c_double), ("face_bc", C.c_int32 * 6), ("face_T", C.c_double * 6),
                ("inflow_n", C.c_double), ("inflow_U", C.c_double), ("inflow_T", C.c_double),
                ("capacity", C.c_int64), ("n_init", C.c_int64), ("init_U", C.c_double * 3),
                ("init_T", C.c_double), ("run_id", C.c_uint32), ("seed", C.c_uint32),
                ("ensemble", C.c_int32), ("subcells", C.c_int32), ("solid_mask", C.c_void_p),
                ("solid_T", C.c_double), ("ntc_nbar_alpha", C.c_double)]


class dsmc_options(C.Structure):
    _fields_ = [("state_fp64", C.c_int32), ("n_groups", C.c_int32), ("n_samples", C.c_int32),
                ("sample_steps", C.POINTER(C.c_int32)), ("use_graph", C.c_int32),
                ("tile_chunks", C.c_int32), ("collide_mode", C.c_int32), ("n_streams", C.c_int32),
                ("window_steps", C.c_int32), ("window_stride", C.c_int32), ("sched", C.c_int32),
                ("sched_blocks", C.c_int32)]


_lib = None


def lib():
    """Load libdsmc.so (never builds it, never falls back)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise DsmcError(-4, "load", f"{LIB_PATH} is not built "
                            "(run paper_cs_9902024_amd.build.build())")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_size_t
        dp = C.POINTER(C.c_double)
        L.dsmc_required_bytes.argtypes = [C.POINTER(dsmc_run_spec), i32, C.POINTER(dsmc_options),
                                          C.POINTER(sz)]
        L.dsmc_init_runs.argtypes = [C.POINTER(dsmc_run_spec), i32, C.POINTER(dsmc_options), vp, sz,
                                     vp, C.POINTER(vp)]
        L.dsmc_step.argtypes = [vp, i32]
        L.dsmc_sample.argtypes = [vp, i32]
        L.dsmc_read_moments.argtypes = [vp, i32, i32, dp, dp, sz]
        L.dsmc_read_accum.argtypes = [vp, i32, i32, dp, sz]
        L.dsmc_sync.argtypes = [vp]
        L.dsmc_destroy.argtypes = [vp]
        L.dsmc_destroy.restype = None
        L.dsmc_last_error.argtypes = [vp]
        L.dsmc_last_error.restype = C.c_char_p
        L.dsmc_get_info.argtypes = [vp, C.POINTER(i64)]
        L.dsmc_get_state.argtypes = [vp, i32, dp, i64, C.POINTER(i64)]
        L.dsmc_set_state.argtypes = [vp, i32, dp, i64]
        L.dsmc_get_lcr.argtypes = [vp, i32, vp, vp, vp, i64, C.POINTER(i64)]
        L.dsmc_get_cell_state.argtypes = [vp, i32, vp, vp, vp, vp]
        L.dsmc_get_counts.argtypes = [vp, C.POINTER(i64), i32]
        L.dsmc_counting_sort_bytes.argtypes = [i64, i32, C.POINTER(sz)]
        L.dsmc_counting_sort.argtypes = [vp, i64, i32, vp, vp, vp, sz, vp]
        L.dsmc_counting_sort_noalloc.argtypes = [vp, i64, i32, vp, vp, vp]
        L.dsmc_get_sample_counts.argtypes = [vp, C.POINTER(i64), i32]
        L.dsmc_get_diag.argtypes = [vp, dp, i32]
        L.dsmc_checkpoint_bytes.argtypes = [vp, C.POINTER(sz)]
        L.dsmc_checkpoint.argtypes = [vp, vp, sz]
        L.dsmc_restore.argtypes = [vp, vp, sz]
        L.dsmc_set_profiling.argtypes = [vp, i32]
        L.dsmc_kernel_times.argtypes = [vp, dp, C.POINTER(i64), i32]
        L.dsmc_kernel_name.argtypes = [i32]
        L.dsmc_autotune_bytes.argtypes = [C.POINTER(dsmc_run_spec), i32, C.POINTER(dsmc_options),
                                          C.POINTER(sz)]
        L.dsmc_autotune.argtypes = [C.POINTER(dsmc_run_spec), i32, C.POINTER(dsmc_options), vp, sz, vp, i32,
                                    vp, sz, C.c_char_p, C.POINTER(dsmc_options), dp]
        L.dsmc_kernel_name.restype = C.c_char_p
        for f in EXPORTS:
            if f not in ("dsmc_destroy", "dsmc_last_error", "dsmc_kernel_name"):
                getattr(L, f).restype = C.c_int32
        _lib = L
    return _lib


# calls whose failures without a context leave their message for
# dsmc_last_error(NULL)
_FREE_MSG = ("dsmc_required_bytes", "dsmc_init_runs", "dsmc_autotune", "dsmc_autotune_bytes")


def _check(st: int, where: str, ctx=None):
    if st != DSMC_OK:
        msg = lib().dsmc_last_error(ctx).decode() if ctx or where in _FREE_MSG else ""
        raise DsmcError(st, where, msg)


# ---------------------------------------------------------------------------
# Argument structs
# ---------------------------------------------------------------------------

def make_run_spec(rs) -> dsmc_run_spec:
    """dsmc_run_spec from a ``workloads.RunSpec``.  A solid mask is passed as
    a pointer to a contiguous byte copy that the returned struct keeps alive."""
    s = dsmc_run_spec()
    if rs.solid is not None:
        mask = np.ascontiguousarray(rs.solid, dtype=np.uint8).ravel()
        if mask.size != rs.nx * rs.ny * rs.nz:
            raise DsmcError(-1, "make_run_spec", "solid mask must have one entry per cell")
        s._mask = mask
        s.solid_mask = mask.ctypes.data
        s.solid_T = rs.solid_T
    s.dim, s.nx, s.ny, s.nz = rs.dim, rs.nx, rs.ny, rs.nz
    s.lx, s.ly, s.lz = rs.lx, rs.ly, rs.lz
    s.dt, s.fnum_sigma, s.omega, s.c_ref = rs.dt, rs.fnum_sigma, rs.omega, rs.c_ref
    for f in range(6):
        s.face_bc[f] = BC[rs.face_bc[f]]
        s.face_T[f] = rs.face_T[f]
    s.inflow_n, s.inflow_U, s.inflow_T = rs.inflow_n, rs.inflow_U, rs.inflow_T
    s.capacity, s.n_init = rs.capacity, rs.n_init
    for a in range(3):
        s.init_U[a] = rs.init_U[a]
    s.init_T = rs.init_T
    s.run_id, s.seed = rs.run_id & 0xFFFFFFFF, rs.seed & 0xFFFFFFFF
    s.ensemble = rs.ensemble
    s.subcells = getattr(rs, "subcells", 1)
    s.ntc_nbar_alpha = getattr(rs, "ntc_nbar_alpha", 0.0)
    return s


def make_options(state_fp64: bool, n_groups: int, sample_steps: Sequence[int],
                 use_graph: bool = False, tile_chunks: int = 0, collide_mode: int = 0,
                 n_streams: int = 0, window_steps: int = 0, window_stride: int = 0, sched: int = 0,
                 sched_blocks: int = 0):
    steps = (C.c_int32 * max(1, len(sample_steps)))(*sample_steps)
    o = dsmc_options()
    o.state_fp64 = int(bool(state_fp64))
    o.n_groups = int(n_groups)
    o.n_samples = len(sample_steps)
    o.sample_steps = C.cast(steps, C.POINTER(C.c_int32))
    o.use_graph = int(bool(use_graph))
    o.tile_chunks = int(tile_chunks)
    o.collide_mode = int(collide_mode)
    o.n_streams = int(n_streams)
    o.window_steps = int(window_steps)
    o.window_stride = int(window_stride)
    o.sched = int(sched)
    o.sched_blocks = int(sched_blocks)
    o._keep = steps
    return o


def _specs(runs):
    keep = [make_run_spec(r) for r in runs]
    arr = (dsmc_run_spec * len(runs))(*keep)
    arr._keep = keep          # the masks the array points to
    return arr


# ---------------------------------------------------------------------------
# The C ABI, one wrapper per entry point
# ---------------------------------------------------------------------------

def dsmc_autotune_bytes(specs, opt) -> int:
    n = C.c_size_t(0)
    _check(lib().dsmc_autotune_bytes(specs, len(specs), C.byref(opt), C.byref(n)), "dsmc_autotune_bytes")
    return n.value


def dsmc_autotune(specs, opt, arena_ptr: int, arena_bytes: int, stream: int, n_steps: int,
                  tune_cache: Optional[str] = None, start: Optional[np.ndarray] = None):
    """Returns (best dsmc_options, ms per step).  start: a checkpoint (uint8
    array from dsmc_checkpoint) every candidate is restored from."""
    best = dsmc_options()
    ms = C.c_double(0)
    path = tune_cache.encode() if tune_cache else None
    if start is not None:
        start = np.ascontiguousarray(start, dtype=np.uint8)
    sp, sb = (start.ctypes.data, start.size) if start is not None else (None, 0)
    _check(lib().dsmc_autotune(specs, len(specs), C.byref(opt), C.c_void_p(arena_ptr), arena_bytes,
                               C.c_void_p(stream), n_steps, C.c_void_p(sp), sb, path, C.byref(best),
                               C.byref(ms)), "dsmc_autotune")
    best._keep = getattr(opt, "_keep", None)
    return best, ms.value


def dsmc_required_bytes(specs, opt) -> int:
    n = C.c_size_t(0)
    _check(lib().dsmc_required_bytes(specs, len(specs), C.byref(opt), C.byref(n)), "dsmc_required_bytes")
    return n.value


def dsmc_init_runs(specs, opt, arena_ptr: int, arena_bytes: int, stream: int):
    ctx = C.c_void_p(0)
    _check(lib().dsmc_init_runs(specs, len(specs), C.byref(opt), C.c_void_p(arena_ptr), arena_bytes,
                                C.c_void_p(stream), C.byref(ctx)), "dsmc_init_runs")
    return ctx


def dsmc_step(ctx, n_steps: int = 1):
    _check(lib().dsmc_step(ctx, n_steps), "dsmc_step", ctx)


def dsmc_sample(ctx, sample_index: int):
    _check(lib().dsmc_sample(ctx, sample_index), "dsmc_sample", ctx)


def dsmc_read_moments(ctx, sample_index: int, ensemble: int, n_cells: int):
    out = np.zeros((n_cells, NMOM))
    se = np.zeros((n_cells, NMOM))
    dp = C.POINTER(C.c_double)
    _check(lib().dsmc_read_moments(ctx, sample_index, ensemble, out.ctypes.data_as(dp),
                                   se.ctypes.data_as(dp), out.size), "dsmc_read_moments", ctx)
    return out, se


def dsmc_read_accum(ctx, sample_index: int, ensemble: int, n_groups: int, n_cells: int):
    out = np.zeros((n_groups, n_cells, NSUM))
    _check(lib().dsmc_read_accum(ctx, sample_index, ensemble,
                                 out.ctypes.data_as(C.POINTER(C.c_double)), out.size),
           "dsmc_read_accum", ctx)
    return out


def dsmc_sync(ctx):
    _check(lib().dsmc_sync(ctx), "dsmc_sync", ctx)


def dsmc_destroy(ctx):
    lib().dsmc_destroy(ctx)


def dsmc_last_error(ctx) -> str:
    return lib().dsmc_last_error(ctx).decode()


def dsmc_get_info(ctx) -> dict:
    a = (C.c_int64 * NINFO)()
    _check(lib().dsmc_get_info(ctx, a), "dsmc_get_info", ctx)
    return dict(zip(("steps", "runs", "ensembles", "fp64", "passes", "tiles", "slots", "error", "lanes",
                     "graph"), list(a)))


def dsmc_get_state(ctx, run: int) -> np.ndarray:
    n = C.c_int64(0)
    _check(lib().dsmc_get_state(ctx, run, None, 0, C.byref(n)), "dsmc_get_state", ctx)
    out = np.zeros((6, n.value))
    _check(lib().dsmc_get_state(ctx, run, out.ctypes.data_as(C.POINTER(C.c_double)), n.value,
                                C.byref(n)), "dsmc_get_state", ctx)
    return out[:, :n.value]


def dsmc_set_state(ctx, run: int, state: np.ndarray):
    st = np.ascontiguousarray(state, dtype=np.float64)
    _check(lib().dsmc_set_state(ctx, run, st.ctypes.data_as(C.POINTER(C.c_double)), st.shape[1]),
           "dsmc_set_state", ctx)


def dsmc_get_lcr(ctx, run: int, capacity: int, n_cells: int):
    lcr = np.zeros(capacity, np.int32)
    cell = np.zeros(capacity, np.int32)
    start = np.zeros(n_cells + 2, np.int64)
    n = C.c_int64(0)
    _check(lib().dsmc_get_lcr(ctx, run, lcr.ctypes.data, cell.ctypes.data, start.ctypes.data, capacity,
                              C.byref(n)), "dsmc_get_lcr", ctx)
    return lcr[:n.value], cell[:n.value], start


def dsmc_get_cell_state(ctx, run: int, n_cells: int) -> dict:
    rem, gmax, nbar = np.zeros(n_cells), np.zeros(n_cells), np.zeros(n_cells)
    ncoll = np.zeros(n_cells, np.int64)
    _check(lib().dsmc_get_cell_state(ctx, run, rem.ctypes.data, gmax.ctypes.data, ncoll.ctypes.data,
                                     nbar.ctypes.data), "dsmc_get_cell_state", ctx)
    return {"rem": rem, "gmax": gmax, "ncoll": ncoll, "nbar": nbar}


def dsmc_get_counts(ctx, n_runs: int) -> np.ndarray:
    out = np.zeros((n_runs, 2), np.int64)
    _check(lib().dsmc_get_counts(ctx, out.ctypes.data_as(C.POINTER(C.c_int64)), n_runs),
           "dsmc_get_counts", ctx)
    return out


def dsmc_get_sample_counts(ctx, n_samples: int) -> np.ndarray:
    out = np.zeros(max(n_samples, 1), np.int64)
    _check(lib().dsmc_get_sample_counts(ctx, out.ctypes.data_as(C.POINTER(C.c_int64)), n_samples),
           "dsmc_get_sample_counts", ctx)
    return out[:n_samples]


def dsmc_get_diag(ctx, n_runs: int) -> np.ndarray:
    out = np.zeros((n_runs, NDIAG))
    _check(lib().dsmc_get_diag(ctx, out.ctypes.data_as(C.POINTER(C.c_double)), n_runs),
           "dsmc_get_diag", ctx)
    return out


def dsmc_checkpoint_bytes(ctx) -> int:
    n = C.c_size_t(0)
    _check(lib().dsmc_checkpoint_bytes(ctx, C.byref(n)), "dsmc_checkpoint_bytes", ctx)
    return n.value


def dsmc_checkpoint(ctx) -> np.ndarray:
    """The checkpoint as a host byte array (8-byte aligned)."""
    n = dsmc_checkpoint_bytes(ctx)
    buf = np.zeros((n + 7) // 8, np.uint64).view(np.uint8)[:n]
    _check(lib().dsmc_checkpoint(ctx, buf.ctypes.data, n), "dsmc_checkpoint", ctx)
    return buf


def dsmc_restore(ctx, buf: np.ndarray):
    b = np.ascontiguousarray(buf, dtype=np.uint8)
    if b.ctypes.data % 8:      # the library wants an 8-byte aligned buffer
        al = np.zeros((b.size + 7) // 8, np.uint64).view(np.uint8)[:b.size]
        al[:] = b
        b = al
    _check(lib().dsmc_restore(ctx, b.ctypes.data, b.size), "dsmc_restore", ctx)


def dsmc_set_profiling(ctx, on: bool):
    _check(lib().dsmc_set_profiling(ctx, int(bool(on))), "dsmc_set_profiling", ctx)


def dsmc_kernel_name(kind: int) -> Optional[str]:
    n = lib().dsmc_kernel_name(kind)
    return n.decode() if n else None


def dsmc_kernel_times(ctx) -> dict:
    """{kernel name: (total ms, launches)} since the last call (resets)."""
    ms = np.zeros(NKERNELS)
    k = np.zeros(NKERNELS, np.int64)
    _check(lib().dsmc_kernel_times(ctx, ms.ctypes.data_as(C.POINTER(C.c_double)),
                                   k.ctypes.data_as(C.POINTER(C.c_int64)), NKERNELS),
           "dsmc_kernel_times", ctx)
    return {dsmc_kernel_name(i): (float(ms[i]), int(k[i])) for i in range(NKERNELS) if k[i]}


def dsmc_counting_sort_bytes(n: int, nbins: int) -> int:
    b = C.c_size_t(0)
    _check(lib().dsmc_counting_sort_bytes(n, nbins, C.byref(b)), "dsmc_counting_sort_bytes")
    return b.value


def dsmc_counting_sort(keys_ptr: int, n: int, nbins: int, lcr_ptr: int, start_ptr: int, work_ptr: int,
                       work_bytes: int, stream: int):
    _check(lib().dsmc_counting_sort(C.c_void_p(keys_ptr), n, nbins, C.c_void_p(lcr_ptr),
                                    C.c_void_p(start_ptr), C.c_void_p(work_ptr), work_bytes,
                                    C.c_void_p(stream)), "dsmc_counting_sort")


SORT_SCRATCH_BYTES = 32 << 20  # DSMC_SORT_SCRATCH_BYTES


def dsmc_counting_sort_noalloc(keys_ptr: int, n: int, nbins: int, lcr_ptr: int, start_ptr: int,
                               stream: int):
    _check(lib().dsmc_counting_sort_noalloc(C.c_void_p(keys_ptr), n, nbins, C.c_void_p(lcr_ptr),
                                            C.c_void_p(start_ptr), C.c_void_p(stream)),
           "dsmc_counting_sort_noalloc")


# ---------------------------------------------------------------------------
# Convenience: one context over torch-owned device memory
# ---------------------------------------------------------------------------

class Ensemble:
    """Runs of a ``workloads.Workload`` (or an explicit run list) in one
    context on the current CUDA/HIP device and stream."""

    def __init__(self, runs, sample_steps: Sequence[int] = (), state_fp64: bool = False,
                 n_groups: int = 1, use_graph: bool = False, tile_chunks: int = 0,
                 collide_mode: int = 0, n_streams: int = 0, window_steps: int = 0,
                 window_stride: int = 0, sched: int = 0, sched_blocks: int = 0, device=None,
                 stream=None):
        import torch
        if not torch.cuda.is_available():
            raise DsmcError(-4, "Ensemble", "no GPU visible to torch")
        self.runs = list(runs)
        self.specs = _specs(self.runs)
        self.opt = make_options(state_fp64, n_groups, list(sample_steps), use_graph, tile_chunks,
                                collide_mode, n_streams, window_steps, window_stride, sched,
                                sched_blocks)
        self.nbytes = dsmc_required_bytes(self.specs, self.opt)
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.arena = torch.empty(self.nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self.ctx = dsmc_init_runs(self.specs, self.opt, self.arena.data_ptr(), self.nbytes,
                                  self.stream.cuda_stream)
        self.ensembles = []
        for r in self.runs:
            if r.ensemble not in self.ensembles:
                self.ensembles.append(r.ensemble)

    @staticmethod
    def autotune(runs, sample_steps: Sequence[int] = (), state_fp64: bool = False, n_groups: int = 1,
                 use_graph: bool = False, n_steps: int = 5, device=None, stream=None,
                 tune_cache: Optional[str] = None, window_steps: int = 0, window_stride: int = 0,
                 start: Optional[np.ndarray] = None) -> dict:
        """Measures the library's candidate tuning settings on these runs
        (dsmc_autotune) in a scratch arena, from the initial fill or from the
        checkpoint `start` (Ensemble.checkpoint() of the same problem), or
        takes them from the tune cache file when it holds this problem;
        returns the fastest as keyword arguments for Ensemble (tile_chunks,
        collide_mode, n_streams, sched, sched_blocks) plus its ms_per_step and
        whether it came from the cache.  Tuning never changes results."""
        import torch
        if not torch.cuda.is_available():
            raise DsmcError(-4, "autotune", "no GPU visible to torch")
        specs = _specs(list(runs))
        opt = make_options(state_fp64, n_groups, list(sample_steps), use_graph,
                           window_steps=window_steps, window_stride=window_stride)
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        cached = True
        try:      # a cached result needs no arena
            best, ms = dsmc_autotune(specs, opt, 0, 0, st.cuda_stream, n_steps, tune_cache, start)
        except DsmcError as e:
            if e.status != -2:
                raise
            cached = False
            nbytes = dsmc_autotune_bytes(specs, opt)
            arena = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            best, ms = dsmc_autotune(specs, opt, arena.data_ptr(), nbytes, st.cuda_stream, n_steps, tune_cache,
                                     start)
            del arena
            torch.cuda.empty_cache()
        return {"tile_chunks": best.tile_chunks, "collide_mode": best.collide_mode,
                "n_streams": best.n_streams, "sched": best.sched, "sched_blocks": best.sched_blocks,
                "ms_per_step": ms, "from_cache": cached}

    @classmethod
    def from_workload(cls, wl, **kw):
        kw.setdefault("state_fp64", wl.state_fp64)
        kw.setdefault("n_groups", wl.n_groups)
        kw.setdefault("window_steps", getattr(wl, "window_steps", 1))
        kw.setdefault("window_stride", getattr(wl, "window_stride", 1))
        return cls(wl.runs, wl.sample_steps, **kw)

    def close(self):
        if getattr(self, "ctx", None):
            dsmc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        dsmc_step(self.ctx, n)

    def sample(self, k: int):
        dsmc_sample(self.ctx, k)

    def sync(self):
        dsmc_sync(self.ctx)

    def n_cells(self, ensemble: int = 0) -> int:
        for r in self.runs:
            if r.ensemble == ensemble:
                return r.n_cells
        raise KeyError(ensemble)

    def moments(self, k: int, ensemble: int = 0):
        return dsmc_read_moments(self.ctx, k, ensemble, self.n_cells(ensemble))

    def accum(self, k: int, ensemble: int = 0) -> np.ndarray:
        nr = sum(1 for r in self.runs if r.ensemble == ensemble)
        G = min(self.opt.n_groups if self.opt.n_groups > 0 else 1, nr)
        return dsmc_read_accum(self.ctx, k, ensemble, G, self.n_cells(ensemble))

    def info(self) -> dict:
        return dsmc_get_info(self.ctx)

    def state(self, run: int) -> np.ndarray:
        return dsmc_get_state(self.ctx, run)

    def set_state(self, run: int, st: np.ndarray):
        dsmc_set_state(self.ctx, run, st)

    def lcr(self, run: int):
        """(lcr, bin of each slot, bin starts) of the run's last Indexing; the
        bins are the cells, or the sub-cells with sub-cells."""
        rs = self.runs[run]
        k = max(1, getattr(rs, "subcells", 1))
        return dsmc_get_lcr(self.ctx, run, rs.capacity + 64 * 1024, rs.n_cells * k ** rs.dim)

    def cell_state(self, run: int) -> dict:
        return dsmc_get_cell_state(self.ctx, run, self.runs[run].n_cells)

    def counts(self) -> np.ndarray:
        return dsmc_get_counts(self.ctx, len(self.runs))

    def sample_counts(self) -> np.ndarray:
        return dsmc_get_sample_counts(self.ctx, self.opt.n_samples)

    def diag(self) -> np.ndarray:
        """[run][7]: particles, generated, collisions, sum u, v, w, |c|^2."""
        return dsmc_get_diag(self.ctx, len(self.runs))

    def checkpoint(self) -> np.ndarray:
        return dsmc_checkpoint(self.ctx)

    def restore(self, buf: np.ndarray):
        dsmc_restore(self.ctx, buf)

    def profiling(self, on: bool):
        dsmc_set_profiling(self.ctx, on)

    def kernel_times(self) -> dict:
        return dsmc_kernel_times(self.ctx)


def counting_sort(keys, nbins: int):
    """Stable counting sort of a 1-D int32 CUDA tensor on the current stream:
    returns (lcr, start) CUDA tensors."""
    import torch
    n = keys.numel()
    keys = keys.contiguous()
    lcr = torch.empty(max(n, 1), dtype=torch.int32, device=keys.device)
    start = torch.empty(nbins + 1, dtype=torch.int32, device=keys.device)
    wb = dsmc_counting_sort_bytes(n, nbins)
    work = torch.empty(wb + 256, dtype=torch.uint8, device=keys.device)
    wp = (work.data_ptr() + 255) & ~255
    dsmc_counting_sort(keys.data_ptr(), n, nbins, lcr.data_ptr(), start.data_ptr(), wp, wb,
                       torch.cuda.current_stream(keys.device).cuda_stream)
    return lcr[:n], start
