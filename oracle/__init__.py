"""Python access to the plain FP64 DSMC oracle (``oracle/dsmc_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke entry point and the CPU
baseline leg of the benchmark may use this package; the GPU library never
does.  The oracle follows the sequential unsteady-DSMC algorithm of Sec. 1.1
of the paper (Generation -> Motion -> Enumeration/Indexing -> Interaction ->
Sampling each time step; LCR rebuilt every step; runs made independent by
their random-number key) with standard DSMC kinetics written from the
mathematics.  It shares no code with the HIP path; both read only the problem
descriptions in ``workloads``.

``moments`` below is the final FP64 division of the sampled sums into
density, mean velocity and temperature (Sec. 1.1: macroparameters averaged
over the particles of a cell and over the runs).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dsmc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

BC_CODES = {"specular": 0, "diffuse": 1, "inflow": 2, "outflow": 3}
NFIELD = 7  # N, sum u, sum v, sum w, sum u^2, sum v^2, sum w^2

STATUS = {0: "ok", -1: "invalid argument", -3: "capacity exceeded", -6: "unsupported",
          -7: "too many wall interactions in one step", -8: "inflow sampler did not accept",
          -9: "out of memory"}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm", "-lpthread"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class OrSpec(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("dt", C.c_double), ("fnum_sigma", C.c_double),
                ("omega", C.c_double), ("c_ref", C.c_double),
                ("face_bc", C.c_int32 * 6), ("face_T", C.c_double * 6),
                ("inflow_n", C.c_double), ("inflow_U", C.c_double), ("inflow_T", C.c_double),
                ("solid", C.c_void_p), ("solid_T", C.c_double),
                ("capacity", C.c_int64), ("n_init", C.c_int64),
                ("init_U", C.c_double * 3), ("init_T", C.c_double),
                ("run_id", C.c_uint32), ("seed", C.c_uint32), ("subcells", C.c_int32),
                ("pad", C.c_int32), ("nbar_alpha", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH) or (os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
            build()
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.or_philox4x32_10.argtypes = [C.POINTER(C.c_uint32)] * 3
        L.or_u01.argtypes = [C.c_uint32, C.c_uint32]
        L.or_u01.restype = C.c_double
        L.or_index.argtypes = [C.c_uint32, C.c_uint32]
        L.or_index.restype = C.c_uint32
        L.or_run_new.argtypes = [C.POINTER(OrSpec), C.POINTER(C.c_int32)]
        L.or_run_new.restype = P
        for f in ("or_run_free", "or_init", "or_generation", "or_motion", "or_indexing",
                  "or_permute", "or_interaction", "or_step", "or_step_begin"):
            getattr(L, f).argtypes = [P]
            getattr(L, f).restype = None
        L.or_sample.argtypes = [P, dp]
        L.or_get_info.argtypes = [P, C.POINTER(C.c_int64)]
        L.or_get_consts.argtypes = [P, dp]
        L.or_get_state.argtypes = [P, dp]
        L.or_set_state.argtypes = [P, C.c_int64, dp]
        L.or_set_state.restype = C.c_int32
        L.or_set_step.argtypes = [P, C.c_uint32]
        L.or_get_cells.argtypes = [P, P, P, P, P]
        L.or_get_cell_state.argtypes = [P, P, P, P]
        L.or_get_face_rem.argtypes = [P, dp]
        L.or_get_solid_hits.argtypes = [P]
        L.or_get_solid_hits.restype = C.c_int64
        L.or_set_cell_state.argtypes = [P, dp, dp]
        L.or_get_nbar.argtypes = [P, dp]
        L.or_set_nbar.argtypes = [P, dp]
        L.or_counting_sort.argtypes = [P, C.c_int64, C.c_int64, P, P, P]
        L.or_collide_cell.argtypes = [C.POINTER(OrSpec), C.c_uint32, C.c_uint32, C.c_int64,
                                      dp, dp, dp, dp, dp, P, P, C.c_int64, C.POINTER(C.c_int64)]
        L.or_collide_cell.restype = C.c_int64
        L.or_ensemble.argtypes = [C.POINTER(OrSpec), C.c_int32, C.c_int32, P, C.c_int32,
                                  C.c_int32, C.c_int32, C.c_int32, C.c_int32, dp,
                                  C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.or_ensemble.restype = C.c_int32
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_spec(rs) -> OrSpec:
    """Build the oracle's argument struct from a ``workloads.RunSpec``."""
    s = OrSpec()
    s.dim, s.nx, s.ny, s.nz = rs.dim, rs.nx, rs.ny, rs.nz
    s.lx, s.ly, s.lz = rs.lx, rs.ly, rs.lz
    s.dt, s.fnum_sigma, s.omega, s.c_ref = rs.dt, rs.fnum_sigma, rs.omega, rs.c_ref
    for f in range(6):
        s.face_bc[f] = BC_CODES[rs.face_bc[f]]
        s.face_T[f] = rs.face_T[f]
    s.inflow_n, s.inflow_U, s.inflow_T = rs.inflow_n, rs.inflow_U, rs.inflow_T
    if rs.solid is None:
        s.solid = None
    else:
        # one byte per cell, cell index (iz * ny + iy) * nx + ix; the run copies it
        mask = np.ascontiguousarray(rs.solid, dtype=np.uint8).ravel()
        if mask.size != rs.n_cells:
            raise ValueError("solid mask must have one entry per cell")
        s._mask = mask
        s.solid = mask.ctypes.data
    s.solid_T = rs.solid_T
    s.capacity, s.n_init = rs.capacity, rs.n_init
    for a in range(3):
        s.init_U[a] = rs.init_U[a]
    s.init_T = rs.init_T
    s.run_id, s.seed = rs.run_id & 0xFFFFFFFF, rs.seed & 0xFFFFFFFF
    s.subcells = getattr(rs, "subcells", 1)
    s.nbar_alpha = getattr(rs, "ntc_nbar_alpha", 0.0)
    return s


# ---------------------------------------------------------------------------
# Random numbers
# ---------------------------------------------------------------------------

def philox(ctr: Sequence[int], key: Sequence[int]) -> tuple:
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return tuple(o)


def u01(a: int, b: int) -> float:
    return lib().or_u01(a & 0xFFFFFFFF, b & 0xFFFFFFFF)


def index(a: int, n: int) -> int:
    return lib().or_index(a & 0xFFFFFFFF, n)


# ---------------------------------------------------------------------------
# One run
# ---------------------------------------------------------------------------

class OracleRun:
    """One independent run: P, LCR and C of Sec. 1.1 in FP64."""

    def __init__(self, rs, init: bool = True):
        self.rs = rs
        self._spec = make_spec(rs)
        st = C.c_int32(0)
        self._h = lib().or_run_new(C.byref(self._spec), C.byref(st))
        if not self._h:
            raise ValueError(f"oracle rejected the run spec: {STATUS.get(st.value, st.value)}")
        self.nc = rs.n_cells
        if init:
            lib().or_init(self._h)
            self._check()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().or_run_free(h)
            self._h = None

    # -- the step and its parts ------------------------------------------------
    def step(self, n: int = 1):
        for _ in range(n):
            lib().or_step(self._h)
            self._check()

    def step_begin(self):
        lib().or_step_begin(self._h)

    def generation(self):
        lib().or_generation(self._h); self._check()

    def motion(self):
        lib().or_motion(self._h); self._check()

    def indexing(self):
        lib().or_indexing(self._h)

    def permute(self):
        lib().or_permute(self._h)

    def interaction(self):
        lib().or_interaction(self._h)

    def solid_hits(self) -> int:
        """Solid-cell faces hit in the last Motion."""
        return int(lib().or_get_solid_hits(self._h))

    def _check(self):
        err = self.info()["err"]
        if err:
            raise RuntimeError(f"oracle run error: {STATUS.get(err, err)}")

    # -- accessors -------------------------------------------------------------
    def info(self) -> dict:
        a = (C.c_int64 * 11)()
        lib().or_get_info(self._h, a)
        keys = ("n", "step", "err", "nc", "n_sorted", "ncoll", "ngen", "nremoved", "nmoved",
                "nface", "nbin")
        return dict(zip(keys, list(a)))

    def consts(self) -> dict:
        a = np.zeros(7)
        lib().or_get_consts(self._h, _dp(a))
        return dict(zip(("coef", "vhs_exp", "gmax0", "mbar", "beta", "s_inf", "p_branch"), a))

    @property
    def n(self) -> int:
        return self.info()["n"]

    def state(self) -> np.ndarray:
        """[6][n] = x, y, z, u, v, w in slot order."""
        n = self.n
        out = np.zeros((6, n))
        lib().or_get_state(self._h, _dp(out))
        return out

    def set_state(self, st: np.ndarray):
        st = np.ascontiguousarray(st, dtype=np.float64)
        rc = lib().or_set_state(self._h, st.shape[1], _dp(st))
        if rc:
            raise ValueError(STATUS.get(rc, rc))

    def set_step(self, step: int):
        lib().or_set_step(self._h, step)

    def cells(self) -> dict:
        """The last Indexing: bin of each slot (cell, or sub-cell with
        sub-cells; nbin = DEAD), LCR, bin starts [nbin+2] and counts [nbin+1]."""
        info = self.info()
        ns, nc = info["n_sorted"], info["nbin"]
        cell = np.zeros(ns, np.int32)
        lcr = np.zeros(ns, np.int32)
        cstart = np.zeros(nc + 2, np.int64)
        ccount = np.zeros(nc + 1, np.int64)
        lib().or_get_cells(self._h, cell.ctypes.data, lcr.ctypes.data, cstart.ctypes.data,
                           ccount.ctypes.data)
        return {"cell": cell, "lcr": lcr, "start": cstart, "count": ccount}

    def cell_state(self) -> dict:
        rem = np.zeros(self.nc); gmax = np.zeros(self.nc); ncoll = np.zeros(self.nc, np.int64)
        lib().or_get_cell_state(self._h, rem.ctypes.data, gmax.ctypes.data, ncoll.ctypes.data)
        nbar = np.zeros(self.nc)
        lib().or_get_nbar(self._h, _dp(nbar))
        return {"rem": rem, "gmax": gmax, "ncoll": ncoll, "nbar": nbar}

    def set_cell_state(self, rem: np.ndarray, gmax: np.ndarray, nbar: np.ndarray = None):
        rem = np.ascontiguousarray(rem, dtype=np.float64)
        gmax = np.ascontiguousarray(gmax, dtype=np.float64)
        assert rem.size == self.nc and gmax.size == self.nc
        lib().or_set_cell_state(self._h, _dp(rem), _dp(gmax))
        if nbar is not None:
            nbar = np.ascontiguousarray(nbar, dtype=np.float64)
            assert nbar.size == self.nc
            lib().or_set_nbar(self._h, _dp(nbar))

    def face_rem(self) -> np.ndarray:
        nf = self.info()["nface"]
        out = np.zeros(max(nf, 0))
        if nf:
            lib().or_get_face_rem(self._h, _dp(out))
        return out

    def sample(self) -> np.ndarray:
        """Per-cell sums [nc][7] of the current (cell-sorted) state."""
        out = np.zeros((self.nc, NFIELD))
        lib().or_sample(self._h, _dp(out))
        return out


# ---------------------------------------------------------------------------
# Stand-alone pieces
# ---------------------------------------------------------------------------

def counting_sort(keys: np.ndarray, nbins: int):
    """Stable counting sort: returns (lcr, start[nbins+1], count[nbins])."""
    keys = np.ascontiguousarray(keys, dtype=np.int32)
    n = keys.size
    lcr = np.zeros(n, np.int32)
    start = np.zeros(nbins + 1, np.int64)
    count = np.zeros(nbins, np.int64)
    lib().or_counting_sort(keys.ctypes.data, n, nbins, lcr.ctypes.data, start.ctypes.data,
                           count.ctypes.data)
    return lcr, start, count


def collide_cell(rs, step: int, cell: int, vel: np.ndarray, gmax: float, rem: float = 0.0,
                 trace_cap: int = 0, sub_off: Optional[Sequence[int]] = None):
    """Interaction in one cell with given velocities [3][N] (modified copy
    returned); with sub-cells (rs.subcells > 1) sub_off holds the S + 1
    sub-cell starts of the N particles.  Returns dict(vel, gmax, rem, ncoll,
    nsel, trace[nsel][3])."""
    spec = make_spec(rs)
    v = np.array(vel, dtype=np.float64, copy=True)
    u, vv, w = (np.ascontiguousarray(v[a]) for a in range(3))
    g = np.array([gmax]); r = np.array([rem])
    tr = np.zeros((max(trace_cap, 1), 3), np.int32)
    nsel = C.c_int64(0)
    off = None if sub_off is None else np.ascontiguousarray(sub_off, dtype=np.int64)
    k = lib().or_collide_cell(C.byref(spec), step, cell, u.size, _dp(u), _dp(vv), _dp(w), _dp(g),
                              _dp(r), off.ctypes.data if off is not None else None,
                              tr.ctypes.data if trace_cap else None, trace_cap, C.byref(nsel))
    if k < 0:
        raise ValueError(STATUS.get(k, k))
    return {"vel": np.stack([u, vv, w]), "gmax": g[0], "rem": r[0], "ncoll": k,
            "nsel": nsel.value, "trace": tr[:min(nsel.value, trace_cap)] if trace_cap else None}


def ensemble(workload, n_threads: int = 0, runs: Optional[Sequence] = None,
             n_steps: Optional[int] = None, n_groups: Optional[int] = None,
             window_steps: Optional[int] = None, window_stride: Optional[int] = None):
    """Runs the outer loop over independent runs.  Returns
    (acc[n_samples][n_groups][nc][7], stats dict); stats["n_snap"][k] is the
    number of snapshots each run added to slot k (the slot's time window:
    the steps sample_steps[k] - j * window_stride, j < window_steps)."""
    runs = list(workload.runs if runs is None else runs)
    n_steps = workload.n_steps if n_steps is None else n_steps
    G = workload.n_groups if n_groups is None else n_groups
    G = max(1, min(G, len(runs)))
    W = getattr(workload, "window_steps", 1) if window_steps is None else window_steps
    q = getattr(workload, "window_stride", 1) if window_stride is None else window_stride
    W, q = max(1, W), max(1, q)
    # slots whose window has started by n_steps
    samples = np.array([s for s in workload.sample_steps if s - (W - 1) * q <= n_steps], np.int32)
    keep = [make_spec(r) for r in runs]       # holds the masks while the C side copies them
    specs = (OrSpec * len(runs))(*keep)
    nc = runs[0].n_cells
    acc = np.zeros((len(samples), G, nc, NFIELD))
    nsnap = np.zeros(max(len(samples), 1), np.int64)
    stats = (C.c_int64 * 2)()
    if n_threads <= 0:
        n_threads = len(os.sched_getaffinity(0))
    rc = lib().or_ensemble(specs, len(runs), n_steps, samples.ctypes.data, len(samples), W, q, G,
                           n_threads, _dp(acc), nsnap.ctypes.data_as(C.POINTER(C.c_int64)), stats)
    if rc:
        raise RuntimeError(f"oracle ensemble failed: {STATUS.get(rc, rc)}")
    return acc, {"particle_steps": stats[0], "collisions": stats[1],
                 "threads": min(n_threads, G), "sample_steps": samples.tolist(),
                 "n_snap": nsnap[:len(samples)].tolist()}


def moments(sums: np.ndarray, n_runs: int, n_snap: int = 1) -> np.ndarray:
    """FP64 division of pooled sums [..., 7] (summed over ``n_runs`` runs and
    ``n_snap`` snapshots of each run) into [..., 8] = n (particles per cell
    per run and snapshot), ux, uy, uz, T, Tx, Ty, Tz.  Cells with no
    particles give NaN."""
    s = np.asarray(sums, dtype=np.float64)
    N = s[..., 0]
    with np.errstate(invalid="ignore", divide="ignore"):
        inv = np.where(N > 0, 1.0 / N, np.nan)
        ux, uy, uz = s[..., 1] * inv, s[..., 2] * inv, s[..., 3] * inv
        Tx = s[..., 4] * inv - ux * ux
        Ty = s[..., 5] * inv - uy * uy
        Tz = s[..., 6] * inv - uz * uz
        T = (Tx + Ty + Tz) / 3.0
    out = np.stack([N / (n_runs * n_snap), ux, uy, uz, T, Tx, Ty, Tz], axis=-1)
    return out
