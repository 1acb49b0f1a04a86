"""Seeded synthetic workloads for the unsteady-DSMC inner loop.

This module only *describes* problems: domain, cell grid, boundary kind of
each face, gas model, time step, particle counts, run keys and the sample
schedule.  It holds none of the method's arithmetic (no particle draws, no
motion, no collisions, no sorting).  Both the HIP library binding and the CPU
oracle read these descriptions and build their own argument structures from
them; the two never import each other.

Units are reduced: Boltzmann constant k = 1, molecular mass m = 1, and
temperatures in units of the reference (initial or free-stream) temperature.

The five problem families follow the workloads stated for this path:

* ``box``      equilibrium gas in a closed specular box (the plain FP64
               single-run case at 20,000 particles and the batched ensemble at
               1M particles per run, 512 runs);
* ``channel``  2-D impulsive start: drifting-Maxwellian inflow at -x, vacuum
               outflow at +x, diffuse wall at T=2 on -y, specular +y;
* ``uneven``   256 channel runs of uneven grids and particle counts;
* ``body3d``   3-D Mach-5 flow past a sphere-like voxel obstacle;
* ``box3d``    a 3-D closed box (exercises the z axis without an obstacle).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Face order used by every spec: -x, +x, -y, +y, -z, +z.
FACES = ("-x", "+x", "-y", "+y", "-z", "+z")
BC_NAMES = ("specular", "diffuse", "inflow", "outflow")

GAMMA_MONATOMIC = 5.0 / 3.0


def mean_speed(T: float) -> float:
    """Mean molecular speed of a Maxwellian at temperature T (k = m = 1)."""
    return math.sqrt(8.0 * T / math.pi)


def sound_speed(T: float) -> float:
    return math.sqrt(GAMMA_MONATOMIC * T)


def fnum_sigma_for(lam: float, n_density: float) -> float:
    """Fnum * sigma_ref giving hard-sphere mean free path ``lam`` at simulated
    number density ``n_density`` (particles per unit volume):
    lam = 1 / (sqrt(2) * n_real * sigma) with n_real = Fnum * n_density."""
    return 1.0 / (math.sqrt(2.0) * lam * n_density)


@dataclass
class RunSpec:
    """One independent unsteady run (one iteration of the outer loop)."""
    dim: int = 2
    nx: int = 32
    ny: int = 32
    nz: int = 1
    lx: float = 1.0
    ly: float = 1.0
    lz: float = 1.0
    dt: float = 1e-3
    fnum_sigma: float = 0.0
    omega: float = 0.5            # VHS viscosity index; 0.5 = hard sphere
    c_ref: float = 4.0 / math.sqrt(math.pi)
    face_bc: Tuple[str, ...] = ("specular",) * 6
    face_T: Tuple[float, ...] = (1.0,) * 6
    inflow_n: float = 0.0         # simulated particles per unit volume
    inflow_U: float = 0.0
    inflow_T: float = 1.0
    capacity: int = 0
    n_init: int = 0
    init_U: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    init_T: float = 1.0
    run_id: int = 0
    seed: int = 0
    ensemble: int = 0
    solid: Optional[np.ndarray] = None   # uint8 [nz][ny][nx], 1 = solid voxel
    solid_T: float = 1.0
    subcells: int = 1             # collision partners from k x k (x k) sub-cells (1 = none)
    ntc_nbar_alpha: float = 0.0   # NTC count N * Nbar / 2 with this running-mean weight (0 = N(N-1)/2)

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def cell_volume(self) -> float:
        return (self.lx / self.nx) * (self.ly / self.ny) * (self.lz / self.nz)

    @property
    def has_inflow(self) -> bool:
        return self.face_bc[0] == "inflow"


@dataclass
class Workload:
    name: str
    runs: List[RunSpec]
    n_steps: int
    sample_steps: List[int]
    n_groups: int
    state_fp64: bool = False
    note: str = ""
    # sampling window: slot k averages the snapshots after steps
    # sample_steps[k] - j * window_stride, j < window_steps (1 = one snapshot)
    window_steps: int = 1
    window_stride: int = 1

    @property
    def n_runs(self) -> int:
        return len(self.runs)

    def with_runs(self, runs: Sequence[RunSpec]) -> "Workload":
        return replace(self, runs=list(runs))

    def with_seed(self, seed: int) -> "Workload":
        return replace(self, runs=[replace(r, seed=seed) for r in self.runs])


def _round_up(x: int, m: int) -> int:
    return ((x + m - 1) // m) * m


# ---------------------------------------------------------------------------
# Closed specular box at equilibrium
# ---------------------------------------------------------------------------

def box(n_per_run: int = 20_000, n_runs: int = 1, n_steps: int = 200,
        sample_every: int = 10, seed: int = 1, grid: Tuple[int, int] = (32, 32),
        lam: float = 0.05, dt_over_tau: float = 0.2, T: float = 1.0,
        state_fp64: bool = True, n_groups: Optional[int] = None,
        omega: float = 0.5, name: str = "box") -> Workload:
    """Uniform Maxwellian gas at rest in a 1x1 specular box.

    Fnum*sigma is chosen for hard-sphere mean free path ``lam`` at the mean
    density; dt = ``dt_over_tau`` mean collision times."""
    nx, ny = grid
    fs = fnum_sigma_for(lam, n_per_run / 1.0)
    dt = dt_over_tau * lam / mean_speed(T)
    runs = [RunSpec(dim=2, nx=nx, ny=ny, nz=1, lx=1.0, ly=1.0, lz=1.0, dt=dt,
                    fnum_sigma=fs, omega=omega,
                    face_bc=("specular",) * 6, face_T=(T,) * 6,
                    capacity=_round_up(n_per_run, 256), n_init=n_per_run,
                    init_T=T, run_id=r, seed=seed)
            for r in range(n_runs)]
    samples = list(range(sample_every, n_steps + 1, sample_every))
    g = n_groups if n_groups is not None else min(n_runs, 32)
    return Workload(name, runs, n_steps, samples, g, state_fp64)


def plain_box() -> Workload:
    """The plain single-run FP64 case: 20,000 hard spheres, 32x32 cells,
    Knudsen 0.05, dt = 0.2 mean collision times, 200 steps, sample every 10."""
    return box(20_000, 1, 200, 10, seed=1, state_fp64=True, name="plain_box_fp64")


def ensemble_box(n_runs: int = 512, n_per_run: int = 1_000_000, n_steps: int = 1000,
                 sample_every: int = 20, seed: int = 3,
                 state_fp64: bool = False) -> Workload:
    """The batched ensemble: the plain-box problem at 1M particles per run,
    512 runs, 1,000 steps, moments at 50 sample times."""
    return box(n_per_run, n_runs, n_steps, sample_every, seed=seed,
               state_fp64=state_fp64, name="ensemble_box")


# ---------------------------------------------------------------------------
# 2-D channel, impulsive start
# ---------------------------------------------------------------------------

def channel_run(nx: int = 256, ny: int = 64, lx: float = 4.0, ly: float = 1.0,
                mach: float = 2.0, ppc_inf: float = 122.0, lam: float = 0.05,
                omega: float = 0.74, wall_T: float = 2.0, T_inf: float = 1.0,
                capacity_factor: float = 1.3, run_id: int = 0, seed: int = 2,
                ensemble: int = 0, fnum_sigma: Optional[float] = None) -> RunSpec:
    dx = lx / nx
    vc = (lx / nx) * (ly / ny)
    n_inf = ppc_inf / vc
    U = mach * sound_speed(T_inf)
    tau = lam / mean_speed(T_inf)
    dt = min(0.2 * tau, 0.5 * dx / U) if U > 0 else 0.2 * tau
    fs = fnum_sigma_for(lam, n_inf) if fnum_sigma is None else fnum_sigma
    fill = n_inf * lx * ly
    return RunSpec(dim=2, nx=nx, ny=ny, nz=1, lx=lx, ly=ly, lz=1.0, dt=dt,
                   fnum_sigma=fs, omega=omega,
                   face_bc=("inflow", "outflow", "diffuse", "specular",
                            "specular", "specular"),
                   face_T=(T_inf, T_inf, wall_T, T_inf, T_inf, T_inf),
                   inflow_n=n_inf, inflow_U=U, inflow_T=T_inf,
                   capacity=_round_up(int(math.ceil(capacity_factor * fill)) + 4096, 256),
                   n_init=0, init_T=T_inf, run_id=run_id, seed=seed,
                   ensemble=ensemble)


def channel(n_runs: int = 16, nx: int = 256, ny: int = 64, ppc_inf: float = 122.0,
            n_steps: int = 2000, sample_every: int = 100, seed: int = 2,
            state_fp64: bool = False, n_groups: Optional[int] = None,
            mach: float = 2.0, omega: float = 0.74, lam: float = 0.05,
            fnum_sigma: Optional[float] = None) -> Workload:
    """Impulsively started Mach-2 channel flow: 4x1 domain on a 256x64 grid,
    diffuse bottom wall at T=2, inflow of a drifting Maxwellian, vacuum
    outflow, VHS omega=0.74, ~2M particles per run at steady fill, 2,000
    steps, samples at 20 fixed times, 16 runs."""
    runs = [channel_run(nx=nx, ny=ny, lx=4.0 * (nx / 256) / (ny / 64), ly=1.0,
                        mach=mach, ppc_inf=ppc_inf, omega=omega, lam=lam,
                        run_id=r, seed=seed, fnum_sigma=fnum_sigma)
            for r in range(n_runs)]
    samples = list(range(sample_every, n_steps + 1, sample_every))
    g = n_groups if n_groups is not None else min(n_runs, 32)
    return Workload("channel", runs, n_steps, samples, g, state_fp64)


# ---------------------------------------------------------------------------
# Uneven ensemble
# ---------------------------------------------------------------------------

UNEVEN_GRIDS = ((64, 64), (128, 128), (256, 128), (512, 256))


def uneven(n_runs: int = 256, n_steps: int = 1000, n_samples: int = 20, seed: int = 4,
           count_range: Tuple[float, float] = (50e3, 4e6),
           grids: Sequence[Tuple[int, int]] = UNEVEN_GRIDS,
           state_fp64: bool = False) -> Workload:
    """256 channel runs with grids drawn from {64x64, 128x128, 256x128,
    512x256}, target particle counts log-uniform in [50k, 4M], omega in
    {0.5, 0.74} and inflow Mach log-uniform in [0.5, 5]; every draw comes from
    numpy's default_rng(seed).  Ly = 1 and Lx = Nx/Ny (square cells); each run
    is its own ensemble (its own flow)."""
    rng = np.random.default_rng(seed)
    gi = rng.integers(0, len(grids), size=n_runs)
    logn = rng.uniform(math.log(count_range[0]), math.log(count_range[1]), size=n_runs)
    om = rng.integers(0, 2, size=n_runs)
    logm = rng.uniform(math.log(0.5), math.log(5.0), size=n_runs)
    runs = []
    for r in range(n_runs):
        nx, ny = grids[int(gi[r])]
        lx, ly = nx / ny, 1.0
        n_target = float(math.exp(logn[r]))
        ppc = n_target / (nx * ny)
        runs.append(channel_run(nx=nx, ny=ny, lx=lx, ly=ly, mach=float(math.exp(logm[r])),
                                ppc_inf=ppc, omega=(0.5, 0.74)[int(om[r])],
                                capacity_factor=1.5, run_id=r, seed=seed, ensemble=r))
    every = max(1, n_steps // n_samples)
    samples = list(range(every, n_steps + 1, every))[:n_samples]
    return Workload("uneven", runs, n_steps, samples, 1, state_fp64)


# ---------------------------------------------------------------------------
# 3-D
# ---------------------------------------------------------------------------

def box3d(n_per_run: int = 50_000, n_runs: int = 1, grid=(16, 16, 16), n_steps: int = 50,
          sample_every: int = 10, seed: int = 6, lam: float = 0.05,
          state_fp64: bool = True, wall: str = "specular", wall_T: float = 1.0) -> Workload:
    nx, ny, nz = grid
    T = 1.0
    fs = fnum_sigma_for(lam, float(n_per_run))
    dt = 0.2 * lam / mean_speed(T)
    runs = [RunSpec(dim=3, nx=nx, ny=ny, nz=nz, lx=1.0, ly=1.0, lz=1.0, dt=dt,
                    fnum_sigma=fs, omega=0.5, face_bc=(wall,) * 6, face_T=(wall_T,) * 6,
                    capacity=_round_up(n_per_run, 256), n_init=n_per_run, init_T=T,
                    run_id=r, seed=seed)
            for r in range(n_runs)]
    samples = list(range(sample_every, n_steps + 1, sample_every))
    return Workload("box3d", runs, n_steps, samples, min(n_runs, 32), state_fp64)


def sphere_mask(nx: int, ny: int, nz: int, lx: float, ly: float, lz: float,
                centre=(0.5, 0.5, 0.5), radius: float = 0.15) -> np.ndarray:
    """Voxel obstacle: a voxel is solid iff its centre lies inside the sphere."""
    xc = (np.arange(nx) + 0.5) * (lx / nx)
    yc = (np.arange(ny) + 0.5) * (ly / ny)
    zc = (np.arange(nz) + 0.5) * (lz / nz)
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")
    r2 = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 + (Z - centre[2]) ** 2
    return (r2 <= radius * radius).astype(np.uint8)


def body3d(n_runs: int = 32, grid=(200, 100, 100), n_per_run: int = 60_000_000,
           n_steps: int = 500, n_samples: int = 10, seed: int = 5, lam: float = 0.02,
           mach: float = 5.0, state_fp64: bool = False) -> Workload:
    """3-D Mach-5 flow past a sphere (r = 0.15 at (0.5, 0.5, 0.5)) given as a
    voxel mask with diffuse walls at T = 3: 2x1x1 box on a 200x100x100 grid,
    60M particles per run (free-stream fill), 500 steps, 32 runs."""
    nx, ny, nz = grid
    lx, ly, lz = 2.0, 1.0, 1.0
    T = 1.0
    U = mach * sound_speed(T)
    dx = lx / nx
    mask = sphere_mask(nx, ny, nz, lx, ly, lz)
    fluid_vol = (nx * ny * nz - int(mask.sum())) * (lx / nx) * (ly / ny) * (lz / nz)
    n_inf = n_per_run / fluid_vol
    fs = fnum_sigma_for(lam, n_inf)
    dt = 0.3 * dx / U
    runs = [RunSpec(dim=3, nx=nx, ny=ny, nz=nz, lx=lx, ly=ly, lz=lz, dt=dt, fnum_sigma=fs,
                    omega=0.5, face_bc=("inflow", "outflow", "specular", "specular",
                                        "specular", "specular"),
                    face_T=(T,) * 6, inflow_n=n_inf, inflow_U=U, inflow_T=T,
                    capacity=_round_up(int(1.3 * n_per_run) + 4096, 256), n_init=n_per_run,
                    init_U=(U, 0.0, 0.0), init_T=T, run_id=r, seed=seed,
                    solid=mask, solid_T=3.0)
            for r in range(n_runs)]
    every = max(1, n_steps // n_samples)
    samples = list(range(every, n_steps + 1, every))[:n_samples]
    return Workload("body3d", runs, n_steps, samples, min(n_runs, 32), state_fp64)


# ---------------------------------------------------------------------------
# Inputs for the Indexing step alone
# ---------------------------------------------------------------------------

def random_cells(n: int, n_bins: int, seed: int, near_sorted: bool = False,
                 jump: int = 1, dead_fraction: float = 0.0) -> np.ndarray:
    """Seeded cell-index arrays for the counting-sort tests.

    ``near_sorted`` mimics a cell-sorted particle array after one step: sorted
    cells, each moved by at most ``jump`` bins.  ``dead_fraction`` of the
    entries get the DEAD bin ``n_bins - 1``."""
    rng = np.random.default_rng(seed)
    live = n_bins - 1
    if live < 1:
        return np.zeros(n, np.int32)
    if near_sorted:
        c = np.sort(rng.integers(0, live, size=n))
        c = np.clip(c + rng.integers(-jump, jump + 1, size=n), 0, live - 1)
    else:
        c = rng.integers(0, live, size=n)
    if dead_fraction > 0:
        c[rng.random(n) < dead_fraction] = live
    return c.astype(np.int32)
