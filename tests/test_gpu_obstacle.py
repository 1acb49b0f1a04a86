"""Voxel obstacle (solid cells with diffuse faces) on the GPU.

- FP64: identical inputs and Philox streams as the oracle, step by step: LCR
  and cells bit-exact, state to 1e-12 (the walk's plane-crossing decisions
  and the face-rounding rule taken in the same precision on both sides).
- FP32 ensembles of a Mach-5 flow past a sphere against the oracle's own
  ensemble (disjoint seeds), 3 standard errors per entry.
- Invariant at FP32: no particle ever in a solid cell.
"""
from dataclasses import replace

import numpy as np
import pytest

import workloads as W
from test_gpu_parity import _parity
from test_gpu_ensemble import _per_run_moments, _z_gate

pytestmark = pytest.mark.gpu


def _body_runs(n_runs, grid=(24, 12, 12), n_per_run=30_000, radius=0.25, seed=5, **kw):
    base = W.body3d(n_runs=n_runs, grid=grid, n_per_run=n_per_run, n_steps=1, n_samples=1, seed=seed)
    mask = W.sphere_mask(*grid, 2.0, 1.0, 1.0, centre=(0.5, 0.5, 0.5), radius=radius)
    return [replace(r, solid=mask, **kw) for r in base.runs]


def test_body3d_fp64_parity(dsmc_gpu, oracle_lib):
    """Mach-5 inflow past a sphere of solid cells at T = 3, two runs."""
    O = _parity(dsmc_gpu, oracle_lib, _body_runs(2), 6)
    assert O[0].info()["ngen"] > 0


def test_large_sphere_fp64_parity(dsmc_gpu, oracle_lib):
    """A sphere of radius ~7 cells: flights inside its box of solid cells
    (widened by two) but starting three or more cells from every solid cell
    take Motion's fast path instead of the full flight; step by step equal to
    the oracle's full flight for every particle."""
    from scipy.ndimage import binary_dilation
    grid = (48, 24, 24)
    runs = _body_runs(2, grid=grid, n_per_run=60_000, radius=0.3, seed=7)
    m = np.asarray(runs[0].solid, bool).reshape(grid[2], grid[1], grid[0])
    near = binary_dilation(m, structure=np.ones((5, 5, 5), bool))
    idx = np.argwhere(m)
    box = np.zeros_like(m)
    lo, hi = idx.min(0) - 2, idx.max(0) + 3
    box[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] = True
    assert (box & ~near).sum() > 1000      # cells of the box the fast path serves
    _parity(dsmc_gpu, oracle_lib, runs, 4)


def test_channel_with_block_2d_fp64_parity(dsmc_gpu, oracle_lib):
    """2-D channel (inflow, diffuse floor at T = 2, outflow) with a 4x6-cell
    block at T = 1.5 in the stream, started half full and drifting."""
    a = W.channel_run(nx=48, ny=16, lx=3.0, ly=1.0, ppc_inf=30.0, run_id=0, seed=31)
    mask = np.zeros((1, 16, 48), np.uint8)
    mask[0, 5:11, 14:18] = 1
    a = replace(a, n_init=12000, init_U=(a.inflow_U, 0.0, 0.0), solid=mask, solid_T=1.5)
    b = replace(a, run_id=1, n_init=0)
    _parity(dsmc_gpu, oracle_lib, [a, b], 6)


def test_cold_obstacle_face_rounding_fp64_parity(dsmc_gpu, oracle_lib):
    """A block at T = 1e-40: particles that hit it stay on its faces, so end
    points round onto solid cells and are moved into the fluid cell on both
    sides alike."""
    wl = W.box3d(n_per_run=20000, n_runs=1, grid=(10, 8, 6), seed=33)
    mask = np.zeros((6, 8, 10), np.uint8)
    mask[2:4, 3:5, 4:7] = 1
    runs = [replace(r, solid=mask, solid_T=1e-40) for r in wl.runs]
    _parity(dsmc_gpu, oracle_lib, runs, 5)


def test_no_particle_in_solid_cells_fp32(dsmc_gpu):
    """16 FP32 runs of the body flow for 60 steps: every particle's cell is
    fluid after each checked step."""
    runs = [replace(r, run_id=i) for i, r in enumerate(_body_runs(1, n_per_run=40_000) * 16)]
    E = dsmc_gpu.Ensemble(runs, [], state_fp64=False, n_groups=1)
    solid = runs[0].solid.ravel().astype(bool)
    nc = runs[0].n_cells
    for s in range(60):
        E.step(1)
        if s % 15 == 14:
            for r in (0, 7, 15):
                lcr, cell, start = E.lcr(r)
                keep = int(start[nc])
                assert keep > 20_000
                assert not np.any(solid[cell[lcr[:keep]]]), (s, r)
                assert E.state(r).shape[1] == keep


def test_body3d_fp32_ensemble_matches_oracle_ensemble(dsmc_gpu, oracle_lib):
    """32 runs per side (disjoint seeds) of the body flow, sampled at steps
    20 and 40: density, velocity and temperature per (cell, time) entry
    within 3 standard errors (normal-theory gate)."""
    n = 32
    gpu_runs = _body_runs(n, n_per_run=20_000, seed=41)
    ora_runs = _body_runs(n, n_per_run=20_000, seed=42)
    samples = [20, 40]
    E = dsmc_gpu.Ensemble(gpu_runs, samples, state_fp64=False, n_groups=n)
    E.step(40)
    acc_g = np.stack([E.accum(k) for k in range(2)])
    wl = W.Workload("body", ora_runs, 40, samples, n)
    acc_o, _ = oracle_lib.ensemble(wl, n_threads=16)
    fields = [0, 1, 2, 4]
    mg, sg, ng = _per_run_moments(acc_g, fields)
    mo, so, no = _per_run_moments(acc_o, fields)
    ok = (np.nanmean(ng, axis=1) >= 5) & (np.nanmean(no, axis=1) >= 5)
    z = (mg - mo) / np.sqrt(sg ** 2 + so ** 2)
    z = np.where(ok[..., None], z, np.nan)
    M = _z_gate(z, "body3d")
    assert M > 2000
    # solid cells hold nothing on either side
    solid = gpu_runs[0].solid.ravel().astype(bool)
    assert np.all(acc_g[:, :, solid, 0] == 0) and np.all(acc_o[:, :, solid, 0] == 0)
