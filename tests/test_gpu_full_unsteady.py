"""The two unsteady batches at full size, in the launch configuration
bench.py times (HIP-graph replay, FP32 state), after the 600 steps from
vacuum bench.py fills them with: the impulsively started Mach-2 channel (16
runs of 256x64 cells, ~2M particles each) and the uneven batch (256 runs of
four grid sizes, 50k-4M particles).  Sampled outputs the oracle can compute
one by one, and properties that hold at any size:

- Indexing: each sampled run's LCR equals the oracle's stable counting sort
  of the same cell array (bit-exact; two-level sort beyond 2047 cells), and
  the particles sit in the cells their positions floor to.
- One oracle step (FP64) from a sampled run's GPU state and cell state
  reproduces the GPU step particle by particle for the particles present
  before it (the entrants depend on the faces' carried remainders).
- Generation: the entrants of a step over all runs match the one-sided
  Maxwellian flux n (exp(-s^2) + sqrt(pi) s (1 + erf s)) / (2 sqrt(pi) beta)
  through the inflow face (beta = 1/sqrt(2T), s = U beta) within 4 standard
  errors.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FILL = 600


def _cells_of(st, rs):
    inv_x = np.float32(np.float64(rs.nx) / rs.lx)
    inv_y = np.float32(np.float64(rs.ny) / rs.ly)
    ix = np.clip(np.floor(st[0].astype(np.float32) * inv_x), 0, rs.nx - 1).astype(np.int64)
    iy = np.clip(np.floor(st[1].astype(np.float32) * inv_y), 0, rs.ny - 1).astype(np.int64)
    return iy * rs.nx + ix


def _flux_per_step(rs):
    beta = 1.0 / math.sqrt(2.0 * rs.inflow_T)
    s = rs.inflow_U * beta
    gamma = rs.inflow_n * (math.exp(-s * s) + math.sqrt(math.pi) * s * (1.0 + math.erf(s))) / (
        2.0 * math.sqrt(math.pi) * beta)
    return gamma * rs.ly * rs.lz * rs.dt


def _check_sampled(E, wl, runs, oracle_lib):
    step0 = E.info()["steps"]
    before = {r: (E.state(r), E.cell_state(r)) for r in runs}
    E.step(1)
    for r in runs:
        rs = wl.runs[r]
        st1 = E.state(r)
        lcr, cell, start = E.lcr(r)
        ref_lcr, ref_start, _ = oracle_lib.counting_sort(cell, rs.n_cells + 1)
        np.testing.assert_array_equal(lcr, ref_lcr, err_msg=f"run {r}")
        np.testing.assert_array_equal(start[: rs.n_cells + 2], ref_start, err_msg=f"run {r}")
        keep = int(start[rs.n_cells])
        assert st1.shape[1] == keep
        np.testing.assert_array_equal(_cells_of(st1, rs), cell[lcr[:keep]], err_msg=f"run {r}")
        st0, cs0 = before[r]
        n0 = st0.shape[1]
        O = oracle_lib.OracleRun(rs, init=False)
        O.set_state(st0)
        O.set_cell_state(cs0["rem"], cs0["gmax"])
        O.set_step(step0)
        O.step()
        so, ol = O.state(), O.cells()
        okeep = int(ol["start"][rs.n_cells])
        ids_g, ids_o = lcr[:keep], ol["lcr"][:okeep]
        pos_g = np.full(n0, -1, np.int64)
        pos_o = np.full(n0, -1, np.int64)
        mg, mo = ids_g < n0, ids_o < n0
        pos_g[ids_g[mg]] = np.nonzero(mg)[0]
        pos_o[ids_o[mo]] = np.nonzero(mo)[0]
        both = (pos_g >= 0) & (pos_o >= 0)
        assert both.mean() > 0.99, (r, both.mean())
        a, b = st1[:, pos_g[both]], so[:, pos_o[both]]
        close = np.all(np.abs(a - b) <= 1e-5 * (1 + np.abs(b)), axis=0)
        assert close.mean() > 0.995, (r, close.mean())
        # the collisions of the step agree up to the cells FP32 rounding moved
        ncoll_g = int(E.cell_state(r)["ncoll"].sum() - cs0["ncoll"].sum())
        assert abs(ncoll_g - int(O.info()["ncoll"])) <= max(20, 0.002 * O.info()["ncoll"]), r


def _check_flux(E, wl):
    gen = E.counts()[:, 1].astype(float)           # entrants of the last step, per run
    expect = np.array([_flux_per_step(rs) for rs in wl.runs])
    # per face element the count is floor(mean + carried remainder): the
    # remainders carry the fractions, so a step's count differs from the
    # mean by the sampling spread only; Poisson bound on its variance
    z = (gen.sum() - expect.sum()) / math.sqrt(expect.sum())
    assert abs(z) < 4.0, (gen.sum(), expect.sum(), z)


def test_channel_full_size_after_the_fill(dsmc_gpu, oracle_lib):
    import torch
    wl = W.channel()
    E = dsmc_gpu.Ensemble.from_workload(wl, use_graph=True)
    E.step(FILL)
    counts = E.counts()[:, 0]
    assert counts.min() > 1_700_000 and counts.max() < 2_400_000, counts
    _check_flux(E, wl)
    _check_sampled(E, wl, (0, 7, 15), oracle_lib)
    E.close()
    del E
    torch.cuda.empty_cache()


def test_uneven_full_size_after_the_fill(dsmc_gpu, oracle_lib):
    import torch
    wl = W.uneven()
    E = dsmc_gpu.Ensemble.from_workload(wl, use_graph=True)
    E.step(FILL)
    _check_flux(E, wl)
    # one run of each grid size, the smallest and the largest batch members
    counts = E.counts()[:, 0]
    by_grid = {}
    for r, rs in enumerate(wl.runs):
        by_grid.setdefault((rs.nx, rs.ny), []).append(r)
    sampled = sorted({g[len(g) // 2] for g in by_grid.values()} | {int(np.argmin(counts)), int(np.argmax(counts))})
    _check_sampled(E, wl, sampled, oracle_lib)
    E.close()
    del E
    torch.cuda.empty_cache()
