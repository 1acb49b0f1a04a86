"""The benchmark workload at full size, in the launch configuration bench.py
times (512 runs x 1M particles, FP32 state, HIP-graph replay): sampled outputs
the oracle can compute one by one, and properties that hold at any size.

- Indexing: the LCR of sampled runs equals the oracle's stable counting sort
  of the same cell arrays (bit-exact) and the cells equal the floor of the
  positions (Enumeration, Sec. 1.1).
- One oracle step from a sampled run's GPU state reproduces the GPU step
  (FP32 vs FP64 rounding only).
- Whole ensemble: particle counts and energies conserved in the specular box,
  collisions per step at the hard-sphere equilibrium rate, and every cell's
  density and temperature within 1 % of the exact equilibrium values (about
  977 particles per cell per run) and within 3 of the returned batch-means
  standard errors.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

N_RUNS, N_PER = 512, 1_000_000
SAMPLED = (0, 137, 511)


@pytest.fixture(scope="module")
def full(dsmc_gpu):
    import torch
    wl = W.ensemble_box(n_runs=N_RUNS, n_per_run=N_PER, n_steps=1000, sample_every=20, seed=3)
    wl.sample_steps = [3, 6]
    E = dsmc_gpu.Ensemble.from_workload(wl, use_graph=True)
    yield wl, E
    E.close()
    del E
    torch.cuda.empty_cache()


def _cells_of(st, rs):
    inv_x = np.float32(np.float64(rs.nx) / rs.lx)
    inv_y = np.float32(np.float64(rs.ny) / rs.ly)
    ix = np.clip(np.floor(st[0].astype(np.float32) * inv_x), 0, rs.nx - 1).astype(np.int64)
    iy = np.clip(np.floor(st[1].astype(np.float32) * inv_y), 0, rs.ny - 1).astype(np.int64)
    return iy * rs.nx + ix


def test_full_size_indexing_and_one_step(full, oracle_lib):
    wl, E = full
    rs = wl.runs[0]
    E.step(2)
    before = {r: (E.state(r), E.cell_state(r)) for r in SAMPLED}
    ncoll0 = sum(int(E.cell_state(r)["ncoll"].sum()) for r in range(0, N_RUNS, 64))
    E.step(1)
    for r in SAMPLED:
        st1 = E.state(r)
        lcr, cell, start = E.lcr(r)
        assert lcr.size == N_PER and st1.shape == (6, N_PER)
        ref_lcr, ref_start, _ = oracle_lib.counting_sort(cell, rs.n_cells + 1)
        np.testing.assert_array_equal(lcr, ref_lcr)
        np.testing.assert_array_equal(start[: rs.n_cells + 2], ref_start)
        # the sorted particles sit in the cells Enumeration gave them
        np.testing.assert_array_equal(_cells_of(st1, rs), cell[lcr])
        # one oracle step (FP64) from the GPU's FP32 state and cell state
        st0, cs0 = before[r]
        O = oracle_lib.OracleRun(wl.runs[r], init=False)
        O.set_state(st0)
        O.set_cell_state(cs0["rem"], cs0["gmax"])
        O.set_step(2)
        O.step()
        so = O.state()
        assert so.shape == st1.shape
        # compare particle by particle (identity = slot before the step), so a
        # particle put in a different cell by FP32 rounding at a cell face
        # only affects the particles of the two cells involved
        by_id_gpu = np.empty_like(st1)
        by_id_gpu[:, lcr] = st1
        by_id_ora = np.empty_like(so)
        by_id_ora[:, O.cells()["lcr"]] = so
        close = np.all(np.abs(by_id_ora - by_id_gpu) <= 1e-5 * (1 + np.abs(by_id_ora)), axis=0)
        assert close.mean() > 0.995, (r, close.mean())
        assert abs(int(O.info()["ncoll"]) - int(E.cell_state(r)["ncoll"].sum() - cs0["ncoll"].sum())) \
            <= max(20, 0.001 * O.info()["ncoll"])
    ncoll1 = sum(int(E.cell_state(r)["ncoll"].sum()) for r in range(0, N_RUNS, 64))
    # hard-sphere equilibrium rate, 8 sampled runs
    T = np.mean([(before[r][0][3:] ** 2).sum() / (3 * N_PER) for r in SAMPLED])
    rate = 0.5 * N_PER * (N_PER - 1) * rs.fnum_sigma * 4 * math.sqrt(T / math.pi) * rs.dt
    got = (ncoll1 - ncoll0) / 8
    # (sigma c_r)_max is still settling in these first steps: 2 % allowance
    assert abs(got - rate) < 0.02 * rate, (got, rate)


def test_full_size_conservation_and_equilibrium_moments(full, dsmc_gpu):
    wl, E = full
    rs = wl.runs[0]
    info = E.info()
    assert info["runs"] == N_RUNS and info["fp64"] == 0
    e_before = {r: float((E.state(r)[3:] ** 2).sum()) for r in SAMPLED}
    E.step(6 - info["steps"])          # reach the second sample step
    counts = E.counts()
    assert np.all(counts[:, 0] == N_PER)
    for r in SAMPLED:
        e = float((E.state(r)[3:] ** 2).sum())
        assert abs(e - e_before[r]) < 2e-5 * e_before[r]
    m, se = E.moments(1)
    n_exact = N_PER / rs.n_cells
    assert np.all(np.abs(m[:, 0] / n_exact - 1) < 0.01)
    T = np.nanmean(m[:, 4])
    assert abs(T - 1.0) < 0.01
    assert np.all(np.abs(m[:, 4] / T - 1) < 0.01)
    assert np.all(np.abs(m[:, 1:4]) < 0.01 * math.sqrt(3 * T))
    # batch-means errors are small and finite
    assert np.all(np.isfinite(se)) and np.all(se[:, 0] < 0.005 * n_exact)
    # within 3 standard errors of the exact equilibrium: n = N/1024 per run,
    # zero mean velocity, and the temperature of the whole gas (energy is
    # conserved, so every cell's expected T is the realised one, taken from
    # the sums over all cells and runs); 32 run groups: Student t with 31
    # degrees of freedom, whose |t| > 3 rate is 0.53 %
    tot = E.accum(1).sum(axis=(0, 1))
    u_all = tot[1:4] / tot[0]
    T_all = ((tot[4] + tot[5] + tot[6]) / tot[0] - float(u_all @ u_all)) / 3.0
    assert tot[0] == 512 * N_PER
    exact = np.array([n_exact, 0.0, 0.0, T_all])
    z = (m[:, [0, 1, 2, 4]] - exact) / se[:, [0, 1, 2, 4]]
    assert np.all(np.isfinite(z))
    M = z.size
    assert np.mean(np.abs(z) > 3) <= 0.0053 + 3 * math.sqrt(0.0053 / M), np.mean(np.abs(z) > 3)
    assert np.max(np.abs(z)) < 6.5, np.max(np.abs(z))
    for f in range(4):
        assert abs(z[:, f].mean()) <= 3 / math.sqrt(z.shape[0]) + 0.05, (f, z[:, f].mean())
