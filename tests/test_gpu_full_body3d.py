"""The flow past a body at full size (32 runs x 60M particles, 200x100x100
cells, sphere of solid cells, Mach-5 inflow, FP32 state, HIP-graph replay):
sampled outputs the oracle can compute one by one, and properties that hold
at any size.

- Indexing: the LCR of sampled runs equals the oracle's stable counting sort
  of the same cell arrays (bit-exact; two 11-bit passes at 2M cells).
- No particle in a solid cell; every particle sits in the cell its position
  floors to.
- One oracle step (FP64) from a sampled run's GPU state reproduces the GPU
  step particle by particle (FP32 vs FP64 rounding only).
- Sampling: upstream of the body the ensemble moments equal the free-stream
  values (density, drift, temperature) the inflow and the fill are drawn
  from; solid cells hold no particles; an explicit sample over all 64M cells
  adds exactly the per-cell sums of the particle state.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

SAMPLED = (0, 17, 31)


@pytest.fixture(scope="module")
def body(dsmc_gpu):
    import torch
    wl = W.body3d()
    wl.sample_steps = [2, 4]
    E = dsmc_gpu.Ensemble.from_workload(wl, use_graph=True)
    yield wl, E
    E.close()
    del E
    torch.cuda.empty_cache()


def _cells_of(st, rs):
    out = np.zeros(st.shape[1], np.int64)
    mul = 1
    for a, (n, L) in enumerate(((rs.nx, rs.lx), (rs.ny, rs.ly), (rs.nz, rs.lz))):
        inv = np.float32(np.float64(n) / L)
        i = np.clip(np.floor(st[a].astype(np.float32) * inv), 0, n - 1).astype(np.int64)
        out += i * mul
        mul *= n
    return out


def test_body3d_full_size_indexing_and_one_step(body, oracle_lib):
    wl, E = body
    rs = wl.runs[0]
    solid = rs.solid.ravel().astype(bool)
    E.step(2)
    before = {r: (E.state(r), E.cell_state(r)) for r in SAMPLED}
    E.step(1)
    for r in SAMPLED:
        st1 = E.state(r)
        lcr, cell, start = E.lcr(r)
        ref_lcr, ref_start, _ = oracle_lib.counting_sort(cell, rs.n_cells + 1)
        np.testing.assert_array_equal(lcr, ref_lcr)
        np.testing.assert_array_equal(start[: rs.n_cells + 2], ref_start)
        keep = int(start[rs.n_cells])
        assert st1.shape[1] == keep and keep > 59_000_000
        live = cell[lcr[:keep]]
        assert not np.any(solid[live])
        # positions floor to their cells except where rounding put an end
        # point on a solid face and it was moved into the fluid cell
        same = _cells_of(st1, rs) == live
        assert same.mean() > 0.999999
        # one oracle step from the GPU's FP32 state and cell state
        st0, cs0 = before[r]
        n0 = st0.shape[1]
        O = oracle_lib.OracleRun(wl.runs[r], init=False)
        O.set_state(st0)
        O.set_cell_state(cs0["rem"], cs0["gmax"])
        O.set_step(2)
        O.step()
        so = O.state()
        ol = O.cells()
        okeep = int(ol["start"][rs.n_cells])
        # particle identity = slot before the step; compare the particles both
        # sides kept (the inflow count may differ by the face remainders)
        ids_g = lcr[:keep]
        ids_o = ol["lcr"][:okeep]
        pos_g = np.full(n0, -1, np.int64)
        pos_o = np.full(n0, -1, np.int64)
        mg = ids_g < n0
        mo = ids_o < n0
        pos_g[ids_g[mg]] = np.nonzero(mg)[0]
        pos_o[ids_o[mo]] = np.nonzero(mo)[0]
        both = (pos_g >= 0) & (pos_o >= 0)
        assert both.mean() > 0.99
        a = st1[:, pos_g[both]]
        b = so[:, pos_o[both]]
        close = np.all(np.abs(a - b) <= 1e-5 * (1 + np.abs(b)), axis=0)
        assert close.mean() > 0.995, (r, close.mean())
        del O, so, ol


def test_body3d_full_size_free_stream_moments(body):
    wl, E = body
    rs = wl.runs[0]
    info = E.info()
    E.step(4 - info["steps"])
    m, se = E.moments(1)                      # after step 4
    solid = rs.solid.ravel().astype(bool)
    assert np.all(np.isnan(m[solid, 0]) | (m[solid, 0] == 0))
    # upstream slab x < 0.2 (20 cell layers), away from the side walls
    ix = np.arange(rs.n_cells) % rs.nx
    iy = (np.arange(rs.n_cells) // rs.nx) % rs.ny
    iz = np.arange(rs.n_cells) // (rs.nx * rs.ny)
    up = (ix >= 2) & (ix < 20) & (iy >= 5) & (iy < 95) & (iz >= 5) & (iz < 95)
    ppc = rs.inflow_n * rs.cell_volume
    n = m[up, 0]
    assert abs(n.mean() / ppc - 1) < 0.002, (n.mean(), ppc)
    assert abs(np.mean(m[up, 1]) / rs.inflow_U - 1) < 0.002
    assert abs(np.mean(m[up, 4]) - rs.inflow_T) < 0.005
    assert np.all(np.abs(m[up, 2:4]).mean(axis=0) < 0.05)


def test_body3d_full_size_explicit_sample_matches_the_particles(body):
    """dsmc_sample over 64M cells (more workgroups than one launch takes, so
    the sampling kernel goes out in two launches): the sums it adds to a
    slot equal, run by run (each run its own group), per-cell sums of the
    particle state computed on the host."""
    wl, E = body
    rs = wl.runs[0]
    nc = rs.n_cells
    before = E.accum(1)
    E.sample(1)
    snap = E.accum(1) - before
    for r in SAMPLED:
        st = E.state(r)
        _, _, start = E.lcr(r)
        cells = np.repeat(np.arange(nc), np.diff(start[: nc + 1]))
        assert cells.size == st.shape[1]
        u, v, w = st[3], st[4], st[5]
        ref = np.stack([np.bincount(cells, weights=x, minlength=nc)
                        for x in (np.ones_like(u), u, v, w, u * u, v * v, w * w)], axis=1)
        np.testing.assert_allclose(snap[r], ref, rtol=1e-9, atol=1e-6, err_msg=f"run {r}")
