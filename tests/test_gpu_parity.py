"""FP64 GPU path vs the FP64 oracle on identical inputs and identical Philox
streams: LCR and cell counts bit-exact, particle state, per-cell interaction
state and sampled sums within 1e-12 relative, step by step (Sec. 1.1 order:
Generation, Motion, Enumeration/Indexing, Interaction, Sampling)."""
import math
from dataclasses import replace

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12
WORST = {"pos": 0.0, "vel": 0.0}   # largest differences seen (printed at the end)


def _t_ref(rs):
    T = [rs.init_T if rs.n_init else 0.0, rs.inflow_T if rs.has_inflow else 0.0]
    T += [rs.face_T[f] for f in range(2 * rs.dim) if rs.face_bc[f] == "diffuse"]
    if rs.solid is not None:
        T.append(rs.solid_T)
    return max(max(T), 1e-300)


def _compare_run(E, r, O, rs, where):
    lcr, cell, start = E.lcr(r)
    cl = O.cells()
    assert lcr.size == cl["lcr"].size, where
    np.testing.assert_array_equal(cell, cl["cell"], err_msg=where)
    np.testing.assert_array_equal(lcr, cl["lcr"], err_msg=where)
    np.testing.assert_array_equal(start[: cl["start"].size], cl["start"], err_msg=where)
    g, o = E.state(r), O.state()
    assert g.shape == o.shape, where
    L = np.array([rs.lx, rs.ly, rs.lz])[:, None]
    if g.shape[1]:
        # positions relative to the box, velocities relative to the thermal
        # speed of the hottest gas or wall of the run
        pos_err = np.max(np.abs(g[:3] - o[:3]) / L)
        vel_err = np.max(np.abs(g[3:] - o[3:])) / math.sqrt(_t_ref(rs))
        WORST["pos"] = max(WORST["pos"], pos_err)
        WORST["vel"] = max(WORST["vel"], vel_err)
        assert pos_err < TOL and vel_err < TOL, (where, pos_err, vel_err)
    cg, co = E.cell_state(r), O.cell_state()
    np.testing.assert_array_equal(cg["ncoll"], co["ncoll"], err_msg=where)
    np.testing.assert_allclose(cg["gmax"], co["gmax"], rtol=TOL, err_msg=where)
    np.testing.assert_allclose(cg["rem"], co["rem"], rtol=0, atol=TOL, err_msg=where)
    np.testing.assert_allclose(cg["nbar"], co["nbar"], rtol=TOL, atol=TOL, err_msg=where)


def _parity(dsmc_gpu, oracle_lib, runs, n_steps, check_every=1, squeeze=None, **kw):
    E = dsmc_gpu.Ensemble(runs, sample_steps=[n_steps], state_fp64=True, n_groups=len(runs), **kw)
    O = [oracle_lib.OracleRun(r) for r in runs]
    for r, rs in enumerate(runs):
        g, o = E.state(r), O[r].state()
        np.testing.assert_allclose(g, o, rtol=0, atol=1e-13)
        if squeeze is not None:      # same crowded initial state on both sides
            o[1] *= squeeze
            O[r].set_state(o)
            E.set_state(r, o)
    for s in range(1, n_steps + 1):
        E.step(1)
        for o in O:
            o.step()
        if s % check_every == 0 or s == n_steps:
            for r, rs in enumerate(runs):
                _compare_run(E, r, O[r], rs, f"run {r} step {s}")
    acc = E.accum(0)
    for r in range(len(runs)):
        ref = O[r].sample()
        np.testing.assert_allclose(acc[r], ref, rtol=TOL, atol=TOL)
    counts = E.counts()
    for r in range(len(runs)):
        assert counts[r, 0] == O[r].n
        assert counts[r, 1] == O[r].info()["ngen"]
    E.close()
    return O


def test_plain_box_fp64(dsmc_gpu, oracle_lib):
    """20,000 hard spheres, 32x32 cells, specular walls, 5 steps."""
    O = _parity(dsmc_gpu, oracle_lib, W.plain_box().runs, 5)
    assert O[0].info()["ncoll"] > 1500


def test_channel_inflow_diffuse_vhs_fp64(dsmc_gpu, oracle_lib):
    """Two batched channel runs: inflow generation, diffuse wall at T=2,
    vacuum outflow, VHS; one starts half full and drifting, one empty."""
    a = W.channel_run(nx=64, ny=16, lx=4.0, ly=1.0, ppc_inf=30.0, run_id=0, seed=11)
    a = replace(a, n_init=15000, init_U=(a.inflow_U, 0.0, 0.0))
    b = W.channel_run(nx=64, ny=16, lx=4.0, ly=1.0, ppc_inf=30.0, run_id=1, seed=11)
    O = _parity(dsmc_gpu, oracle_lib, [a, b], 8)
    assert O[1].n > 0 and O[0].info()["nremoved"] >= 0


def test_two_pass_indexing_fp64(dsmc_gpu, oracle_lib):
    """> 2047 cells: Indexing sorts by bucket (bin >> 11), then each bucket by
    its low 11 bits."""
    a = W.channel_run(nx=64, ny=40, lx=1.6, ly=1.0, ppc_inf=12.0, mach=1.0, run_id=3, seed=12)
    a = replace(a, n_init=20000, init_U=(a.inflow_U, 0.0, 0.0))
    b = replace(a, run_id=4)
    _parity(dsmc_gpu, oracle_lib, [a, b], 5)


def test_two_pass_indexing_edges_fp64(dsmc_gpu, oracle_lib):
    """Two-level Indexing edge cases in one batch: 4095 cells (the bin after
    the DEAD bin starts a bucket that does not exist), a channel filling from
    empty (most buckets empty at first, one bucket item holding the inflow
    layer), and a run of 100 cells (one bucket) beside them."""
    edge = replace(W.box(12000, 1, 3, 3, seed=21, grid=(91, 45)).runs[0], run_id=0)
    empty = replace(W.channel_run(nx=96, ny=48, lx=2.0, ly=1.0, ppc_inf=6.0, mach=2.0, run_id=1, seed=21),
                    n_init=0, ensemble=1)
    small = replace(W.box(3000, 1, 3, 3, seed=21, grid=(10, 10)).runs[0], run_id=2, ensemble=2)
    runs = [edge, empty, small]
    E = dsmc_gpu.Ensemble(runs, sample_steps=[4], state_fp64=True, n_groups=1)
    O = [oracle_lib.OracleRun(r) for r in runs]
    for s in range(1, 5):
        E.step(1)
        for o in O:
            o.step()
        for r, rs in enumerate(runs):
            _compare_run(E, r, O[r], rs, f"run {r} step {s}")
    for r in range(3):
        np.testing.assert_allclose(E.accum(0, ensemble=r)[0], O[r].sample(), rtol=TOL, atol=TOL)
    E.close()


def test_box3d_diffuse_fp64(dsmc_gpu, oracle_lib):
    wl = W.box3d(n_per_run=20000, n_runs=2, grid=(10, 8, 6), wall="diffuse", wall_T=1.3, seed=13)
    _parity(dsmc_gpu, oracle_lib, wl.runs, 5)


def test_uneven_runs_fp64(dsmc_gpu, oracle_lib):
    """Runs of different grids and particle counts in one launch."""
    a = W.box(6000, 1, 5, 5, seed=14, grid=(16, 16)).runs[0]
    b = replace(W.box(17000, 1, 5, 5, seed=14, grid=(32, 16)).runs[0], run_id=1, ensemble=1)
    c = replace(W.channel_run(nx=24, ny=24, lx=1.0, ly=1.0, ppc_inf=20.0, run_id=2, seed=14),
                ensemble=2)
    E_runs = [a, b, c]
    E = dsmc_gpu.Ensemble(E_runs, sample_steps=[5], state_fp64=True, n_groups=1)
    O = [oracle_lib.OracleRun(r) for r in E_runs]
    for s in range(1, 6):
        E.step(1)
        for o in O:
            o.step()
        for r, rs in enumerate(E_runs):
            _compare_run(E, r, O[r], rs, f"run {r} step {s}")
    for r in range(3):
        np.testing.assert_allclose(E.accum(0, ensemble=r)[0], O[r].sample(), rtol=TOL, atol=TOL)


@pytest.mark.parametrize("graph,lanes", [(False, 1), (True, 1), (False, 2)])
def test_mixed_interaction_modes_fp64(dsmc_gpu, oracle_lib, graph, lanes):
    """One batch whose runs need all three Interaction modes (~20, ~160 and
    ~620 expected particles per cell: a lane, a wavefront and a block per
    cell), eagerly and replayed from a graph, in one or two stream lanes:
    step by step equal to the oracle."""
    sparse = W.box(5000, 1, 4, 4, seed=16, grid=(16, 16)).runs[0]
    mid = replace(W.box(40000, 1, 4, 4, seed=16, grid=(16, 16)).runs[0], run_id=1, ensemble=1)
    dense = replace(W.box(40000, 1, 4, 4, seed=16, grid=(8, 8)).runs[0], run_id=2, ensemble=2)
    runs = [sparse, mid, dense, replace(sparse, run_id=3, ensemble=3)]
    E = dsmc_gpu.Ensemble(runs, sample_steps=[4], state_fp64=True, n_groups=1, use_graph=graph,
                          n_streams=lanes)
    O = [oracle_lib.OracleRun(r) for r in runs]
    for s in range(1, 5):
        E.step(1)
        for o in O:
            o.step()
        for r, rs in enumerate(runs):
            _compare_run(E, r, O[r], rs, f"run {r} step {s}")
    for r in range(len(runs)):
        np.testing.assert_allclose(E.accum(0, ensemble=r)[0], O[r].sample(), rtol=TOL, atol=TOL)
    E.close()


def test_dense_cells_one_wave_per_cell_fp64(dsmc_gpu, oracle_lib):
    """~390 particles per cell: one 256-thread block per cell (the auto
    mode), 256 selections per window in conflict-free levels; the first steps
    exceed (sigma c_r)_max often, so windows are undone and replayed."""
    wl = W.box(100_000, 2, 5, 5, seed=15, grid=(16, 16))
    O = _parity(dsmc_gpu, oracle_lib, wl.runs, 5)
    assert O[0].info()["ncoll"] > 5000


def test_sparse_cells_forced_block_mode_fp64(dsmc_gpu, oracle_lib):
    _parity(dsmc_gpu, oracle_lib, W.plain_box().runs, 4, collide_mode=2)


def test_wavefront_per_cell_fp64(dsmc_gpu, oracle_lib):
    """~130 particles per cell: one wavefront per cell (the auto mode), 64
    selections per window with wavefront-level synchronisation, undone and
    replayed when (sigma c_r)_max grows inside a window."""
    wl = W.box(33_000, 2, 5, 5, seed=19, grid=(16, 16))
    O = _parity(dsmc_gpu, oracle_lib, wl.runs, 5)
    assert O[0].info()["ncoll"] > 1000


def test_wavefront_per_cell_beyond_its_stage_fp64(dsmc_gpu, oracle_lib):
    """~390 particles per cell forced into the wavefront mode, whose FP64
    stage holds 256: every cell takes the sequential fallback on P'."""
    wl = W.box(100_000, 1, 3, 3, seed=20, grid=(16, 16))
    _parity(dsmc_gpu, oracle_lib, wl.runs, 3, collide_mode=3)


def test_dense_cells_forced_lane_mode_fp64(dsmc_gpu, oracle_lib):
    wl = W.box(60_000, 1, 3, 3, seed=16, grid=(16, 16))
    _parity(dsmc_gpu, oracle_lib, wl.runs, 3, collide_mode=1)


def test_cells_beyond_lds_capacity_fp64(dsmc_gpu, oracle_lib):
    """A cell (block mode) and a 64-cell group (lane mode) holding more
    particles than the LDS stage: the global-memory fallbacks."""
    big_cell = W.box(20_000, 1, 3, 3, seed=17, grid=(4, 4)).runs      # 1250 per cell
    _parity(dsmc_gpu, oracle_lib, big_cell, 3)
    # 31 per cell on average, but every particle starts in the bottom rows:
    # the first lane-mode group holds all 2000
    big_group = W.box(2_000, 1, 3, 3, seed=18, grid=(8, 8)).runs
    _parity(dsmc_gpu, oracle_lib, big_group, 3, squeeze=0.2)


@pytest.mark.parametrize("ppc", [150, 400])
@pytest.mark.parametrize("mode", [0, 1, 2, 3])
def test_box3d_crowded_cells_fp64(dsmc_gpu, oracle_lib, ppc, mode):
    """3-D cells of ~150 and ~400 particles (auto: a wavefront, then a block
    per cell), and every forced mode: a lane per cell, a block per cell, a
    wavefront per cell (beyond its 256-particle FP64 stage at 400)."""
    wl = W.box3d(n_per_run=ppc * 120, n_runs=2, grid=(6, 5, 4), seed=70 + ppc + mode, wall="diffuse",
                 wall_T=1.2)
    O = _parity(dsmc_gpu, oracle_lib, wl.runs, 4, collide_mode=mode)
    assert O[0].info()["ncoll"] > 200


def test_box3d_cells_beyond_lds_capacity_fp64(dsmc_gpu, oracle_lib):
    """3-D cells holding more particles than each mode's LDS stage: 1250 per
    cell (block mode, stage 1024; wavefront mode, stage 256) and a lane-mode
    group of cells holding all 2000 particles of a run (stage 512)."""
    big = W.box3d(n_per_run=22_500, n_runs=1, grid=(3, 3, 2), seed=75).runs
    _parity(dsmc_gpu, oracle_lib, big, 3)
    _parity(dsmc_gpu, oracle_lib, big, 2, collide_mode=3)
    grp = W.box3d(n_per_run=2000, n_runs=1, grid=(8, 8, 2), seed=76).runs
    _parity(dsmc_gpu, oracle_lib, grp, 3, squeeze=0.1)


def _sub(runs, k):
    return [replace(r, subcells=k) for r in runs]


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
@pytest.mark.parametrize("ppc", [30, 150, 400])
def test_subcell_partners_fp64(dsmc_gpu, oracle_lib, mode, ppc):
    """Sub-cell partner choice (2 x 2 sub-cells): Enumeration bins by
    sub-cell, the LCR is sorted by bin, and every selection's second partner
    comes from the first one's sub-cell when it holds two or more; ~30, ~150
    and ~400 particles per cell in the auto mode and every forced mode."""
    wl = W.box(ppc * 64, 2, 4, 4, seed=90 + ppc + mode, grid=(8, 8))
    O = _parity(dsmc_gpu, oracle_lib, _sub(wl.runs, 2), 4, collide_mode=mode)
    assert O[0].info()["nbin"] == 64 * 4 and O[0].info()["ncoll"] > 50


@pytest.mark.parametrize("mode", [0, 1, 3])
def test_subcell_partners_3d_fp64(dsmc_gpu, oracle_lib, mode):
    """3-D, 2 x 2 x 2 sub-cells per cell, diffuse walls."""
    wl = W.box3d(n_per_run=150 * 120, n_runs=2, grid=(6, 5, 4), seed=95 + mode, wall="diffuse", wall_T=1.2)
    O = _parity(dsmc_gpu, oracle_lib, _sub(wl.runs, 2), 4, collide_mode=mode)
    assert O[0].info()["nbin"] == 120 * 8


def test_subcell_partners_channel_and_beyond_lds_fp64(dsmc_gpu, oracle_lib):
    """3 x 3 sub-cells in a channel with inflow, diffuse wall and outflow;
    cells beyond each mode's LDS stage (1250 per cell: block and wavefront
    modes) take the global-memory fallbacks with sub-cells too; more than
    2047 bins (2304 and 4096) take the two-level Indexing."""
    ch = W.channel_run(nx=32, ny=8, lx=2.0, ly=0.5, ppc_inf=30.0, run_id=0, seed=97)
    ch = replace(ch, subcells=3, n_init=4000, init_U=(ch.inflow_U, 0.0, 0.0))
    _parity(dsmc_gpu, oracle_lib, [ch], 5)
    big = _sub(W.box(20_000, 1, 3, 3, seed=98, grid=(4, 4)).runs, 4)
    _parity(dsmc_gpu, oracle_lib, big, 3)
    _parity(dsmc_gpu, oracle_lib, big, 2, collide_mode=3)
    wide = _sub(W.box(30_000, 1, 3, 3, seed=99, grid=(32, 32)).runs, 2)     # 4096 bins
    _parity(dsmc_gpu, oracle_lib, wide, 3)


@pytest.mark.parametrize("mode", [0, 1, 2, 3])
@pytest.mark.parametrize("alpha", [0.3, 1.0])
def test_ntc_running_mean_count_fp64(dsmc_gpu, oracle_lib, mode, alpha):
    """Bird's N * Nbar / 2 count with a running mean per cell, in the auto
    mode and every forced mode, on cells of ~150 particles (2-D) and ~40
    (3-D): the running means and remainders within 1e-12, everything else as
    for the pair count."""
    wl = W.box(150 * 64, 2, 4, 4, seed=110 + mode, grid=(8, 8))
    runs = [replace(r, ntc_nbar_alpha=alpha) for r in wl.runs]
    O = _parity(dsmc_gpu, oracle_lib, runs, 4, collide_mode=mode)
    nb = O[0].cell_state()["nbar"]
    assert not np.allclose(nb, 150.0)      # the means moved with the counts
    w3 = W.box3d(n_per_run=40 * 120, n_runs=1, grid=(6, 5, 4), seed=115 + mode, wall="diffuse", wall_T=1.2)
    _parity(dsmc_gpu, oracle_lib, [replace(r, ntc_nbar_alpha=alpha) for r in w3.runs], 3, collide_mode=mode)


def test_ntc_running_mean_count_channel_fp64(dsmc_gpu, oracle_lib):
    """A channel filling through its inflow face (counts change step by step,
    empty cells start at a zero mean) with a slow running mean, next to a run
    that keeps the pair count."""
    a = W.channel_run(nx=32, ny=8, lx=2.0, ly=0.5, ppc_inf=30.0, run_id=0, seed=118)
    a = replace(a, n_init=3000, init_U=(a.inflow_U, 0.0, 0.0), ntc_nbar_alpha=0.1)
    b = replace(a, run_id=1, ntc_nbar_alpha=0.0)
    _parity(dsmc_gpu, oracle_lib, [a, b], 6)


def test_zz_worst_parity_differences():
    """Reports the largest position and velocity differences of the parity
    tests above (all below 1e-12)."""
    print(f"worst FP64 parity differences: positions/L {WORST['pos']:.3e}, "
          f"velocities/sqrt(T_ref) {WORST['vel']:.3e}")
    assert WORST["pos"] < TOL and WORST["vel"] < TOL
