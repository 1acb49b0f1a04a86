"""The 3-D crowded-cell Interaction kernels in FP32 (the precision of the
batched path): a wavefront per cell at ~150 particles per cell and a block
per cell at ~400 in 3-D, against one oracle step (FP64) from the same GPU
state, particle by particle, and against each other (every mode runs each
cell's selections in the sequential order, Sec. 1.1 Interaction per cell)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _box3d(ppc, seed, n_runs=2):
    return W.box3d(n_per_run=ppc * 8 * 6 * 5, n_runs=n_runs, grid=(8, 6, 5), seed=seed,
                   state_fp64=False, wall="diffuse", wall_T=1.5)


@pytest.mark.parametrize("ppc", [150, 400])
def test_fp32_crowded_3d_step_matches_one_oracle_step(dsmc_gpu, oracle_lib, ppc):
    wl = _box3d(ppc, 80 + ppc)
    E = dsmc_gpu.Ensemble(wl.runs, [], state_fp64=False)
    E.step(2)
    before = {r: (E.state(r), E.cell_state(r)) for r in range(2)}
    E.step(1)
    for r in range(2):
        st1 = E.state(r)
        lcr, cell, start = E.lcr(r)
        st0, cs0 = before[r]
        O = oracle_lib.OracleRun(wl.runs[r], init=False)
        O.set_state(st0)
        O.set_cell_state(cs0["rem"], cs0["gmax"])
        O.set_step(2)
        O.step()
        so = O.state()
        assert so.shape == st1.shape
        # particle by particle (identity = slot before the step): a particle
        # that FP32 rounding puts in another cell changes only its two cells
        by_id_gpu = np.empty_like(st1)
        by_id_gpu[:, lcr] = st1
        by_id_ora = np.empty_like(so)
        by_id_ora[:, O.cells()["lcr"]] = so
        close = np.all(np.abs(by_id_ora - by_id_gpu) <= 1e-5 * (1 + np.abs(by_id_ora)), axis=0)
        assert close.mean() > 0.995, (r, close.mean())
        got = int(E.cell_state(r)["ncoll"].sum() - cs0["ncoll"].sum())
        assert abs(int(O.info()["ncoll"]) - got) <= max(20, 0.002 * got), (got, O.info()["ncoll"])


@pytest.mark.parametrize("ppc", [150, 400])
@pytest.mark.parametrize("mode", [1, 2, 3])
def test_fp32_3d_interaction_modes_give_identical_results(dsmc_gpu, ppc, mode):
    wl = _box3d(ppc, 90 + ppc)
    A = dsmc_gpu.Ensemble(wl.runs, [3], state_fp64=False, n_groups=1, collide_mode=0)
    B = dsmc_gpu.Ensemble(wl.runs, [3], state_fp64=False, n_groups=1, collide_mode=mode)
    A.step(3)
    B.step(3)
    for r in range(2):
        np.testing.assert_array_equal(A.state(r), B.state(r))
        np.testing.assert_array_equal(A.cell_state(r)["ncoll"], B.cell_state(r)["ncoll"])
        np.testing.assert_array_equal(A.cell_state(r)["gmax"], B.cell_state(r)["gmax"])


def test_fp32_3d_cells_beyond_the_stage(dsmc_gpu):
    """1600 particles per cell: beyond the FP32 block stage (1280) and the
    wavefront stage (512): the fallbacks agree with each other and with the
    lane mode bit for bit."""
    wl = W.box3d(n_per_run=1600 * 12, n_runs=1, grid=(3, 2, 2), seed=95, state_fp64=False)
    res = []
    for mode in (0, 1, 3):
        E = dsmc_gpu.Ensemble(wl.runs, [], state_fp64=False, collide_mode=mode)
        E.step(2)
        res.append((E.state(0), E.cell_state(0)["ncoll"]))
    for st, nc in res[1:]:
        np.testing.assert_array_equal(st, res[0][0])
        np.testing.assert_array_equal(nc, res[0][1])
    assert res[0][1].sum() > 100
