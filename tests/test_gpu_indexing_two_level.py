"""The two-level Indexing (runs with 2049 .. 2^22 bins: a pass by bucket,
bin >> 11, then each bucket by its low 11 bits) against the oracle's stable
counting sort of the same cell array, bit for bit, step after step: after the
initial fill and in steady stepping, with tiles of 256, 768 and 16384 slots
(bucket items cut by many tile edges, buckets inside one tile), for a channel
filling from vacuum (empty buckets, most particles generated), with
sub-cells, in 2-D and 3-D; at the largest two-level grid and the first
grid past it (three LSD passes); and after a run's state was replaced by a
shuffled, shorter one, where the next steps must equal those of a context
restored from the same checkpoint and given the same state."""
from dataclasses import replace

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _bins(rs):
    k = max(1, getattr(rs, "subcells", 1))
    return rs.n_cells * k ** rs.dim + 1


def _check_lcr(E, runs, oracle_lib, where):
    for r, rs in enumerate(runs):
        lcr, cell, start = E.lcr(r)
        ref_lcr, ref_start, _ = oracle_lib.counting_sort(cell, _bins(rs))
        np.testing.assert_array_equal(lcr, ref_lcr, err_msg=f"{where} run {r}")
        np.testing.assert_array_equal(start[: ref_start.size], ref_start, err_msg=f"{where} run {r}")


def _runs(dim):
    if dim == 2:
        box = replace(W.box(30_000, 1, 1, 1, seed=31, grid=(64, 64)).runs[0], run_id=0)      # 4097 bins
        chan = replace(W.channel_run(nx=96, ny=48, lx=2.0, ly=1.0, ppc_inf=8.0, mach=2.0, run_id=2, seed=33),
                       n_init=0, ensemble=1)
        sub = replace(W.box(20_000, 1, 1, 1, seed=34, grid=(24, 24)).runs[0], run_id=3, ensemble=2, subcells=2)
        return [box, chan, sub]
    cube = replace(W.box3d(40_000, 1, grid=(20, 20, 20), seed=32).runs[0], run_id=1)
    sub3 = replace(W.box3d(30_000, 1, grid=(10, 10, 10), seed=36).runs[0], run_id=4, ensemble=1, subcells=2)
    return [cube, sub3]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("tc", [4, 12, 256])
def test_two_level_sort_is_the_stable_counting_sort(dsmc_gpu, oracle_lib, tc, dim):
    runs = _runs(dim)
    E = dsmc_gpu.Ensemble(runs, [8], state_fp64=False, n_groups=1, tile_chunks=tc)
    for s in range(1, 9):
        E.step(1)
        _check_lcr(E, runs, oracle_lib, f"tile_chunks {tc} step {s}")
    E.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_two_level_sort_after_state_replacement(dsmc_gpu, oracle_lib, dim):
    """A run's particles replaced by a shuffled 70 % of them: the next steps
    equal, particle by particle, those of a context restored from the same
    checkpoint and given the same states, and the LCRs are the counting
    sort."""
    runs = _runs(dim)
    E = dsmc_gpu.Ensemble(runs, [], state_fp64=True, n_groups=1, tile_chunks=4)
    E.step(4)
    F = dsmc_gpu.Ensemble(runs, [], state_fp64=True, n_groups=1, tile_chunks=4)
    F.restore(E.checkpoint())
    rng = np.random.default_rng(35)
    for r in range(len(runs)):
        st = E.state(r)
        keep = rng.permutation(st.shape[1])[: int(0.7 * st.shape[1])]
        st = st[:, keep]
        E.set_state(r, st)
        F.set_state(r, st)
    for s in range(3):
        E.step(1)
        F.step(1)
        _check_lcr(E, runs, oracle_lib, f"replaced, step {s}")
        for r in range(len(runs)):
            np.testing.assert_array_equal(E.lcr(r)[0], F.lcr(r)[0], err_msg=f"run {r} step {s}")
            np.testing.assert_array_equal(E.state(r), F.state(r), err_msg=f"run {r} step {s}")
    E.close()
    F.close()


@pytest.mark.parametrize("ny", [2047, 2049])
def test_largest_two_level_and_first_three_pass_grids(dsmc_gpu, oracle_lib, ny):
    """2048 x 2047 cells (4,192,257 bins with the DEAD bin: the largest
    two-level sort, 2047 buckets) and 2048 x 2049 (past 2^22 bins: three LSD
    passes), 1M particles: the step's LCR is the stable counting sort."""
    rs = replace(W.box(1_000_000, 1, 1, 1, seed=37, grid=(2048, ny)).runs[0], run_id=0)
    E = dsmc_gpu.Ensemble([rs], [], state_fp64=False, n_groups=1)
    for s in range(2):
        E.step(1)
        _check_lcr(E, [rs], oracle_lib, f"{ny} rows, step {s + 1}")
    E.close()
