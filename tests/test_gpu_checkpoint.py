"""Checkpoint and resume, per-run diagnostics, sampling windows (the
steady-flow variant) and the error paths of the C ABI, on the GPU.

A run is replayable from its Philox key and the step counter (Sec. 1.1: runs
made independent by shifting the generator), so a context restored from a
checkpoint must continue bit for bit as the checkpointed one does."""
import math
from dataclasses import replace

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _channel_runs(n, seed=41, fp64=False):
    # inflow (face remainders), a diffuse wall, outflow; a partial fill
    return [replace(W.channel_run(nx=48, ny=12, lx=3.0, ly=0.75, ppc_inf=35.0, run_id=r, seed=seed),
                    n_init=6000, init_U=(2.0, 0.0, 0.0))
            for r in range(n)]


def _same(A, B, n_runs, tag):
    for r in range(n_runs):
        np.testing.assert_array_equal(A.state(r), B.state(r), err_msg=f"{tag}: state of run {r}")
        ca, cb = A.cell_state(r), B.cell_state(r)
        for k in ("rem", "gmax", "ncoll", "nbar"):
            np.testing.assert_array_equal(ca[k], cb[k], err_msg=f"{tag}: {k} of run {r}")
    np.testing.assert_array_equal(A.counts(), B.counts(), err_msg=tag)
    np.testing.assert_array_equal(A.sample_counts(), B.sample_counts(), err_msg=tag)
    for k in range(A.opt.n_samples):
        np.testing.assert_array_equal(A.accum(k), B.accum(k), err_msg=f"{tag}: slot {k}")
    np.testing.assert_array_equal(A.diag(), B.diag(), err_msg=tag)


@pytest.mark.parametrize("fp64,sub,alpha", [(False, 1, 0.0), (True, 1, 0.0), (False, 3, 0.0), (True, 1, 0.4),
                                            (False, 1, 0.4)])
def test_checkpoint_resume_is_bit_identical(dsmc_gpu, fp64, sub, alpha):
    """Checkpoint after 7 steps, restore into a fresh context with another
    tile size and graph replay, and step both 9 more: identical particles,
    cell state, accumulators (slots on both sides of the checkpoint and one
    window across it), counts and diagnostics; LCR of the next step too
    (with 3 x 3 sub-cells: the LCR and bin starts are by sub-cell; with the
    running-mean count: the per-cell means too)."""
    runs = [replace(r, subcells=sub, ntc_nbar_alpha=alpha) for r in _channel_runs(5)]
    kw = dict(state_fp64=fp64, n_groups=2, window_steps=3, window_stride=2)
    A = dsmc_gpu.Ensemble(runs, [4, 9, 16], **kw)
    A.step(7)
    ck = A.checkpoint()
    assert ck.size == dsmc_gpu.dsmc_checkpoint_bytes(A.ctx)
    B = dsmc_gpu.Ensemble(runs, [4, 9, 16], tile_chunks=128, use_graph=True, **kw)
    B.restore(ck)
    _same(A, B, len(runs), "at the checkpoint")
    assert B.info()["steps"] == 7
    A.step(9)
    B.step(9)
    _same(A, B, len(runs), "9 steps after")
    for r in range(len(runs)):
        la, lb = A.lcr(r), B.lcr(r)
        for x, y in zip(la, lb):
            np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(A.sample_counts(), [2, 3, 3])   # slot 0: steps 2 and 4


def test_checkpoint_of_a_fresh_context_and_foreign_checkpoints(dsmc_gpu):
    runs = _channel_runs(2)
    A = dsmc_gpu.Ensemble(runs, [3], state_fp64=False)
    ck0 = A.checkpoint()                       # before any step
    A.step(3)
    B = dsmc_gpu.Ensemble(runs, [3], state_fp64=False)
    B.restore(ck0)
    B.step(3)
    _same(A, B, 2, "restored from step 0")
    ck = A.checkpoint()
    other = dsmc_gpu.Ensemble(_channel_runs(2, seed=42), [3], state_fp64=False)
    f64 = dsmc_gpu.Ensemble(runs, [3], state_fp64=True)
    for ctx, buf in ((other, ck), (f64, ck), (B, ck[:-8]), (B, np.zeros_like(ck))):
        before = ctx.state(0)
        with pytest.raises(dsmc_gpu.DsmcError) as e:
            ctx.restore(buf)
        assert e.value.status == -1
        np.testing.assert_array_equal(ctx.state(0), before)   # nothing changed


def test_diag_against_the_oracle_fp64(dsmc_gpu, oracle_lib):
    """Diagnostics of the plain box against the oracle after the same steps:
    counts and collisions exact, momentum and energy sums to 1e-12; energy
    stays what it was (specular walls, elastic collisions)."""
    wl = W.plain_box()
    E = dsmc_gpu.Ensemble(wl.runs, [], state_fp64=True)
    O = oracle_lib.OracleRun(wl.runs[0])
    d0 = E.diag()[0]
    for s in (1, 4):
        E.step(s)
        O.step(s)
    d = E.diag()[0]
    np.testing.assert_array_equal(E.diag(), E.diag())    # same bits each call
    st = O.state()
    assert d[0] == O.n and d[1] == 0
    assert d[2] == O.cell_state()["ncoll"].sum()
    for a in range(3):
        assert math.isclose(d[3 + a], math.fsum(st[3 + a]), rel_tol=1e-12, abs_tol=1e-9)
    e = math.fsum((st[3:] ** 2).ravel())
    assert math.isclose(d[6], e, rel_tol=1e-12)
    assert math.isclose(d[6], d0[6], rel_tol=1e-12)


def test_sampling_window_parity_fp64(dsmc_gpu, oracle_lib):
    """Windowed slots against the oracle ensemble on the same Philox streams:
    snapshot counts exact, sums to 1e-12, moments and batch-means errors
    element by element from the oracle's FP64 division of the same sums."""
    runs = [replace(r, n_init=0) for r in _channel_runs(4, seed=43)]
    wl = W.Workload("win", runs, 20, [9, 20], 2, state_fp64=True, window_steps=4, window_stride=2)
    E = dsmc_gpu.Ensemble.from_workload(wl)
    E.step(20)
    acc_o, st = oracle_lib.ensemble(wl, n_threads=2)
    np.testing.assert_array_equal(E.sample_counts(), st["n_snap"])
    assert st["n_snap"] == [4, 4]
    for k in range(2):
        g = E.accum(k)
        np.testing.assert_allclose(g, acc_o[k], rtol=1e-12, atol=1e-9)
        m, se = E.moments(k)
        mo = oracle_lib.moments(g.sum(axis=0), n_runs=4, n_snap=4)
        np.testing.assert_allclose(m, mo, rtol=1e-12, atol=1e-12, equal_nan=True)
        mg = np.stack([oracle_lib.moments(g[q], n_runs=2, n_snap=4) for q in range(2)])
        with np.errstate(invalid="ignore"):
            seo = mg.std(axis=0, ddof=1) / math.sqrt(2)
        np.testing.assert_allclose(se, seo, rtol=1e-9, atol=1e-12, equal_nan=True)


def test_set_state_rejects_non_finite_and_outside(dsmc_gpu):
    runs = [W.box(2000, 1, 1, 1, seed=61, grid=(8, 8)).runs[0]]
    E = dsmc_gpu.Ensemble(runs, [], state_fp64=False)
    before = E.state(0)
    good = np.zeros((6, 10))
    good[0:2] = 0.5
    good[3:] = 1.0
    for a, v in ((0, np.nan), (4, np.inf), (5, -np.inf), (0, 1.5), (1, -0.01)):
        bad = good.copy()
        bad[a, 3] = v
        with pytest.raises(dsmc_gpu.DsmcError) as e:
            E.set_state(0, bad)
        assert e.value.status == -1
    np.testing.assert_array_equal(E.state(0), before)
    edge = good.copy()
    edge[0, 0], edge[1, 1] = 1.0, 0.0         # on the faces: accepted
    E.set_state(0, edge)


def test_too_many_wall_hits_is_reported(dsmc_gpu):
    """A finite speed that crosses the box ~100 times in one step: the wall
    loop stops at its bound of 64 interactions and latches DSMC_EBOUNCE."""
    rs = W.box(500, 1, 1, 1, seed=62, grid=(4, 4)).runs[0]
    E = dsmc_gpu.Ensemble([rs], [], state_fp64=True)
    st = E.state(0)
    st[3, 0] = 100.0 * rs.lx / rs.dt
    E.set_state(0, st)
    E.step(1)
    with pytest.raises(dsmc_gpu.DsmcError) as e:
        E.sync()
    assert e.value.status == -7


@pytest.mark.parametrize("fp64", [False, True])
def test_absurd_collision_rate_is_reported(dsmc_gpu, fp64):
    """A finite but enormous w (2-D: it takes no part in the flight) makes the
    pair's g enormous; the next step's NTC count exceeds 1e9 selections in
    that cell and latches DSMC_ENUMERIC."""
    rs = W.box(3000, 1, 1, 1, seed=63, grid=(2, 2)).runs[0]
    E = dsmc_gpu.Ensemble([rs], [], state_fp64=fp64)
    st = E.state(0)
    st[5, :] = 1e15
    st[5, ::2] = -1e15
    E.set_state(0, st)
    E.step(3)
    with pytest.raises(dsmc_gpu.DsmcError) as e:
        E.sync()
    assert e.value.status == -9


def test_fill_of_an_almost_solid_run_is_reported(dsmc_gpu):
    """One fluid cell among 1000: most fill positions need more than 100
    draws, so dsmc_init_runs returns DSMC_EREJECT."""
    rs = W.box3d(2000, 1, grid=(10, 10, 10), seed=64).runs[0]
    mask = np.ones((10, 10, 10), np.uint8)
    mask[5, 5, 5] = 0
    rs = replace(rs, solid=mask, solid_T=1.0)
    with pytest.raises(dsmc_gpu.DsmcError) as e:
        dsmc_gpu.Ensemble([rs], [], state_fp64=True)
    assert e.value.status == -8
