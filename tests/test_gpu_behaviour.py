"""Behaviour of the batched GPU path: bitwise determinism, independence of a
run from the rest of its batch (runs are the paper's statistically
independent runs, Sec. 1.3), HIP-graph replay equal to eager launches, and
device-side error reporting through the C ABI."""
from dataclasses import replace

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _small_channel_runs(n, seed=31):
    return [replace(W.channel_run(nx=64, ny=16, lx=4.0, ly=1.0, ppc_inf=30.0, run_id=r, seed=seed),
                    n_init=8000, init_U=(2.5, 0.0, 0.0))
            for r in range(n)]


def test_bitwise_determinism_fp32(dsmc_gpu):
    runs = _small_channel_runs(6)
    A = dsmc_gpu.Ensemble(runs, [5, 10], state_fp64=False, n_groups=3)
    B = dsmc_gpu.Ensemble(runs, [5, 10], state_fp64=False, n_groups=3)
    A.step(10)
    B.step(10)
    for r in range(6):
        np.testing.assert_array_equal(A.state(r), B.state(r))
    np.testing.assert_array_equal(A.accum(1), B.accum(1))


def test_run_does_not_depend_on_its_batch(dsmc_gpu):
    """A run advanced alone and inside a batch of other runs (other grids,
    other sizes) follows the identical trajectory."""
    runs = _small_channel_runs(3)
    other = replace(W.box(30_000, 1, 1, 1, seed=9, grid=(20, 10)).runs[0], run_id=99, ensemble=7)
    alone = dsmc_gpu.Ensemble([runs[1]], [8], state_fp64=False)
    batch = dsmc_gpu.Ensemble([runs[0], other, runs[1], runs[2]], [8], state_fp64=False)
    alone.step(8)
    batch.step(8)
    np.testing.assert_array_equal(alone.state(0), batch.state(2))
    np.testing.assert_array_equal(alone.cell_state(0)["ncoll"], batch.cell_state(2)["ncoll"])


@pytest.mark.parametrize("fp64", [False, True])
def test_graph_replay_equals_eager(dsmc_gpu, fp64):
    """Every replay of the captured step graph (two graphs: even and odd
    steps) gives the state the eager launch sequence gives."""
    import torch
    runs = _small_channel_runs(4)
    E = dsmc_gpu.Ensemble(runs, [3, 6, 9], state_fp64=fp64, n_groups=2, use_graph=False)
    G = dsmc_gpu.Ensemble(runs, [3, 6, 9], state_fp64=fp64, n_groups=2, use_graph=True)
    for s in range(9):
        E.step(1)
        G.step(1)
        torch.cuda.synchronize()
        for r in range(4):
            np.testing.assert_array_equal(E.state(r), G.state(r), err_msg=f"step {s + 1}")
    for k in range(3):
        np.testing.assert_array_equal(E.accum(k), G.accum(k))
        m1, _ = E.moments(k)
        m2, _ = G.moments(k)
        np.testing.assert_array_equal(m1, m2)


@pytest.mark.parametrize("fp64,graph", [(False, True), (True, False)])
def test_tile_size_does_not_change_results(dsmc_gpu, fp64, graph):
    """Indexing tiles of 1, 3 and 5 rounds of 256 slots give the same runs,
    cell states and sample sums as the default 64 rounds: Motion's reads of
    in-place cells four rounds at a time, their remainder, and the switch to
    generated particles inside a tile (inflow channels) decide nothing about
    the result; neither do the tile histograms and wall-queue segments.  The
    64x64-cell box takes the two-level sort."""
    import torch
    big = replace(W.box(30_000, 1, 1, 1, seed=9, grid=(64, 64)).runs[0], run_id=50, ensemble=7)
    small = replace(W.box(3_001, 1, 1, 1, seed=9, grid=(8, 8)).runs[0], run_id=51, ensemble=8)
    runs = _small_channel_runs(3) + [big, small]
    ref = dsmc_gpu.Ensemble(runs, [3, 6], state_fp64=fp64, n_groups=2, use_graph=graph)
    ref.step(6)
    torch.cuda.synchronize()
    for tc in (4, 12, 20):
        E = dsmc_gpu.Ensemble(runs, [3, 6], state_fp64=fp64, n_groups=2, use_graph=graph, tile_chunks=tc)
        E.step(6)
        torch.cuda.synchronize()
        for r in range(len(runs)):
            np.testing.assert_array_equal(ref.state(r), E.state(r), err_msg=f"tile_chunks {tc} run {r}")
            np.testing.assert_array_equal(ref.cell_state(r)["ncoll"], E.cell_state(r)["ncoll"])
        for ens in (0, 7, 8):
            for k in range(2):
                np.testing.assert_array_equal(ref.accum(k, ensemble=ens), E.accum(k, ensemble=ens))
        np.testing.assert_array_equal(ref.counts(), E.counts())
        E.close()


@pytest.mark.parametrize("fp64,graph", [(False, True), (True, False)])
def test_stream_lanes_do_not_change_results(dsmc_gpu, fp64, graph):
    """The batch split into 2, 3 or 4 run groups stepped concurrently on
    their own streams (one group's Indexing and Interaction overlapping the
    next group's Motion) gives bit-identical runs, cell states and sample
    sums.  The batch mixes inflow channels with a 64x64-cell box (two
    indexing passes) and uneven sizes, so the groups are uneven too."""
    import torch
    big = replace(W.box(30_000, 1, 1, 1, seed=9, grid=(64, 64)).runs[0], run_id=50, ensemble=7)
    small = replace(W.box(3_000, 1, 1, 1, seed=9, grid=(8, 8)).runs[0], run_id=51, ensemble=8)
    runs = _small_channel_runs(4) + [big, small] + _small_channel_runs(2, seed=77)
    ref = dsmc_gpu.Ensemble(runs, [3, 6], state_fp64=fp64, n_groups=2, use_graph=graph, n_streams=1)
    ref.step(6)
    torch.cuda.synchronize()
    for lanes in (2, 3, 4):
        E = dsmc_gpu.Ensemble(runs, [3, 6], state_fp64=fp64, n_groups=2, use_graph=graph, n_streams=lanes)
        E.step(6)
        torch.cuda.synchronize()
        for r in range(len(runs)):
            np.testing.assert_array_equal(ref.state(r), E.state(r), err_msg=f"lanes {lanes} run {r}")
            np.testing.assert_array_equal(ref.cell_state(r)["ncoll"], E.cell_state(r)["ncoll"])
        for ens in (0, 7, 8):
            for k in range(2):
                np.testing.assert_array_equal(ref.accum(k, ensemble=ens), E.accum(k, ensemble=ens))
        np.testing.assert_array_equal(ref.counts(), E.counts())
        E.close()


def test_autotuned_settings_give_identical_results(dsmc_gpu):
    """dsmc_autotune picks tuning fields by timing; a context built with them
    follows the default context bit for bit."""
    import torch
    runs = _small_channel_runs(8)
    tuned = dsmc_gpu.Ensemble.autotune(runs, [3, 6], state_fp64=False, n_groups=2, use_graph=True, n_steps=2)
    assert tuned["tile_chunks"] in (64, 128, 256) and tuned["n_streams"] in (1, 2)
    assert tuned["collide_mode"] in (0, 1, 2, 3) and tuned["ms_per_step"] > 0
    assert tuned["sched"] in (0, 1) and tuned["sched_blocks"] in (0, 1024) and not tuned["from_cache"]
    kw = {k: tuned[k] for k in ("tile_chunks", "collide_mode", "n_streams", "sched", "sched_blocks")}
    A = dsmc_gpu.Ensemble(runs, [3, 6], state_fp64=False, n_groups=2, use_graph=True)
    B = dsmc_gpu.Ensemble(runs, [3, 6], state_fp64=False, n_groups=2, use_graph=True, **kw)
    A.step(6)
    B.step(6)
    torch.cuda.synchronize()
    for r in range(len(runs)):
        np.testing.assert_array_equal(A.state(r), B.state(r))
    for k in range(2):
        np.testing.assert_array_equal(A.accum(k), B.accum(k))


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_interaction_modes_give_identical_results(dsmc_gpu, mode):
    """The lane-per-cell, block-per-cell and wavefront-per-cell interaction
    kernels all run each cell's selections in the sequential order and add
    each cell's sample sums in one shared order: FP32 states, collision
    counts and sample sums are identical, and so are FP64 ones."""
    import torch
    runs = _small_channel_runs(3)
    for fp64 in (False, True):
        A = dsmc_gpu.Ensemble(runs, [2, 4], state_fp64=fp64, n_groups=1, collide_mode=0)
        B = dsmc_gpu.Ensemble(runs, [2, 4], state_fp64=fp64, n_groups=1, collide_mode=mode)
        A.step(4)
        B.step(4)
        torch.cuda.synchronize()
        for r in range(len(runs)):
            np.testing.assert_array_equal(A.state(r), B.state(r))
            np.testing.assert_array_equal(A.cell_state(r)["ncoll"], B.cell_state(r)["ncoll"])
        for k in range(2):
            np.testing.assert_array_equal(A.accum(k), B.accum(k))


def test_capacity_overflow_is_reported(dsmc_gpu):
    rs = replace(W.channel_run(nx=32, ny=8, lx=2.0, ly=0.5, ppc_inf=40.0, seed=3), capacity=2000)
    E = dsmc_gpu.Ensemble([rs], [], state_fp64=False)
    E.step(50)          # enqueues fine; the device latches the overflow
    with pytest.raises(dsmc_gpu.DsmcError) as e:
        E.sync()
    assert e.value.status == -3
    with pytest.raises(dsmc_gpu.DsmcError) as e:
        E.step(1)
    assert e.value.status == -3
    assert "slots" in dsmc_gpu.dsmc_last_error(E.ctx)


def test_argument_errors(dsmc_gpu):
    E = dsmc_gpu.Ensemble(W.plain_box().runs, [2], state_fp64=True)
    with pytest.raises(dsmc_gpu.DsmcError) as e:
        E.sample(0)                  # no step yet: state not cell-sorted
    assert e.value.status == -5
    with pytest.raises(dsmc_gpu.DsmcError) as e:
        E.sample(3)
    assert e.value.status == -1
    with pytest.raises(dsmc_gpu.DsmcError) as e:
        dsmc_gpu.dsmc_read_moments(E.ctx, 0, 12345, 1024)
    assert e.value.status == -1
    E.step(2)
    m, se = E.moments(0)
    assert abs(np.nansum(m[:, 0]) - 20_000) < 1e-9
    assert np.all(np.isnan(se))      # one group: no batch-means error


def test_manual_sample_equals_scheduled_sample(dsmc_gpu):
    runs = _small_channel_runs(2)
    A = dsmc_gpu.Ensemble(runs, [4], state_fp64=True, n_groups=2)
    B = dsmc_gpu.Ensemble(runs, [-1], state_fp64=True, n_groups=2)
    A.step(4)
    B.step(4)
    B.sample(0)
    np.testing.assert_allclose(A.accum(0), B.accum(0), rtol=1e-13, atol=1e-13)


def test_fp32_tracks_fp64_statistically(dsmc_gpu):
    """Same Philox streams, FP32 vs FP64 state: the trajectories separate
    (chaos), but conserved totals and collision rates agree."""
    wl = W.box(20_000, 8, 30, 30, seed=41)
    E32 = dsmc_gpu.Ensemble(wl.runs, [30], state_fp64=False, n_groups=8)
    E64 = dsmc_gpu.Ensemble(wl.runs, [30], state_fp64=True, n_groups=8)
    e0 = [float((E64.state(r)[3:] ** 2).sum()) for r in range(8)]
    E32.step(30)
    E64.step(30)
    for r in range(8):
        s32, s64 = E32.state(r), E64.state(r)
        assert s32.shape == s64.shape == (6, 20_000)
        assert abs((s32[3:] ** 2).sum() - e0[r]) < 1e-4 * e0[r]
        assert abs((s64[3:] ** 2).sum() - e0[r]) < 1e-12 * e0[r]
    n32 = sum(int(E32.cell_state(r)["ncoll"].sum()) for r in range(8))
    n64 = sum(int(E64.cell_state(r)["ncoll"].sum()) for r in range(8))
    assert abs(n32 - n64) < 5 * np.sqrt(n64)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("fp64", [True, False])
def test_state_round_trip(dsmc_gpu, dim, fp64):
    """A replaced state reads back component for component (the device keeps
    (x, y, u, v) records plus w, or the (z, w) pair in 3-D), also in a second
    run of the batch, and stepping from it matches stepping from the same
    state in a fresh context."""
    if dim == 2:
        runs = [W.box(3000, 1, 1, 1, seed=51, grid=(8, 8)).runs[0],
                replace(W.box(2000, 1, 1, 1, seed=52, grid=(6, 5)).runs[0], run_id=1, ensemble=1)]
    else:
        runs = [W.box3d(4000, 1, grid=(5, 4, 3), seed=53).runs[0],
                replace(W.box3d(3000, 1, grid=(4, 4, 4), seed=54).runs[0], run_id=1, ensemble=1)]
    rng = np.random.default_rng(7)
    E = dsmc_gpu.Ensemble(runs, [], state_fp64=fp64)
    n = 1500
    st = np.empty((6, n))
    st[0] = rng.random(n)
    st[1] = rng.random(n)
    st[2] = rng.random(n) if dim == 3 else 0.0
    st[3:] = rng.normal(size=(3, n))
    if not fp64:
        st = st.astype(np.float32).astype(np.float64)
    E.set_state(1, st)
    np.testing.assert_array_equal(E.state(1), st)
    E.step(2)
    F = dsmc_gpu.Ensemble(runs, [], state_fp64=fp64)
    F.set_state(1, st)
    F.step(2)
    np.testing.assert_array_equal(E.state(1), F.state(1))
    np.testing.assert_array_equal(E.state(0), F.state(0))


def _mixed_mode_runs():
    """Runs whose cells take each Interaction mode (a lane, a wavefront and a
    block per cell: ~30, ~150 and ~400 particles per cell), plus a channel
    with inflow, in one batch."""
    lane = replace(W.box(64 * 30, 1, 1, 1, seed=71, grid=(8, 8)).runs[0], run_id=0, ensemble=0)
    wave = replace(W.box(64 * 150, 1, 1, 1, seed=72, grid=(8, 8)).runs[0], run_id=1, ensemble=1)
    cell = replace(W.box(64 * 400, 1, 1, 1, seed=73, grid=(8, 8)).runs[0], run_id=2, ensemble=2)
    ch = replace(W.channel_run(nx=32, ny=8, lx=2.0, ly=0.5, ppc_inf=30.0, run_id=3, seed=74), ensemble=3)
    lane2 = replace(lane, run_id=4, ensemble=4)
    return [lane, wave, cell, ch, lane2]


@pytest.mark.parametrize("fp64", [False, True])
@pytest.mark.parametrize("sched,streams", [(1, 1), (2, 1), (1, 2), (2, 2)])
def test_interaction_scheduling_gives_identical_results(dsmc_gpu, fp64, sched, streams):
    """Persistent Interaction grids drawing items from a device queue shared
    by all runs (1) or from per-run queues (2) compute every item exactly as
    the grid with one item per workgroup does (0); with one workgroup per
    grid (fewer units than runs with items) every run is still served."""
    runs = _mixed_mode_runs()
    A = dsmc_gpu.Ensemble(runs, [3], state_fp64=fp64, n_groups=1, sched=0)
    B = dsmc_gpu.Ensemble(runs, [3], state_fp64=fp64, n_groups=1, sched=sched, n_streams=streams,
                          use_graph=True)
    C = dsmc_gpu.Ensemble(runs, [3], state_fp64=fp64, n_groups=1, sched=sched, sched_blocks=7)
    A2 = dsmc_gpu.Ensemble(runs, [3], state_fp64=fp64, n_groups=1, sched=0, collide_mode=2)
    D = dsmc_gpu.Ensemble(runs, [3], state_fp64=fp64, n_groups=1, sched=sched, sched_blocks=1,
                          collide_mode=2)
    for E in (A, B, C, A2, D):
        E.step(4)
    for r in range(len(runs)):
        for X, E in ((A, B), (A, C), (A2, D)):
            np.testing.assert_array_equal(X.state(r), E.state(r))
            np.testing.assert_array_equal(X.cell_state(r)["ncoll"], E.cell_state(r)["ncoll"])
    for e in range(len(runs)):
        for X, E in ((A, B), (A, C), (A, D), (A2, D)):
            np.testing.assert_array_equal(X.accum(0, ensemble=e), E.accum(0, ensemble=e))


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_subcell_interaction_modes_give_identical_results(dsmc_gpu, mode):
    """With 2 x 2 sub-cells the FP32 lane, block (the pipelined FP32 kernel)
    and wavefront kernels, on the hardware grid and on the persistent queue,
    make the same selections in the same order: identical results."""
    runs = [replace(r, subcells=2) for r in _mixed_mode_runs()]
    A = dsmc_gpu.Ensemble(runs, [3], state_fp64=False, n_groups=1, collide_mode=0)
    B = dsmc_gpu.Ensemble(runs, [3], state_fp64=False, n_groups=1, collide_mode=mode)
    C = dsmc_gpu.Ensemble(runs, [3], state_fp64=False, n_groups=1, collide_mode=mode, sched=1,
                          use_graph=True)
    for E in (A, B, C):
        E.step(4)
    for r in range(len(runs)):
        for E in (B, C):
            np.testing.assert_array_equal(A.state(r), E.state(r))
            np.testing.assert_array_equal(A.cell_state(r)["ncoll"], E.cell_state(r)["ncoll"])
    for e in range(len(runs)):
        for E in (B, C):
            np.testing.assert_array_equal(A.accum(0, ensemble=e), E.accum(0, ensemble=e))
    assert sum(int(A.cell_state(r)["ncoll"].sum()) for r in range(len(runs))) > 1000


@pytest.mark.parametrize("mode", [1, 2, 3])
def test_running_mean_count_modes_give_identical_results(dsmc_gpu, mode):
    """With Bird's N * Nbar / 2 count the FP32 lane, block and wavefront
    kernels still make the same selections: identical states, collision
    counts, running means and sample sums."""
    runs = [replace(r, ntc_nbar_alpha=0.2) for r in _mixed_mode_runs()]
    A = dsmc_gpu.Ensemble(runs, [3], state_fp64=False, n_groups=1, collide_mode=0)
    B = dsmc_gpu.Ensemble(runs, [3], state_fp64=False, n_groups=1, collide_mode=mode, sched=1)
    for E in (A, B):
        E.step(4)
    for r in range(len(runs)):
        np.testing.assert_array_equal(A.state(r), B.state(r))
        for k in ("ncoll", "nbar", "rem"):
            np.testing.assert_array_equal(A.cell_state(r)[k], B.cell_state(r)[k])
    for e in range(len(runs)):
        np.testing.assert_array_equal(A.accum(0, ensemble=e), B.accum(0, ensemble=e))


def test_tune_cache_returns_the_stored_result(dsmc_gpu, tmp_path):
    """The first autotune of a problem times the candidates and appends its
    pick to the cache file; the second finds it there (no timing); another
    problem (other seed) is not taken from it."""
    runs = _small_channel_runs(4)
    path = str(tmp_path / "tune.txt")
    a = dsmc_gpu.Ensemble.autotune(runs, [3], n_steps=1, tune_cache=path)
    b = dsmc_gpu.Ensemble.autotune(runs, [3], n_steps=1, tune_cache=path)
    assert not a["from_cache"] and b["from_cache"]
    for k in ("tile_chunks", "collide_mode", "n_streams", "sched", "sched_blocks"):
        assert a[k] == b[k]
    assert abs(a["ms_per_step"] - b["ms_per_step"]) < 1e-3 * a["ms_per_step"]
    c = dsmc_gpu.Ensemble.autotune(_small_channel_runs(4, seed=32), [3], n_steps=1, tune_cache=path)
    assert not c["from_cache"]
    assert len(open(path).read().splitlines()) == 2
    # a later line for the same problem with settings the library refuses
    # (tile_chunks 3) is no answer: the problem is timed again
    key = " ".join(open(path).read().splitlines()[0].split()[:2])
    with open(path, "a") as f:
        f.write(f"{key} 3 0 1 0 0 0.5\n")
    d = dsmc_gpu.Ensemble.autotune(runs, [3], n_steps=1, tune_cache=path)
    assert not d["from_cache"] and d["tile_chunks"] in (64, 128, 256)


def test_autotune_from_a_checkpoint(dsmc_gpu, tmp_path):
    """The autotuner restores every candidate from a checkpoint (a filled
    unsteady state, not the start) and caches the pick under that state's
    step; its settings then continue the checkpointed run bit for bit."""
    runs = [replace(r, n_init=0) for r in _small_channel_runs(4)]     # from vacuum
    E = dsmc_gpu.Ensemble(runs, [60], state_fp64=False, n_groups=2)
    E.step(40)
    ck = E.checkpoint()
    path = str(tmp_path / "tune.txt")
    a = dsmc_gpu.Ensemble.autotune(runs, [60], n_groups=2, n_steps=1, tune_cache=path, start=ck)
    b = dsmc_gpu.Ensemble.autotune(runs, [60], n_groups=2, n_steps=1, tune_cache=path, start=ck)
    c = dsmc_gpu.Ensemble.autotune(runs, [60], n_groups=2, n_steps=1, tune_cache=path)
    assert not a["from_cache"] and b["from_cache"] and not c["from_cache"]
    kw = {k: a[k] for k in ("tile_chunks", "collide_mode", "n_streams", "sched", "sched_blocks")}
    F = dsmc_gpu.Ensemble(runs, [60], state_fp64=False, n_groups=2, **kw)
    F.restore(ck)
    E.step(25)
    F.step(25)
    for r in range(len(runs)):
        np.testing.assert_array_equal(E.state(r), F.state(r))
    np.testing.assert_array_equal(E.accum(0), F.accum(0))
    # a checkpoint of another problem is refused
    with pytest.raises(dsmc_gpu.DsmcError) as e:
        dsmc_gpu.Ensemble.autotune(runs, [60], n_groups=3, n_steps=1, start=ck)
    assert e.value.status == -1


def test_forced_block_mode_beyond_one_launch(dsmc_gpu):
    """3000 x 3000 cells with the block-per-cell mode forced: 9M cell items
    are more workgroups than one launch takes (2^23), so the Interaction
    kernel goes out as two launches over consecutive items, eagerly and in a
    graph; the run equals the lane-per-cell mode's, sample sums included."""
    import torch
    rs = replace(W.box(1_000_000, 1, 1, 1, seed=38, grid=(3000, 3000)).runs[0], run_id=0)
    for graph in (False, True):
        A = dsmc_gpu.Ensemble([rs], [2], state_fp64=False, n_groups=1, collide_mode=1, use_graph=graph)
        B = dsmc_gpu.Ensemble([rs], [2], state_fp64=False, n_groups=1, collide_mode=2, use_graph=graph)
        A.step(2)
        B.step(2)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(A.state(0), B.state(0))
        np.testing.assert_array_equal(A.cell_state(0)["ncoll"], B.cell_state(0)["ncoll"])
        np.testing.assert_array_equal(A.accum(0), B.accum(0))
        A.close()
        B.close()

