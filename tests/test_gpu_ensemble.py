"""Ensemble statistics of the batched FP32 path (FP32 particle state, FP64
cross-run accumulators and final division) against the FP64 oracle's own
ensemble and against closed forms.

Sec. 1.1 of the paper: macroparameters of an unsteady flow are averaged over
the particles of a cell and over n statistically independent runs.  Here the
GPU ensemble and the oracle ensemble use disjoint Philox seeds, so they are
independent samples of the same distribution; every (cell, sample time,
field) entry gives z = (GPU - oracle) / sqrt(SE_gpu^2 + SE_oracle^2) with
standard errors from the run-to-run spread.  The gate (3 standard errors):
the fraction of |z| > 3 stays within its normal-theory rate 0.27 % plus
three binomial standard errors, no |z| exceeds 6, and the mean z of each
field stays within 3/sqrt(M) + 0.05.
"""
import math
from dataclasses import replace

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _z_gate(z, label):
    # a zero standard error on both sides with different means is a failure,
    # not a missing entry (entries masked out on purpose are NaN)
    assert not np.any(np.isinf(z)), (label, "zero standard error but different means")
    z = z[np.isfinite(z)]
    M = z.size
    assert M > 200, label
    frac = np.mean(np.abs(z) > 3)
    assert frac <= 0.0027 + 3 * math.sqrt(0.0027 / M) + 0.002, (label, frac, M)
    assert np.max(np.abs(z)) < 6.0, (label, np.max(np.abs(z)))
    return M


def _per_run_moments(acc, fields):
    """acc[k][run][cell][7] (one run per group) -> per-run moments and the
    pooled estimate with its run-to-run standard error."""
    import oracle
    S = acc.sum(axis=1)
    pooled = oracle.moments(S, acc.shape[1])
    per_run = oracle.moments(acc, 1)
    n = acc.shape[1]
    se = np.nanstd(per_run, axis=1, ddof=1) / math.sqrt(n)
    return pooled[..., fields], se[..., fields], per_run[..., 0]


def test_channel_fp32_ensemble_matches_oracle_ensemble(dsmc_gpu, oracle_lib):
    """Impulsively started Mach-2 channel (inflow, diffuse wall at T = 2,
    vacuum outflow, VHS), 64 runs on each side, three sample times."""
    n_runs = 64
    base = W.channel(n_runs=n_runs, nx=32, ny=8, ppc_inf=40.0, n_steps=120, sample_every=40,
                     seed=101, n_groups=n_runs)
    gpu_wl = base
    ora_wl = base.with_seed(202)
    E = dsmc_gpu.Ensemble.from_workload(gpu_wl, state_fp64=False)
    E.step(gpu_wl.n_steps)
    acc_g = np.stack([E.accum(k) for k in range(len(gpu_wl.sample_steps))])
    acc_o, _ = oracle_lib.ensemble(ora_wl, n_threads=16)
    fields = [0, 1, 2, 4]       # n, ux, uy, T
    mg, sg, ng = _per_run_moments(acc_g, fields)
    mo, so, no = _per_run_moments(acc_o, fields)
    # normal theory needs a few particles per cell and run on both sides
    ok = (np.nanmean(ng, axis=1) >= 5) & (np.nanmean(no, axis=1) >= 5)
    z = (mg - mo) / np.sqrt(sg ** 2 + so ** 2)
    z = np.where(ok[..., None], z, np.nan)
    M = _z_gate(z, "channel")
    for f in range(len(fields)):
        zf = z[..., f][np.isfinite(z[..., f])]
        assert abs(zf.mean()) <= 3 / math.sqrt(zf.size) + 0.05, (f, zf.mean())
    assert M > 1000
    _library_moments_equal_oracle_division(E, acc_g, n_runs)


def _library_moments_equal_oracle_division(E, acc, n_runs):
    """dsmc_read_moments (FP64 division on the device) element by element
    against the oracle's division of the same sums, values and batch-means
    errors (one group per run here)."""
    import oracle
    for k in range(acc.shape[0]):
        m, se = E.moments(k)
        G = acc.shape[1]
        np.testing.assert_allclose(m, oracle.moments(acc[k].sum(axis=0), n_runs), rtol=1e-12, atol=1e-14,
                                   equal_nan=True)
        per = oracle.moments(acc[k], n_runs // G)
        with np.errstate(invalid="ignore"):
            se_o = np.nanstd(per, axis=0, ddof=1) / math.sqrt(G)
        # cells without particles in some group: NaN on both sides
        se_o = np.where(np.isnan(per).any(axis=0), np.nan, se_o)
        np.testing.assert_allclose(se, se_o, rtol=1e-9, atol=1e-14, equal_nan=True)


def test_channel_fp32_at_122_per_cell_matches_oracle_ensemble(dsmc_gpu, oracle_lib):
    """The channel at its free-stream fill of 122 particles per cell, where
    the auto mode gives each cell a wavefront: 64 runs on each side, three
    sample times, the same 3-standard-error gate, and the library's moments
    equal to the oracle's division of the same sums."""
    n_runs = 64
    base = W.channel(n_runs=n_runs, nx=32, ny=8, ppc_inf=122.0, n_steps=120, sample_every=40,
                     seed=111, n_groups=n_runs)
    E = dsmc_gpu.Ensemble.from_workload(base, state_fp64=False)
    assert E.info()["runs"] == n_runs
    E.step(base.n_steps)
    acc_g = np.stack([E.accum(k) for k in range(len(base.sample_steps))])
    acc_o, _ = oracle_lib.ensemble(base.with_seed(222), n_threads=16)
    fields = [0, 1, 2, 4]
    mg, sg, ng = _per_run_moments(acc_g, fields)
    mo, so, no = _per_run_moments(acc_o, fields)
    ok = (np.nanmean(ng, axis=1) >= 5) & (np.nanmean(no, axis=1) >= 5)
    z = (mg - mo) / np.sqrt(sg ** 2 + so ** 2)
    z = np.where(ok[..., None], z, np.nan)
    M = _z_gate(z, "channel at 122 per cell")
    for f in range(len(fields)):
        zf = z[..., f][np.isfinite(z[..., f])]
        assert abs(zf.mean()) <= 3 / math.sqrt(zf.size) + 0.05, (f, zf.mean())
    assert M > 1000
    # the fill the auto rule saw: cells behind the front hold ~122 per run
    full = mg[-1][..., 0][ok[-1]]
    assert np.nanmax(full) > 100
    _library_moments_equal_oracle_division(E, acc_g, n_runs)


def test_box_fp32_ensemble_equilibrium_closed_form(dsmc_gpu):
    """Equilibrium box: every cell's expected density is N/1024 per run, the
    mean velocity 0 and the temperature the realised one; 128 runs at ~20
    particles per cell, sampled after 20 and 40 steps."""
    wl = W.box(20_000, 128, 40, 20, seed=77, state_fp64=False, n_groups=128)
    E = dsmc_gpu.Ensemble.from_workload(wl)
    T0 = np.mean([(E.state(r)[3:] ** 2).sum() / 60_000 for r in range(128)])
    E.step(40)
    for k in range(2):
        acc = E.accum(k)[None]                  # [1][run][cell][7]
        m, se, _ = _per_run_moments(acc, [0, 1, 2, 4])
        m, se = m[0], se[0]
        exact = np.array([20_000 / 1024, 0.0, 0.0, T0])
        z = (m - exact) / se
        _z_gate(z, f"box sample {k}")
        # energy is conserved exactly in a specular box: the pooled T agrees
        # with the realised initial T to FP32 roundoff
        mom, _ = E.moments(k)
        assert abs(np.nanmean(mom[:, 4]) - T0) < 0.01


def test_uneven_batch_fp32_matches_oracle_runs(dsmc_gpu, oracle_lib):
    """Uneven runs (different grids, counts, HS/VHS, Mach numbers) in one
    launch: each run's per-cell density, velocity and temperature agree with
    the oracle's ensemble of the same run spec (disjoint seeds) within the
    3-standard-error gate."""
    wl = W.uneven(n_runs=4, n_steps=60, n_samples=1, seed=4, count_range=(20e3, 60e3),
                  grids=((32, 32), (64, 32)))
    reps = 24
    gpu_runs, ora_runs = [], []
    for r, rs in enumerate(wl.runs):
        for k in range(reps):
            gpu_runs.append(replace(rs, run_id=1000 * r + k, seed=7, ensemble=r))
            ora_runs.append(replace(rs, run_id=1000 * r + k, seed=8, ensemble=r))
    E = dsmc_gpu.Ensemble(gpu_runs, wl.sample_steps, state_fp64=False, n_groups=reps)
    E.step(wl.n_steps)
    zs = []
    for r, rs in enumerate(wl.runs):
        ag = E.accum(0, ensemble=r)                                    # [reps][cell][7]
        sub = W.Workload("u", ora_runs[r * reps:(r + 1) * reps], wl.n_steps, wl.sample_steps, reps)
        ao, _ = oracle_lib.ensemble(sub, n_threads=16)
        # per cell: n, ux, uy, T with run-to-run standard errors
        mg, sg, ng = _per_run_moments(ag[None], [0, 1, 2, 4])
        mo, so, no = _per_run_moments(ao, [0, 1, 2, 4])
        ok = (np.nanmean(ng, axis=1) >= 5) & (np.nanmean(no, axis=1) >= 5)
        z = (mg - mo) / np.sqrt(sg ** 2 + so ** 2)
        zs.append(np.where(ok[..., None], z, np.nan).ravel())
    z = np.concatenate(zs)
    M = _z_gate(z, "uneven runs, per cell")
    assert M > 1000
