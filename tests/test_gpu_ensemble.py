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
    launch: each run's sampled density profile agrees with the oracle's
    ensemble of the same run spec (disjoint seeds), integrated over columns."""
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
    for r, rs in enumerate(wl.runs):
        ag = E.accum(0, ensemble=r)                                    # [reps][cell][7]
        sub = W.Workload("u", ora_runs[r * reps:(r + 1) * reps], wl.n_steps, wl.sample_steps, reps)
        ao, _ = oracle_lib.ensemble(sub, n_threads=16)
        cols_g = ag[..., 0].reshape(reps, rs.ny, rs.nx).sum(axis=1)   # per run, per column
        cols_o = ao[0, ..., 0].reshape(reps, rs.ny, rs.nx).sum(axis=1)
        d = cols_g.mean(0) - cols_o.mean(0)
        se = np.sqrt(cols_g.var(0, ddof=1) / reps + cols_o.var(0, ddof=1) / reps)
        ok = se > 0
        z = d[ok] / se[ok]
        assert np.max(np.abs(z)) < 5.0, (r, z)
        assert np.mean(np.abs(z) > 3) < 0.05, (r, z)
