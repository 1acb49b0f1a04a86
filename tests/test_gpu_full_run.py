"""The benchmark workload run to its end: 512 runs x 1M particles, 1000
steps, every one of its 50 sample slots (every 20 steps), FP32 state, FP64
accumulators, HIP-graph replay.  The box is at equilibrium from the start
(uniform Maxwellian fill, specular walls), so at every sample time each
cell's density, velocity and temperature must be the exact equilibrium
values within the returned batch-means standard errors: the |t| > 3 rate at
Student-t's (31 degrees of freedom) over all slots, no bias per slot, and
every cell within 1 % of the exact density and temperature."""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

N_RUNS, N_PER = 512, 1_000_000


def test_every_sample_of_the_full_run_is_at_equilibrium(dsmc_gpu):
    import torch
    wl = W.ensemble_box(n_runs=N_RUNS, n_per_run=N_PER, n_steps=1000, sample_every=20, seed=11)
    assert len(wl.sample_steps) == 50
    E = dsmc_gpu.Ensemble.from_workload(wl, use_graph=True)
    e0 = sum(float((E.state(r)[3:] ** 2).sum()) for r in (0, 255, 511))
    for _ in range(10):
        E.step(100)
        E.sync()
    rs = wl.runs[0]
    n_exact = N_PER / rs.n_cells
    counts = E.counts()
    assert np.all(counts[:, 0] == N_PER)
    assert np.all(E.sample_counts() == 1)
    e1 = sum(float((E.state(r)[3:] ** 2).sum()) for r in (0, 255, 511))
    assert abs(e1 - e0) < 1e-4 * e0           # specular walls and collisions conserve energy
    zs = []
    for k in range(50):
        m, se = E.moments(k)
        tot = E.accum(k).sum(axis=(0, 1))
        assert tot[0] == N_RUNS * N_PER
        u_all = tot[1:4] / tot[0]
        T_all = ((tot[4] + tot[5] + tot[6]) / tot[0] - float(u_all @ u_all)) / 3.0
        assert np.all(np.abs(m[:, 0] / n_exact - 1) < 0.01), k
        assert np.all(np.abs(m[:, 4] / T_all - 1) < 0.01), k
        z = (m[:, [0, 1, 2, 4]] - np.array([n_exact, 0.0, 0.0, T_all])) / se[:, [0, 1, 2, 4]]
        assert np.all(np.isfinite(z)), k
        for f in range(4):
            assert abs(z[:, f].mean()) <= 4 / math.sqrt(z.shape[0]) + 0.05, (k, f, z[:, f].mean())
        zs.append(z)
    z = np.concatenate(zs)
    M = z.size
    frac = np.mean(np.abs(z) > 3)
    assert frac <= 0.0053 + 6 * math.sqrt(0.0053 / M), frac
    assert np.max(np.abs(z)) < 7.5, np.max(np.abs(z))
    E.close()
    del E
    torch.cuda.empty_cache()
