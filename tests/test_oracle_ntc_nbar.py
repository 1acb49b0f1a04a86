"""Pins of the oracle's N * Nbar / 2 selection count (the NTC variant of
Bird, whose method the paper's collision step follows, Sec. 1.1): the count
of selections in a cell is M = N Nbar / 2 * Fnum sigma_ref dt / V_c *
(sigma c_r)_max + remainder, with Nbar a running mean of the cell's count,
moved towards this step's N by the weight alpha before the count and started
at the expected count of the initial fill.  alpha = 1 makes Nbar = N."""
import math
from dataclasses import replace

import numpy as np
import pytest

import workloads as W


def _counts(R):
    """Particles per cell after the last Indexing."""
    cl = R.cells()
    start = cl["start"]
    S = R.info()["nbin"] // R.info()["nc"]
    return np.diff(start[: R.info()["nbin"] + 1][::S]).astype(np.float64)


def test_running_mean_starts_at_the_fill_and_follows_the_counts(oracle_lib):
    rs = replace(W.plain_box().runs[0], ntc_nbar_alpha=0.25)
    R = oracle_lib.OracleRun(rs)
    nb = R.cell_state()["nbar"]
    np.testing.assert_array_equal(nb, np.full(rs.n_cells, rs.n_init / rs.n_cells))
    for _ in range(4):
        R.step()
        N = _counts(R)
        nb = nb + 0.25 * (N - nb)
        np.testing.assert_array_equal(R.cell_state()["nbar"], nb)


def test_zero_weight_keeps_the_plain_count(oracle_lib):
    """alpha = 0 is the N(N-1)/2 count: the running mean is never touched and
    the run is the pinned plain method's."""
    base = W.plain_box().runs[0]
    a = oracle_lib.OracleRun(base)
    b = oracle_lib.OracleRun(replace(base, ntc_nbar_alpha=0.0))
    a.step(3)
    b.step(3)
    np.testing.assert_array_equal(a.state(), b.state())
    np.testing.assert_array_equal(b.cell_state()["nbar"], np.full(base.n_cells, base.n_init / base.n_cells))


def _rate(oracle_lib, rs, burn=20, steps=100):
    R = oracle_lib.OracleRun(rs)
    c = R.state()[3:]
    T = ((c - c.mean(axis=1, keepdims=True)) ** 2).sum() / (3 * c.shape[1])
    tot = 0
    for s in range(burn + steps):
        R.step()
        if s >= burn:
            tot += R.info()["ncoll"]
    per_step = tot / steps
    return per_step, math.sqrt(per_step / steps), T


def test_slow_running_mean_keeps_the_equilibrium_collision_frequency(oracle_lib):
    """With the cell counts of a uniform gas multinomial, E[N_c] * N / cells
    summed over the cells is N^2 / cells against N(N-1) / cells for the pair
    count: the hard-sphere rate 1/2 N^2 Fnum sigma <c_r> dt / V."""
    rs = replace(W.plain_box().runs[0], ntc_nbar_alpha=0.02)
    per_step, se, T = _rate(oracle_lib, rs)
    N = rs.n_init
    expect = 0.5 * N * N * rs.fnum_sigma * 4 * math.sqrt(T / math.pi) * rs.dt / (rs.lx * rs.ly)
    assert abs(per_step - expect) < 4 * se + 0.002 * expect, (per_step, expect)


def test_unit_weight_counts_n_squared(oracle_lib):
    """alpha = 1: Nbar = N, so the count follows E[N_c^2] = N(N-1)/cells^2 +
    N/cells for multinomial cell counts, a rate higher than the pair count's
    by 1 + cells/(N-1) (5 % at 20 particles per cell)."""
    rs = replace(W.plain_box().runs[0], ntc_nbar_alpha=1.0)
    per_step, se, T = _rate(oracle_lib, rs)
    N, nc = rs.n_init, rs.n_cells
    pair = 0.5 * N * (N - 1) * rs.fnum_sigma * 4 * math.sqrt(T / math.pi) * rs.dt / (rs.lx * rs.ly)
    expect = pair * (1 + nc / (N - 1))
    assert abs(per_step - expect) < 4 * se + 0.002 * expect, (per_step, expect, pair)
    assert per_step > pair * 1.03


@pytest.mark.parametrize("alpha", [-0.1, 1.5, float("nan")])
def test_weights_outside_0_1_are_refused(oracle_lib, alpha):
    with pytest.raises(ValueError):
        oracle_lib.OracleRun(replace(W.plain_box().runs[0], ntc_nbar_alpha=alpha))
