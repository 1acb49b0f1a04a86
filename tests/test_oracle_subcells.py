"""Pins of the oracle's sub-cell partner selection (a refinement of the
collision-partner choice of the DSMC method the paper builds on, Sec. 1.1
and its reference to Bird): the first partner is drawn uniformly from the
cell, the second from the other particles of the first one's sub-cell when it
holds two or more, else from the cell.  The NTC count stays the cell's."""
import math
from dataclasses import replace

import numpy as np
import pytest
from scipy import stats

import workloads as W


def _box(k, dim=2, seed=31, n=6000, grid=(8, 8)):
    if dim == 2:
        rs = W.box(n, 1, 10, 5, seed=seed, grid=grid).runs[0]
    else:
        rs = W.box3d(n, 1, grid=(4, 4, 3), seed=seed).runs[0]
    return replace(rs, subcells=k)


def test_one_subcell_is_the_plain_method(oracle_lib):
    a = oracle_lib.OracleRun(_box(1))
    b = oracle_lib.OracleRun(replace(_box(1), subcells=0))
    a.step(3)
    b.step(3)
    np.testing.assert_array_equal(a.state(), b.state())
    np.testing.assert_array_equal(a.cells()["lcr"], b.cells()["lcr"])


@pytest.mark.parametrize("k,dim", [(2, 2), (3, 2), (2, 3)])
def test_subcell_bins_are_the_floor_of_the_sub_grid(oracle_lib, k, dim):
    """Enumeration with sub-cells: bin = cell * S + sub-cell, from the floor of
    the position on the sub-cell grid; LCR is the stable sort by bin."""
    rs = _box(k, dim)
    R = oracle_lib.OracleRun(rs)
    R.step()
    st, cl = R.state(), R.cells()
    info = R.info()
    S = k ** dim
    assert info["nbin"] == rs.n_cells * S
    n = [rs.nx, rs.ny, rs.nz]
    L = [rs.lx, rs.ly, rs.lz]
    f = [np.clip(np.floor(st[a] * ((n[a] * k) / L[a])), 0, n[a] * k - 1).astype(np.int64) if a < dim
         else np.zeros(st.shape[1], np.int64) for a in range(3)]
    cell = ((f[2] // k) * rs.ny + f[1] // k) * rs.nx + f[0] // k
    sub = ((f[2] % k) * k + f[1] % k) * k + f[0] % k
    bins = cell * S + sub
    # the state is cell-sorted: slot p holds particle lcr[p] of the step; its
    # bin is cl["cell"][lcr[p]]
    np.testing.assert_array_equal(bins, cl["cell"][cl["lcr"]])
    np.testing.assert_array_equal(cl["lcr"], np.argsort(cl["cell"], kind="stable"))


def test_subcell_first_selection_probabilities_brute_force(oracle_lib):
    """N = 7 particles in sub-cells of 3, 1, 0 and 3: P(first selection =
    ordered pair (i, j) and accepted) = 1/N * 1/(n_s - 1) * g_ij/gmax for j in
    i's sub-cell of n_s >= 2 particles, 1/N * 1/(N - 1) * g_ij/gmax for any
    j != i when i is alone in its sub-cell."""
    rng = np.random.default_rng(7)
    N = 7
    off = [0, 3, 4, 4, 7]
    sub_of = [0, 0, 0, 1, 3, 3, 3]
    vel = rng.normal(size=(3, N))
    gmax = 6.0
    rs = replace(W.plain_box().runs[0], fnum_sigma=1.0, subcells=2)
    trials = 40000
    counts = {}
    for step in range(1, trials + 1):
        out = oracle_lib.collide_cell(rs, step=step, cell=5, vel=vel, gmax=gmax, rem=0.999999, trace_cap=1,
                                      sub_off=off)
        i, j, acc = (int(x) for x in out["trace"][0])
        counts[(i, j, acc)] = counts.get((i, j, acc), 0) + 1
    obs, exp = [], []
    for i in range(N):
        ns = off[sub_of[i] + 1] - off[sub_of[i]]
        for j in range(N):
            if j == i:
                continue
            if ns >= 2:
                if sub_of[j] != sub_of[i]:
                    assert counts.get((i, j, 0), 0) + counts.get((i, j, 1), 0) == 0
                    continue
                p = 1.0 / N / (ns - 1)
            else:
                p = 1.0 / N / (N - 1)
            g = np.linalg.norm(vel[:, i] - vel[:, j])
            obs += [counts.get((i, j, 1), 0), counts.get((i, j, 0), 0)]
            exp += [p * g / gmax * trials, p * (1 - g / gmax) * trials]
    assert sum(obs) == trials
    assert stats.chisquare(obs, exp).pvalue > 1e-4


@pytest.mark.parametrize("k", [1, 2, 3])
def test_subcells_shorten_the_partner_separation(oracle_lib, k):
    """Particles uniform in one square cell of side a, 1200 of them, sorted
    into k x k sub-cells: the selected pairs lie on average 0.5214 a/k apart
    (the mean distance of two uniform points in a square is
    (2 + sqrt 2 + 5 ln(1 + sqrt 2))/15 of its side)."""
    rng = np.random.default_rng(11 + k)
    a = 1.0
    n = 1200
    x, y = rng.random(n) * a, rng.random(n) * a
    sub = (np.floor(y * k / a) * k + np.floor(x * k / a)).astype(int)
    order = np.argsort(sub, kind="stable")
    x, y, sub = x[order], y[order], sub[order]
    off = np.searchsorted(sub, np.arange(k * k + 1))
    vel = rng.normal(size=(3, n))
    rs = replace(W.plain_box().runs[0], fnum_sigma=0.0, subcells=k)
    nsel = 6000
    out = oracle_lib.collide_cell(rs, step=3, cell=0, vel=vel, gmax=10.0, rem=float(nsel), trace_cap=nsel,
                                  sub_off=off if k > 1 else None)
    tr = out["trace"]
    assert len(tr) == nsel
    d = np.hypot(x[tr[:, 0]] - x[tr[:, 1]], y[tr[:, 0]] - y[tr[:, 1]])
    mean_sq = (2 + math.sqrt(2) + 5 * math.log(1 + math.sqrt(2))) / 15
    expect = mean_sq * a / k
    assert abs(d.mean() - expect) < 5 * d.std() / math.sqrt(nsel), (d.mean(), expect)


def test_subcells_keep_the_equilibrium_collision_frequency(oracle_lib):
    """In equilibrium velocities are independent of positions, so sub-cell
    partners leave the rate 1/2 N(N-1) Fnum sigma <c_r> dt / V unchanged."""
    wl = W.plain_box()
    rs = replace(wl.runs[0], subcells=2)
    R = oracle_lib.OracleRun(rs)
    st = R.state()
    c = st[3:]
    T = ((c - c.mean(axis=1, keepdims=True)) ** 2).sum() / (3 * c.shape[1])
    N = rs.n_init
    expect = 0.5 * N * (N - 1) * rs.fnum_sigma * 4 * math.sqrt(T / math.pi) * rs.dt / (rs.lx * rs.ly)
    tot = 0
    e0 = float((c ** 2).sum())
    for s in range(120):
        R.step()
        if s >= 20:
            tot += R.info()["ncoll"]
    per_step = tot / 100
    se = math.sqrt(per_step / 100)
    assert abs(per_step - expect) < 4 * se + 0.002 * expect, (per_step, expect)
    # energy is conserved by every collision and by the specular walls
    assert abs(float((R.state()[3:] ** 2).sum()) - e0) < 1e-9 * e0


def test_subcells_with_a_body_are_refused(oracle_lib):
    rs = W.body3d(n_runs=1, grid=(20, 10, 10), n_per_run=2000, n_steps=2, n_samples=1).runs[0]
    with pytest.raises(ValueError):
        oracle_lib.OracleRun(replace(rs, subcells=2))
