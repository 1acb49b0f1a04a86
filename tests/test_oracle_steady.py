"""Pins of the oracle's sampling windows -- the steady-flow variant: a slot
averages the snapshots of a time window (an averaging time much longer than
dt once the flow is steady, Sec. 1.1) on top of the average over the runs
(end of Sec. 3).  Pinned against exact conservation sums, against the
definition (a window equals the sum of its single snapshots), and against the
closed form of a collisionless inflow."""
import math
from dataclasses import replace

import numpy as np
import pytest
from scipy import special

import workloads as W


def test_window_sums_in_a_closed_box_are_exact(oracle_lib):
    """Specular box with collisions: every snapshot holds all particles and the
    same energy (conserved to rounding), so a window of W snapshots sums to
    exactly W times N per run, W times the energy, and n averages to N/nc."""
    wl = W.box(3000, 4, 40, 20, seed=11, grid=(8, 8), state_fp64=True, n_groups=2)
    wl = replace(wl, sample_steps=[20, 40], window_steps=5, window_stride=3)
    acc, st = oracle_lib.ensemble(wl, n_threads=2)
    assert st["n_snap"] == [5, 5]
    e0 = 0.0
    for rs in wl.runs:
        O = oracle_lib.OracleRun(rs)
        s = O.state()
        e0 += float(np.sum(s[3:] ** 2))
    for k in range(2):
        tot = acc[k].sum(axis=(0, 1))
        assert tot[0] == 5 * 4 * 3000
        np.testing.assert_allclose(tot[4] + tot[5] + tot[6], 5 * e0, rtol=1e-12)
        m = oracle_lib.moments(acc[k].sum(axis=0), n_runs=4, n_snap=st["n_snap"][k])
        assert math.isclose(float(np.sum(m[:, 0])), 3000.0, rel_tol=1e-13)


def test_window_is_the_sum_of_its_snapshots(oracle_lib):
    """By definition a window slot is the sum of single-snapshot slots at its
    steps (same runs, same streams): compare both schedules bit for bit up to
    the order of additions."""
    runs = [replace(W.channel_run(nx=24, ny=6, lx=1.5, ly=0.5, mach=2.0, ppc_inf=25.0,
                                  capacity_factor=3.0, run_id=r, seed=13)) for r in range(3)]
    wl = W.Workload("win", runs, 30, [17, 30], 1, state_fp64=True, window_steps=4, window_stride=2)
    acc_w, st = oracle_lib.ensemble(wl, n_threads=1)
    assert st["n_snap"] == [4, 4]
    single = [11, 13, 15, 17, 24, 26, 28, 30]
    acc_s, st1 = oracle_lib.ensemble(replace(wl, sample_steps=single, window_steps=1), n_threads=1)
    assert st1["n_snap"] == [1] * 8
    np.testing.assert_allclose(acc_w[0], acc_s[:4].sum(axis=0), rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(acc_w[1], acc_s[4:].sum(axis=0), rtol=1e-13, atol=1e-12)


def test_window_clipped_at_the_first_step_and_overlap_rejected(oracle_lib):
    wl = W.box(500, 1, 12, 6, seed=2, grid=(4, 4), state_fp64=True, n_groups=1)
    acc, st = oracle_lib.ensemble(replace(wl, sample_steps=[3, 12], window_steps=5,
                                          window_stride=1))
    assert st["n_snap"] == [3, 5]                      # steps 1..3 and 8..12
    assert acc[0].sum(axis=(0, 1))[0] == 3 * 500
    with pytest.raises(RuntimeError):
        oracle_lib.ensemble(replace(wl, sample_steps=[6, 8], window_steps=3, window_stride=1))


def _fm_sums(x0, x1, t, U, T):
    """Expected number and x-momentum (per unit inflow density and unit
    cross-section) in [x0, x1] at time t after a drifting Maxwellian (1-D
    marginal N(U, T)) starts flowing in through x = 0 with no collisions: a
    particle of speed u entered at a uniform time and is found at x < u t, so
    n(x, t) = 1/2 erfc((x/t - U)/sqrt(2T)) and n u_x(x, t) =
    U n(x, t) + sqrt(T/2pi) exp(-(x/t - U)^2/(2T))."""
    from scipy import integrate
    sg = math.sqrt(T)
    n = integrate.quad(lambda x: 0.5 * special.erfc((x / t - U) / (sg * math.sqrt(2))), x0, x1)[0]
    nu = integrate.quad(lambda x: U * 0.5 * special.erfc((x / t - U) / (sg * math.sqrt(2)))
                        + sg / math.sqrt(2 * math.pi) * math.exp(-(x / t - U) ** 2 / (2 * T)),
                        x0, x1)[0]
    return n, nu


def test_windowed_collisionless_inflow_matches_closed_form(oracle_lib):
    """sigma = 0, empty start: the window sums of N and of u per cell against
    the closed form summed over the window's snapshot times, gated with
    batch-means errors over 32 one-run groups."""
    nx, ny, lx, ly = 40, 2, 2.0, 0.1
    runs = [replace(W.channel_run(nx=nx, ny=ny, lx=lx, ly=ly, mach=1.0, ppc_inf=40.0,
                                  capacity_factor=3.0, run_id=r, seed=91),
                    fnum_sigma=0.0, face_bc=("inflow", "outflow", "specular", "specular",
                                             "specular", "specular"))
            for r in range(32)]
    Wn, q, S = 10, 4, 100
    wl = W.Workload("fm_window", runs, S, [S], 32, window_steps=Wn, window_stride=q)
    acc, st = oracle_lib.ensemble(wl, n_threads=8)
    assert st["n_snap"] == [Wn]
    rs = runs[0]
    dx = lx / nx
    U, T = rs.inflow_U, rs.inflow_T
    times = [(S - j * q) * rs.dt for j in range(Wn)]
    per_group = acc[0].reshape(32, ny, nx, 7).sum(axis=1)           # [group][x cell][field]
    for f in (0, 1):
        z = []
        for i in range(nx):
            e = sum(_fm_sums(i * dx, (i + 1) * dx, t, U, T)[f] for t in times) * rs.inflow_n * ly
            g = per_group[:, i, f]
            se = g.std(ddof=1) / math.sqrt(len(g))
            if e * 32 < 50:       # cells the front has hardly reached
                continue
            z.append((g.mean() - e) / se)
        z = np.array(z)
        assert len(z) > 20
        assert np.max(np.abs(z)) < 4.5, (f, z)
        assert abs(np.mean(z)) < 3.0 / math.sqrt(len(z)) + 0.35, (f, z)
