"""Pins of the oracle's voxel obstacle (solid cells with diffuse faces, the
body of the flow-past-a-body problem), against geometry worked out by hand
and against kinetic theory, not against the oracle itself.

- A particle aimed at a solid cell hits the crossed face at the time and
  point of the straight line, leaves it into the fluid and flies on for the
  rest of the step; a path beside the cell is untouched.
- Corner crossings take the lower axis first (x, then y): the three corner
  cases give the face the rule names.
- An all-fluid mask changes nothing, bit for bit.
- The initial fill avoids solid cells and is uniform over the fluid.
- Equilibrium gas at the obstacle's temperature: the number of solid faces hit
  per step is the one-sided Maxwellian flux n sqrt(T / 2 pi) times the
  exposed face area times dt, and the gas temperature does not drift (the
  re-emission distribution is the flux-weighted one).
- Closed box, every wall and the obstacle diffuse at T_w: the gas relaxes to
  uniform density over the fluid, zero mean velocity and T = T_w.
- No particle ever ends a step in a solid cell.
"""
import math
from dataclasses import replace

import numpy as np
import pytest

import workloads as W

def _box3d(n=(8, 8, 8), L=(1.0, 1.0, 1.0), dt=0.01, n_init=0, T=1.0, solid=None, solid_T=1.0,
           wall="specular", wall_T=1.0, fnum_sigma=0.0, capacity=None, run_id=0, seed=11):
    nx, ny, nz = n
    return W.RunSpec(dim=3, nx=nx, ny=ny, nz=nz, lx=L[0], ly=L[1], lz=L[2], dt=dt,
                     fnum_sigma=fnum_sigma, omega=0.5, face_bc=(wall,) * 6, face_T=(wall_T,) * 6,
                     capacity=capacity or max(256, n_init), n_init=n_init, init_T=T,
                     run_id=run_id, seed=seed, solid=solid, solid_T=solid_T)


def _mask(n, cells):
    nx, ny, nz = n
    m = np.zeros((nz, ny, nx), np.uint8)
    for ix, iy, iz in cells:
        m[iz, iy, ix] = 1
    return m


def _one_particle(oracle_lib, rs, pos, vel, step=1):
    O = oracle_lib.OracleRun(rs, init=False)
    st = np.zeros((6, 1))
    st[:3, 0] = pos
    st[3:, 0] = vel
    O.set_state(st)
    O.set_step(step - 1)
    O.step()
    return O, O.state()[:, 0]


def test_face_hit_time_point_and_departure(oracle_lib):
    """Cell size 0.1; solid cell (5, 2, 2).  From x = 0.12 at u = 1 the path
    reaches the plane x = 0.5 at t = 0.38 inside the solid cell's face; the
    particle leaves it with u < 0 for the remaining 0.12 of the step.  A cold
    wall (T = 0.01) keeps the departure short of every other face."""
    n = (10, 4, 4)
    rs = _box3d(n, L=(1.0, 0.4, 0.4), dt=0.5, solid=_mask(n, [(5, 2, 2)]), solid_T=0.01)
    O, p = _one_particle(oracle_lib, rs, (0.12, 0.25, 0.25), (1.0, 0.0, 0.0))
    assert O.solid_hits() == 1
    u, v, w = p[3:]
    assert u < 0
    t_left = 0.5 - 0.38
    np.testing.assert_allclose(p[0], 0.5 + u * t_left, rtol=0, atol=1e-15)
    np.testing.assert_allclose(p[1], 0.25 + v * t_left, rtol=0, atol=1e-15)
    np.testing.assert_allclose(p[2], 0.25 + w * t_left, rtol=0, atol=1e-15)
    # the same path one cell to the side passes the solid cell untouched
    O, p = _one_particle(oracle_lib, rs, (0.12, 0.15, 0.25), (1.0, 0.0, 0.0))
    assert O.solid_hits() == 0
    np.testing.assert_allclose(p[:3], [0.62, 0.15, 0.25], rtol=0, atol=1e-15)
    np.testing.assert_array_equal(p[3:], [1.0, 0.0, 0.0])


def test_face_hit_moving_down_and_in_y(oracle_lib):
    """Approach from +x (u < 0) and along y: the face hit is the solid cell's
    upper x face (x = 0.6) or its lower y face (y = 0.2), left with the
    normal velocity reversed in sign."""
    n = (10, 4, 4)
    rs = _box3d(n, L=(1.0, 0.4, 0.4), dt=0.5, solid=_mask(n, [(5, 2, 2)]), solid_T=0.01)
    O, p = _one_particle(oracle_lib, rs, (0.9, 0.25, 0.25), (-1.0, 0.0, 0.0))
    assert O.solid_hits() == 1 and p[3] > 0
    np.testing.assert_allclose(p[0], 0.6 + p[3] * 0.2, rtol=0, atol=1e-15)
    O, p = _one_particle(oracle_lib, rs, (0.55, 0.05, 0.25), (0.0, 1.0, 0.0))
    assert O.solid_hits() == 1 and p[4] < 0
    np.testing.assert_allclose(p[1], 0.2 + p[4] * 0.35, rtol=0, atol=1e-15)
    np.testing.assert_allclose(p[0], 0.55 + p[3] * 0.35, rtol=0, atol=1e-15)


@pytest.mark.parametrize("solid_cells,hit_axis", [([(4, 1, 0)], 0),   # x neighbour solid: x face
                                                  ([(3, 2, 0)], None),  # only the y neighbour: passes
                                                  ([(4, 2, 0)], 1)])  # diagonal cell: y face of it
def test_corner_crossing_takes_x_first(oracle_lib, solid_cells, hit_axis):
    """Cell size 0.125 (exact); start (0.4375, 0.1875) in cell (3, 1) moving
    (1, 1): both planes x = 0.5 and y = 0.25 are reached at t = 0.0625.  The x
    plane is crossed first, into (4, 1), then the y plane, into (4, 2)."""
    n = (8, 8, 1)
    rs = _box3d(n, L=(1.0, 1.0, 0.125), dt=0.125, solid=_mask(n, solid_cells), solid_T=1e-4)
    O, p = _one_particle(oracle_lib, rs, (0.4375, 0.1875, 0.0625), (1.0, 1.0, 0.0))
    if hit_axis is None:
        assert O.solid_hits() == 0
        np.testing.assert_array_equal(p[:2], [0.5625, 0.3125])
    else:
        assert O.solid_hits() == 1
        assert p[3 + hit_axis] < 0                   # left the crossed face backwards
        other = 1 - hit_axis
        # the hit point is the corner (0.5, 0.25); 0.0625 of the step remains
        np.testing.assert_allclose(p[hit_axis], [0.5, 0.25][hit_axis] + p[3 + hit_axis] * 0.0625,
                                   rtol=0, atol=1e-15)
        np.testing.assert_allclose(p[other], [0.5, 0.25][other] + p[3 + other] * 0.0625,
                                   rtol=0, atol=1e-15)


def test_all_fluid_mask_changes_nothing(oracle_lib):
    base = W.channel_run(nx=32, ny=8, lx=2.0, ly=0.5, ppc_inf=20.0, seed=5)
    base = replace(base, dim=3, nz=4, lz=0.25, n_init=3000, init_U=(2.0, 0.0, 0.0),
                   face_bc=base.face_bc[:4] + ("diffuse", "specular"),
                   face_T=base.face_T[:4] + (1.5, 1.0))
    A = oracle_lib.OracleRun(base)
    B = oracle_lib.OracleRun(replace(base, solid=np.zeros((4, 8, 32), np.uint8), solid_T=2.0))
    A.step(6)
    B.step(6)
    np.testing.assert_array_equal(A.state(), B.state())
    np.testing.assert_array_equal(A.cells()["lcr"], B.cells()["lcr"])


def test_initial_fill_is_uniform_over_the_fluid(oracle_lib):
    n = (12, 12, 12)
    mask = W.sphere_mask(*n, 1.0, 1.0, 1.0, radius=0.3)
    rs = _box3d(n, n_init=60_000, solid=mask)
    O = oracle_lib.OracleRun(rs)
    st = O.state()
    ix = np.minimum((st[0] * 12).astype(int), 11)
    iy = np.minimum((st[1] * 12).astype(int), 11)
    iz = np.minimum((st[2] * 12).astype(int), 11)
    c = (iz * 12 + iy) * 12 + ix
    solid = mask.ravel().astype(bool)
    counts = np.bincount(c, minlength=12 ** 3)
    assert counts[solid].sum() == 0
    fl = counts[~solid]
    e = 60_000 / fl.size
    chi2 = ((fl - e) ** 2 / e).sum()
    dof = fl.size - 1
    assert abs(chi2 - dof) < 5 * math.sqrt(2 * dof), (chi2, dof)


def test_equilibrium_flux_to_the_obstacle_and_no_drift(oracle_lib):
    """Collisionless gas at T = 1 in a specular box around a 2x2x2 solid
    block at T = 1.  Hits per step = n sqrt(T / 2 pi) A dt with A = 24 faces
    of area 1/64; the mean energy stays at its start (no heating by the
    re-emission) within sampling error."""
    n = (8, 8, 8)
    block = [(ix, iy, iz) for ix in (3, 4) for iy in (3, 4) for iz in (3, 4)]
    N = 20_000
    rs = _box3d(n, dt=0.01, n_init=N, solid=_mask(n, block), solid_T=1.0)
    O = oracle_lib.OracleRun(rs)
    e0 = (O.state()[3:] ** 2).sum() / (3 * N)
    hits = 0
    steps = 500
    for _ in range(steps):
        O.step()
        hits += O.solid_hits()
    n_dens = N / (1.0 - 8 / 512)
    A = 24 * (1 / 8) ** 2
    expect = n_dens * math.sqrt(1.0 / (2 * math.pi)) * A * rs.dt * steps
    assert abs(hits - expect) < 4 * math.sqrt(expect) + 0.01 * expect, (hits, expect)
    e1 = (O.state()[3:] ** 2).sum() / (3 * N)
    # energy changes only at the block, by the difference of an arriving and
    # a departing |c|^2 (both of mean 4T and s.d. about 3T) per hit
    sigma = math.sqrt(hits) * 4.5 / (3 * N)
    assert abs(e1 - e0) < 5 * sigma, (e0, e1, sigma)
    assert abs(e1 - 1.0) < 0.03


def test_closed_diffuse_box_relaxes_to_the_wall_state(oracle_lib):
    """2-D box, every wall and a 4x4-cell obstacle diffuse at T_w = 2, gas
    started at T = 1 with collisions (Kn 0.2): late-time samples are uniform
    in density over the fluid, at rest and at T_w."""
    nx = ny = 16
    mask = np.zeros((1, ny, nx), np.uint8)
    mask[0, 6:10, 6:10] = 1
    N = 4000
    fs = W.fnum_sigma_for(0.2, N)
    rs = W.RunSpec(dim=2, nx=nx, ny=ny, lx=1.0, ly=1.0, dt=0.2 * 0.2 / W.mean_speed(1.0),
                   fnum_sigma=fs, face_bc=("diffuse",) * 6, face_T=(2.0,) * 6, capacity=4096,
                   n_init=N, init_T=1.0, run_id=3, seed=21, solid=mask, solid_T=2.0)
    O = oracle_lib.OracleRun(rs)
    O.step(600)
    S = np.zeros((nx * ny, 7))
    for _ in range(400):
        O.step()
        S += O.sample()
    fluid = ~mask.ravel().astype(bool)
    assert np.all(S[~fluid, 0] == 0)
    m = oracle_lib.moments(S[fluid].sum(axis=0), 400)
    assert abs(m[4] - 2.0) < 0.03, m
    assert np.all(np.abs(m[1:3]) < 0.02)
    # density: chi^2 of the per-cell counts over time (samples 1 step apart
    # are correlated, so the allowance is generous)
    cnt = S[fluid, 0]
    e = cnt.mean()
    assert np.all(np.abs(cnt / e - 1) < 0.12)


def test_no_particle_ends_a_step_in_a_solid_cell(oracle_lib):
    """Mach-5 inflow past a sphere of solid cells (diffuse, T = 3), with
    collisions: after every step each particle's cell is fluid, and the
    particle count changes by generated minus removed."""
    n = (24, 12, 12)
    mask = W.sphere_mask(*n, 2.0, 1.0, 1.0, centre=(0.5, 0.5, 0.5), radius=0.25)
    base = W.body3d(n_runs=1, grid=n, n_per_run=12_000, n_steps=1, n_samples=1).runs[0]
    rs = replace(base, solid=mask)
    O = oracle_lib.OracleRun(rs)
    solid = mask.ravel().astype(bool)
    n_prev = O.info()["n"]
    total_hits = 0
    for _ in range(40):
        O.step()
        info = O.info()
        assert info["n"] == n_prev + info["ngen"] - info["nremoved"]
        n_prev = info["n"]
        cells = O.cells()
        keep = cells["count"][:-1].sum()
        live = cells["cell"][cells["lcr"][:keep]]
        assert not np.any(solid[live])
        total_hits += O.solid_hits()
    assert total_hits > 1000


def test_end_point_rounded_onto_a_solid_face_stays_in_the_fluid(oracle_lib):
    """A wall so cold (T = 1e-40) that the departure is far below one ulp:
    the end point rounds onto the face x = 0.5, whose floor is the solid cell
    5.  It is moved by rounding steps into cell 4, the fluid cell the path
    ended in."""
    n = (10, 4, 4)
    rs = _box3d(n, L=(1.0, 0.4, 0.4), dt=0.5, solid=_mask(n, [(5, 2, 2)]), solid_T=1e-40)
    O, p = _one_particle(oracle_lib, rs, (0.12, 0.25, 0.25), (1.0, 0.0, 0.0))
    assert O.solid_hits() == 1
    assert p[0] < 0.5 and 0.5 - p[0] < 1e-15
    assert int(np.floor(p[0] * 10.0)) == 4
    cells = O.cells()
    assert cells["cell"][0] == (2 * 4 + 2) * 10 + 4
