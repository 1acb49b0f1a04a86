"""Pins of the FP64 oracle to things other than itself (CPU only).

Each test checks the oracle against a value the mathematics or a published
source fixes: known-answer vectors of Philox4x32-10, library stable sorting,
exact conservation laws, closed-form kinetic-theory rates and distributions,
and brute-force enumeration on tiny cells.  The kinetics are those of the
DSMC inner loop of Sec. 1.1 of the paper (Generation, Motion,
Enumeration/Indexing, Interaction, Sampling), written from standard DSMC
practice (the paper's reference Bird 1994).
"""
import math
import os
from dataclasses import replace

import numpy as np
import pytest
from scipy import integrate, special, stats

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# Random numbers
# ---------------------------------------------------------------------------

def test_philox_known_answers(oracle_lib):
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert oracle_lib.philox(v[0:4], v[4:6]) == tuple(v[6:10])


def test_uniform_and_index_edges(oracle_lib):
    # 52-bit centred uniform: extremes are 2^-53 and 1 - 2^-53, never 0 or 1
    assert oracle_lib.u01(0, 0) == 2.0 ** -53
    assert oracle_lib.u01(0xFFFFFFFF, 0xFFFFFFFF) == 1.0 - 2.0 ** -53
    assert oracle_lib.u01(0x80000000, 0) == 0.5 + 2.0 ** -53
    # multiply-shift index: full range maps onto [0, n)
    for n in (1, 2, 3, 977, 2 ** 31 + 5):
        assert oracle_lib.index(0, n) == 0
        assert oracle_lib.index(0xFFFFFFFF, n) == n - 1
    assert oracle_lib.index(0x80000000, 10) == 5


def test_philox_uniformity_and_key_independence(oracle_lib):
    n = 20000
    a = np.array([oracle_lib.philox([i, 3, 7, 0], [11, 5])[0] for i in range(n)], np.float64)
    b = np.array([oracle_lib.philox([i, 3, 7, 0], [12, 5])[0] for i in range(n)], np.float64)
    ua, ub = a / 2 ** 32, b / 2 ** 32
    assert stats.kstest(ua, "uniform").pvalue > 1e-4
    # different keys (runs) give uncorrelated streams
    assert abs(np.corrcoef(ua, ub)[0, 1]) < 4.0 / math.sqrt(n)


# ---------------------------------------------------------------------------
# Indexing: stable counting sort == library stable sort
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,nbins,near,dead", [(1, 2, False, 0.0), (1000, 17, False, 0.1),
                                               (200_000, 1025, True, 0.01),
                                               (100_000, 16385, False, 0.0),
                                               (50_000, 3, False, 0.5)])
def test_counting_sort_is_stable_sort(oracle_lib, n, nbins, near, dead):
    keys = W.random_cells(n, nbins, seed=n + nbins, near_sorted=near, jump=40,
                          dead_fraction=dead)
    lcr, start, count = oracle_lib.counting_sort(keys, nbins)
    np.testing.assert_array_equal(lcr, np.argsort(keys, kind="stable"))
    np.testing.assert_array_equal(count, np.bincount(keys, minlength=nbins))
    np.testing.assert_array_equal(start[1:], np.cumsum(count))


def test_counting_sort_empty(oracle_lib):
    lcr, start, count = oracle_lib.counting_sort(np.zeros(0, np.int32), 5)
    assert lcr.size == 0 and start.tolist() == [0] * 6 and count.tolist() == [0] * 5


def test_step_lcr_and_cells_match_floor(oracle_lib):
    wl = W.plain_box()
    R = oracle_lib.OracleRun(wl.runs[0])
    R.step_begin(); R.generation(); R.motion()
    st = R.state()
    R.indexing()
    cl = R.cells()
    rs = wl.runs[0]
    ix = np.clip(np.floor(st[0] * (rs.nx / rs.lx)), 0, rs.nx - 1).astype(np.int64)
    iy = np.clip(np.floor(st[1] * (rs.ny / rs.ly)), 0, rs.ny - 1).astype(np.int64)
    np.testing.assert_array_equal(cl["cell"], iy * rs.nx + ix)
    np.testing.assert_array_equal(cl["lcr"], np.argsort(cl["cell"], kind="stable"))
    # after the permutation P is cell-sorted
    R.permute()
    st2 = R.state()
    np.testing.assert_array_equal(st2, st[:, cl["lcr"]])


# ---------------------------------------------------------------------------
# Interaction
# ---------------------------------------------------------------------------

def _spec(**kw):
    base = W.plain_box().runs[0]
    return replace(base, **kw)


def test_collision_conserves_momentum_and_energy(oracle_lib):
    rng = np.random.default_rng(5)
    rs = _spec(fnum_sigma=0.5)
    for N in (2, 3, 10, 200):
        vel = rng.normal(size=(3, N)) + np.array([[0.3], [-1.0], [2.0]])
        out = oracle_lib.collide_cell(rs, step=7, cell=3, vel=vel, gmax=5.0)
        assert out["ncoll"] > 0
        p0, p1 = vel.sum(axis=1), out["vel"].sum(axis=1)
        e0, e1 = (vel ** 2).sum(), (out["vel"] ** 2).sum()
        np.testing.assert_allclose(p1, p0, rtol=0, atol=1e-12 * N)
        assert abs(e1 - e0) <= 1e-13 * e0 * N


def test_collision_scattering_is_isotropic(oracle_lib):
    # two particles, one accepted collision per call: cos(chi) of the relative
    # velocity after the collision is uniform on [-1, 1]
    rs = _spec(fnum_sigma=1.0)
    cosx = []
    vel = np.array([[1.0, -1.0], [0.0, 0.0], [0.0, 0.0]])
    for step in range(1, 3001):
        out = oracle_lib.collide_cell(rs, step=step, cell=0, vel=vel, gmax=2.0, rem=0.0,
                                      trace_cap=1)
        if out["trace"][0][2]:
            g = out["vel"][:, out["trace"][0][0]] - out["vel"][:, out["trace"][0][1]]
            cosx.append(g[0] / np.linalg.norm(g) * np.sign(vel[0, out["trace"][0][0]] - vel[0, out["trace"][0][1]]))
    cosx = np.array(cosx)
    assert len(cosx) > 2500
    assert stats.kstest(cosx, stats.uniform(loc=-1, scale=2).cdf).pvalue > 1e-4


@pytest.mark.parametrize("N", [3, 4, 6])
def test_first_selection_probabilities_brute_force(oracle_lib, N):
    """P(first selection = unordered pair {i,j} and accepted) =
    2/(N(N-1)) * g_ij / gmax, enumerated over all pairs."""
    rng = np.random.default_rng(N)
    vel = rng.normal(size=(3, N))
    gmax = 6.0
    rs = _spec(fnum_sigma=1.0)
    # make the first selection happen: rem close to 1
    trials = 30000
    counts = {}
    for step in range(1, trials + 1):
        out = oracle_lib.collide_cell(rs, step=step, cell=N, vel=vel, gmax=gmax, rem=0.999999,
                                      trace_cap=1)
        assert out["nsel"] >= 1
        i, j, acc = (int(x) for x in out["trace"][0])
        key = (min(i, j), max(i, j), acc)
        counts[key] = counts.get(key, 0) + 1
    npairs = N * (N - 1) // 2
    obs, exp = [], []
    for i in range(N):
        for j in range(i + 1, N):
            g = np.linalg.norm(vel[:, i] - vel[:, j])
            p_acc = g / gmax / npairs
            p_rej = (1 - g / gmax) / npairs
            obs += [counts.get((i, j, 1), 0), counts.get((i, j, 0), 0)]
            exp += [p_acc * trials, p_rej * trials]
    chi2 = stats.chisquare(obs, exp)
    assert chi2.pvalue > 1e-4, (obs, exp)


def test_ntc_expected_collisions(oracle_lib):
    """Mean accepted collisions in one step of a cell approach
    sum_{i<j} coef * g_ij (NTC is unbiased while gmax is not exceeded)."""
    rng = np.random.default_rng(2)
    N = 8
    vel = rng.normal(size=(3, N))
    rs = _spec(fnum_sigma=0.001)
    R = oracle_lib.OracleRun(rs, init=False)
    coef = R.consts()["coef"]
    g = np.array([np.linalg.norm(vel[:, i] - vel[:, j]) for i in range(N) for j in range(i + 1, N)])
    expect = coef * g.sum()
    tot, rem = 0, 0.0
    trials = 40000
    for step in range(1, trials + 1):
        out = oracle_lib.collide_cell(rs, step=step, cell=1, vel=vel, gmax=8.0, rem=rem)
        rem = out["rem"]
        tot += out["ncoll"]
    assert expect < 0.5
    # each trial restarts from the same velocities; to first order in expect
    assert abs(tot / trials - expect) < 0.03 * expect + 4 * math.sqrt(expect / trials)


def _realised_T(st):
    c = st[3:]
    return ((c - c.mean(axis=1, keepdims=True)) ** 2).sum() / (3 * c.shape[1])


def test_hard_sphere_equilibrium_collision_frequency(oracle_lib):
    """Collisions per step = 1/2 N(N-1) Fnum sigma <c_r> dt / V with
    <c_r> = 4 sqrt(T/pi) (multinomial cell occupancy makes this exact in
    expectation); ~2000 per step in the plain 20,000-particle box."""
    wl = W.plain_box()
    R = oracle_lib.OracleRun(wl.runs[0])
    rs = wl.runs[0]
    T = _realised_T(R.state())
    N = rs.n_init
    expect = 0.5 * N * (N - 1) * rs.fnum_sigma * 4 * math.sqrt(T / math.pi) * rs.dt / (rs.lx * rs.ly)
    assert abs(expect - 2000) < 20
    tot = 0
    for s in range(200):
        R.step()
        if s >= 20:   # skip the first steps while (sigma c_r)_max settles
            tot += R.info()["ncoll"]
    per_step = tot / 180
    se = math.sqrt(per_step / 180)
    assert abs(per_step - expect) < 4 * se + 0.002 * expect, (per_step, expect)


def test_vhs_equilibrium_collision_frequency(oracle_lib):
    """VHS: <sigma c_r>/sigma_ref = c_ref^(2w-1) <c_r^(2-2w)>, with
    <c_r^q> = (2/sqrt(pi)) Gamma((q+3)/2) (4T)^(q/2)."""
    om = 0.74
    wl = W.box(20_000, 1, 120, 10, seed=9, omega=om)
    rs = wl.runs[0]
    R = oracle_lib.OracleRun(rs)
    T = _realised_T(R.state())
    q = 2 - 2 * om
    mean_crq = 2 / math.sqrt(math.pi) * math.gamma((q + 3) / 2) * (4 * T) ** (q / 2)
    assert abs(2 / math.sqrt(math.pi) * math.gamma(2) * 2 - 4 / math.sqrt(math.pi)) < 1e-15
    sc = rs.c_ref ** (2 * om - 1) * mean_crq
    N = rs.n_init
    expect = 0.5 * N * (N - 1) * rs.fnum_sigma * sc * rs.dt
    tot = 0
    for s in range(120):
        R.step()
        if s >= 20:
            tot += R.info()["ncoll"]
    per_step = tot / 100
    se = math.sqrt(per_step / 100)
    assert abs(per_step - expect) < 4 * se + 0.003 * expect, (per_step, expect)


def test_specular_box_conserves_energy_and_stays_maxwellian(oracle_lib):
    wl = W.plain_box()
    R = oracle_lib.OracleRun(wl.runs[0])
    e0 = (R.state()[3:] ** 2).sum()
    R.step(200)
    st = R.state()
    e1 = (st[3:] ** 2).sum()
    assert abs(e1 - e0) < 1e-12 * e0
    assert R.n == 20_000
    T = e1 / (3 * st.shape[1])
    for a in (3, 4, 5):
        assert stats.kstest(st[a] / math.sqrt(T), "norm").pvalue > 1e-3
    c2 = (st[3:] ** 2).sum(axis=0)
    ratio = (c2 ** 2).mean() / c2.mean() ** 2
    assert abs(ratio - 5 / 3) < 0.06


def test_relaxation_to_maxwellian_from_a_speed_shell(oracle_lib):
    """All particles start at speed sqrt(3) (<c^4>/<c^2>^2 = 1); collisions
    must relax the gas to a Maxwellian (ratio 5/3) at the same energy."""
    wl = W.box(10_000, 1, 150, 10, seed=4, lam=0.05)
    rs = wl.runs[0]
    R = oracle_lib.OracleRun(rs)
    st = R.state()
    rng = np.random.default_rng(0)
    d = rng.normal(size=(3, st.shape[1]))
    st[3:] = d / np.linalg.norm(d, axis=0) * math.sqrt(3)
    R.set_state(st)
    c2 = (st[3:] ** 2).sum(axis=0)
    assert abs((c2 ** 2).mean() / c2.mean() ** 2 - 1) < 1e-12
    R.step(150)   # 30 mean collision times
    st = R.state()
    c2 = (st[3:] ** 2).sum(axis=0)
    assert abs((c2 ** 2).mean() / c2.mean() ** 2 - 5 / 3) < 0.07
    assert abs(c2.mean() - 3.0) < 1e-10


# ---------------------------------------------------------------------------
# Motion
# ---------------------------------------------------------------------------

def test_ballistic_and_specular_mirror(oracle_lib):
    rs = _spec(fnum_sigma=0.0, capacity=256, n_init=0)
    R = oracle_lib.OracleRun(rs, init=False)
    dt = rs.dt
    st = np.array([
        # x, y, z, u, v, w
        [0.5, 0.5, 0.0, 1.0, -2.0, 0.3],            # free flight
        [0.999, 0.5, 0.0, 1.0, 0.0, 0.0],           # +x wall
        [0.5, 0.001, 0.0, 0.0, -1.0, 0.0],          # -y wall
        [0.0005, 0.9995, 0.0, -1.0, 1.0, 5.0],      # corner
    ]).T.copy()
    R.set_state(st)
    R.step_begin(); R.motion()
    out = R.state()
    exp = st.copy()
    exp[0, 0] += 1.0 * dt; exp[1, 0] += -2.0 * dt
    exp[0, 1] = 2 * 1.0 - (0.999 + dt); exp[3, 1] = -1.0
    exp[1, 2] = -(0.001 - dt); exp[4, 2] = 1.0
    exp[0, 3] = -(0.0005 - dt); exp[1, 3] = 2 * 1.0 - (0.9995 + dt); exp[3, 3] = 1.0; exp[4, 3] = -1.0
    np.testing.assert_allclose(out, exp, rtol=0, atol=1e-15)


def _diffuse_hits(oracle_lib, Tw, n=20000):
    rs = _spec(fnum_sigma=0.0, capacity=n, n_init=0,
               face_bc=("specular", "specular", "diffuse", "specular", "specular", "specular"),
               face_T=(1.0, 1.0, Tw, 1.0, 1.0, 1.0))
    R = oracle_lib.OracleRun(rs, init=False)
    st = np.zeros((6, n))
    st[0] = np.linspace(0.1, 0.9, n)
    st[1] = 1e-9
    st[4] = -1.0       # every particle hits -y right away
    R.set_state(st)
    R.step_begin(); R.motion()
    return R.state(), rs


def test_diffuse_wall_reemission_distribution(oracle_lib):
    """Full accommodation at T_w: the normal component has the flux-weighted
    (Rayleigh) density v e^{-v^2/2T_w}, the tangential ones are N(0, T_w)."""
    Tw = 2.0
    out, rs = _diffuse_hits(oracle_lib, Tw)
    vn = out[4]
    assert (vn > 0).all()
    assert stats.kstest(vn, stats.rayleigh(scale=math.sqrt(Tw)).cdf).pvalue > 1e-3
    for a in (3, 5):
        assert stats.kstest(out[a] / math.sqrt(Tw), "norm").pvalue > 1e-3
    # re-emitted particle flies the rest of the step from y = 0
    np.testing.assert_allclose(out[1], vn * (rs.dt - 1e-9), rtol=1e-6)


def test_closed_diffuse_box_keeps_wall_temperature(oracle_lib):
    """Gas at the wall temperature in an all-diffuse box stays at it (wall
    flux balance), with collisions."""
    Tw = 1.5
    wl = W.box(20_000, 1, 300, 10, seed=12, T=Tw)
    rs = replace(wl.runs[0], face_bc=("diffuse",) * 6, face_T=(Tw,) * 6)
    R = oracle_lib.OracleRun(rs)
    R.step(300)
    st = R.state()
    T = (st[3:] ** 2).sum() / (3 * st.shape[1])
    assert abs(T - Tw) < 0.02 * Tw


# ---------------------------------------------------------------------------
# Generation
# ---------------------------------------------------------------------------

def _flux_quad(n, U, T):
    f = lambda u: u * math.exp(-(u - U) ** 2 / (2 * T)) / math.sqrt(2 * math.pi * T)
    return n * integrate.quad(f, 0, np.inf, epsabs=0, epsrel=1e-13)[0]


@pytest.mark.parametrize("mach", [0.0, 0.5, 2.0, 5.0])
def test_inflow_mean_count_is_the_flux(oracle_lib, mach):
    rs = W.channel_run(nx=16, ny=8, lx=1.0, ly=1.0, mach=mach, ppc_inf=30.0, capacity_factor=50.0)
    R = oracle_lib.OracleRun(rs, init=False)
    c = R.consts()
    dy = rs.ly / rs.ny
    assert abs(c["mbar"] - _flux_quad(rs.inflow_n, rs.inflow_U, rs.inflow_T) * dy * rs.dt) \
        < 1e-10 * c["mbar"]
    S = 40
    for _ in range(S):
        R.step_begin(); R.generation()
    per_face = R.n / rs.ny
    assert abs(per_face - S * c["mbar"]) < 1.0
    assert np.all(R.face_rem() >= 0) and np.all(R.face_rem() < 1)


def _flux_cdf(z, s):
    """CDF of z = beta*u for density ~ z exp(-(z-s)^2), z > 0."""
    num = 0.5 * (math.exp(-s * s) - np.exp(-(z - s) ** 2)) + s * math.sqrt(math.pi) / 2 * (
        special.erf(z - s) + special.erf(s))
    den = 0.5 * math.exp(-s * s) + s * math.sqrt(math.pi) / 2 * (1 + special.erf(s))
    return num / den


@pytest.mark.parametrize("mach", [0.0, 0.7, 2.0, 5.0])
def test_inflow_velocity_distributions(oracle_lib, mach):
    rs = W.channel_run(nx=16, ny=8, lx=1.0, ly=1.0, mach=mach, ppc_inf=400.0, capacity_factor=50.0)
    R = oracle_lib.OracleRun(rs, init=False)
    for _ in range(200):
        R.step_begin(); R.generation()
        if R.n > 5000:
            break
    st = R.state()
    beta = 1 / math.sqrt(2 * rs.inflow_T)
    s = rs.inflow_U * beta
    # the closed-form CDF agrees with direct quadrature of u f(u)
    for zt in (0.3, 1.0, s + 0.5):
        q = integrate.quad(lambda z: z * math.exp(-(z - s) ** 2), 0, zt)[0] / \
            integrate.quad(lambda z: z * math.exp(-(z - s) ** 2), 0, np.inf)[0]
        assert abs(q - _flux_cdf(np.array(zt), s)) < 1e-10
    assert st.shape[1] > 3000
    assert stats.kstest(st[3] * beta, lambda z: _flux_cdf(z, s)).pvalue > 1e-3
    for a in (4, 5):
        assert stats.kstest(st[a] / math.sqrt(rs.inflow_T), "norm").pvalue > 1e-3
    assert stats.kstest(st[1] / rs.ly, "uniform").pvalue > 1e-3
    # placed upstream so that a full step carries it in at a uniform time
    frac = 1 + st[0] / (st[3] * rs.dt)
    assert (st[0] <= 0).all() and stats.kstest(frac, "uniform").pvalue > 1e-3
    # entrants are independent draws: no two alike, and successive entrants
    # (mostly of one face element) uncorrelated
    n = st.shape[1]
    assert len(np.unique(st[3])) == n and len(np.unique(st[4])) == n
    yf = np.mod(st[1] * rs.ny / rs.ly, 1.0)        # offset within the face element
    for name, q in (("u", st[3]), ("v", st[4]), ("y offset", yf)):
        r1 = np.corrcoef(q[:-1], q[1:])[0, 1]
        assert abs(r1) < 4.5 / math.sqrt(n), (name, r1)


def test_collisionless_impulsive_start_density(oracle_lib):
    """sigma = 0, empty start: n(x,t) = n_inf 1/2 erfc((x/t - U)/sqrt(2T))."""
    nx, ny = 40, 2
    lx, ly = 2.0, 0.1
    runs = [replace(W.channel_run(nx=nx, ny=ny, lx=lx, ly=ly, mach=1.0, ppc_inf=60.0,
                                  capacity_factor=3.0, run_id=r, seed=77),
                    fnum_sigma=0.0, face_bc=("inflow", "outflow", "specular", "specular",
                                             "specular", "specular"))
            for r in range(16)]
    S = 100
    wl = W.Workload("fm", runs, S, [S], 16)
    acc, st = oracle_lib.ensemble(wl, n_threads=4)
    rs = runs[0]
    t = S * rs.dt
    counts = acc[0].sum(axis=0)[:, 0].reshape(ny, nx).sum(axis=0)   # over groups and y
    dx = lx / nx
    vol = dx * ly * len(runs)
    U, T = rs.inflow_U, rs.inflow_T
    z = []
    for i in range(nx):
        a, b = i * dx, (i + 1) * dx
        m = integrate.quad(lambda x: 0.5 * special.erfc((x / t - U) / math.sqrt(2 * T)), a, b)[0] / dx
        expect = rs.inflow_n * m * vol
        z.append((counts[i] - expect) / math.sqrt(max(expect, 1.0)))
    z = np.array(z)
    assert np.max(np.abs(z)) < 4.5, z
    assert np.mean(z ** 2) < 2.0, z


# ---------------------------------------------------------------------------
# Sampling, moments, runs
# ---------------------------------------------------------------------------

def test_sampling_matches_fsum(oracle_lib):
    wl = W.plain_box()
    R = oracle_lib.OracleRun(wl.runs[0])
    R.step(3)
    st = R.state()
    cl = R.cells()
    s = R.sample()
    for c in (0, 1, 500, 1023):
        b, n = cl["start"][c], cl["count"][c]
        seg = st[3:, b:b + n]
        ref = [n] + [math.fsum(seg[a]) for a in range(3)] + [math.fsum(seg[a] ** 2) for a in range(3)]
        np.testing.assert_allclose(s[c], ref, rtol=1e-13, atol=1e-13)
    assert s[:, 0].sum() == 20_000


def test_moments_closed_form(oracle_lib):
    rng = np.random.default_rng(3)
    vel = rng.normal(size=(3, 5000)) * math.sqrt(2.0) + np.array([[1.0], [-0.5], [0.25]])
    sums = np.array([vel.shape[1], *vel.sum(axis=1), *(vel ** 2).sum(axis=1)])
    m = oracle_lib.moments(sums, n_runs=2)
    assert m[0] == 2500
    np.testing.assert_allclose(m[1:4], vel.mean(axis=1), rtol=1e-12)
    np.testing.assert_allclose(m[5:8], vel.var(axis=1), rtol=1e-10)
    np.testing.assert_allclose(m[4], vel.var(axis=1).mean(), rtol=1e-10)
    assert np.isnan(oracle_lib.moments(np.zeros(7), 1)[1])


def test_runs_replay_and_are_independent(oracle_lib):
    wl = W.box(2000, 2, 5, 5, seed=8)
    a = oracle_lib.OracleRun(wl.runs[0]); a.step(5)
    b = oracle_lib.OracleRun(wl.runs[0]); b.step(5)
    c = oracle_lib.OracleRun(wl.runs[1]); c.step(5)
    np.testing.assert_array_equal(a.state(), b.state())
    assert not np.allclose(a.state()[3], c.state()[3])


def test_ensemble_independent_of_thread_count(oracle_lib):
    wl = W.box(1500, 6, 12, 4, seed=21, n_groups=3)
    a1, s1 = oracle_lib.ensemble(wl, n_threads=1)
    a3, s3 = oracle_lib.ensemble(wl, n_threads=3)
    np.testing.assert_array_equal(a1, a3)
    assert s1["particle_steps"] == 6 * 12 * 1500
    assert a1.shape == (3, 3, 1024, 7)
    assert np.all(a1[:, :, :, 0].sum(axis=(1, 2)) == 6 * 1500)


def test_sigma_cr_max_updates_immediately(oracle_lib):
    """Two particles, (sigma c_r)_max set below their g: the first selection
    raises it to g exactly and is accepted (g/g = 1 > U); scattering keeps
    |c_r|, so every later selection in the step is accepted too."""
    rs = _spec(fnum_sigma=1.0)
    vel = np.array([[1.5, -0.5], [0.2, 0.1], [-0.3, 0.4]])
    g = np.linalg.norm(vel[:, 0] - vel[:, 1])
    out = oracle_lib.collide_cell(rs, step=3, cell=9, vel=vel, gmax=0.1 * g, rem=0.0)
    assert out["nsel"] >= 1
    assert out["gmax"] == g
    assert out["ncoll"] == out["nsel"]
    np.testing.assert_allclose(np.linalg.norm(out["vel"][:, 0] - out["vel"][:, 1]), g, rtol=1e-14)


def test_upstream_particle_that_never_enters_is_removed(oracle_lib):
    rs = _spec(fnum_sigma=0.0, capacity=256, n_init=0,
               face_bc=("inflow", "outflow", "specular", "specular", "specular", "specular"))
    R = oracle_lib.OracleRun(rs, init=False)
    st = np.array([[-1.0, 0.5, 0.0, 1.0, 0.0, 0.0],      # still upstream after dt
                   [-1e-4, 0.5, 0.0, 1.0, 0.0, 0.0],     # enters
                   [1e-4, 0.5, 0.0, -1.0, 0.0, 0.0]]).T.copy()   # leaves through the inflow plane
    R.set_state(st)
    R.step_begin(); R.motion(); R.indexing()
    cl = R.cells()
    assert cl["cell"].tolist() == [1024, 16 * 32, 1024]
    assert R.info()["nremoved"] == 2
