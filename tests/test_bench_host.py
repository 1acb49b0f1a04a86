"""Host-side arithmetic of bench.py (no GPU): the Amdahl fit of the
reallocation experiment (eq. (11) with PRI = 0 is T(p) = T(1)(beta +
(1 - beta)/p)), the FP32-accumulator emulation of the precision report, the
byte accounting of the roofline, and the refusal of more than one GPU."""
import importlib.util
import math
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("beta", [0.0, 0.004, 0.05, 0.3])
@pytest.mark.parametrize("overhead", [0.0, 1e-4])
def test_amdahl_fit_recovers_beta(bench, beta, overhead):
    """T(p) = T(1) (beta + (1 - beta)/p) plus a per-processor start-up cost
    that grows with p; the smallest p timed is 2, not 1."""
    p = [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048]
    t = [10.0 * (beta + (1 - beta) / x) + overhead * x for x in p]
    fit = bench.amdahl_fit(p, t)
    T1 = 10.0 + overhead
    assert abs(fit["beta"] - 10.0 * beta / T1) < 1e-9
    assert abs(fit["overhead"] - overhead / T1) < 1e-9


def test_amdahl_fit_limits(bench):
    # a time that no processor count changes is all sequential; times
    # falling faster than 1/p clamp beta to 0
    assert bench.amdahl_beta([1, 2, 4, 8], [3.0, 3.0, 3.0, 3.0]) == pytest.approx(1.0)
    assert bench.amdahl_beta([1, 2, 4, 8], [1.0, 0.3, 0.05, 0.005]) == 0.0


def _sums(rng, groups, cells, drift):
    acc = np.zeros((groups, cells, 7))
    for g in range(groups):
        N = rng.poisson(30, cells).astype(float)
        u = rng.normal(drift, 1.0, (cells, 3))
        acc[g, :, 0] = N
        acc[g, :, 1:4] = N[:, None] * u
        acc[g, :, 4:7] = N[:, None] * (u * u + 1.0)
    return acc


def _moments64(acc, runs):
    tot = acc.sum(axis=0)
    m = np.zeros((tot.shape[0], 5))
    m[:, 0] = tot[:, 0] / runs
    u = tot[:, 1:4] / tot[:, 0:1]
    m[:, 1:4] = u
    m[:, 4] = ((tot[:, 4:7] / tot[:, 0:1]) - u * u).mean(axis=1)
    return m


def test_fp32_accumulator_error_grows_with_the_drift(bench):
    """The emulated FP32 accumulation loses T to cancellation as the flow
    speed grows (T = <c^2> - u^2): the report must show it, and be exact for
    the counts."""
    rng = np.random.default_rng(3)
    out = {}
    for drift in (0.0, 6.0, 30.0):
        acc = _sums(rng, 32, 400, drift)
        m = _moments64(acc, 32)
        se = np.abs(m) * 0.01 + 0.01
        out[drift] = bench.accumulator_precision(acc, m, se, 32)
        assert out[drift]["n"]["max_err"] == 0.0
        assert out[drift]["cells"] == 400
    assert out[0.0]["T"]["max_err"] < 1e-5
    assert out[30.0]["T"]["median_err"] > 10 * out[0.0]["T"]["median_err"]


def test_fp32_accumulator_emulation_rounds_every_add(bench):
    """A group sum that FP32 cannot hold next to the running total is lost
    in FP32 but kept in FP64."""
    acc = np.zeros((2, 1, 7))
    acc[0, 0] = [2**25, 0, 0, 0, 2**25, 2**25, 2**25]
    acc[1, 0] = [1, 1, 1, 1, 1, 1, 1]
    m = _moments64(acc, 2)
    rep = bench.accumulator_precision(acc, m, np.ones_like(m), 2)
    assert rep["n"]["max_err"] == pytest.approx(1 / (2**25 + 1))


def test_byte_accounting(bench):
    n, c = 1_000_000, 1024
    assert bench.scope_bytes("motion", n, c, 4) == n * bench.SCOPE_BYTES["motion"]
    assert bench.scope_bytes("collide_cells", n, c, 4) == n * bench.SCOPE_BYTES["collide"] + c * 28
    # as built: LCR 4 + particle 20 read + 20 written + next cell 4 = 48 (2-D FP32)
    assert bench.algorithmic_bytes("collide_cells", n, c, 2, 4) == n * 48 + c * 28
    assert bench.algorithmic_bytes("collide_lanes", n, c, 3, 4) == n * 56 + c * 28
    assert bench.algorithmic_bytes("motion", n, c, 2, 4) == n * 4
    assert bench.algorithmic_bytes("scatter", n, c, 2, 4) == n * 8
    assert sum(bench.SCOPE_BYTES.values()) == 80


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_line_is_strict_json(bench):
    import json
    line = {"a": float("nan"), "b": [1.0, float("inf")], "c": {"d": 2, "e": -float("inf")}}
    out = json.dumps(bench._json_safe(line), allow_nan=False)
    assert json.loads(out) == {"a": None, "b": [1.0, None], "c": {"d": 2, "e": None}}
