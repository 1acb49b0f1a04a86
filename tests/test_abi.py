"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/dsmc.h declares, and validates / sizes run specs on the host."""
import ctypes as C
import os
import re
import subprocess

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def dsmc():
    import paper_cs_9902024_amd as P
    if not os.path.exists(P.LIB_PATH):
        from paper_cs_9902024_amd import build
        build.build()
    return P


def _header_symbols():
    src = open(os.path.join(ROOT, "include", "dsmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dsmc_[a-z_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(dsmc):
    syms = _header_symbols()
    assert len(syms) >= 17
    L = C.CDLL(dsmc.LIB_PATH)
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(dsmc.EXPORTS) == syms


def test_struct_sizes_match_header(dsmc, tmp_path):
    """The binding's ctypes layouts equal the C compiler's for the header:
    size and every field offset of the two public structs."""
    fields = {"dsmc_run_spec": [f for f, _ in dsmc.dsmc_run_spec._fields_],
              "dsmc_options": [f for f, _ in dsmc.dsmc_options._fields_]}
    src = ["#include <stddef.h>", "#include <stdio.h>", '#include "dsmc.h"', "int main(void) {"]
    for st, fs in fields.items():
        src.append(f'  printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            src.append(f'  printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    src.append("  return 0; }")
    c_file = tmp_path / "layout.c"
    c_file.write_text("\n".join(src) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(c_file), "-o", str(exe)],
                   check=True)
    out = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                        check=True).stdout.splitlines())
    for st, fs in fields.items():
        cls = getattr(dsmc, st)
        assert int(out[st]) == C.sizeof(cls), st
        for f in fs:
            assert int(out[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)
    assert C.sizeof(dsmc.dsmc_run_spec) == 256 and C.sizeof(dsmc.dsmc_options) == 56


def test_array_lengths_match_header(dsmc):
    src = open(os.path.join(ROOT, "include", "dsmc.h")).read()
    defs = dict(re.findall(r"#define (DSMC_N[A-Z]+) (\d+)", src))
    assert int(defs["DSMC_NINFO"]) == dsmc.NINFO
    assert int(defs["DSMC_NKERNELS"]) == dsmc.NKERNELS
    assert int(defs["DSMC_NDIAG"]) == dsmc.NDIAG == len(dsmc.DIAG_NAMES)


def test_stream_lane_option_is_validated(dsmc):
    specs = dsmc._specs(W.plain_box().runs)
    for bad in (-1, 5):
        opt = dsmc.make_options(True, 1, [], n_streams=bad)
        with pytest.raises(dsmc.DsmcError) as e:
            dsmc.dsmc_required_bytes(specs, opt)
        assert e.value.status == -1
    for ok in range(5):
        dsmc.dsmc_required_bytes(specs, dsmc.make_options(True, 1, [], n_streams=ok))


def test_tile_option_is_validated(dsmc):
    # a tile is whole rounds of 256 slots: 64-slot chunks in multiples of 4
    specs = dsmc._specs(W.plain_box().runs)
    for bad in (-4, 1, 3, 6, 4097, 4100):
        with pytest.raises(dsmc.DsmcError) as e:
            dsmc.dsmc_required_bytes(specs, dsmc.make_options(True, 1, [], tile_chunks=bad))
        assert e.value.status == -1
    for ok in (0, 4, 8, 64, 4096):
        dsmc.dsmc_required_bytes(specs, dsmc.make_options(True, 1, [], tile_chunks=ok))


def _bytes(dsmc, wl, fp64=False, groups=None):
    specs = dsmc._specs(wl.runs)
    opt = dsmc.make_options(fp64, groups or wl.n_groups, wl.sample_steps)
    return dsmc.dsmc_required_bytes(specs, opt)


def test_required_bytes_scale_with_the_workload(dsmc):
    small = _bytes(dsmc, W.plain_box(), fp64=True)
    assert 1e6 < small < 1e8
    big = _bytes(dsmc, W.ensemble_box())
    # 512 runs x ~1M slots x (2 x 5 fp32 + cell + lcr) ~ 25 GB
    assert 20e9 < big < 32e9
    big64 = _bytes(dsmc, W.ensemble_box(), fp64=True)
    assert big64 > 1.6 * big


INF, NAN = float("inf"), float("nan")


@pytest.mark.parametrize("field,value", [("dim", 4), ("nx", 0), ("dt", 0.0), ("dt", -1.0), ("dt", INF),
                                         ("omega", 0.3), ("capacity", 10), ("n_init", -1),
                                         ("fnum_sigma", -1.0), ("fnum_sigma", INF), ("ntc_nbar_alpha", -0.1),
                                         ("ntc_nbar_alpha", 1.5), ("ntc_nbar_alpha", NAN), ("lx", INF),
                                         ("ly", NAN), ("c_ref", INF), ("init_T", INF),
                                         ("init_U", (NAN, 0.0, 0.0)), ("init_U", (0.0, INF, 0.0))])
def test_invalid_specs_are_rejected_on_the_host(dsmc, field, value):
    from dataclasses import replace
    rs = replace(W.plain_box().runs[0], **{field: value})
    with pytest.raises(dsmc.DsmcError) as e:
        _bytes(dsmc, W.plain_box().with_runs([rs]))
    assert e.value.status == -1


def test_failures_without_a_context_carry_a_message(dsmc):
    from dataclasses import replace
    rs = replace(W.plain_box().runs[0], omega=0.3)
    with pytest.raises(dsmc.DsmcError) as e:
        _bytes(dsmc, W.plain_box().with_runs([rs]))
    assert "omega" in str(e.value)
    assert "omega" in dsmc.lib().dsmc_last_error(None).decode()


def test_inflow_only_on_minus_x(dsmc):
    from dataclasses import replace
    rs = W.channel_run(nx=16, ny=8, lx=1.0)
    bad = replace(rs, face_bc=("specular", "inflow") + rs.face_bc[2:])
    with pytest.raises(dsmc.DsmcError):
        _bytes(dsmc, W.plain_box().with_runs([bad]))


@pytest.mark.parametrize("field,value", [("inflow_n", INF), ("inflow_U", NAN), ("inflow_T", INF),
                                         ("face_T", (INF,) * 6)])
def test_non_finite_boundary_state_is_rejected(dsmc, field, value):
    from dataclasses import replace
    rs = W.channel_run(nx=16, ny=8, lx=1.0)
    if field == "face_T":
        rs = replace(rs, face_bc=("inflow", "outflow", "diffuse", "diffuse", "specular", "specular"))
    _bytes(dsmc, W.plain_box().with_runs([rs]))
    with pytest.raises(dsmc.DsmcError) as e:
        _bytes(dsmc, W.plain_box().with_runs([replace(rs, **{field: value})]))
    assert e.value.status == -1


def test_ensemble_runs_must_share_a_grid(dsmc):
    from dataclasses import replace
    a = W.plain_box().runs[0]
    b = replace(a, nx=16, run_id=1)
    with pytest.raises(dsmc.DsmcError):
        _bytes(dsmc, W.plain_box().with_runs([a, b]))
    _bytes(dsmc, W.plain_box().with_runs([a, replace(b, ensemble=1)]))


def test_init_rejects_before_touching_the_device(dsmc):
    specs = dsmc._specs(W.plain_box().runs)
    opt = dsmc.make_options(True, 1, [])
    ctx = C.c_void_p(0)
    # arena missing -> size error, nothing enqueued
    st = dsmc.lib().dsmc_init_runs(specs, 1, C.byref(opt), None, 0, None, C.byref(ctx))
    assert st == -2 and not ctx.value
    st = dsmc.lib().dsmc_init_runs(specs, 0, C.byref(opt), None, 0, None, C.byref(ctx))
    assert st == -1


def test_obstacle_specs(dsmc):
    """Solid masks are sized into the arena and validated on the host."""
    from dataclasses import replace
    # masks of 2 x 2M cells: larger than the 2 MiB alignment of the arena's
    # large arrays, so the difference shows
    big = W.body3d(n_runs=2, grid=(200, 100, 100), n_per_run=100_000, n_steps=1, n_samples=1)
    with_mask = _bytes(dsmc, big)
    without = _bytes(dsmc, big.with_runs([replace(r, solid=None) for r in big.runs]))
    assert with_mask - without >= 2 * 200 * 100 * 100 - (2 << 20)
    wl = W.body3d(n_runs=2, grid=(40, 20, 20), n_per_run=100_000, n_steps=1, n_samples=1)
    bad_T = replace(wl.runs[0], solid_T=0.0)
    with pytest.raises(dsmc.DsmcError) as e:
        _bytes(dsmc, wl.with_runs([bad_T]))
    assert e.value.status == -1
    m = wl.runs[0].solid.copy()
    m[3, 4, 0] = 1                      # a solid cell in the inflow layer
    with pytest.raises(dsmc.DsmcError) as e:
        _bytes(dsmc, wl.with_runs([replace(wl.runs[0], solid=m)]))
    assert e.value.status == -1
    with pytest.raises(dsmc.DsmcError):
        dsmc.make_run_spec(replace(wl.runs[0], solid=m[:, :, :5]))


def test_subcell_specs(dsmc):
    """Sub-cells: 0..4 per axis; the LCR and bin starts are sized by bin
    (cells x k^dim); a body with sub-cells is refused as unsupported."""
    from dataclasses import replace
    wl = W.plain_box()
    plain = _bytes(dsmc, wl)
    sub = _bytes(dsmc, wl.with_runs([replace(wl.runs[0], subcells=4)]))
    assert sub - plain >= 4 * 32 * 32 * 15
    assert _bytes(dsmc, wl.with_runs([replace(wl.runs[0], subcells=1)])) == plain
    for k in (-1, 5):
        with pytest.raises(dsmc.DsmcError) as e:
            _bytes(dsmc, wl.with_runs([replace(wl.runs[0], subcells=k)]))
        assert e.value.status == -1
    body = W.body3d(n_runs=1, grid=(20, 10, 10), n_per_run=10_000, n_steps=1, n_samples=1)
    with pytest.raises(dsmc.DsmcError) as e:
        _bytes(dsmc, body.with_runs([replace(body.runs[0], subcells=2)]))
    assert e.value.status == -6


def test_autotune_workspace_covers_every_candidate(dsmc):
    # 100 expected particles per cell: all three interaction modes are candidates
    wl = W.channel(n_runs=8, nx=64, ny=16, ppc_inf=100.0, n_steps=10, sample_every=5)
    specs = dsmc._specs(wl.runs)
    opt = dsmc.make_options(False, 2, wl.sample_steps)
    tune = dsmc.dsmc_autotune_bytes(specs, opt)
    for tc in (64, 128, 256):
        for mode in (1, 2, 3):
            for lanes in (1, 2):
                o = dsmc.make_options(False, 2, wl.sample_steps, tile_chunks=tc, collide_mode=mode,
                                      n_streams=lanes)
                assert dsmc.dsmc_required_bytes(specs, o) <= tune
    # argument errors before any device work
    best = dsmc.dsmc_options()
    assert dsmc.lib().dsmc_autotune(specs, len(specs), C.byref(opt), None, 0, None, 0, None, 0, None,
                                    C.byref(best), None) == -1
    assert dsmc.lib().dsmc_autotune(specs, len(specs), C.byref(opt), None, 0, None, 3, None, 0, None,
                                    C.byref(best), None) == -2
    # a starting state that is not a checkpoint, or a pointer without a size
    junk = (C.c_uint8 * 200)()
    assert dsmc.lib().dsmc_autotune(specs, len(specs), C.byref(opt), None, 0, None, 3, junk, 200, None,
                                    C.byref(best), None) == -1
    assert dsmc.lib().dsmc_autotune(specs, len(specs), C.byref(opt), None, 0, None, 3, junk, 0, None,
                                    C.byref(best), None) == -1


def test_counting_sort_workspace_query(dsmc):
    assert dsmc.dsmc_counting_sort_bytes(0, 1) > 0
    assert dsmc.dsmc_counting_sort_bytes(1 << 20, 1025) < dsmc.dsmc_counting_sort_bytes(1 << 20, 20000)
    with pytest.raises(dsmc.DsmcError):
        dsmc.dsmc_counting_sort_bytes(-1, 5)


def test_no_oracle_in_the_product():
    """The product path never imports, links or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_cs_9902024_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "dsmc_oracle" not in txt and "liboracle" not in txt, f


def test_no_alloc_sort_validates_on_the_host(dsmc):
    # size and argument checks come before any device call (none is made here)
    assert dsmc.dsmc_counting_sort_bytes(4_000_000, 4097) > dsmc.SORT_SCRATCH_BYTES
    with pytest.raises(dsmc.DsmcError) as e:
        dsmc.dsmc_counting_sort_noalloc(8, 4_000_000, 4097, 8, 8, 0)
    assert e.value.status == -2
    for n, nbins, start in ((-1, 5, 8), (10, 0, 8), (10, 5, 0)):
        with pytest.raises(dsmc.DsmcError) as e:
            dsmc.dsmc_counting_sort_noalloc(8, n, nbins, 8, start, 0)
        assert e.value.status == -1


def test_sort_scratch_size_matches_header(dsmc):
    src = open(os.path.join(ROOT, "include", "dsmc.h")).read()
    m = re.search(r"#define DSMC_SORT_SCRATCH_BYTES \(\(size_t\)(\d+) << (\d+)\)", src)
    assert m and int(m.group(1)) << int(m.group(2)) == dsmc.SORT_SCRATCH_BYTES


def test_sampling_windows_are_validated(dsmc):
    specs = dsmc._specs(W.plain_box().runs)
    ok = [([10, 20], 5, 2), ([3, 20], 5, 1), ([10, 20], 0, 0), ([0, 20], 30, 1)]
    for steps, w, q in ok:
        dsmc.dsmc_required_bytes(specs, dsmc.make_options(True, 1, steps, window_steps=w, window_stride=q))
    # windows that share a step, and negative fields
    bad = [([10, 12], 3, 1), ([10, 20], 6, 2), ([10, 20], -1, 1), ([10, 20], 2, -3)]
    for steps, w, q in bad:
        with pytest.raises(dsmc.DsmcError) as e:
            dsmc.dsmc_required_bytes(specs, dsmc.make_options(True, 1, steps, window_steps=w,
                                                              window_stride=q))
        assert e.value.status == -1
