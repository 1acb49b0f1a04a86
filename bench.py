#!/usr/bin/env python3
"""Throughput of the unsteady-DSMC inner loop on one MI355X.

A step is one pass of the whole inner loop (Generation, Motion,
Enumeration/Indexing, Interaction, Sampling at the scheduled steps) over every
run of the batch.  The default workload is the batched ensemble: 512
independent runs of the 32x32-cell specular box at 1M hard-sphere particles
each (512M particle slots, FP32 SoA state, FP64 sampling accumulators, a
sample every 20 steps), stepped by HIP-graph replay with inputs resident in
HBM.  ``value`` = particle-steps per second over the timed steps (particles
moved per step, summed over runs and steps, divided by the wall time between
two device synchronisations).

Before the timed region the library's autotuner (dsmc_autotune) picks the
tuning settings (Indexing tile, interaction mode, stream lanes) by timing its
candidates on the same batch in a scratch arena; tuning never changes results.

Beside it the line carries:
  roofline      the dominant kernel's algorithmic bytes per launch over its
                mean HIP-event duration (events recorded on the streams the
                kernels run on), against MI355X's 8 TB/s HBM peak, with the
                per-particle bytes of the hot-path scope table (Interaction
                with the permutation: 4 + 20 read + 20 written);
                roofline_as_built: the same with the bytes this design moves
                (48: the next flight's cell is also written), and the whole
                step's bytes per particle-step under both accountings;
  plain_fp64    the plain path: the same problem, one run at a time, FP64
                state, one launch per kernel;
  cpu_baseline  the FP64 oracle timed on the host cores on a bounded sample
                (128 runs x 20 steps, 16 threads) and on one thread;
  oracle_match  each macroparameter of the timed batch at step 20 (512 FP32
                runs, FP64 accumulators) against the oracle's ensemble of
                the same problem at step 20 (the 128 runs above, other seeds):
                z = difference / combined standard error per cell, and the
                relative error; also against the exact equilibrium values;
  paper_figures the paper's own speedup and efficiency parameters with the
                machine it names (context: a whole program on an SPP-1600);
  accumulator_precision  per macroparameter, the error FP32 accumulators and
                division would have added to the batch's first sample (its
                run groups' sums added and divided in FP32) against the FP64
                ones, beside the sample's relative standard error (the
                first ensemble of the batch).

``--workload body3d`` times the flow past a body at full size instead (32 runs
x 60M particles, 2M cells, solid-cell obstacle); ``channel`` (16 runs of the
impulsively started Mach-2 channel, 256x64 cells, ~2M particles each at fill)
and ``uneven`` (256 runs of uneven grids, particle counts, collision models
and inflow speeds) start from vacuum and are timed after FILL_STEPS steps, by
when the flow has crossed the domain; the autotuner then times its candidates
from a checkpoint of that state (not from the empty start).  These are
informational, not the benchmark line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/sec (batched FP32 vs plain FP64) at 3σ/1% oracle match; HBM GB/s"
HBM_PEAK_GBS = 8000.0
FILL_STEPS = 600  # steps from vacuum before the unsteady workloads are timed
# The paper's own figures, with the machine it names: parallel-efficiency
# parameters of a whole DSMC program on a shared-memory multiprocessor (Sec.
# 2-3), not throughputs of this path, so they are context, not a baseline.
PAPER_FIGURES = {
    "machine": "HP/Convex Exemplar SPP-1600: 8 processors, 2 GB memory, 1600 Mflops peak",
    "tlp_comet_flow": {"problem": "unsteady 3-D water-vapour flow in a comet's inner atmosphere",
                       "p1": 6, "p2": "1..6", "alpha1": 0.998, "alpha2": 0.97},
    "tlpdpr_body_flow": {"problem": "unsteady flow past a body", "beta": 0.437, "p1": 6, "p": 36,
                         "max_level2_speedup_eq11": 2.3, "tlp_fraction_of_max": 0.80,
                         "tlpdpr_fraction_of_max_at_optimal_pri": 0.93,
                         "tlpdpr_equivalent_tlp_processors": 120},
}
WORKLOAD_TEXT = {
    "ensemble_box": ("ensemble_box: {runs} independent runs x {per_run} hard-sphere particles, 2-D 1x1 "
                     "specular box, 32x32 cells, Kn 0.05, dt = 0.2 mean collision times, FP32 state, FP64 "
                     "sampling accumulators, sample every 20 steps, HIP graph"),
    "body3d": ("body3d: 32 independent runs x 60M hard-sphere particles, 3-D 2x1x1 box, 200x100x100 "
               "cells, Mach-5 inflow past a sphere of solid cells (diffuse, T = 3), FP32 state, FP64 "
               "sampling accumulators, HIP graph"),
    "channel": ("channel: 16 independent runs of the impulsively started Mach-2 channel, 4x1 domain, "
                "256x64 cells, VHS omega 0.74, diffuse wall at T = 2, ~2M particles per run at fill, "
                "timed after 600 steps from vacuum, FP32 state, HIP graph"),
    "uneven": ("uneven: 256 independent runs, grids 64x64..512x256, 50k..4M particles, HS/VHS, Mach "
               "0.5..5 inflow, timed after 600 steps from vacuum, FP32 state, HIP graph"),
}


# Algorithmic bytes per particle-step of the hot-path scope table (2-D, FP32
# state): Motion with Enumeration 16 read + 12 written, the Indexing scatter
# 4 + 4, Interaction with the permutation 4 + 20 read + 20 written.
SCOPE_BYTES = {"motion": 28, "scatter": 8, "collide": 44}


def scope_bytes(kind: str, n_particles: int, n_cells: int, es: int) -> float:
    """Bytes per launch by the hot-path scope table's per-particle figures,
    plus the same per-cell terms as below."""
    if kind == "motion":
        return n_particles * SCOPE_BYTES["motion"]
    if kind == "scatter":
        return n_particles * SCOPE_BYTES["scatter"]
    if kind in ("collide", "collide_cells", "collide_waves", "collide_lanes"):
        return n_particles * SCOPE_BYTES["collide"] + n_cells * (4 + 4 * es + 8)
    return 0.0


def algorithmic_bytes(kind: str, n_particles: int, n_cells: int, dim: int, es: int) -> float:
    """Bytes a kernel of this design must move per launch (each byte once, no
    re-reads).

    motion         reads the cell the last Interaction found for the
                   particle's flight (4); only particles generated in the
                   step (none in a closed box) are read whole and tested here
    scatter        reads the cell index (4), writes the LCR entry (4)
    collide_cells  (Interaction fused with the flight, the permutation
    collide_waves   P' = P[LCR], Sampling and the next flight's test) reads
    collide_lanes   the LCR entry (4) and the particle (dim+3)*es, writes it to
                   P' and its next flight cell (4); per cell the two bin
                   starts (4), remainder and (sigma c_r)_max read and written
                   (4*es) and the collision counter read and written (8)
    """
    if kind == "motion":
        return n_particles * 4
    if kind == "scatter":
        return n_particles * 8
    if kind in ("collide", "collide_cells", "collide_waves", "collide_lanes"):
        return n_particles * (8 + 2 * (dim + 3) * es) + n_cells * (4 + 4 * es + 8)
    return 0.0


TRAFFIC_GLOB = os.path.join(ROOT, "profiles", "ensemble_box_512x1M_fp32_tile*_traffic.md")
KERNEL_SRC = os.path.join(ROOT, "paper_cs_9902024_amd", "csrc", "dsmc_kernels.hip")


def measured_traffic(kernel: str, lanes: int, tile: int):
    """HBM bytes per launch of ``kernel`` from a committed FETCH_SIZE /
    WRITE_SIZE summary (scaled by the copy-kernel calibration) taken with the
    same kernel source, the same split of the batch into lanes and the same
    Indexing tile size as this run; None when there is none."""
    import glob
    import hashlib
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    for path in sorted(glob.glob(TRAFFIC_GLOB)):
        found, ok, same_lanes, same_tile = None, False, False, False
        for line in open(path):
            f = line.split()
            if len(f) == 3 and f[0] == "traffic" and f[1] == kernel:
                found = float(f[2])
            if len(f) == 2 and f[0] == "source_sha256":
                ok = f[1] == sha
            if len(f) == 2 and f[0] == "lanes":
                same_lanes = int(f[1]) == lanes
            if len(f) == 2 and f[0] == "tile":
                same_tile = int(f[1]) == tile
        if found is not None and ok and same_lanes and same_tile:
            return found
    return None


def copy_calibration(nbytes: int = 1 << 31):
    """A plain device-to-device copy of known size (torch's copy kernel):
    the streaming bandwidth this GPU delivers, and the reference kernel whose
    FETCH_SIZE / WRITE_SIZE counters scale the traffic of the DSMC kernels."""
    import torch
    x = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    y = torch.empty_like(x)
    for _ in range(2):
        y.copy_(x)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    n = 5
    a.record()
    for _ in range(n):
        y.copy_(x)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / n
    del x, y
    torch.cuda.empty_cache()
    return {"bytes_per_copy": 2 * nbytes, "ms": ms, "GBs": 2 * nbytes / (ms * 1e-3) / 1e9}


def run_gpu(args):
    import torch
    import paper_cs_9902024_amd as P
    import workloads as W

    torch.cuda.set_device(0)
    calib = copy_calibration()
    if args.workload == "body3d":
        wl = W.body3d()
    elif args.workload == "channel":
        wl = W.channel()
    elif args.workload == "uneven":
        wl = W.uneven()
    else:
        wl = W.ensemble_box(n_runs=args.runs, n_per_run=args.per_run, n_steps=1000, sample_every=20,
                            seed=3, state_fp64=False)
    dim = wl.runs[0].dim
    tuned = None
    kw = {"n_streams": args.streams, "tile_chunks": args.tile_chunks, "collide_mode": args.collide_mode,
          "sched": args.sched, "sched_blocks": args.sched_blocks}
    unsteady = args.workload in ("channel", "uneven")
    tune_kw = dict(state_fp64=False, n_groups=wl.n_groups, use_graph=True, n_steps=3, tune_cache=args.tune_cache,
                   window_steps=getattr(wl, "window_steps", 1), window_stride=getattr(wl, "window_stride", 1))
    if not args.no_tune and not unsteady:
        # the library's autotuner times its candidate settings on this batch
        # (a scratch arena, before the timed region); tuning never changes results
        tuned = P.Ensemble.autotune(wl.runs, wl.sample_steps, **tune_kw)
        kw = {k: tuned[k] for k in ("tile_chunks", "collide_mode", "n_streams", "sched", "sched_blocks")
              if k in tuned}
    E = P.Ensemble.from_workload(wl, use_graph=True, **kw)
    n_runs = wl.n_runs
    nc = wl.runs[0].n_cells

    warmup = args.warmup
    if unsteady:
        # fill from vacuum; then tune at the filled state (every candidate
        # restored from its checkpoint) and carry on from the same state
        E.step(FILL_STEPS)
        warmup += FILL_STEPS
        if not args.no_tune:
            ck = E.checkpoint()
            E.close()
            del E
            torch.cuda.empty_cache()
            tuned = P.Ensemble.autotune(wl.runs, wl.sample_steps, start=ck, **tune_kw)
            kw = {k: tuned[k] for k in ("tile_chunks", "collide_mode", "n_streams", "sched", "sched_blocks")}
            E = P.Ensemble.from_workload(wl, use_graph=True, **kw)
            E.restore(ck)
            del ck
    E.step(args.warmup)
    E.sync()
    torch.cuda.synchronize()
    n0 = int(E.counts()[:, 0].sum())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    E.step(args.steps)
    E.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n1 = int(E.counts()[:, 0].sum())
    elapsed = t1 - t0
    if args.workload == "ensemble_box":
        assert n0 == n1, "closed box must keep its particle count"
        psteps = n0 * args.steps
    else:
        # inflow and outflow change the count by ~0.01 % per step: the mean of
        # the counts before and after the timed steps
        psteps = (n0 + n1) // 2 * args.steps
    value = psteps / elapsed

    # the timed batch's moments at the first sample step (FP64 division of
    # the FP64 accumulators), for the comparison with the oracle
    match_gpu = None
    if args.workload == "ensemble_box" and wl.sample_steps and warmup + args.steps >= wl.sample_steps[0]:
        m, se = E.moments(0)
        tot = E.accum(0).sum(axis=(0, 1))
        match_gpu = {"step": wl.sample_steps[0], "m": m, "se": se, "tot": tot, "runs": n_runs,
                     "groups": wl.n_groups}

    # per-kernel HIP-event durations over a second, profiled window
    E.profiling(True)
    E.step(args.prof_steps)
    kt = E.kernel_times()
    E.profiling(False)
    info = E.info()
    # FP64 against FP32 accumulation of the batch's first sample, per
    # macroparameter (after the timed and profiled steps; the body flow steps
    # on to its first sample step)
    acc_prec = None
    if wl.sample_steps:
        done = warmup + args.steps + args.prof_steps
        if done < wl.sample_steps[0]:
            E.step(wl.sample_steps[0] - done)
        m64, se = E.moments(0)                         # ensemble 0
        acc_prec = accumulator_precision(E.accum(0), m64, se, sum(1 for r in wl.runs if r.ensemble == 0))
        acc_prec["step"] = wl.sample_steps[0]
        acc_prec["ensemble"] = 0
    E.close()
    del E
    torch.cuda.empty_cache()

    # a step launches each kernel once per lane (run group); the lanes split
    # the runs, so a launch's algorithmic bytes are the step's over the
    # launches per step
    kernels = {k: {"ms_total": ms, "launches": n, "ms_avg": ms / n} for k, (ms, n) in kt.items()}
    # with several Interaction kernels (cells split between the modes) each
    # moves only its own cells' particles: the roofline then takes
    # Interaction as a whole (every particle once, the kernels' summed time)
    modes = [k for k in kernels if k.startswith("collide_")]
    view = {k: v for k, v in kernels.items() if k not in modes or len(modes) == 1}
    if len(modes) > 1:
        tot = sum(kernels[k]["ms_total"] for k in modes)
        n_l = max(kernels[k]["launches"] for k in modes)
        view["collide"] = {"ms_total": tot, "launches": n_l, "ms_avg": tot / n_l,
                           "kernels": {k: kernels[k]["ms_total"] for k in modes}}
    dom = max(view, key=lambda k: view[k]["ms_total"])
    rl = rl_built = None
    tr = measured_traffic(dom, info["lanes"], info["slots"] // info["tiles"]) \
        if args.workload == "ensemble_box" else None
    n_cells_all = sum(r.n_cells for r in wl.runs)
    for acct, fn in (("scope", lambda k: scope_bytes(k, n0, n_cells_all, 4) if dim == 2 else 0.0),
                     ("built", lambda k: algorithmic_bytes(k, n0, n_cells_all, dim, 4))):
        per_step = fn(dom)
        if per_step <= 0:
            continue
        ab = per_step * args.prof_steps / view[dom]["launches"]
        ach = ab / (view[dom]["ms_avg"] * 1e-3) / 1e9
        obj = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": tr, "kernel": dom,
               "algorithmic_bytes_per_launch": ab, "avg_launch_ms": view[dom]["ms_avg"]}
        if dom == "collide":
            obj["kernels"] = view[dom]["kernels"]
        if acct == "scope":
            rl = obj
        else:
            rl_built = obj
    if rl is None:
        rl, rl_built = rl_built, None
    for k, v in (kernels.items() if len(modes) < 2 else [(k, v) for k, v in kernels.items() if k not in modes]):
        b = algorithmic_bytes(k, n0, n_cells_all, dim, 4)
        if b > 0:
            v["algorithmic_GBs"] = round(b * args.prof_steps / (v["ms_total"] * 1e-3) / 1e9, 1)
            v["frac_of_hbm_peak"] = round(v["algorithmic_GBs"] / HBM_PEAK_GBS, 4)

    plain = None
    if args.plain_runs > 0 and args.workload == "ensemble_box":
        plain = run_plain_fp64(args, P, W)
    # the whole step's bytes per particle-step, both accountings
    step_bytes = None
    if args.workload == "ensemble_box":
        bpp = {"scope": sum(SCOPE_BYTES.values()), "built": 4 + 8 + 48}
        step_bytes = {a: {"bytes_per_particle_step": b, "GBs": round(b * value / 1e9, 1),
                          "frac": round(b * value / 1e9 / HBM_PEAK_GBS, 4)} for a, b in bpp.items()}
    return {"value": value, "elapsed": elapsed, "psteps": psteps, "n_runs": n_runs, "nc": nc, "tuned": tuned,
            "warmup": warmup, "n_mean": psteps // args.steps, "rl_built": rl_built, "step_bytes": step_bytes,
            "kernels": kernels, "roofline": rl, "plain": plain, "info": info, "calib": calib,
            "match_gpu": match_gpu, "acc_prec": acc_prec}


def run_plain_fp64(args, P, W):
    """The plain path: one run at a time, FP64 state, a launch per kernel."""
    import torch
    total_ps, total_t = 0, 0.0
    for r in range(args.plain_runs):
        wl = W.ensemble_box(n_runs=1, n_per_run=args.per_run, n_steps=1000, sample_every=20, seed=3,
                            state_fp64=True)
        from dataclasses import replace
        runs = [replace(wl.runs[0], run_id=r)]
        E = P.Ensemble(runs, wl.sample_steps, state_fp64=True, n_groups=1, use_graph=False)
        E.step(2)
        E.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        E.step(args.plain_steps)
        E.sync()
        torch.cuda.synchronize()
        total_t += time.perf_counter() - t0
        total_ps += args.per_run * args.plain_steps
        E.close()
    return {"value": total_ps / total_t, "unit": "particle-steps/s", "runs_timed": args.plain_runs,
            "steps_per_run": args.plain_steps, "dtype": "f64",
            "note": "same box problem, one run per context, FP64 state, no graph"}


def interaction_ms(E, steps: int) -> float:
    """Mean Interaction time per step (all interaction kernels) over `steps`
    profiled steps of context E."""
    E.profiling(True)
    E.step(steps)
    kt = E.kernel_times()
    E.profiling(False)
    return sum(ms for k, (ms, n) in kt.items() if k.startswith("collide")) / steps


def accumulator_precision(acc, m64, se, n_runs: int) -> dict:
    """What FP32 sampling accumulators would have cost, per macroparameter:
    the run groups' sums (FP64, [groups][cells][7]) rounded to FP32 and added
    in FP32 in group order, then divided in FP32 (n = N/R, u = sum c / N,
    T = mean over axes of sum c_a^2 / N - u_a^2), against the library's FP64
    moments m64 of the same sums.  Errors over the cells holding particles:
    n and T relative, u, v, w relative to sqrt(T); beside them the median
    relative standard error (run groups) for scale."""
    import numpy as np
    acc = np.asarray(acc).reshape(-1, acc.shape[-2], acc.shape[-1])
    f = np.float32
    tot = np.zeros(acc.shape[1:], f)
    for g in range(acc.shape[0]):
        tot = (tot + acc[g].astype(f)).astype(f)
    N = tot[:, 0]
    ok = (N > 0) & (m64[:, 0] > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        n32 = N / f(n_runs)
        u32 = tot[:, 1:4] / N[:, None]
        T32 = ((tot[:, 4:7] / N[:, None]) - u32 * u32).mean(axis=1, dtype=f)
    T64 = m64[:, 4]
    scale = np.sqrt(np.maximum(T64, 1e-300))
    out = {"cells": int(ok.sum()), "runs": n_runs, "groups": int(acc.shape[0])}
    errs = {"n": np.abs(n32 - m64[:, 0]) / np.abs(m64[:, 0]),
            "u": np.abs(u32[:, 0] - m64[:, 1]) / scale, "v": np.abs(u32[:, 1] - m64[:, 2]) / scale,
            "w": np.abs(u32[:, 2] - m64[:, 3]) / scale, "T": np.abs(T32 - T64) / np.abs(T64)}
    cols = {"n": 0, "u": 1, "v": 2, "w": 3, "T": 4}
    for k, e in errs.items():
        e = e[ok & np.isfinite(e)]
        c = cols[k]
        with np.errstate(divide="ignore", invalid="ignore"):
            rel_se = se[ok, c] / (np.abs(m64[ok, c]) if k in ("n", "T") else scale[ok])
        rel_se = rel_se[np.isfinite(rel_se)]      # none with a single run group
        out[k] = {"max_err": float(e.max()) if e.size else None, "median_err": float(np.median(e)) if e.size else None,
                  "median_rel_se": float(np.median(rel_se)) if rel_se.size else None}
    return out


def amdahl_fit(units, times) -> dict:
    """Amdahl's beta from times T(p) on p processors (wavefronts): a
    least-squares fit, in relative terms (each point weighted by 1/T(p)), of
    T(p) = A + B/p + C p -- the part more processors do not shorten, the
    part they share, and a per-processor cost of starting and draining the
    persistent grid that shows at large p.  With T(1) = A + B + C: beta =
    A / T(1) and overhead = C / T(1) (both clamped to [0, 1]).  The smallest
    p need not be 1."""
    import numpy as np
    p = np.asarray(units, float)
    T = np.asarray(times, float)
    X = np.stack([np.ones_like(p), 1.0 / p, p], axis=1) / T[:, None]
    (A, B, C), *_ = np.linalg.lstsq(X, np.ones_like(T), rcond=None)
    T1 = A + B + C
    if T1 <= 0:
        return {"beta": 1.0 if A > 0 else 0.0, "overhead": 0.0}
    clamp = lambda x: float(min(max(x, 0.0), 1.0))
    return {"beta": clamp(A / T1), "overhead": clamp(C / T1)}


def amdahl_beta(units, times) -> float:
    return amdahl_fit(units, times)["beta"]


def balance_experiment(args):
    """Dynamic against static allocation of Interaction's workgroups to the
    runs of the uneven batch (the two-level split of Sec. 2 against the
    dynamic processor reallocation of Sec. 3), every run in the lane-per-cell
    mode (one kernel; its processors are wavefronts).

    - beta of sampled runs: each run alone, its Interaction timed on persistent
      grids of 2 .. 2048 wavefronts drawing from its queue; Amdahl fit.
    - the batch after the fill: static (sched 2: p2 wavefronts tied to each
      run) and dynamic (sched 1: p2 x runs wavefronts drawing from one queue)
      for p2 = 1, 2, 4, 8; achieved level-2 speedups S = T_static(1) / T.
    - beside them eq. (11), S_p2 = 1 / (beta + (1 - beta) / (p2 (1 + PRI))),
      at PRI = 0 and at PRI* = beta / (1 - beta) (p2 - 1) from eq. (13)."""
    import numpy as np
    import paper_cs_9902024_amd as P
    import workloads as W
    wl = W.uneven()
    R = wl.n_runs
    wpb = 2  # wavefronts per workgroup of the lane-per-cell kernel
    kw = dict(collide_mode=1, use_graph=False)
    base = P.Ensemble.from_workload(wl, sched=1, **kw)
    base.step(FILL_STEPS)
    counts = base.counts()[:, 0]
    ck = base.checkpoint()
    base.close()
    # sampled runs: smallest, two middle, largest by particles at fill, and
    # the most crowded (particles per cell: in the lane mode a cell's chain
    # grows as N^2, so it is the run a static split waits for)
    order = np.argsort(counts)
    ppc = counts / np.array([r.n_cells for r in wl.runs], float)
    sample = [int(order[0]), int(order[R // 3]), int(order[2 * R // 3]), int(order[-1])]
    if int(np.argmax(ppc)) not in sample:
        sample.append(int(np.argmax(ppc)))
    runs_beta = []
    for r in sample:
        one = W.Workload("one", [wl.runs[r]], wl.n_steps, wl.sample_steps, 1)
        E = P.Ensemble.from_workload(one, sched=1, **kw)
        E.step(FILL_STEPS)
        ck1 = E.checkpoint()
        E.close()
        units, times = [], []
        for G in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024):
            E = P.Ensemble.from_workload(one, sched=1, sched_blocks=G, **kw)
            E.restore(ck1)
            E.step(1)
            units.append(G * wpb)
            times.append(interaction_ms(E, 3))
            E.close()
        fit = amdahl_fit(units, times)
        runs_beta.append({"run": r, "particles": int(counts[r]), "cells": wl.runs[r].n_cells,
                          "beta": fit["beta"], "overhead_per_wavefront": fit["overhead"],
                          "wavefronts": units, "ms": [round(t, 4) for t in times]})
    beta = float(np.mean([b["beta"] for b in runs_beta]))
    rows = []
    t_static_1 = None
    for p2 in (1, 2, 4, 8):
        row = {"p2": p2}
        for name, sched in (("static", 2), ("dynamic", 1)):
            E = P.Ensemble.from_workload(wl, sched=sched, sched_blocks=max(1, p2 * R // wpb), **kw)
            E.restore(ck)
            E.step(1)
            row[name + "_ms"] = round(interaction_ms(E, 3), 4)
            E.close()
        if t_static_1 is None:
            t_static_1 = row["static_ms"]
        pri = beta / (1 - beta) * (p2 - 1) if beta < 1 else 0.0
        row.update({"S_static": round(t_static_1 / row["static_ms"], 3),
                    "S_dynamic": round(t_static_1 / row["dynamic_ms"], 3),
                    "eq11_PRI0": round(1 / (beta + (1 - beta) / p2), 3),
                    "PRI_star_eq13": round(pri, 3),
                    "eq11_PRI_star": round(1 / (beta + (1 - beta) / (p2 * (1 + pri))), 3)})
        rows.append(row)
    E = P.Ensemble.from_workload(wl, sched=0, **kw)
    E.restore(ck)
    E.step(1)
    grid_ms = interaction_ms(E, 3)
    E.close()
    return {"workload": "uneven, 256 runs after %d steps from vacuum, every run a lane per cell" % FILL_STEPS,
            "runs": R, "processors": "wavefronts of the persistent lane-per-cell Interaction grid",
            "beta_sampled_runs": runs_beta, "beta_mean": beta, "p2_rows": rows,
            "hardware_grid_ms": round(grid_ms, 4)}


ORACLE_SEED = 1003   # the oracle's runs: same problem, seeds disjoint from the GPU batch's


def cpu_baseline(args):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    problem: `oracle_runs` runs of per_run particles for 20 steps (init
    included), one run per thread at a time on `threads` threads, sampled at
    step 20 into 32 run groups; and one run's steps on one thread (the
    per-core rate).  Returns (baseline, the oracle's sums at step 20)."""
    import oracle
    import workloads as W
    oracle.build(force=False)
    affinity = len(os.sched_getaffinity(0))
    threads = max(1, min(16, affinity))
    # one thread: one run for 1 and for k steps (init included in both), k
    # giving about 2e7 particle-steps
    k = max(3, -(-20_000_000 // args.per_run))
    wl1 = W.ensemble_box(n_runs=1, n_per_run=args.per_run, n_steps=k, sample_every=1000, seed=ORACLE_SEED)
    t0 = time.perf_counter()
    oracle.ensemble(wl1, n_threads=1, n_steps=1)
    t1 = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.ensemble(wl1, n_threads=1, n_steps=k)
    tk = time.perf_counter() - t0
    per_core = (k - 1) * args.per_run / max(tk - t1, 1e-6)
    steps = 20
    wl = W.ensemble_box(n_runs=args.oracle_runs, n_per_run=args.per_run, n_steps=steps, sample_every=20,
                        seed=ORACLE_SEED)
    t0 = time.perf_counter()
    acc, st = oracle.ensemble(wl, n_threads=threads, n_steps=steps)
    el = time.perf_counter() - t0
    base = {"value": st["particle_steps"] / el, "unit": "particle-steps/s", "cores": st["threads"],
            "kind": "oracle", "affinity_cpus": affinity, "per_core_value": per_core,
            "sample": f"{args.oracle_runs} runs x {args.per_run} particles x {steps} steps of the same box "
                      f"problem (init included), {st['threads']} threads, one run per thread at a time, "
                      f"{el:.1f} s; per_core_value: one run's steps 2-{k} on one thread"}
    return base, {"acc": acc[0], "runs": args.oracle_runs, "step": st["sample_steps"][0]}


def oracle_match(gpu, ora, rs):
    """Per macroparameter (n, ux, uy, T): z = (GPU - oracle) / combined
    batch-means standard error over the cells, the fraction of |z| > 3, the
    mean z and the largest relative error (velocities relative to the thermal
    speed sqrt(3T)); against the oracle's ensemble and against the exact
    equilibrium (n = N/cells per run, zero velocity, the gas's T)."""
    import math
    import numpy as np
    import oracle
    acc = ora["acc"]                                   # [groups][cell][7]
    G = acc.shape[0]
    mo = oracle.moments(acc.sum(axis=0), ora["runs"])
    per = oracle.moments(acc, ora["runs"] // G)
    so = per.std(axis=0, ddof=1) / math.sqrt(G)
    mg, sg, tot = gpu["m"], gpu["se"], gpu["tot"]
    u_all = tot[1:4] / tot[0]
    T_all = ((tot[4] + tot[5] + tot[6]) / tot[0] - float(u_all @ u_all)) / 3.0
    exact = {0: rs.n_init / rs.n_cells, 1: 0.0, 2: 0.0, 4: T_all}
    scale = {0: exact[0], 1: math.sqrt(3 * T_all), 2: math.sqrt(3 * T_all), 4: T_all}
    out = {}
    for f, name in ((0, "n"), (1, "ux"), (2, "uy"), (4, "T")):
        z = (mg[:, f] - mo[:, f]) / np.sqrt(sg[:, f] ** 2 + so[:, f] ** 2)
        ze = (mg[:, f] - exact[f]) / sg[:, f]
        rel = np.abs(mg[:, f] - mo[:, f]) / scale[f]
        out[name] = {"max_abs_z": round(float(np.max(np.abs(z))), 3),
                     "frac_abs_z_gt_3": round(float(np.mean(np.abs(z) > 3)), 5),
                     "mean_z": round(float(np.mean(z)), 4),
                     "max_rel_err": float(rel.max()),
                     "frac_cells_within_1pct": round(float(np.mean(rel < 0.01)), 5),
                     "median_3se_comb_rel": float(np.median(3 * np.sqrt(sg[:, f] ** 2 + so[:, f] ** 2)) / scale[f]),
                     "vs_exact_max_abs_z": round(float(np.max(np.abs(ze))), 3),
                     "vs_exact_max_rel_err": float(np.max(np.abs(mg[:, f] - exact[f])) / scale[f])}
    return {"step": gpu["step"], "gpu_runs": gpu["runs"], "gpu_groups": gpu["groups"],
            "oracle_runs": ora["runs"], "oracle_groups": G, "cells": int(mg.shape[0]),
            "fields": out, "max_frac_abs_z_gt_3": max(out[k]["frac_abs_z_gt_3"] for k in out),
            "vs_exact_all_within_1pct": bool(all(out[k]["vs_exact_max_rel_err"] < 0.01 for k in out)),
            "note": "GPU: FP32 state, FP64 accumulators and division; oracle: FP64 throughout, "
                    "independent seeds; standard errors from run groups (batch means)"}


def _json_safe(x):
    """The line as strict JSON: non-finite numbers become null."""
    import math
    if isinstance(x, dict):
        return {k: _json_safe(v) for k, v in x.items()}
    if isinstance(x, (list, tuple)):
        return [_json_safe(v) for v in x]
    if isinstance(x, float) and not math.isfinite(x):
        return None
    return x


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--runs", type=int, default=512)
    ap.add_argument("--per-run", type=int, default=1_000_000)
    ap.add_argument("--prof-steps", type=int, default=5)
    ap.add_argument("--streams", type=int, default=0,
                    help="run groups stepped concurrently (0 = the library's choice; with --no-tune)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner; use --streams / --tile-chunks / --collide-mode (0 = default)")
    ap.add_argument("--tile-chunks", type=int, default=0)
    ap.add_argument("--workload", choices=("ensemble_box", "body3d", "channel", "uneven"), default="ensemble_box",
                    help="ensemble_box (the benchmark); body3d, channel or uneven (informational)")
    ap.add_argument("--collide-mode", type=int, default=0,
                    help="interaction work item: 0 auto, 1 a lane per cell, 2 a block per cell, "
                         "3 a wavefront per cell")
    ap.add_argument("--sched", type=int, default=0,
                    help="Interaction work distribution (with --no-tune): 0 a workgroup per item, 1 a "
                         "persistent grid drawing from a queue shared by all runs, 2 workgroups tied to runs")
    ap.add_argument("--sched-blocks", type=int, default=0,
                    help="workgroups of each persistent grid (0 = as many as fit)")
    ap.add_argument("--tune-cache", default=None,
                    help="file of earlier autotune results to reuse and extend (default: none, always time)")
    ap.add_argument("--balance", action="store_true",
                    help="with --workload uneven: also run the static vs dynamic allocation experiment")
    ap.add_argument("--plain-runs", type=int, default=2)
    ap.add_argument("--plain-steps", type=int, default=10)
    ap.add_argument("--oracle-runs", type=int, default=128,
                    help="runs of the oracle leg (20 steps each), a multiple of 32")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(runs would shard across GPUs, with one final reduction of the accumulators)",
              file=sys.stderr)
        sys.exit(2)

    g = run_gpu(args)
    balance = balance_experiment(args) if (args.balance and args.workload == "uneven") else None
    cpu = match = None
    if not args.no_cpu_baseline and args.workload == "ensemble_box":
        cpu, ora = cpu_baseline(args)
        if g["match_gpu"] is not None and ora["step"] == g["match_gpu"]["step"]:
            import workloads as W
            match = oracle_match(g["match_gpu"], ora, W.ensemble_box(n_runs=1, n_per_run=args.per_run).runs[0])
    ms_per_step = g["elapsed"] / args.steps * 1e3
    line = {
        "metric": METRIC,
        "value": g["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": g["warmup"],
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[args.workload].format(runs=g["n_runs"], per_run=args.per_run),
                   "runs": g["n_runs"],
                   "particles_per_run": args.per_run if args.workload == "ensemble_box" else None,
                   "mean_particles": g["n_mean"],
                   "cells_per_run": g["nc"], "lanes": g["info"]["lanes"],
                   "tile_slots": g["info"]["slots"] // g["info"]["tiles"], "tuned": g["tuned"],
                   "parallelism": "one GPU; runs batched in each launch, split into "
                                  f"{g['info']['lanes']} concurrent stream lanes"},
        "roofline": g["roofline"],
        "roofline_as_built": g["rl_built"],
        "step_bytes": g["step_bytes"],
        "cpu_baseline": cpu,
        "oracle_match": match,
        "accumulator_precision": g["acc_prec"],
        "paper_figures": PAPER_FIGURES,
        "plain_fp64": g["plain"],
        "batched_over_plain": (g["value"] / g["plain"]["value"]) if g["plain"] else None,
        "kernels": g["kernels"],
        "stream_copy": g["calib"],
    }
    if balance is not None:
        line["balance"] = balance
    print(json.dumps(_json_safe(line)))


if __name__ == "__main__":
    main()
