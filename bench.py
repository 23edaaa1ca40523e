#!/usr/bin/env python3
"""Throughput of the RK4 block stage loop on one MI355X.

Workload: a fixed, seeded random 2:1-balanced periodic octree on [0, 2 pi]^3
(levels 3..7, >= 20000 blocks of 24^3 interior points, 4 ghost layers), seeded
smooth random-Fourier velocity and pressure (16 modes per field, |k| <= 8),
nu 1e-2, C0 20, C_gamma 1, no mask, CFL 0.5 (time step recomputed on the GPU
every step).  A step is one classical RK4 step: 4 x (ghost synchronisation +
fused rhs/RK stage) plus the CFL time step.  The K timed steps are one
wacm_rk4_steps call (each step's CFL maximum is formed by the previous step's
last stage).  Inputs are resident in HBM before the timed region.

Metric: RK4 block-point updates/s = interior points x 4 stages / s.  The
primary line is the FP64 path; the FP32 path is reported beside it with its
speed-up.  The roofline object refers to the fused rhs + RK stage kernel: its
algorithmic bytes divided by its average duration, measured with HIP events
on the launch stream inside the timed region.  Algorithmic bytes are the
compulsory interior traffic of classical RK4 with 3 + 1 registers, 16 values
per interior point and stage (stage 1 reads U^n and writes the accumulator
and the next input, 12; stages 2 and 3 read the input, U^n and the
accumulator and write two registers, 20; stage 4 reads the input and the
accumulator and writes U^{n+1}, 12).  The implementation itself moves 12
(8, 16, 12, 12 for stages 1-4: only stage 2 writes a second register, which
with the stage-4 input gives U^{n+1}); `moved_min_bytes_per_launch` states
that figure, and `traffic` the bytes the hardware counters saw.

    python bench.py [--gpus 1] [--steps 50] [--warmup 5]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def build_case(target: int, seed: int):
    from paper_1912_05371_amd import cases
    return cases.random_octree(bs=24, ng=4, target=target, j0=3, jmax=7, seed=seed,
                               with_fields=False)


def run_gpu(case, dtype_code: int, steps: int, warmup: int, use_graph: bool, tune: bool,
            schedule=None, shipped: bool = True, write_tuned: str = ""):
    import torch

    from paper_1912_05371_amd import inputs, wacm

    g = wacm.Grid.from_case(case, dtype=dtype_code)
    slots, codes, levels = g.info()
    pool = g.pool()
    modes = inputs.fourier_modes(case_seed(case), 4, 16, 8, 1.0 / 16.0)
    # leaf i of the case is in pool slot i
    inputs.fourier_fill_device(pool, modes, case.bs, case.ng, case.L, case.lev, case.ix, case.iy,
                               case.iz, np.arange(case.nb))
    work = g.work()
    t_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    p = wacm.make_params(case.params)
    stream = torch.cuda.current_stream()
    trials = []
    if schedule:
        g.set_schedule(**schedule)
    elif write_tuned:
        # a careful search (longer calls, best of two passes) for the table
        # shipped with the package
        from paper_1912_05371_amd import autotune
        schedule, trials = autotune.tune(g, case.params, pool, steps=6, reps=2, use_cache=False,
                                         shipped=False)
        data = {}
        if os.path.exists(write_tuned):
            with open(write_tuned) as f:
                data = json.load(f)
        best_ms = min(ms for ms, _ in trials)
        data[autotune.workload_key(g)] = {"schedule": schedule, "ms_per_step": best_ms,
                                          "candidates": len(trials)}
        with open(write_tuned, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        log(f"  tuned schedule {schedule} written to {write_tuned}")
    elif tune:
        from paper_1912_05371_amd import autotune
        schedule, trials = autotune.tune(g, case.params, pool, steps=2, use_cache=False,
                                         shipped=shipped)
        log(f"  schedule {schedule} " + (f"(best of {len(trials)} timed)" if trials else
                                          "(the tuner's stored choice for this workload)"))
    schedule = g.get_schedule()
    g.rk4_steps(None, t_dev, dt_dev, pool, work, warmup, dt_mode=wacm.DT_CFL, _p=p)
    torch.cuda.synchronize()

    # timed region: K steps, kernel classes timed with events on the stream
    g.profile_enable(True)
    g.profile_read()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    g.rk4_steps(None, t_dev, dt_dev, pool, work, steps, dt_mode=wacm.DT_CFL, _p=p)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms_total = ev0.elapsed_time(ev1)
    kms, kn = g.profile_read()
    g.profile_enable(False)

    res = dict(ms_per_step=ms_total / steps, wall_s=wall, kernel_ms=kms.tolist(),
               kernel_launches=kn.tolist(), schedule=schedule,
               tuning=[[ms, s] for ms, s in trials])
    if use_graph:
        graph = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            g.rk4_steps(None, t_dev, dt_dev, pool, work, 1, dt_mode=wacm.DT_CFL, _p=p)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph):
            g.rk4_steps(None, t_dev, dt_dev, pool, work, steps, dt_mode=wacm.DT_CFL, _p=p)
        graph.replay()
        torch.cuda.synchronize()
        ev0.record()
        graph.replay()
        ev1.record()
        torch.cuda.synchronize()
        res["graph_ms_per_step"] = ev0.elapsed_time(ev1) / steps
    out = torch.zeros(10, dtype=torch.float64, device="cuda")
    g.diagnostics(case.params, float(t_dev.item()), pool, out)
    res["t_end"] = float(t_dev.item())
    res["dt_last"] = float(dt_dev.item())
    res["diag"] = out.cpu().tolist()
    res["finite"] = bool(np.isfinite(res["diag"]).all())
    del pool, work
    g.close()
    torch.cuda.empty_cache()
    return res


def fp32_error(case):
    """R23 on the benchmark workload: one CFL step in FP64 and one in FP32
    from the same state (the FP64 state rounded to FP32), max |U32 - U64| /
    max |U64| over the interiors of the 4-component state; outside the timed
    region, each precision with its shipped schedule."""
    import torch

    from paper_1912_05371_amd import autotune, inputs, wacm

    res = {}
    for name, code in (("f64", wacm.F64), ("f32", wacm.F32)):
        g = wacm.Grid.from_case(case, dtype=code)
        pool = g.pool() if name == "f64" else None
        if name == "f64":
            modes = inputs.fourier_modes(case_seed(case), 4, 16, 8, 1.0 / 16.0)
            inputs.fourier_fill_device(pool, modes, case.bs, case.ng, case.L, case.lev, case.ix,
                                       case.iy, case.iz, np.arange(case.nb))
            start = pool.float()  # the FP32 input: the FP64 state rounded
        else:
            pool = start
        autotune.tune(g, case.params, pool, steps=1, use_cache=False)
        work = g.work()
        t = torch.zeros(1, dtype=torch.float64, device="cuda")
        dt = torch.zeros(1, dtype=torch.float64, device="cuda")
        g.rk4_steps(case.params, t, dt, pool, work, 1, dt_mode=wacm.DT_CFL)
        torch.cuda.synchronize()
        I = slice(case.ng, case.ng + case.bs)
        res[name] = (pool[:case.nb, :, I, I, I].double() if name == "f32"
                     else pool[:case.nb, :, I, I, I].clone(), float(dt.item()))
        del work, pool, g
        torch.cuda.empty_cache()
    a, b = res["f64"][0], res["f32"][0]
    err = float((b - a).abs().max() / a.abs().max())
    return {"rel_err_one_step": err, "tolerance": 1e-5, "metric": "max|U32-U64|/max|U64| over "
            "interiors of (u,v,w,p) after one CFL step from the same state",
            "dt_f64": res["f64"][1], "dt_f32": res["f32"][1]}


def case_seed(case):
    return case.extra.get("seed", 12345)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage_kernel_traffic_random_octree_bs24.md")


def counter_traffic(dtype: str, schedule: dict):
    """HBM bytes per stage-kernel launch (FETCH_SIZE + WRITE_SIZE, scaled by
    the copy probe) from the committed counter summary, if it was taken with
    the current stage-kernel sources and this schedule; else None."""
    from paper_1912_05371_amd import profile_summary
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    # the tuning knobs; pen_split changes nothing without a mask or sponge
    key = ",".join(f"{k}={schedule[k]}" for k in sorted(schedule) if k != "pen_split")
    cur = profile_summary.stage_source_sha1()
    sha, inside = None, False
    for ln in lines:
        f = ln.split()
        if ln.strip() == "traffic-data":
            inside, sha = True, None
        elif ln.strip() == "end-traffic-data":
            inside = False
        elif inside and f and f[0] == "source_sha1":
            sha = f[1]
        elif inside and len(f) == 6 and f[0] == dtype and f[1] == key and sha == cur:
            return float(f[3]) + float(f[5])
    return None


def roofline(res, npts: int, es: int):
    stage_ms = res["kernel_ms"][2] / max(res["kernel_launches"][2], 1)
    bytes_per_launch = 16 * es * npts  # classical RK4, 3 + 1 registers: 12, 20, 20, 12 values
    achieved = bytes_per_launch / (stage_ms * 1e-3) / 1e9
    step_bytes = 64 * es * npts
    return {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": None,  # filled from the counter summary when it applies
        "kernel": "stage_kernel (fused rhs + RK4 stage)",
        "kernel_avg_ms": round(stage_ms, 4),
        "bytes_per_launch": bytes_per_launch,
        # interior bytes the implementation itself moves per launch (8, 16, 12, 12 values)
        "moved_min_bytes_per_launch": 12 * es * npts,
        "whole_step_frac": round(step_bytes / (res["ms_per_step"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                 4),
    }


def aux_timings(case):
    """Timings of the other hot-path calls, outside the timed region (FP64):
    on the benchmark grid the stand-alone ghost synchronisation, wavelet
    thresholding, diagnostics, time step and wavelet filtering of every
    block, each with its compulsory bytes and the fraction of the HBM peak
    they imply; on the adaptive plate case one
    full adaptive step (refine all, one RK4 step, coarsening passes until no
    block merges), by phase."""
    import torch

    from paper_1912_05371_amd import cases, inputs, wacm

    out = {}
    g = wacm.Grid.from_case(case, dtype=wacm.F64)
    pool = g.pool()
    modes = inputs.fourier_modes(case_seed(case), 4, 16, 8, 1.0 / 16.0)
    inputs.fourier_fill_device(pool, modes, case.bs, case.ng, case.L, case.lev, case.ix, case.iy,
                               case.iz, np.arange(case.nb))
    nb = g.nb
    dmax = torch.zeros(nb, dtype=torch.float64, device="cuda")
    mr = torch.zeros(nb, dtype=torch.float64, device="cuda")
    fl = torch.zeros(nb, dtype=torch.int8, device="cuda")
    diag = torch.zeros(10, dtype=torch.float64, device="cuda")
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    calls = {
        "sync_ghosts": lambda: g.sync_ghosts(pool),
        "threshold_blocks": lambda: g.threshold_blocks(case.params, 0.0, pool, 1e-3, True, dmax,
                                                       mr, fl),
        "diagnostics": lambda: g.diagnostics(case.params, 0.0, pool, diag),
        "compute_dt": lambda: g.compute_dt(case.params, pool, dt_dev),
        # in place, so every repetition filters already filtered blocks: the
        # same loads and stores each time
        "filter_blocks": lambda: g.filter_blocks(pool, -1),
    }
    # compulsory bytes per call (FP64): the ghost shell written once and its
    # sources read once; interiors read by the norm and detail passes; 4
    # values read per point; 3 velocity values read per point; every interior
    # value written plus the even lattice (a quarter of the padded rows of
    # every other plane) read
    es = 8
    npts = case.nb * case.bs ** 3
    P = case.bs + 2 * case.ng
    shell = case.nb * (P ** 3 - case.bs ** 3)
    even = case.nb * (case.bs // 2 + 3) ** 2 * P
    algo = {"sync_ghosts": 2 * shell * 4 * es, "threshold_blocks": 8 * npts * es,
            "diagnostics": 4 * npts * es, "compute_dt": 3 * npts * es,
            "filter_blocks": (4 * npts + 4 * even) * es}
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    roof = {}
    for name, fn in calls.items():
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(3):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 3
        out[name + "_ms"] = round(ms, 4)
        gbs = algo[name] / (ms * 1e-3) / 1e9
        roof[name] = {"bytes": algo[name], "GBps": round(gbs, 1),
                      "frac": round(gbs / HBM_PEAK_GBS, 4)}
    out["roofline"] = roof
    del pool
    g.close()
    torch.cuda.empty_cache()

    out["cdf44"] = lifting_timings(case_seed(case))
    out["mr_transform"] = mr_timings(case_seed(case))

    # one adaptive step of the rotating plate (levels 2..6, bs 16)
    from paper_1912_05371_amd.adaptive import adaptive_step
    c = cases.plate_adaptive()
    eps, dealias = c.extra["eps"], c.extra["dealias"]
    ga = wacm.Grid.from_case(c, dtype=wacm.F64, capacity=10 * c.nb + 64)
    U = ga.pool()
    U[: c.nb].copy_(torch.from_numpy(c.padded()))
    work = ga.work()
    t_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    # the first step from the start grid, then 3 steps from the adapted grid,
    # each phase synchronised and split into host and device time
    steps = []
    for i in range(4):
        ph = {}
        nb0 = ga.nb
        r = adaptive_step(ga, c.params, U, work, t_dev, dt_dev, eps, dealias, timings=ph)
        steps.append((nb0, r, ph))
    out["adaptive_plate_step"] = {
        "first": _adaptive_record(*steps[0], 1),
        "steady_mean_of_3": _adaptive_record(steps[1][0], steps[3][1],
                                             _sum_phases([s[2] for s in steps[1:]]), 3)}
    del U, work
    ga.close()
    torch.cuda.empty_cache()
    return out


def _sum_phases(phs):
    tot = {}
    for ph in phs:
        for k, v in ph.items():
            rec = tot.setdefault(k, {"wall": 0.0, "host": 0.0, "device": 0.0})
            for q in rec:
                rec[q] += v[q]
    return tot


def _adaptive_record(nb0, r, ph, nsteps):
    """Per-phase wall / host / device ms (mean over nsteps adaptive steps) and
    the host share of the step's wall time."""
    wall = sum(v["wall"] for v in ph.values())
    host = sum(v["host"] for v in ph.values())
    return {"blocks": [nb0, r["refined"], r["blocks"]], "merging_passes": r["merged_passes"],
            "ms_by_phase": {k: {q: round(x / nsteps, 3) for q, x in v.items()}
                            for k, v in ph.items()},
            "wall_ms": round(wall / nsteps, 3), "host_ms": round(host / nsteps, 3),
            "host_share": round(host / wall, 3) if wall > 0 else None}


def c3_run(nsteps: int = 200, every: int = 10):
    """The rotating-plate adaptive case as configured (levels 2..6, bs 16, 4
    ghost layers, eps 1e-3 on the max-norm details, dealiasing, adapt every
    step): FP64 runs free (its own coarsening flags, CFL time step), FP32
    follows it in lockstep -- the same time steps and FP64's flags in every
    merge pass (replay), its own flags computed and counted where they
    differ.  Per step: block counts, FP32-vs-FP64 relative interior
    difference (drift, not gated), own-flag disagreements.  Host wall time
    per phase of the FP64 run."""
    import torch

    from paper_1912_05371_amd import cases, wacm

    c = cases.plate_adaptive()
    eps, dealias = c.extra["eps"], c.extra["dealias"]
    cap = 40000  # refine-all of the largest grid of the run must fit
    grids = {k: wacm.Grid.from_case(c, dtype=d, capacity=cap)
             for k, d in (("f64", wacm.F64), ("f32", wacm.F32))}
    pools, works = {}, {}
    for k, g in grids.items():
        pools[k] = g.pool()
        pools[k][:c.nb] = torch.from_numpy(c.padded()).to("cuda", g.torch_dtype())
        works[k] = None
    t64 = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt64 = torch.zeros(1, dtype=torch.float64, device="cuda")
    t32 = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt32 = torch.zeros(1, dtype=torch.float64, device="cuda")
    I = slice(c.ng, c.ng + c.bs)
    recs, phases = [], {}

    def timed(name, fn):
        # wall ms of the phase; host ms: for the adaptation calls the
        # library's host share, else the wall time outside the stream events
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0.record()
        r = fn()
        e1.record()
        torch.cuda.synchronize()
        w = (time.perf_counter() - t0) * 1e3
        dev = grids["f64"].adapt_timing()[1] if name in ("refine_all", "coarsen") else \
            min(e0.elapsed_time(e1), w)
        rec = phases.setdefault(name, {"wall": 0.0, "host": 0.0, "device": 0.0})
        rec["wall"] += w
        rec["device"] += dev
        rec["host"] += w - dev
        return r

    def flags_of(k, t):
        g, U = grids[k], pools[k]
        n = g.nb
        dm = torch.empty(n, dtype=torch.float64, device="cuda")
        mr = torch.empty(n, dtype=torch.float64, device="cuda")
        fl = torch.empty(n, dtype=torch.int8, device="cuda")
        g.sync_ghosts_lattice(U)
        g.threshold_blocks(c.params, t, U, eps, dealias, dm, mr, fl)
        return fl.cpu().numpy()

    wall0 = time.perf_counter()
    for step in range(nsteps):
        nb0 = grids["f64"].nb
        for k in grids:
            n = (timed if k == "f64" else (lambda _n, f: f()))(
                "refine_all", lambda: grids[k].adapt(wacm.REFINE_ALL, pools[k]))
            if works[k] is None or works[k].numel() < grids[k].work_bytes():
                works[k] = grids[k].work()
        nref = grids["f64"].nb
        timed("rk4_step", lambda: grids["f64"].rk4_step(c.params, t64, dt64, pools["f64"],
                                                        works["f64"], dt_mode=wacm.DT_CFL))
        dt32.copy_(dt64)
        grids["f32"].rk4_step(c.params, t32, dt32, pools["f32"], works["f32"],
                              dt_mode=wacm.DT_FIXED)
        t = float(t64.item())
        disagree, passes = 0, 0
        while True:
            a, b = grids["f64"].info(), grids["f32"].info()
            assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
            f64 = timed("sync_threshold", lambda: flags_of("f64", t))
            f32 = flags_of("f32", t)
            disagree += int(np.sum(f64 != f32))
            n = grids["f64"].nb
            if timed("coarsen", lambda: grids["f64"].adapt(wacm.COARSEN, pools["f64"], f64)) == n:
                grids["f32"].adapt(wacm.COARSEN, pools["f32"], f64)
                break
            grids["f32"].adapt(wacm.COARSEN, pools["f32"], f64)
            passes += 1
        s64 = torch.as_tensor(grids["f64"].info()[0], device="cuda")
        s32 = torch.as_tensor(grids["f32"].info()[0], device="cuda")
        A = pools["f64"][:, :, I, I, I].index_select(0, s64)
        B = pools["f32"][:, :, I, I, I].index_select(0, s32).double()
        drift = float((A - B).abs().max() / A.abs().max())
        recs.append({"step": step, "t": t, "dt": float(dt64.item()), "blocks": [nb0, nref,
                     grids["f64"].nb], "merge_passes": passes, "drift": drift,
                     "flag_disagreements": disagree})
        if step % every == 0 or step == nsteps - 1:
            log(f"  C3 step {step}: t {t:.5f} blocks {nb0}->{nref}->{grids['f64'].nb} "
                f"passes {passes} drift {drift:.2e} flag disagreements {disagree}")
    wall = time.perf_counter() - wall0
    nbs = [r["blocks"][2] for r in recs]
    return {"case": "rotating plate, levels 2-6, bs 16, ng 4, eps 1e-3, dealiasing",
            "steps": nsteps, "t_end": float(t64.item()), "wall_s": round(wall, 2),
            "blocks_min_max": [min(nbs), max(nbs)],
            "refined_max": max(r["blocks"][1] for r in recs),
            "drift_max": max(r["drift"] for r in recs), "drift_end": recs[-1]["drift"],
            "flag_disagreements_total": sum(r["flag_disagreements"] for r in recs),
            "steps_with_disagreements": sum(1 for r in recs if r["flag_disagreements"]),
            "f64_ms_per_step_by_phase": {k: {q: round(x / nsteps, 3) for q, x in v.items()}
                                         for k, v in phases.items()},
            "f64_host_share": round(sum(v["host"] for v in phases.values()) /
                                    sum(v["wall"] for v in phases.values()), 3),
            "records": recs}


def small_configs_gpu():
    """The Taylor-Green (64 blocks, 10 steps) and two-level sphere (736 blocks,
    20 steps) configurations in full on the GPU, FP64 and FP32: one
    wacm_rk4_steps call of the configuration's step count, HIP events on the
    launch stream, median of 5 repetitions from the same initial state."""
    import torch

    from paper_1912_05371_amd import cases, wacm

    out = {}
    for name, mk in (("taylor_green_64blocks_10steps", cases.taylor_green),
                     ("sphere_two_level_736blocks_20steps", cases.sphere_two_level)):
        c = mk()
        npts = c.nb * c.bs ** 3
        rec = {"blocks": c.nb, "steps": c.steps, "interior_points": npts}
        for dname, code in (("f64", wacm.F64), ("f32", wacm.F32)):
            g = wacm.Grid.from_case(c, dtype=code)
            U0 = g.pool()
            U0[:c.nb] = torch.from_numpy(c.padded()).to("cuda", g.torch_dtype())
            U = U0.clone()
            work = g.work()
            t = torch.zeros(1, dtype=torch.float64, device="cuda")
            dt = torch.zeros(1, dtype=torch.float64, device="cuda")
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            times = []
            for rep in range(6):
                U.copy_(U0)
                t.zero_()
                torch.cuda.synchronize()
                e0.record()
                g.rk4_steps(c.params, t, dt, U, work, c.steps, dt_mode=wacm.DT_CFL)
                e1.record()
                torch.cuda.synchronize()
                if rep:
                    times.append(e0.elapsed_time(e1) / c.steps)
            ms = float(np.median(times))
            rec[dname] = {"ms_per_step": round(ms, 4),
                          "updates_per_s": round(npts * 4 / (ms * 1e-3), 1)}
            del U, U0, work, g
        out[name] = rec
    torch.cuda.empty_cache()
    return out


def _lattice_of(g, pool, N):
    """Interior values of a 2D pool assembled into N x N lattice arrays
    ([c][y, x]) at the points the grid holds (NaN elsewhere)."""
    slots, codes, levels = g.info()
    out = np.full((3, N, N), np.nan)
    bs = g.bs
    P = pool[:, :, g.ng:g.ng + bs, g.ng:g.ng + bs].double().cpu().numpy()
    from paper_1912_05371_amd import wacm
    for s, code, J in zip(slots, codes, levels):
        bx, by, _ = wacm.treecode_decode(int(code), int(J))
        st = N // ((1 << int(J)) * bs)
        gx = (bx * bs + np.arange(bs)) * st
        gy = (by * bs + np.arange(bs)) * st
        out[:, gy[:, None], gx[None, :]] = P[s]
    return out


def vortex_study(T_eq: float = 1.0, T_ad: float = 0.5):
    """The three vortices in two dimensions on the GPU.

    Self-convergence of the equidistant runs: levels J = 3..6 (N = 128..1024
    points per axis, blocks of 16^2), all with the time step of the finest
    (CFL 0.5 at N = 1024), to t = T_eq; the error of each run is the max-norm
    difference of (u, v) from the finest run at its own points, relative to
    the finest field's max norm, and the observed order log2(e_N / e_2N).

    Thresholding error of adaptive runs (refine, step, coarsen every step,
    CDF 4/0): Jmax = 4 (N = 256), eps = 1e-2 .. 1e-6, the start grid obtained
    by coarsening the uniform level-4 initial field until no family merges;
    error against the equidistant level-4 run with the same time step, at the
    adaptive grid's points, to t = T_ad.  Without dealiasing the error is the
    thresholding error alone and vanishes with eps; with dealiasing every
    level-4 block is coarsened after each step, so the runs approach the
    level-4 evolution of level-3 data instead."""
    import torch

    from paper_1912_05371_amd import cases, wacm
    from paper_1912_05371_amd.adaptive import adaptive_step

    prm = cases.three_vortex_params()
    p = wacm.make_params(prm)

    def uniform_run(J, dt, T):
        c = cases.three_vortices(bs=16, ng=4, J=J)
        g = wacm.Grid.from_case(c, dtype=wacm.F64)
        U = g.pool()
        U[:c.nb] = torch.from_numpy(c.padded()).cuda()
        work = g.work()
        t = torch.zeros(1, dtype=torch.float64, device="cuda")
        dtd = torch.tensor([dt], dtype=torch.float64, device="cuda")
        n = int(math.ceil(T / dt - 1e-9))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.rk4_steps(None, t, dtd, U, work, n, dt_mode=wacm.DT_FIXED, _p=p)
        e1.record()
        torch.cuda.synchronize()
        lat = _lattice_of(g, U, (1 << J) * 16)
        return lat, n, e0.elapsed_time(e1) / n, c.nb

    # the finest run's CFL time step
    cf = cases.three_vortices(bs=16, ng=4, J=6)
    gf = wacm.Grid.from_case(cf, dtype=wacm.F64)
    Uf = gf.pool()
    Uf[:cf.nb] = torch.from_numpy(cf.padded()).cuda()
    dtt = torch.zeros(1, dtype=torch.float64, device="cuda")
    gf.compute_dt(prm, Uf, dtt)
    dt_f = float(dtt.item())
    del Uf, gf
    runs = {}
    for J in (6, 5, 4, 3):
        lat, n, ms, nb = uniform_run(J, dt_f, T_eq)
        runs[J] = lat
        log(f"  vortices level {J} ({nb} blocks): {n} steps, {ms:.3f} ms/step")
    ref = runs[6]
    scale = np.max(np.abs(ref[:2]))
    eq = []
    for J in (3, 4, 5):
        st = 1 << (6 - J)
        e = float(np.max(np.abs(runs[J][:2] - ref[:2, ::st, ::st])) / scale)
        eq.append({"level": J, "N": (1 << J) * 16, "rel_err_vs_N1024": e})
    for a, b in zip(eq, eq[1:]):
        a["order_to_next"] = round(math.log2(a["rel_err_vs_N1024"] / b["rel_err_vs_N1024"]), 3)

    # thresholding error
    jmax = 4
    c4 = cases.three_vortices(bs=16, ng=4, J=jmax)
    g4 = wacm.Grid.from_case(c4, dtype=wacm.F64)
    U4 = g4.pool()
    U4[:c4.nb] = torch.from_numpy(c4.padded()).cuda()
    g4.compute_dt(prm, U4, dtt)
    dt4 = float(dtt.item())
    del U4, g4
    ref4, n4, _, _ = uniform_run(jmax, dt4, T_ad)
    scale4 = np.max(np.abs(ref4[:2]))
    ad = {False: [], True: []}
    for dealias, eps in [(d, e) for d in (False, True) for e in (1e-2, 1e-3, 1e-4, 1e-5, 1e-6)]:
        c = cases.three_vortices(bs=16, ng=4, J=jmax)
        c.jmin = 1
        # refine-all holds a grid's blocks and their children at once
        g = wacm.Grid.from_case(c, dtype=wacm.F64, capacity=2 * c.nb)
        U = g.pool()
        U[:c.nb] = torch.from_numpy(c.padded()).cuda()
        # start grid: coarsen the fully resolved initial field
        for _ in range(8):
            n0 = g.nb
            dm = torch.empty(n0, dtype=torch.float64, device="cuda")
            mr = torch.empty(n0, dtype=torch.float64, device="cuda")
            fl = torch.empty(n0, dtype=torch.int8, device="cuda")
            g.sync_ghosts(U)
            g.threshold_blocks(prm, 0.0, U, eps, False, dm, mr, fl)
            if g.adapt(wacm.COARSEN, U, fl.cpu().numpy()) == n0:
                break
        nb_start = g.nb
        work = g.work()
        t = torch.zeros(1, dtype=torch.float64, device="cuda")
        dtd = torch.tensor([dt4], dtype=torch.float64, device="cuda")
        nbs = []
        wall0 = time.perf_counter()
        for _ in range(n4):
            adaptive_step(g, prm, U, work, t, dtd, eps, dealias, dt_mode=wacm.DT_FIXED)
            nbs.append(g.nb)
        wall = time.perf_counter() - wall0
        lat = _lattice_of(g, U, (1 << jmax) * 16)
        m = ~np.isnan(lat[0])
        e = float(np.max(np.abs(lat[:2][:, m] - ref4[:2][:, m])) / scale4)
        ad[dealias].append({"eps": eps, "rel_err_vs_equidistant": e, "blocks_start": nb_start,
                   "blocks_mean": round(float(np.mean(nbs)), 1), "blocks_end": nbs[-1],
                   "grid_fraction_end": round(nbs[-1] * 16 * 16 / float((1 << jmax) * 16) ** 2,
                                              4),
                   "steps": n4, "ms_per_adaptive_step": round(wall / n4 * 1e3, 3)})
        log(f"  adaptive eps {eps:g} dealias {dealias}: {nb_start} -> {nbs[-1]} blocks, "
            f"rel err {e:.3e}")
        del U, work, g
    torch.cuda.empty_cache()
    return {"case": "three Gaussian vortices, [0,2pi)^2, nu 5e-5, C0 10, C_gamma 1, FP64, "
                    "blocks of 16^2, CDF 4/0",
            "equidistant": {"t_end": T_eq, "dt": dt_f, "runs": eq},
            "adaptive": {"t_end": T_ad, "dt": dt4, "jmax": jmax, "runs": ad[False],
                         "runs_dealias": ad[True]}}


def lifting_timings(seed: int):
    """CDF 4/4 (lifted restriction) on a random octree with 6 ghost layers
    (bs 24, levels 3-6, ~4000 blocks, FP64): the full ghost sync with CDF 4/0
    and with CDF 4/4 (the lifted phase on top), and one RK4 step with each
    (CDF 4/4: per stage the ghost fill of what the stage and the face-star
    lifted values read, the lifted face star, and the fused stage)."""
    import torch

    from paper_1912_05371_amd import cases, inputs, wacm

    c = cases.random_octree(bs=24, ng=6, target=4000, j0=3, jmax=6, seed=seed,
                            with_fields=False)
    g = wacm.Grid.from_case(c, dtype=wacm.F64)
    pool = g.pool()
    modes = inputs.fourier_modes(seed, 4, 16, 8, 1.0 / 16.0)
    inputs.fourier_fill_device(pool, modes, c.bs, c.ng, c.L, c.lev, c.ix, c.iy, c.iz,
                               np.arange(c.nb))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return round(e0.elapsed_time(e1) / reps, 3)

    out = {"blocks": c.nb, "sync_cdf40_ms": timed(lambda: g.sync_ghosts(pool))}
    work = g.work()
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    out["rk4_step_cdf40_ms"] = timed(
        lambda: g.rk4_step(c.params, t, dt, pool, work, dt_mode=wacm.DT_CFL), reps=2)
    del work
    g.set_wavelet(wacm.CDF44)
    out["sync_cdf44_ms"] = timed(lambda: g.sync_ghosts(pool))
    work = g.work()
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    out["rk4_step_cdf44_ms"] = timed(
        lambda: g.rk4_step(c.params, t, dt, pool, work, dt_mode=wacm.DT_CFL), reps=2)
    del work, pool
    g.close()
    torch.cuda.empty_cache()
    return out


def mr_timings(seed: int, n: int = 256, nf: int = 4, nlev: int = 5):
    """Multiresolution transform of the equidistant lattice (n^3 points, nf
    fields, nlev levels, periodic; FP64, then FP32 under keys ending in
    _f32): forward and inverse with CDF 4/0 and CDF 4/4, each with the
    compulsory bytes (every lattice value of a
    level read once and its changed values written once: 7/8 of them with
    CDF 4/0, all with CDF 4/4) and the fraction of the HBM peak they imply."""
    import torch

    from paper_1912_05371_amd import wacm

    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    pts = sum((n >> m) ** 3 for m in range(nlev)) * nf
    out = {"n": n, "fields": nf, "levels": nlev, "dtypes": ["f64", "f32 (keys ending in _f32)"]}
    for tdt, es, suffix in ((torch.float64, 8, ""), (torch.float32, 4, "_f32")):
        u = torch.randn((nf, n, n, n), dtype=tdt, device="cuda", generator=g)
        work = wacm.mr_work(u)
        for wname, wav, wfrac in (("cdf40", wacm.CDF40, 7 / 8), ("cdf44", wacm.CDF44, 1.0)):
            nbytes = int(pts * (1 + wfrac) * es)
            for dname, fn in (("forward", wacm.mr_forward), ("inverse", wacm.mr_inverse)):
                fn(u, nlev, wav, work)
                torch.cuda.synchronize()
                e0.record()
                reps = 5
                for _ in range(reps):
                    fn(u, nlev, wav, work)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                gbs = nbytes / (ms * 1e-3) / 1e9
                out[f"{wname}_{dname}{suffix}"] = {"ms": round(ms, 4), "bytes": nbytes,
                                                   "GBps": round(gbs, 1),
                                                   "frac": round(gbs / HBM_PEAK_GBS, 4)}
        del u, work
        torch.cuda.empty_cache()
    return out


def copy_probe(gib: float):
    """Bandwidth of a plain streaming kernel (torch.neg: read and write `gib`
    GiB once each): the achievable rate, and the reference for scaling the
    traffic counters (its FETCH_SIZE / WRITE_SIZE must read `gib` GiB)."""
    import torch
    n = int(gib * (1 << 30)) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    # torch.neg: a plain elementwise kernel that reads and writes n doubles once
    for _ in range(2):
        torch.neg(a, out=b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 10
    e0.record()
    for _ in range(reps):
        torch.neg(a, out=b)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    moved = 2 * n * 8
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_per_buffer": n * 8, "bytes_moved": moved, "ms": round(ms, 4),
            "GBps": round(moved / (ms * 1e-3) / 1e9, 1)}


def cpu_model() -> str:
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_sample(seed: int, min_seconds: float, target: int, j0: int, jmax: int):
    """RK4 steps (each with its CFL time step) of the FP64 oracle on a random
    octree of the benchmark's generator (bs 24, ng 4), repeated until
    `min_seconds` of wall time have passed: (updates/s, steps, seconds,
    blocks, interior points)."""
    from oracle import oracle
    from paper_1912_05371_amd import cases
    oracle.build(force=False)
    c = cases.random_octree(bs=24, ng=4, target=target, j0=j0, jmax=jmax, seed=seed)
    og = oracle.Grid(c.bs, c.ng, c.L, c.jmin, c.jmax, c.lev, c.ix, c.iy, c.iz)
    U = c.padded()
    t, n = 0.0, 0
    t0 = time.perf_counter()
    while True:
        dt = og.dt(c.params, U)
        og.rk4_step(c.params, t, dt, U)
        t += dt
        n += 1
        el = time.perf_counter() - t0
        if el >= min_seconds:
            break
    npts = c.nb * c.bs ** 3
    return npts * 4 * n / el, n, el, c.nb, npts


def oracle_configs():
    """The Taylor-Green (10 steps) and two-level sphere (20 steps)
    configurations in full with the FP64 oracle: updates/s and seconds."""
    from oracle import oracle
    from paper_1912_05371_amd import cases
    oracle.build(force=False)
    out = {}
    for name, mk in (("taylor_green_64blocks_10steps", cases.taylor_green),
                     ("sphere_two_level_736blocks_20steps", cases.sphere_two_level)):
        c = mk()
        og = oracle.Grid(c.bs, c.ng, c.L, c.jmin, c.jmax, c.lev, c.ix, c.iy, c.iz)
        U = c.padded()
        t = 0.0
        t0 = time.perf_counter()
        for _ in range(c.steps):
            dt = og.dt(c.params, U)
            og.rk4_step(c.params, t, dt, U)
            t += dt
        el = time.perf_counter() - t0
        npts = c.nb * c.bs ** 3
        out[name] = {"seconds": round(el, 3), "updates_per_s": round(npts * 4 * c.steps / el, 1)}
    return out


def _child_json(expr: str, threads: int) -> dict:
    """Evaluate `expr` (a call into this module) in a child Python process
    with OMP_NUM_THREADS=threads (the oracle's OpenMP team is fixed when it
    loads, so other thread counts need their own process)."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    code = f"import json, bench; print(json.dumps({expr}))"
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=900)
    if r.returncode != 0:
        raise RuntimeError(r.stderr[-2000:])
    return json.loads(r.stdout.strip().splitlines()[-1])


def cpu_baseline(seed: int, min_seconds: float = 10.0):
    """The FP64 oracle on the host cores: a bounded sample of the benchmark
    workload (a 603-block octree of the same generator, levels 2..4, RK4
    steps repeated for >= min_seconds) with every host core, the same sample
    on one core, and the Taylor-Green and sphere configurations in full (all
    cores; Taylor-Green also on one core)."""
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    rate, n, el, nb, npts = oracle_sample(seed, min_seconds, 600, 2, 4)
    one = _child_json(f"bench.oracle_sample({seed}, {min_seconds}, 600, 2, 4)", 1)
    cfg = _child_json("bench.oracle_configs()", threads)
    cfg1 = _child_json("bench.oracle_configs()['taylor_green_64blocks_10steps']", 1)
    cfg["taylor_green_64blocks_10steps"]["one_thread"] = cfg1
    return {
        "value": round(rate, 1),
        "unit": "block-point updates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"{n} RK4 steps (+CFL dt each) of the FP64 oracle on a {nb}-block random "
                  f"octree (bs 24, ng 4, levels 2-4, {npts} interior points), same generator; "
                  f"{el:.2f} s wall with OpenMP over blocks",
        "seconds": round(el, 3),
        "core_seconds_per_point_rhs": el * threads / (npts * 4 * n),
        "cpu_model": cpu_model(),
        "one_thread": {"value": round(one[0], 1), "steps": one[1], "seconds": round(one[2], 3),
                       "core_seconds_per_point_rhs": one[2] / (one[4] * 4 * one[1])},
        "configs": cfg,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--target", type=int, default=20000, help="minimum number of blocks")
    ap.add_argument("--seed", type=int, default=12345)
    ap.add_argument("--dtype", choices=["both", "f64", "f32"], default="both")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="keep the default schedule")
    ap.add_argument("--retune", action="store_true",
                    help="time all schedules even if the package ships a choice for this GPU")
    ap.add_argument("--write-tuned", default="",
                    help="search the schedules carefully and store the choice in this JSON file")
    ap.add_argument("--no-aux", action="store_true",
                    help="skip the timings of the other calls (sync, thresholding, adaptation)")
    ap.add_argument("--schedule", default="",
                    help="fixed stage-kernel schedule instead of tuning, e.g. "
                         "tile_rows=8,wg_per_cu=2,xcd_map=0,prefetch=0,nontemporal=1")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-probe", type=float, default=2.0,
                    help="GiB per buffer of a plain device copy timed for the achievable "
                         "bandwidth (0: skip)")
    ap.add_argument("--aux-only", action="store_true",
                    help="time only the other calls (the aux block) on the benchmark grid and "
                         "print them")
    ap.add_argument("--c3-run", type=int, default=0, metavar="STEPS",
                    help="run the adaptive rotating-plate case for STEPS steps (FP64 free, "
                         "FP32 replaying its flags) and print drift and flag disagreements")
    ap.add_argument("--vortex-study", action="store_true",
                    help="two-dimensional three-vortex runs: self-convergence of equidistant "
                         "runs and the thresholding error of adaptive runs")
    ap.add_argument("--mr-only", action="store_true",
                    help="time only the multiresolution transform (256^3 x 4, 5 levels) and "
                         "print its figures")
    ap.add_argument("--lifting-only", action="store_true",
                    help="time only the CDF 4/0 and CDF 4/4 syncs and RK4 steps on the "
                         "4012-block octree with 6 ghost layers and print them")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the block pool of this workload is resident on "
              "a single MI355X and no multi-GPU path is built (use --gpus 1).", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_1912_05371_amd import wacm

    wacm.lib()
    if args.c3_run:
        print(json.dumps({"c3_run": c3_run(args.c3_run)}), flush=True)
        return
    if args.vortex_study:
        print(json.dumps({"vortex_study": vortex_study()}), flush=True)
        return
    if args.mr_only:
        if args.copy_probe > 0:
            copy_probe(args.copy_probe)
        print(json.dumps({"mr_transform": mr_timings(args.seed)}), flush=True)
        return
    if args.lifting_only:
        if args.copy_probe > 0:
            copy_probe(args.copy_probe)
        print(json.dumps({"cdf44": lifting_timings(args.seed)}), flush=True)
        return
    t0 = time.perf_counter()
    case = build_case(args.target, args.seed)
    case.extra["seed"] = args.seed
    npts = case.nb * case.bs ** 3
    levels = {int(l): int(n) for l, n in zip(*np.unique(case.lev, return_counts=True))}
    log(f"workload: {case.nb} blocks {levels}, {npts} interior points "
        f"(generated in {time.perf_counter() - t0:.1f} s)")

    if args.aux_only:
        print(json.dumps({"aux": aux_timings(case)}), flush=True)
        return
    copy = copy_probe(args.copy_probe) if args.copy_probe > 0 else None
    if copy:
        log(f"copy probe: {copy['bytes_moved'] / 1e9:.2f} GB moved at {copy['GBps']:.0f} GB/s")
    results = {}
    for name, code, es in (("f64", wacm.F64, 8), ("f32", wacm.F32, 4)):
        if args.dtype not in ("both", name):
            continue
        log(f"running {name}: warmup {args.warmup}, steps {args.steps}")
        sched = dict((k, int(v)) for k, v in (kv.split("=") for kv in args.schedule.split(",")
                                               if kv)) or None
        r = run_gpu(case, code, args.steps, args.warmup, not args.no_graph, not args.no_tune,
                    sched, shipped=not args.retune, write_tuned=args.write_tuned)
        r["value"] = npts * 4 / (r["ms_per_step"] * 1e-3)
        r["roofline"] = roofline(r, npts, es)
        tb = counter_traffic(name, r["schedule"])
        if tb is not None:
            # bytes per launch, like bytes_per_launch
            r["roofline"]["traffic"] = int(round(tb))
            r["roofline"]["traffic_over_algorithmic"] = round(
                tb / r["roofline"]["bytes_per_launch"], 3)
        log(f"  {name}: {r['ms_per_step']:.3f} ms/step, {r['value']:.4e} updates/s, stage kernel "
            f"{r['roofline']['kernel_avg_ms']:.3f} ms = {r['roofline']['achieved']:.0f} GB/s "
            f"({100 * r['roofline']['frac']:.1f} %), graph {r.get('graph_ms_per_step', 0):.3f} "
            f"ms/step, kernels {r['kernel_ms']} ms / {r['kernel_launches']}")
        results[name] = r

    prim = "f64" if "f64" in results else "f32"
    R = results[prim]
    line = {
        "metric": "RK4 block-point updates/s",
        "value": round(R["value"], 1),
        "unit": "block-point updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(R["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prim,
        "data": "synthetic",
        "config": {
            "workload": f"random_octree_bs24_ng4_L3-7_{case.nb}blocks",
            "blocks": case.nb,
            "levels": levels,
            "bs": case.bs,
            "ng": case.ng,
            "interior_points": npts,
            "dt": "CFL 0.5 on device every step",
        },
        "roofline": R["roofline"],
    }
    if "graph_ms_per_step" in R:
        line["graph_ms_per_step"] = round(R["graph_ms_per_step"], 4)
    line["schedule"] = R["schedule"]
    other = "f32" if prim == "f64" else None
    if other and other in results:
        O = results[other]
        line["f32"] = {
            "value": round(O["value"], 1),
            "ms_per_step": round(O["ms_per_step"], 4),
            "roofline": O["roofline"],
            "speedup_vs_f64": round(R["ms_per_step"] / O["ms_per_step"], 3),
            "graph_ms_per_step": round(O.get("graph_ms_per_step", 0.0), 4),
            "schedule": O["schedule"],
        }
    line["kernel_ms_per_step"] = {
        k: round(v / args.steps, 4)
        for k, v in zip(["dt", "face_halo", "stage", "time"], R["kernel_ms"])}
    if copy:
        line["copy_probe"] = copy
        line["roofline"]["frac_of_copy"] = round(R["roofline"]["achieved"] / copy["GBps"], 4)
    if "f64" in results and "f32" in results:
        log("FP32 against FP64 after one step")
        line["f32"]["error_vs_f64"] = fp32_error(case)
        log(f"  rel err {line['f32']['error_vs_f64']['rel_err_one_step']:.3e}")
    if not args.no_aux:
        log("timing the Taylor-Green and sphere configurations")
        line["configs_gpu"] = small_configs_gpu()
    if not args.no_aux and "f64" in results:
        log("timing the other calls")
        line["aux"] = aux_timings(case)
    if not args.no_cpu_baseline:
        log("timing the oracle on a sample")
        line["cpu_baseline"] = cpu_baseline(args.seed)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
