#!/usr/bin/env python3
"""Throughput of the MPC-SRD step on one MI355X.

Prints ONE JSON line.  `value` is FP64 particle-steps/s on the 512^3
periodic box with 10 particles per cell (1,342,177,280 particles, plain SRD:
rotation by 130 degrees, kT = 1, h = 0.1), inputs resident in HBM before the
timed region, `--steps` timed steps (100 by default) after `--warmup`.  The
same line carries:
  roofline     : the collide kernel (dominant) -- algorithmic bytes per launch
                 (particles x state bytes read + written once) / its average
                 duration from HIP events on the launch stream, against the
                 8 TB/s HBM peak and against the copy probe; `traffic` is the
                 HBM bytes per launch from rocprofv3 counter runs of this
                 same command, when they were taken on the current kernels;
  hbm_probe    : a plain copy kernel and a plain read kernel of the library on
                 a 4 GiB buffer -- the bandwidth a kernel attains on this machine;
  forms        : the split-FP32 form on the same 512^3 box from the same
                 initial state (throughput and drift next to FP64); the 256^3
                 box with the thermostat, reorder interval 20, in FP64, FP32
                 and split; the batched ensemble of 64 uneven boxes in FP64
                 and split (graphs of 50 steps); the angular-momentum-
                 conserving collision SRD+a (FP64, split).  More with --forms
                 (fp64_fixed, walls_slip, walls_couette, lees_edwards,
                 density50, features, reorder_sweep, c5);
  cpu_baseline : the single-threaded CPU oracle on a bounded sample of the
                 512^3 workload (with --cpu-configs also on the 16^3, 256^3,
                 64-box and channel workloads).
--copy-probe-gib G adds one torch device-to-device copy of G GiB before the
run: the counter runs use it to scale FETCH_SIZE / WRITE_SIZE to bytes.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                       # MI355X HBM3E peak, GB/s
STATE_BYTES = {"fp64": 48, "fp32": 24, "split": 28}   # stored bytes per particle
METRIC = "MPC particle-steps/s on 1 GPU + % HBM roofline, FP64 vs split-FP32 vs batched"
DEFAULT_FORMS = "split,c2_fp64,c2_fp32,c2_split,batched,batched_split,amc,amc_split,c5"


def log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("mpc_kernels.hip", "mpc_internal.h", "philox_dev.h"):
        with open(os.path.join(ROOT, "paper_2406_15236_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_record(form: str, workload: str, R: int):
    """HBM bytes per collide launch from committed rocprofv3 counter runs, if
    they were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "collide_hbm_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except OSError:
        return None
    r = rec.get(f"{workload}:{form}:R{R}")
    if not r or r.get("kernel_hash") != kernel_source_hash():
        return None
    return r


def run_box(mpc, torch, box, form: str, R: int, steps: int, warmup: int,
            profiled: bool = True, tune: bool = True, graph=True, init_seed: int = 2024):
    """Device-initialised state, autotuned tiling, `warmup` untimed steps, then
    `steps` timed steps (kernel by kernel with HIP events when profiled, else
    graph replays).  Returns (particles, wall seconds, kernel times or None,
    observables before, observables after)."""
    sim = mpc.Sim(box if isinstance(box, list) else [box], form=form, reorder_every=R,
                  graph=graph if not profiled else True)
    sim.init_state(init_seed)
    n = sum(sim.n(b) for b in range(len(sim.params)))
    tiling = None
    if tune:  # the library's autotuner picks the collide tiling (state restored after)
        sim.step(2)
        sim.autotune(3)
        tiling = sim.get_tiling()
        log(f"  autotuned {form}: {tiling}")
        sim.init_state(init_seed)
        sim.set_step(0)
    if warmup:
        sim.step(warmup) if not profiled else sim.step_profiled(warmup)
    o0 = sim.observables(0)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if profiled:
        kt = sim.step_profiled(steps)
    else:
        sim.step(steps)
        kt = None
    sim.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    o1 = sim.observables(0)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    run_box.last_tiling = tiling
    return n, wall, kt, o0, o1


def form_entry(workload: str, form: str, n: int, steps: int, wall: float, kt, extra=None):
    v = n * steps / wall
    e = {"workload": workload, "value": v, "unit": "particle-steps/s",
         "ms_per_step": wall * 1e3 / steps,
         "hbm_roofline_frac_step": v * 2 * STATE_BYTES[form] / (HBM_PEAK_GBS * 1e9),
         "launch": run_box.last_tiling}
    if kt is not None:
        c = kt.collide_ms / max(1, kt.collide_launches)
        gbs = n * 2 * STATE_BYTES[form] / (c * 1e-3) / 1e9
        e.update({"collide_ms": c, "collide_achieved_GBs": gbs,
                  "collide_roofline_frac": gbs / HBM_PEAK_GBS,
                  "scan_draws_ms": kt.scan_ms / steps, "scatter_ms": kt.scatter_ms / steps})
    if extra:
        e.update(extra)
    return e


def hbm_probe(mpc, torch, gib: float = 4.0, reps: int = 5):
    """The library's plain copy and read kernels on a `gib` GiB buffer, over
    several grid sizes: best of `reps` launches each, timed with HIP events on
    torch's stream; the fastest grid is reported."""
    nb = int(gib * 2 ** 30)
    src = torch.empty(nb, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    st = torch.cuda.current_stream().cuda_stream
    grids = (1024, 2048, 4096, 8192, 16384)
    out = torch.empty(max(grids) * 256 * 4, dtype=torch.uint8, device="cuda")
    res = {"bytes": nb}
    for name in ("copy", "read"):
        best, best_grid, per_grid = None, None, {}
        for grid in grids:
            g_best = None
            for r in range(reps + 1):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                if name == "copy":
                    mpc.probe_copy(dst.data_ptr(), src.data_ptr(), nb, grid, st)
                else:
                    mpc.probe_read(src.data_ptr(), nb, out.data_ptr(), out.numel(), grid, st)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1)
                if r and (g_best is None or ms < g_best):   # the first launch is a warm-up
                    g_best = ms
            per_grid[grid] = g_best
            if best is None or g_best < best:
                best, best_grid = g_best, grid
        moved = 2 * nb if name == "copy" else nb
        res[name] = {"ms": best, "GBs": moved / (best * 1e-3) / 1e9, "grid": best_grid,
                     "GBs_by_grid": {str(g): round(moved / (t * 1e-3) / 1e9, 1)
                                     for g, t in per_grid.items()}}
    del src, dst, out
    torch.cuda.empty_cache()
    log(f"[hbm probe] copy {res['copy']['GBs']:.0f} GB/s, read {res['read']['GBs']:.0f} GB/s")
    return res


def srd_viscosity(nc, kT, h, alpha, m=1.0, a=1.0):
    """Shear viscosity of 3D SRD with random grid shift (kinetic + collisional)."""
    c1, c2 = math.cos(alpha), math.cos(2 * alpha)
    f = nc - 1 + math.exp(-nc)
    return (nc * kT * h / a ** 3 * (5 * nc / (f * (4 - 2 * c1 - 2 * c2)) - 0.5)
            + m / (18 * a * h) * f * (1 - c1))


def run_c5(mpc, torch, synth, steps: int):
    """Poiseuille flow, 256 x 256 x 64 cells between no-slip walls, gravity
    1e-3 along x, thermostat, split form: throughput and the time-averaged
    profile v_x(z) against the parabola rho g z (H - z) / (2 eta)."""
    box = synth.config("C5")
    L = box["L"]
    H = L[2]
    sim = mpc.Sim(box, form="split", reorder_every=20, graph=50)
    sim.init_state(5)
    n = sim.n()
    nsnap, gap = 10, 200
    run = steps - nsnap * gap
    sim.step(2)
    sim.autotune(3)  # state and step restored by the tuner
    tiling = sim.get_tiling()
    sim.sync()
    t0 = time.perf_counter()
    done = 0
    while done < run - 2:
        k = min(2000, run - 2 - done)
        sim.step(k)
        sim.sync()
        done += k
        log(f"[C5] {done + 2} steps")
    wall = time.perf_counter() - t0
    acc = np.zeros(H)
    cnt = np.zeros(H)
    for _ in range(nsnap):
        sim.step(gap)
        x, v = sim.get_state()
        zb = np.clip(np.floor(x[2]).astype(np.int64), 0, H - 1)
        acc += np.bincount(zb, weights=v[0], minlength=H)
        cnt += np.bincount(zb, minlength=H)
        del x, v
    o = sim.observables()
    sim.close()
    del sim
    torch.cuda.empty_cache()
    prof = acc / cnt
    zc = np.arange(H) + 0.5
    X = np.stack([zc * (H - zc), np.ones(H)], axis=1)
    (A, B), *_ = np.linalg.lstsq(X, prof, rcond=None)
    resid = prof - X @ np.array([A, B])
    r2 = 1 - float(resid @ resid) / float((prof - prof.mean()) @ (prof - prof.mean()))
    eta = srd_viscosity(box["density"], box["kT"], box["h"], box["alpha"])
    A_th = box["density"] * box["g"][0] / (2 * eta)
    return {"workload": "256x256x64 cells between no-slip walls, 10/cell (41,943,040 particles), "
                        "g=1e-3 along x, MBS, split form, " + f"{steps} steps",
            "value": n * (run - 2) / wall, "unit": "particle-steps/s",
            "ms_per_step": wall * 1e3 / (run - 2),
            "profile_curvature_vs_theory": A / A_th, "slip_over_vmax": B / (A * H * H / 4),
            "profile_r2": r2, "v_max": A * H * H / 4 + B, "T_end": o["T"],
            "eta_theory": eta, "tiling": tiling, "profile": [round(float(q), 5) for q in prof]}


def run_features(mpc, torch, synth, steps: int = 1000):
    """Time per step and per kernel against the collision features (plain
    SRD, + MBS, SRD+a, SRD+a + MBS) on the 100^3 box with 10 particles per
    cell, FP64: the analog of the paper's feature-cost figure (Sec. III.D)."""
    out = {}
    base = dict(synth.config("C1"), L=(100, 100, 100))
    for name, kw in (("plain", {}), ("mbs", {"mbs": True}), ("amc", {"amc": True}),
                     ("amc_mbs", {"amc": True, "mbs": True})):
        n, wall, kt, _, _ = run_box(mpc, torch, dict(base, **kw), "fp64", 20, steps, 10)
        out[name] = {"ms_per_step": wall * 1e3 / steps,
                     "scan_draws_ms": kt.scan_ms / steps, "scatter_ms": kt.scatter_ms / steps,
                     "collide_ms": kt.collide_ms / steps, "advance_ms": kt.other_ms / steps,
                     "particle_steps_per_s": n * steps / wall}
        log(f"[features {name}] {wall * 1e3 / steps:.3f} ms/step (collide "
            f"{kt.collide_ms / steps:.3f})")
    plain = out["plain"]["ms_per_step"]
    for v in out.values():
        v["relative_to_plain"] = v["ms_per_step"] / plain
    return {"workload": "100^3 cells, 10/cell (10,000,000 particles), FP64, R = 20, "
                        f"{steps} steps per feature set", "sets": out}


def run_reorder_sweep(mpc, torch, synth, steps: int = 200):
    """Time per step against the reorder interval R (1, 5, 20, 100, never) on
    the 128^3 box with SRD+a and the thermostat (the paper's reorder-interval
    experiment, Sec. III.B.3)."""
    out = {}
    box = dict(synth.config("C1"), L=(128, 128, 128), amc=True, mbs=True)
    for R in (1, 5, 20, 100, 0):
        n, wall, kt, _, _ = run_box(mpc, torch, box, "fp64", R, steps, 10)
        out[str(R) if R else "never"] = wall * 1e3 / steps
    log("[reorder sweep] " + ", ".join(f"R={k}: {v:.3f}" for k, v in out.items()) + " ms/step")
    return {"workload": "128^3 cells, 10/cell, FP64, SRD+a + MBS, "
                        f"{steps} steps per interval", "ms_per_step_by_interval": out}


def cpu_baseline(steps: int = 3):
    """Single-threaded FP64 oracle on a bounded sample of the 512^3 workload:
    a 256 x 256 x 128-cell periodic box (1/16 of its cells) with the same
    density and collision, `steps` steps."""
    import oracle
    import synth
    box = synth.config("C3")
    L = (256, 256, 128)
    p = oracle.Params(L=L, h=box["h"], alpha=box["alpha"], kT=box["kT"], density=box["density"],
                      seed=1, mbs=False)
    x, v = synth.box_state(L, seed=1)
    n = x.shape[1]
    t0 = time.perf_counter()
    for t in range(steps):
        x, v = oracle.step(p, t, x, v)
    wall = time.perf_counter() - t0
    log(f"[cpu baseline] {n} particles x {steps} steps in {wall:.1f} s")
    return {"value": n * steps / wall, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"256x256x128 periodic cells x 10/cell ({n} particles, 1/16 of the 512^3 "
                      f"workload's cells), plain SRD, FP64, {steps} steps, 1 thread"}


def cpu_configs():
    """The single-threaded FP64 oracle on the other workloads (opt-in, a few
    minutes): the 16^3 box for all 100 steps; the 256^3 box with the
    thermostat, the 64-box ensemble and the Poiseuille channel for 5 steps
    each.  Particle-steps/s per workload, 1 thread."""
    import oracle
    import synth
    out = {}

    def run(name, boxes, steps, kw):
        states = [synth.box_state(b["L"], density=b["density"], kT=b["kT"], seed=7 + i)
                  for i, b in enumerate(boxes)]
        ps = [oracle.Params(L=b["L"], h=b["h"], alpha=b["alpha"], kT=b["kT"],
                            density=b["density"], seed=b["seed"], mbs=b["mbs"],
                            walls=b["walls"], g=b["g"], **kw) for b in boxes]
        n = sum(x.shape[1] for x, _ in states)
        t0 = time.perf_counter()
        for t in range(steps):
            states = [oracle.step(p, t, x, v) for p, (x, v) in zip(ps, states)]
            if n * steps > 10 ** 8:
                log(f"[cpu {name}] step {t + 1} of {steps}")
        wall = time.perf_counter() - t0
        log(f"[cpu {name}] {n} particles x {steps} steps in {wall:.1f} s")
        out[name] = {"value": n * steps / wall, "particles": n, "steps": steps,
                     "seconds": wall}
        del states

    run("16^3, plain SRD", [synth.config("C1")], 100, {})
    run("256^3, thermostat", [synth.config("C2")], 5, {})
    run("64 boxes", synth.batch_boxes(64, seed=4), 5, {})
    run("256x256x64 channel, walls, gravity, thermostat", [synth.config("C5")], 5, {})
    return {"unit": "particle-steps/s", "cores": 1, "kind": "oracle", "configs": out}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--forms", default=DEFAULT_FORMS,
                    help="entries besides the FP64 headline (comma list, or none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-configs", action="store_true",
                    help="also time the CPU oracle on the 16^3, 256^3, 64-box and channel "
                         "workloads (a few minutes)")
    ap.add_argument("--no-probe", action="store_true")
    ap.add_argument("--c2-steps", type=int, default=200)
    ap.add_argument("--batched-steps", type=int, default=500)
    ap.add_argument("--c5-steps", type=int, default=20000)
    ap.add_argument("--copy-probe-gib", type=float, default=0.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU path is not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2406_15236_amd as mpc
    import synth
    mpc.lib()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    copy_probe = None
    if args.copy_probe_gib > 0:
        nb = int(args.copy_probe_gib * 2 ** 30)
        src = torch.empty(nb, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        copy_probe = {"bytes_read": nb, "bytes_written": nb, "ms": ms,
                      "GBs": 2 * nb / (ms * 1e-3) / 1e9}
        del src, dst
        torch.cuda.empty_cache()
    probe = None if args.no_probe else hbm_probe(mpc, torch)

    # headline: 512^3, plain SRD, FP64
    c3 = synth.config("C3")
    R = 0
    n, wall, kt, o0, o1 = run_box(mpc, torch, c3, "fp64", R, args.steps, args.warmup,
                                  init_seed=3)
    value = n * args.steps / wall
    ms_step = wall * 1e3 / args.steps
    coll_ms = kt.collide_ms / max(1, kt.collide_launches)
    alg_bytes = n * 2 * STATE_BYTES["fp64"]
    achieved = alg_bytes / (coll_ms * 1e-3) / 1e9
    tr = traffic_record("fp64", "C3", R)
    drift64 = {"energy_drift_rel": abs(o1["E"] - o0["E"]) / o0["E"],
               "momentum_drift_per_sqrtN": float(np.abs(o1["P"] - o0["P"]).max() / math.sqrt(n)),
               "T_end": o1["T"]}
    log(f"[fp64 512^3] N={n} {ms_step:.3f} ms/step: scan {kt.scan_ms / args.steps:.3f} "
        f"scatter {kt.scatter_ms / args.steps:.3f} collide {coll_ms:.3f} "
        f"other {kt.other_ms / args.steps:.3f} ms; dE/E {drift64['energy_drift_rel']:.2e}")
    roof = {"bound": "hbm", "kernel": "k_collide<fp64>", "achieved": achieved,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": tr["bytes_per_launch"] if tr else None,
            "algorithmic_bytes_per_launch": alg_bytes, "avg_launch_ms": coll_ms}
    if probe:
        roof["attainable_copy_GBs"] = probe["copy"]["GBs"]
        roof["frac_of_attainable"] = achieved / probe["copy"]["GBs"]
    line = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "512^3 periodic cells, 10 particles/cell "
                               f"({n} particles), plain SRD, kT=1, h=0.1, alpha=130deg, "
                               "FP64 SoA, state kept in cell order every step",
                   "particles": n, "cells": 512 ** 3, "reorder_every": R},
        "hbm_roofline_frac_step": value * 2 * STATE_BYTES["fp64"] / (HBM_PEAK_GBS * 1e9),
        "roofline": roof,
        "launch": {"collide_tiling": run_box.last_tiling, "autotuned": True},
        "kernels_ms_per_step": {"scan": kt.scan_ms / args.steps,
                                "scatter": kt.scatter_ms / args.steps,
                                "collide": coll_ms, "advance": kt.other_ms / args.steps},
        "precision": {"fp64": drift64},
    }
    c2 = synth.config("C2")
    c2_work = "256^3 periodic cells, 10/cell, MBS thermostat, reorder every 20 steps"
    forms = {}
    extra = [f for f in args.forms.split(",") if f and f != "none"]
    for form in extra:
        try:
            if form == "split":
                n2, w2, k2, p0, p1 = run_box(mpc, torch, c3, "split", R, args.steps, args.warmup,
                                             init_seed=3)
                ds = {"energy_drift_rel": abs(p1["E"] - p0["E"]) / p0["E"],
                      "momentum_drift_per_sqrtN":
                          float(np.abs(p1["P"] - p0["P"]).max() / math.sqrt(n2)),
                      "T_end": p1["T"]}
                line["precision"]["split"] = ds
                line["precision"]["T_diff_split_vs_fp64"] = p1["T"] - o1["T"]
                forms[form] = form_entry("the same 512^3 box and initial state, split-FP32 form",
                                         "split", n2, args.steps, w2, k2, ds)
                trs = traffic_record("split", "C3", R)
                forms[form]["collide_traffic_bytes"] = trs["bytes_per_launch"] if trs else None
                forms[form]["collide_ms_vs_fp64"] = forms[form]["collide_ms"] / coll_ms
            elif form in ("c2_fp64", "c2_fp32", "c2_split"):
                fm = form[3:]
                n2, w2, k2, _, _ = run_box(mpc, torch, c2, fm, 20, args.c2_steps, args.warmup)
                forms[form] = form_entry(f"{c2_work}, {fm}", fm, n2, args.c2_steps, w2, k2)
                trs = traffic_record(fm, "C2", 20)
                forms[form]["collide_traffic_bytes"] = trs["bytes_per_launch"] if trs else None
            elif form in ("batched", "batched_split"):
                fm = "fp64" if form == "batched" else "split"
                boxes = synth.batch_boxes(64, seed=4)
                nb, wb, _, _, _ = run_box(mpc, torch, boxes, fm, 0, args.batched_steps,
                                          args.warmup, profiled=False, graph=50)
                forms[form] = form_entry(
                    "64 periodic boxes, edges U{16..96}, density U{5,10,20}, alpha "
                    f"U[90,150]deg, kT U[0.5,2], {fm}, graphs of 50 steps, "
                    f"{args.batched_steps} steps", fm, nb, args.batched_steps, wb, None,
                    {"particles": nb})
                _, _, kb, _, _ = run_box(mpc, torch, boxes, fm, 0, 20, 5)
                forms[form]["collide_ms_profiled"] = kb.collide_ms / max(1, kb.collide_launches)
                trb = traffic_record(fm, "C4", 0)
                forms[form]["collide_traffic_bytes"] = trb["bytes_per_launch"] if trb else None
                forms[form]["collide_roofline_frac_profiled"] = (
                    nb * 2 * STATE_BYTES[fm] / (forms[form]["collide_ms_profiled"] * 1e-3) / 1e9
                    / HBM_PEAK_GBS)
            elif form in ("amc", "amc_split"):
                fm = "fp64" if form == "amc" else "split"
                n2, w2, k2, _, p1 = run_box(mpc, torch, dict(c2, amc=True), fm, 20,
                                            args.c2_steps, args.warmup)
                forms[form] = form_entry(f"{c2_work}, {fm}, collision SRD+a", fm, n2,
                                         args.c2_steps, w2, k2, {"T_end": p1["T"]})
                tra = traffic_record("amc_" + fm, "C2", 20)
                forms[form]["collide_traffic_bytes"] = tra["bytes_per_launch"] if tra else None
            elif form == "fp64_fixed":
                n2, w2, k2, _, p1 = run_box(mpc, torch, dict(c2, fixed=True), "fp64", 20,
                                            args.c2_steps, args.warmup)
                forms[form] = form_entry(f"{c2_work}, FP64, fixed-point cell sums", "fp64", n2,
                                         args.c2_steps, w2, k2, {"T_end": p1["T"]})
            elif form in ("walls_slip", "walls_couette"):
                c5 = synth.config("C5")
                wbox = (dict(c5, slip=True) if form == "walls_slip"
                        else dict(c5, g=(0.0, 0.0, 0.0), uwall=0.1))
                n2, w2, k2, _, _ = run_box(mpc, torch, wbox, "fp64", 20, args.c2_steps,
                                           args.warmup)
                forms[form] = form_entry(
                    "256x256x64 channel, FP64, thermostat, " +
                    ("slip walls, g = 1e-3" if form == "walls_slip"
                     else "no-slip walls moving with +-0.1 along x"), "fp64", n2, args.c2_steps,
                    w2, k2)
            elif form == "lees_edwards":
                n2, w2, k2, _, _ = run_box(mpc, torch, dict(c2, le_u=0.5), "fp64", 20,
                                           args.c2_steps, args.warmup)
                forms[form] = form_entry(f"{c2_work}, FP64, Lees-Edwards image velocity 0.5",
                                         "fp64", n2, args.c2_steps, w2, k2)
            elif form == "density50":
                out = {}
                for tag, kw in (("srd", {}), ("amc", {"amc": True})):
                    dbox = dict(synth.config("C1"), L=(128, 128, 128), density=50.0, mbs=True,
                                **kw)
                    n2, w2, k2, _, _ = run_box(mpc, torch, dbox, "fp64", 20, args.c2_steps,
                                               args.warmup)
                    out[tag] = form_entry("128^3 cells x 50 particles, FP64, thermostat", "fp64",
                                          n2, args.c2_steps, w2, k2)
                forms[form] = {"workload": "128^3 cells x 50 particles (104,857,600), FP64, "
                                           "thermostat, reorder every 20 steps", "sets": out}
            elif form == "features":
                forms["features"] = run_features(mpc, torch, synth)
            elif form == "reorder_sweep":
                forms["reorder_sweep"] = run_reorder_sweep(mpc, torch, synth)
            elif form == "c5":
                forms["c5"] = run_c5(mpc, torch, synth, args.c5_steps)
            else:
                raise ValueError(f"unknown form {form}")
            if form in forms and isinstance(forms[form].get("ms_per_step"), float):
                log(f"[{form}] {forms[form]['ms_per_step']:.3f} ms/step"
                    + (f", collide {forms[form]['collide_ms']:.3f} ms"
                       if "collide_ms" in forms[form] else ""))
        except Exception as exc:  # report, keep the headline
            forms[form] = {"error": str(exc)}
            log(f"[{form}] error: {exc}")
    if forms:
        line["forms"] = forms
    if probe:
        line["hbm_probe"] = probe
    if copy_probe:
        line["copy_probe"] = copy_probe
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
        if args.cpu_configs:
            line["cpu_baseline"]["other_workloads"] = cpu_configs()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
