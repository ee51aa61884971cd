#!/usr/bin/env python3
"""Throughput of the MPC-SRD step on one MI355X.

Prints ONE JSON line.  `value` is FP64 particle-steps/s on the 256^3 periodic
box with the Maxwell-Boltzmann-scaling thermostat, 10 particles per cell and
particles reordered by cell every 20 steps (inputs resident in HBM before the
timed region; 200 steps by default).  The same line carries:
  roofline     : the collide kernel (dominant) -- algorithmic bytes per launch
                 (particles x state bytes read + written once) / its average
                 duration from HIP events on the launch stream; `traffic` is
                 the HBM bytes per launch from rocprofv3 counter runs of this
                 same command, when they were taken on the current kernels;
  forms        : FP32 and split-FP32 on the same box, FP64 stored in cell
                 order after every step, the batched ensemble of 64
                 uneven boxes (graph replay), the angular-momentum-
                 conserving collision SRD+a in FP64 and split-FP32, FP64
                 with fixed-point (order-independent) cell sums, the
                 256x256x64 channel with slip walls or moving walls, the
                 256^3 box under Lees-Edwards shear, 128^3 cells at 50
                 particles per cell, the
                 cost of each collision feature on 100^3 and the reorder-
                 interval sweep on 128^3;
  cpu_baseline : the single-threaded CPU oracle on a bounded sample.
--copy-probe-gib G adds one device-to-device copy of G GiB before the run: the
counter runs use it to scale FETCH_SIZE / WRITE_SIZE to bytes.
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


def run_box(mpc, torch, box: dict, form: str, R: int, steps: int, warmup: int,
            profiled: bool = True, tune: bool = True):
    sim = mpc.Sim(box if isinstance(box, list) else [box], form=form, reorder_every=R,
                  graph=not profiled)
    sim.init_state(2024)
    n = sum(sim.n(b) for b in range(len(sim.params)))
    tiling = None
    if tune:  # the library's autotuner picks the collide tiling (state restored after)
        sim.step(2)
        sim.autotune(3)
        tiling = sim.get_tiling()
        print(f"  autotuned {form}: {tiling}", file=sys.stderr, flush=True)
    if warmup:
        sim.step(warmup) if not profiled else sim.step_profiled(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if profiled:
        kt = sim.step_profiled(steps)
    else:
        sim.step(steps)
        kt = None
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sim.sync()
    obs = sim.observables(0)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    run_box.last_tiling = tiling
    return n, wall, kt, obs


def srd_viscosity(nc, kT, h, alpha, m=1.0, a=1.0):
    """Shear viscosity of 3D SRD with random grid shift (kinetic + collisional)."""
    c1, c2 = math.cos(alpha), math.cos(2 * alpha)
    f = nc - 1 + math.exp(-nc)
    return (nc * kT * h / a ** 3 * (5 * nc / (f * (4 - 2 * c1 - 2 * c2)) - 0.5)
            + m / (18 * a * h) * f * (1 - c1))


def run_c3(mpc, torch, synth, steps: int):
    """512^3 plain SRD, FP64 and split from the same device-initialised state
    (seed 3): throughput and energy / momentum drift of each form."""
    box = synth.config("C3")
    out = {"workload": "512^3 periodic cells, 10/cell (1,342,177,280 particles), plain SRD, "
                       f"kT=1, h=0.1, alpha=130deg, same initial state, {steps} steps"}
    for form in ("fp64", "split"):
        sim = mpc.Sim(box, form=form, reorder_every=0, graph=True)
        sim.init_state(3)
        o0 = sim.observables()
        n = o0["N"]
        sim.step(2)
        sim.autotune(2)  # state and step restored by the tuner
        out.setdefault("tiling", {})[form] = sim.get_tiling()
        sim.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        sim.sync()
        wall = time.perf_counter() - t0
        o1 = sim.observables()
        out[form] = {"value": n * steps / wall, "unit": "particle-steps/s",
                     "ms_per_step": wall * 1e3 / steps,
                     "energy_drift_rel": abs(o1["E"] - o0["E"]) / o0["E"],
                     "momentum_drift_per_sqrtN": float(np.abs(o1["P"] - o0["P"]).max()
                                                       / math.sqrt(n)),
                     "T_end": o1["T"]}
        print(f"[C3 {form}] {wall * 1e3 / steps:.2f} ms/step, dE/E {out[form]['energy_drift_rel']:.3e}",
              file=sys.stderr, flush=True)
        sim.close()
        del sim
        torch.cuda.empty_cache()
    out["T_diff_split_vs_fp64"] = out["split"]["T_end"] - out["fp64"]["T_end"]
    return out


def run_c5(mpc, torch, synth, steps: int):
    """Poiseuille flow, 256 x 256 x 64 cells between no-slip walls, gravity
    1e-3 along x, thermostat, split form: throughput and the time-averaged
    profile v_x(z) against the parabola rho g z (H - z) / (2 eta)."""
    box = synth.config("C5")
    L = box["L"]
    H = L[2]
    sim = mpc.Sim(box, form="split", reorder_every=20, graph=True)
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
        print(f"[C5] {done + 2} steps", file=sys.stderr, flush=True)
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
    cell, FP64, 1000 steps each: the analog of the paper's feature-cost figure
    (Sec. III.D)."""
    out = {}
    base = dict(synth.config("C1"), L=(100, 100, 100))
    for name, kw in (("plain", {}), ("mbs", {"mbs": True}), ("amc", {"amc": True}),
                     ("amc_mbs", {"amc": True, "mbs": True})):
        n, wall, kt, obs = run_box(mpc, torch, dict(base, **kw), "fp64", 20, steps, 10)
        out[name] = {"ms_per_step": wall * 1e3 / steps,
                     "scan_draws_ms": kt.scan_ms / steps, "scatter_ms": kt.scatter_ms / steps,
                     "collide_ms": kt.collide_ms / steps, "advance_ms": kt.other_ms / steps,
                     "particle_steps_per_s": n * steps / wall}
        print(f"[features {name}] {wall * 1e3 / steps:.3f} ms/step (collide "
              f"{kt.collide_ms / steps:.3f})", file=sys.stderr, flush=True)
    plain = out["plain"]["ms_per_step"]
    for v in out.values():
        v["relative_to_plain"] = v["ms_per_step"] / plain
    return {"workload": "100^3 cells, 10/cell (10,000,000 particles), FP64, R = 20, "
                        f"{steps} steps per feature set", "sets": out}


def run_reorder_sweep(mpc, torch, synth, steps: int = 200):
    """Time per step against the reorder interval R (1, 5, 20, 100, never) on
    the 128^3 box with SRD+a and the thermostat (the paper's reorder-interval
    experiment, Sec. III.B.3): here R only decides when the logical order is
    renumbered, so the cost should not depend on it."""
    out = {}
    box = dict(synth.config("C1"), L=(128, 128, 128), amc=True, mbs=True)
    for R in (1, 5, 20, 100, 0):
        n, wall, kt, obs = run_box(mpc, torch, box, "fp64", R, steps, 10)
        out[str(R) if R else "never"] = wall * 1e3 / steps
    print("[reorder sweep] " + ", ".join(f"R={k}: {v:.3f}" for k, v in out.items()) + " ms/step",
          file=sys.stderr, flush=True)
    return {"workload": "128^3 cells, 10/cell, FP64, SRD+a + MBS, "
                        f"{steps} steps per interval", "ms_per_step": out}


def cpu_baseline(seconds_hint: float = 15.0):
    """Single-threaded FP64 oracle on a 128^3 sample of the 256^3 workload."""
    import oracle
    import synth
    box = synth.config("C2")
    L = (128, 128, 128)
    p = oracle.Params(L=L, h=box["h"], alpha=box["alpha"], kT=1.0, density=10.0, seed=1,
                      mbs=True)
    x, v = synth.box_state(L, seed=1)
    n = x.shape[1]
    oracle.step(p, 0, x, v)   # warm
    steps = 0
    t0 = time.perf_counter()
    t = 1
    while True:
        x, v = oracle.step(p, t, x, v, reorder=((t + 1) % 20 == 0))
        steps += 1
        t += 1
        if time.perf_counter() - t0 > seconds_hint or steps >= 6:
            break
    wall = time.perf_counter() - t0
    return {"value": n * steps / wall, "unit": "particle-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"128^3 cells x 10/cell ({n} particles), MBS, {steps} steps, "
                      "1 thread (1/8 of the 256^3 workload's cells)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--forms",
                    default="fp32,split,fp64_sorted_every_step,batched,amc,amc_split,fp64_fixed,"
                            "walls_slip,walls_couette,lees_edwards,density50,features,"
                            "reorder_sweep",
                    help="extra entries besides the FP64 headline (comma list, or none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=500)
    ap.add_argument("--reorder-every", type=int, default=20)
    ap.add_argument("--c3-steps", type=int, default=100)
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

    box = synth.config("C2")
    workload = "C2"
    R = args.reorder_every
    n, wall, kt, obs = run_box(mpc, torch, box, "fp64", R, args.steps, args.warmup)
    value = n * args.steps / wall
    ms_step = wall * 1e3 / args.steps
    coll_ms = kt.collide_ms / max(1, kt.collide_launches)
    alg_bytes = n * 2 * STATE_BYTES["fp64"]
    achieved = alg_bytes / (coll_ms * 1e-3) / 1e9
    tr = traffic_record("fp64", workload, R)
    print(f"[fp64 C2] N={n} {ms_step:.3f} ms/step: scan {kt.scan_ms / args.steps:.3f} "
          f"scatter {kt.scatter_ms / args.steps:.3f} collide {coll_ms:.3f} "
          f"other {kt.other_ms / args.steps:.3f} ms; T={obs['T']:.4f}", file=sys.stderr)
    line = {
        "metric": METRIC, "value": value, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "256^3 periodic cells, 10 particles/cell "
                               f"({n} particles), MBS thermostat, kT=1, h=0.1, "
                               f"alpha=130deg, FP64 SoA, reorder every {R} steps",
                   "particles": n, "cells": 256 ** 3, "reorder_every": R},
        "hbm_roofline_frac_step": value * 2 * STATE_BYTES["fp64"] / (HBM_PEAK_GBS * 1e9),
        "roofline": {"bound": "hbm", "kernel": "k_collide<fp64>", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": tr["bytes_per_launch"] if tr else None,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": coll_ms},
        "launch": {"collide_tiling": run_box.last_tiling, "autotuned": True},
        "kernels_ms_per_step": {"scan": kt.scan_ms / args.steps,
                                "scatter": kt.scatter_ms / args.steps,
                                "collide": coll_ms, "advance": kt.other_ms / args.steps},
    }
    forms = {}
    extra = [f for f in args.forms.split(",") if f and f != "none"]
    for form in extra:
        try:
            if form in ("fp32", "split"):
                n2, w2, k2, o2 = run_box(mpc, torch, box, form, R, args.steps, args.warmup)
                v2 = n2 * args.steps / w2
                c2 = k2.collide_ms / max(1, k2.collide_launches)
                forms[form] = {
                    "workload": f"same 256^3 box, reorder every {R} steps", "value": v2, "unit": "particle-steps/s",
                    "ms_per_step": w2 * 1e3 / args.steps,
                    "hbm_roofline_frac_step": v2 * 2 * STATE_BYTES[form] / (HBM_PEAK_GBS * 1e9),
                    "collide_ms": c2,
                    "collide_achieved_GBs": n2 * 2 * STATE_BYTES[form] / (c2 * 1e-3) / 1e9}
                print(f"[{form} C2] {w2 * 1e3 / args.steps:.3f} ms/step collide {c2:.3f} ms",
                      file=sys.stderr)
            elif form == "fp64_sorted_every_step":
                n2, w2, k2, o2 = run_box(mpc, torch, box, "fp64", 1, args.steps, args.warmup)
                v2 = n2 * args.steps / w2
                c2 = k2.collide_ms / max(1, k2.collide_launches)
                forms[form] = {
                    "workload": "same 256^3 box, FP64, state written in cell order every step",
                    "value": v2, "unit": "particle-steps/s",
                    "ms_per_step": w2 * 1e3 / args.steps,
                    "hbm_roofline_frac_step": v2 * 2 * STATE_BYTES["fp64"] / (HBM_PEAK_GBS * 1e9),
                    "collide_ms": c2,
                    "collide_achieved_GBs": n2 * 2 * STATE_BYTES["fp64"] / (c2 * 1e-3) / 1e9}
                print(f"[fp64 R=1 C2] {w2 * 1e3 / args.steps:.3f} ms/step collide {c2:.3f} ms",
                      file=sys.stderr)
            elif form in ("walls_slip", "walls_couette"):
                # the 256 x 256 x 64 channel, FP64, thermostat: slip walls with a
                # body force, or no-slip walls moving with +-0.1 (shear flow)
                c5 = synth.config("C5")
                wbox = (dict(c5, slip=True) if form == "walls_slip"
                        else dict(c5, g=(0.0, 0.0, 0.0), uwall=0.1))
                n2, w2, k2, o2 = run_box(mpc, torch, wbox, "fp64", R, args.steps, args.warmup)
                v2 = n2 * args.steps / w2
                c2 = k2.collide_ms / max(1, k2.collide_launches)
                forms[form] = {
                    "workload": ("256x256x64 channel, FP64, thermostat, " +
                                 ("slip walls, g = 1e-3" if form == "walls_slip"
                                  else "no-slip walls moving with +-0.1 along x")
                                 + f", reorder every {R} steps"),
                    "value": v2, "unit": "particle-steps/s",
                    "ms_per_step": w2 * 1e3 / args.steps,
                    "collide_ms": c2,
                    "collide_achieved_GBs": n2 * 2 * STATE_BYTES["fp64"] / (c2 * 1e-3) / 1e9,
                    "launch": run_box.last_tiling}
                print(f"[{form}] N={n2} {w2 * 1e3 / args.steps:.3f} ms/step collide {c2:.3f} ms",
                      file=sys.stderr)
            elif form == "lees_edwards":
                lbox = dict(box, le_u=0.5)
                n2, w2, k2, o2 = run_box(mpc, torch, lbox, "fp64", R, args.steps, args.warmup)
                v2 = n2 * args.steps / w2
                c2 = k2.collide_ms / max(1, k2.collide_launches)
                forms[form] = {
                    "workload": f"same 256^3 box and thermostat, FP64, Lees-Edwards shear "
                                f"(image velocity 0.5), reorder every {R} steps",
                    "value": v2, "unit": "particle-steps/s",
                    "ms_per_step": w2 * 1e3 / args.steps,
                    "collide_ms": c2,
                    "collide_achieved_GBs": n2 * 2 * STATE_BYTES["fp64"] / (c2 * 1e-3) / 1e9,
                    "launch": run_box.last_tiling}
                print(f"[{form} C2] {w2 * 1e3 / args.steps:.3f} ms/step collide {c2:.3f} ms",
                      file=sys.stderr)
            elif form == "fp64_fixed":
                fbox = dict(box, fixed=True)
                n2, w2, k2, o2 = run_box(mpc, torch, fbox, "fp64", R, args.steps, args.warmup)
                v2 = n2 * args.steps / w2
                c2 = k2.collide_ms / max(1, k2.collide_launches)
                forms[form] = {
                    "workload": f"same 256^3 box and thermostat, FP64, fixed-point cell sums "
                                f"(order-independent), reorder every {R} steps",
                    "value": v2, "unit": "particle-steps/s",
                    "ms_per_step": w2 * 1e3 / args.steps,
                    "collide_ms": c2,
                    "collide_achieved_GBs": n2 * 2 * STATE_BYTES["fp64"] / (c2 * 1e-3) / 1e9,
                    "launch": run_box.last_tiling, "T_end": o2["T"]}
                print(f"[{form} C2] {w2 * 1e3 / args.steps:.3f} ms/step collide {c2:.3f} ms",
                      file=sys.stderr)
            elif form in ("amc", "amc_split"):
                fm = "fp64" if form == "amc" else "split"
                abox = dict(box, amc=True)
                n2, w2, k2, o2 = run_box(mpc, torch, abox, fm, R, args.steps, args.warmup)
                v2 = n2 * args.steps / w2
                c2 = k2.collide_ms / max(1, k2.collide_launches)
                forms[form] = {
                    "workload": f"same 256^3 box and thermostat, {fm}, collision SRD+a "
                                f"(angular momentum conserving), reorder every {R} steps",
                    "value": v2, "unit": "particle-steps/s",
                    "ms_per_step": w2 * 1e3 / args.steps,
                    "hbm_roofline_frac_step": v2 * 2 * STATE_BYTES[fm] / (HBM_PEAK_GBS * 1e9),
                    "collide_ms": c2,
                    "collide_achieved_GBs": n2 * 2 * STATE_BYTES[fm] / (c2 * 1e-3) / 1e9,
                    "collide_roofline_frac": n2 * 2 * STATE_BYTES[fm] / (c2 * 1e-3) / 1e9
                    / HBM_PEAK_GBS,
                    "launch": run_box.last_tiling, "T_end": o2["T"]}
                tra = traffic_record("amc_" + fm, "C2", R)
                forms[form]["collide_traffic_bytes"] = tra["bytes_per_launch"] if tra else None
                print(f"[{form} C2] {w2 * 1e3 / args.steps:.3f} ms/step collide {c2:.3f} ms",
                      file=sys.stderr)
            elif form == "density50":
                # the paper's main-text density: 128^3 cells x 50 particles, FP64,
                # thermostat, with and without SRD+a
                out = {}
                for tag, kw in (("srd", {}), ("amc", {"amc": True})):
                    dbox = dict(synth.config("C1"), L=(128, 128, 128), density=50.0, mbs=True,
                                **kw)
                    n2, w2, k2, o2 = run_box(mpc, torch, dbox, "fp64", R, args.steps,
                                             args.warmup)
                    c2 = k2.collide_ms / max(1, k2.collide_launches)
                    out[tag] = {"value": n2 * args.steps / w2, "unit": "particle-steps/s",
                                "ms_per_step": w2 * 1e3 / args.steps, "collide_ms": c2,
                                "collide_achieved_GBs":
                                    n2 * 2 * STATE_BYTES["fp64"] / (c2 * 1e-3) / 1e9,
                                "launch": run_box.last_tiling}
                    print(f"[density50 {tag}] N={n2} {w2 * 1e3 / args.steps:.3f} ms/step "
                          f"collide {c2:.3f} ms", file=sys.stderr, flush=True)
                forms[form] = {"workload": f"128^3 cells x 50 particles (104,857,600), FP64, "
                                           f"thermostat, reorder every {R} steps", "sets": out}
            elif form == "features":
                forms["features"] = run_features(mpc, torch, synth)
            elif form == "reorder_sweep":
                forms["reorder_sweep"] = run_reorder_sweep(mpc, torch, synth)
            elif form == "c3":
                forms["c3"] = run_c3(mpc, torch, synth, args.c3_steps)
            elif form == "c5":
                forms["c5"] = run_c5(mpc, torch, synth, args.c5_steps)
            elif form == "batched":
                boxes = synth.batch_boxes(64, seed=4)
                nb, wb, _, _ = run_box(mpc, torch, boxes, "fp64", 0, args.batched_steps,
                                       args.warmup, profiled=False)
                vb = nb * args.batched_steps / wb
                forms["batched"] = {
                    "workload": "64 periodic boxes, edges U{16..96}, density U{5,10,20}, "
                                "alpha U[90,150]deg, kT U[0.5,2], FP64, one graph replay "
                                f"per step, {args.batched_steps} steps",
                    "particles": nb, "value": vb, "unit": "particle-steps/s",
                    "ms_per_step": wb * 1e3 / args.batched_steps,
                    "hbm_roofline_frac_step": vb * 2 * STATE_BYTES["fp64"] / (HBM_PEAK_GBS * 1e9)}
                print(f"[batched C4] N={nb} {wb * 1e3 / args.batched_steps:.3f} ms/step",
                      file=sys.stderr)
        except Exception as exc:  # report, keep the headline
            forms[form] = {"error": str(exc)}
    if forms:
        line["forms"] = forms
    if copy_probe:
        line["copy_probe"] = copy_probe
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
