#!/usr/bin/env python3
"""Benchmark of the stochastic-LLG hysteresis-loop path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A bench step is one full field sweep (one dynamic hysteresis loop per
realization) of the named workload, including the per-step loop reduction
and the loop analytics; for the 8.4M-cell block it is a window of Heun steps
(the sweep is 6.4e6 steps).  Inputs are synthetic and seeded, already resident
in HBM when timing starts.  Rank 0 prints one JSON line.

Workloads (sllg_workloads): rod_b1_ens8 (default: 8x24x56 rod, b=1, 8
realizations, 4e6 steps of 1 fs), rod_b4_single, multilevel_ens256,
block_b2_cone10, rod_b4_adjoint64, and the paper's protocol
rod_sine_sr250_ens100 and rod_sine_sr2p5_ens100 (a sweep of 1.6e8 steps:
run it with --steps 1 --warmup 0).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sLLG cell-updates/s & loops/s at 1 GPU (% HBM roofline); batched & adjoint vs plain"

# Algorithmic work of one cell-update (one Heun step of one cell), counted as
# the VALU instructions of the per-cell device functions compiled alone for
# gfx950, without load addressing (an FMA or a transcendental is one):
# Philox4x32-10 (18 wide multiplies, 19 exclusive-ors, most of them
# three-input), four 23-bit uniforms (8), Box-Muller (12, 7 of them
# transcendental), the thermal field scale (3), two neighbour sums (2 x 18),
# two effective fields, two LLG right-hand sides, the predictor and corrector
# updates and two renormalisations: 120 in the predictor, 57 in the corrector.
VALU_OPS_PER_CELL_UPDATE = 177
# HBM: m_n in and m_{n+1} out (12 + 12 bytes); per-cell easy axes add 12.
BYTES_PER_CELL_UPDATE = 24
BYTES_AXES = 12
PEAK_HBM_GBS = 8000.0
# FP32 vector peak 157.3 TFLOP/s = 78.6e12 FMA lane-operations per second
# (256 CUs x 128 lanes x 2.4 GHz); one VALU op per lane counted as one
PEAK_VALU_TOPS = 256 * 128 * 2.4e9 / 1e12
# sweeps longer than this many steps run in pieces that report progress
LONG_SWEEP = 20_000_000


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed bench steps")
    ap.add_argument("--warmup", type=int, default=None, help="untimed bench steps")
    ap.add_argument("--workload", default="rod_b1_ens8")
    ap.add_argument("--window", type=int, default=None,
                    help="Heun steps per bench step (default: the whole sweep; 2000 for the block)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="target CPU time of the oracle sample")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (for counter scaling)")
    return ap.parse_args()


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; --gpus must be 1",
                          "n_gpus_requested": a.gpus}))
        sys.exit(2)
    import numpy as np
    import torch

    import sllg_workloads as W
    from paper_1912_00310_amd import Sim

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    wl = W.workload(a.workload)
    mat, levels = wl["material"], wl["levels"]
    ckpt = wl.get("ckpt_every", 0)
    adjoint = a.workload == "rod_b4_adjoint64"
    t_init = time.time()
    sim = Sim(mat, levels, ckpt_every=ckpt if adjoint else 0)
    torch.cuda.synchronize()
    t_init = time.time() - t_init
    params = [sim.level_params(l) for l in range(len(levels))]
    n_sweep = int(max(p["n_steps"] for p in params))
    window = a.window
    if window is None and "window" in wl:
        window = wl["window"]["timed_steps"]
    window = min(window or n_sweep, n_sweep)
    cells_per_step = sum(sim.ncell(l) * levels[l]["n_real"] for l in range(len(levels)))
    heavy = window >= 1_000_000
    steps = a.steps if a.steps is not None else (2 if heavy else 5)
    warmup = a.warmup if a.warmup is not None else 1

    t_split = {"forward": 0.0, "grad": 0.0}

    def one_step():
        # one sweep (or window) of every level and realization
        t = time.perf_counter()
        if window == n_sweep and n_sweep > LONG_SWEEP:
            # a sweep of minutes: the same steps in pieces, with progress
            sim.reset()
            done = 0
            while done < n_sweep:
                k = min(LONG_SWEEP, n_sweep - done)
                sim.run_steps(k)
                done += k
                sim.synchronize()
                print(f"  {done}/{n_sweep} Heun steps", file=sys.stderr, flush=True)
        elif window == n_sweep:
            sim.reset()
            sim.run_sweep()
        else:
            if sim.step(0) + window > n_sweep:
                sim.reset()
            sim.run_steps(window)
        if adjoint:
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sim.grad(0)          # synchronises
            t_split["forward"] += t1 - t
            t_split["grad"] += time.perf_counter() - t1
        for l in range(len(levels)):
            sim.loop(l, -1)

    if "window" in wl and window < n_sweep:
        sim.run_steps(wl["window"]["warmup_steps"])
    for i in range(warmup):
        one_step()
        print(f"warmup step {i + 1}/{warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_split["forward"] = t_split["grad"] = 0.0
    # HIP events on the library's stream around the dominant kernel's launch
    # units (graph replays of 128 streamed steps, slab launches, or resident
    # launches)
    sim.set_timing(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        one_step()
        # progress on stderr (microseconds against sweeps of seconds)
        print(f"timed step {i + 1}/{steps} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_n, k_cells = sim.kernel_time()
    sim.set_timing(0)
    dt = t1 - t0
    cell_updates = cells_per_step * window * steps
    value = cell_updates / dt
    loops = sum(levels[l]["n_real"] for l in range(len(levels))) * steps * window / n_sweep
    stats = {l: sim.loop(l, -1)[2] for l in range(len(levels))}
    plan_ids = [int(p["plan"]) for p in params]

    # roofline of the dominant kernel from its mean launch time.  The library
    # times streamed launches if a level is streamed, else slab launches, else
    # resident launches; a slab launch covers kSlabChunk steps and the library
    # reports it per step, so it is scaled back to one dispatch here.
    rl = None
    kernels = [sim.kernel_name(l) for l in range(len(levels))]
    fam = next((f for f in ("k_stream", "k_rows", "k_slab", "k_resident")
                if any(k.startswith(f) for k in kernels)), "none")
    if fam == "k_rows" and any(k.startswith("k_stream") for k in kernels):
        fam = "k_stream"
    dom = next(k for k in kernels if k.startswith(fam)) if fam != "none" else "none"
    if k_n > 0 and k_ms > 0:
        spl = 1
        mt = re.search(r"steps/launch (\d+)", dom)
        if mt:
            spl = int(mt.group(1))
        launch_ms = k_ms * spl
        per_launch = k_cells * spl
        has_axes = any(l.get("cone_deg", 0) > 0 for l in levels)
        bpc = BYTES_PER_CELL_UPDATE + (BYTES_AXES if has_axes else 0)
        gbs = per_launch * bpc / (launch_ms * 1e-3) / 1e9
        tops = per_launch * VALU_OPS_PER_CELL_UPDATE / (launch_ms * 1e-3) / 1e12
        f_h, f_a = gbs / PEAK_HBM_GBS, tops / PEAK_VALU_TOPS
        traffic = measured_traffic(dom, a.workload)
        # streamed kernels move the state through HBM every step; the slab and
        # resident kernels keep it on chip (LDS) and are bound by arithmetic
        # and latency, so their fraction is taken against the ALU peak
        if fam in ("k_stream", "k_rows"):
            rl = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                  "frac": round(f_h, 4), "traffic": traffic}
        else:
            rl = {"bound": "alu", "achieved": round(tops, 3), "peak": round(PEAK_VALU_TOPS, 3),
                  "unit": "TOP/s", "frac": round(f_a, 4), "traffic": traffic}
        rl["kernel"] = dom
        rl["mean_launch_ms"] = launch_ms
        rl["steps_per_launch"] = spl
        rl["launches_timed"] = k_n // spl if spl > 1 else k_n
        rl["cell_updates_per_launch"] = per_launch
        rl["algorithmic_bytes_per_launch"] = per_launch * bpc
        rl["hbm_equiv_GBps"] = round(gbs, 1)
        rl["valu_TOPs"] = round(tops, 3)

    extra = {}
    if adjoint:
        extra["adjoint"] = {"forward_s_per_sweep": t_split["forward"] / steps,
                            "grad_s_per_sweep": t_split["grad"] / steps,
                            "grad_over_forward": t_split["grad"] / max(t_split["forward"], 1e-12)}
    if len(levels) > 1 or levels[0]["n_real"] > 8:
        extra["batched_vs_plain"] = plain_leg(Sim, torch, wl, dt / (steps * window))

    cpu = None
    if not a.no_cpu_baseline:
        cpu = cpu_baseline(wl, a.cpu_seconds)

    if a.copy_probe:
        # a plain elementwise copy of known size (1 GiB read, 1 GiB written)
        # whose FETCH_SIZE / WRITE_SIZE calibrate the counters
        n = 1 << 28
        x = torch.ones(n, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            torch.add(x, 0.0, out=y)
        torch.cuda.synchronize()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": dt / steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": a.workload,
            "levels": [f"{l['nx']}x{l['ny']}x{l['nz']} b={l['b']:g} x{l['n_real']}" for l in levels],
            "heun_steps_per_bench_step": window,
            "heun_steps_per_sweep": n_sweep,
            "dt_fs": [round(p["dt"] * 1e15, 3) for p in params],
            "alpha": [p["alpha"] for p in params],
            "plan": plan_ids,
            "loop_accumulators": "f64",
        },
        "loops_per_s": loops / dt,
        "init_s": round(t_init, 3),
        "roofline": rl,
        "cpu_baseline": cpu,
        "loop": {str(l): {k: (None if isinstance(v, float) and math.isnan(v) else v)
                          for k, v in stats[l].items()} for l in stats},
    }
    out.update(extra)
    print(json.dumps(out))
    sim.close()


def plain_leg(Sim, torch, wl, batched_s_per_step, nsteps=2000):
    """The same instances stepped one realization at a time: a context per
    level holding a single realization (its own plan, tuned alike), timed
    over nsteps and scaled by the number of realizations.  Both forms run the
    same per-cell arithmetic, so their states are bit-identical."""
    per_level = []
    plain = 0.0
    for lvd in wl["levels"]:
        one = dict(lvd, n_real=1)
        sim = Sim(wl["material"], [one])
        sim.run_steps(64)
        torch.cuda.synchronize()
        t = time.perf_counter()
        sim.run_steps(nsteps)
        torch.cuda.synchronize()
        s = (time.perf_counter() - t) / nsteps
        per_level.append({"grid": f"{lvd['nx']}x{lvd['ny']}x{lvd['nz']}", "us_per_step_one_realization": s * 1e6,
                          "kernel": sim.kernel_name(0)})
        plain += s * lvd["n_real"]
        sim.close()
    return {"plain_us_per_step": plain * 1e6, "batched_us_per_step": batched_s_per_step * 1e6,
            "speedup": plain / batched_s_per_step, "per_level": per_level}


def source_digest():
    """SHA-256 over the kernel sources (csrc/*.hip, *.hpp, sorted by name)."""
    d = os.path.join(ROOT, "paper_1912_00310_amd", "csrc")
    h = hashlib.sha256()
    for n in sorted(os.listdir(d)):
        if n.endswith((".hip", ".hpp")):
            with open(os.path.join(d, n), "rb") as f:
                h.update(n.encode() + b"\0" + f.read())
    return h.hexdigest()


def kernel_instance(name):
    """'k_rows2<1024,1> tz 43' or 'k_rows2<1024,1,true>' -> 'k_rows2<1024,1'
    (template and its thread and cell counts; the axes flag follows the
    workload)."""
    n = name.split()[0].replace(" ", "")
    for flag in (",true>", ",false>"):
        n = n.replace(flag, ">")
    return n.rstrip(">")


def measured_traffic(kernel, workload):
    """HBM bytes per launch of the dominant kernel (as the library names it,
    e.g. 'k_rows2<1024,1> tz 43') from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by a plain copy of known size), or None
    when there is none, it was taken on another instantiation, or the kernel
    sources changed since."""
    path = os.path.join(ROOT, "profiles", f"{kernel.split('<')[0]}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != source_digest():
        return None
    if "<" in kernel and kernel_instance(kv.get("kernel", "")) != kernel_instance(kernel):
        return None
    try:
        return int(float(kv["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def cpu_baseline(wl, seconds):
    """FP64 oracle on the host cores over a bounded sample of the workload."""
    import oracle
    from oracle import gk
    lvd = max(wl["levels"], key=lambda l: l["nx"] * l["ny"] * l["nz"] * l["n_real"])
    idx = wl["levels"].index(lvd)
    lv = gk.compile_level(wl["material"], lvd, idx)
    ncell = lv["nx"] * lv["ny"] * lv["nz"]
    threads = oracle.max_threads()
    nreal = min(lvd["n_real"], max(1, threads))
    seeds = [lvd["seed_base"] + r for r in range(nreal)]
    # calibrate on a short run, then size the sample to about `seconds`
    probe = max(1, int(2e6 // (ncell * nreal)))
    t = time.perf_counter()
    oracle.run_batch(lv, seeds, probe)
    rate = ncell * nreal * probe / (time.perf_counter() - t)
    nsteps = max(1, min(lv["n_steps"], int(rate * seconds / (ncell * nreal))))
    t = time.perf_counter()
    oracle.run_batch(lv, seeds, nsteps)
    el = time.perf_counter() - t
    return {"value": ncell * nreal * nsteps / el, "unit": "cell-updates/s",
            "cores": min(nreal, threads), "kind": "oracle",
            "sample": f"{nreal} realizations x {nsteps} Heun steps of the "
                      f"{lv['nx']}x{lv['ny']}x{lv['nz']} grid (FP64 C oracle, OpenMP over realizations)",
            "seconds": round(el, 2)}


if __name__ == "__main__":
    main()
