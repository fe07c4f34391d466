#!/usr/bin/env python3
"""Benchmark of the stochastic-LLG hysteresis-loop path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                    [--legs all|none|NAME,...]

Headline (default workload block_b2_cone10): the 128x128x512 block of b = 2
cells with easy axes in a 10 degree cone, the largest single-GPU workload and
the one whose fused step is bound by HBM.  A bench step is a window of 2000
Heun steps (after 200 warm-up steps); its full sweep is 6.4e6 steps.  For the
other workloads a bench step is one full field sweep (one dynamic hysteresis
loop per realization), including the per-step loop reduction and the loop
analytics.  Inputs are synthetic and seeded, already resident in HBM when
timing starts.  Rank 0 prints one JSON line.

Legs in the same line (each a fixed amount of work, independent of --steps):
  rod_b1_ens8            one full sweep of the 8x24x56 rod, 8 realizations
                         (cell-updates/s, loops/s)
  multilevel_ens256      one full sweep of the four-level batch (1024
                         instances) and the same instances stepped one
                         realization at a time (batched_vs_plain)
  rod_b4_adjoint64       forward sweep and gradient of 64 realizations
                         (grad_over_forward)
  block_b2_cone10_z1024  the block at 128x128x1024 (state and axes beyond the
                         256 MB Infinity Cache), a 2000-step window
  macrospin_sr2p5_ens256 the single-macrospin limit (one cell of the rod's
                         volume) at SR = 2.5 Oe/ns, alpha = 1 (SR/alpha =
                         2.5 Oe/ns, Fig. 4): 256 realizations, one per lane,
                         8e5 steps of 1 ps
  rod_b4_demag64         the 2x6x14 b = 4 rod of the adjoint workload with the
                         magnetostatic field (beyond the paper), 64
                         realizations, 4e4 steps

Shape pins for counter runs: --stream-shape kind,a,b,c,planes and
--slab-shape kind,threads,cells,planes switch the tuners off and set the
dominant level's kernel.
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
HEADLINE = "block_b2_cone10"
LEGS = ("rod_b1_ens8", "multilevel_ens256", "rod_b4_adjoint64", "block_b2_cone10_z1024",
        "macrospin_sr2p5_ens256", "rod_b4_demag64")

# Algorithmic work of one cell-update (one Heun step of one cell).
# HBM: m_n in and m_{n+1} out (12 + 12 bytes); stored per-cell easy axes add
# 12 bytes read.
BYTES_PER_CELL_UPDATE = 24
BYTES_AXES = 12
# FP32 flops of the step's arithmetic (two fields, two LLG right-hand sides,
# the Heun updates, two renormalisations, Box-Muller): about 150.
FLOPS_PER_CELL_UPDATE = 150
# VALU lane operations of the per-cell device functions compiled alone for
# gfx950 without load addressing (Philox, uniforms, Box-Muller, fields,
# right-hand sides, updates, renormalisations): 120 predictor + 57 corrector.
VALU_OPS_PER_CELL_UPDATE = 177
PEAK_HBM_GBS = 8000.0                   # MI355X HBM3E
PEAK_FP32_TFLOPS = 157.3                # MI355X vector FP32 (packed, FMA = 2)
# VALU issue rate without packed FP32 (this library issues none): 256 CUs x
# 4 SIMDs x 16 lanes x 2.4 GHz lane-instructions per second
PEAK_VALU_ISSUE_TOPS = 256 * 64 * 2.4e9 / 1e12
# sweeps longer than this many steps run in pieces that report progress
LONG_SWEEP = 20_000_000


def parse():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed bench steps")
    ap.add_argument("--warmup", type=int, default=None, help="untimed bench steps")
    ap.add_argument("--workload", default=HEADLINE)
    ap.add_argument("--window", type=int, default=None,
                    help="Heun steps per bench step (default: the whole sweep; 2000 for the block)")
    ap.add_argument("--legs", default=None,
                    help="'all' (default with the headline workload), 'none', or a comma list")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="target CPU time of each oracle sample (1 thread and all threads)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain device copy of known size (for counter scaling)")
    ap.add_argument("--stream-shape", default=None, help="kind,a,b,c,planes for level 0 (tuners off)")
    ap.add_argument("--slab-shape", default=None, help="kind,threads,cells,planes for level 0 (tuners off)")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def workload(name):
    import sllg_workloads as W
    if name == "block_b2_cone10_z1024":
        wl = W.workload("block_b2_cone10")
        wl["levels"][0]["nz"] = 1024
        return wl
    if name == "macrospin_sr2p5_ens256":
        return W.macrospin_pair(2.5, 1.0, T_K=310.0, n_real=256)
    if name == "rod_b4_demag64":
        wl = W.workload("rod_b4_adjoint64")
        wl["material"]["demag"] = True
        wl["ckpt_every"] = 0
        return wl
    return W.workload(name)


def open_sim(wl, ckpt, stream_shape=None, slab_shape=None):
    from paper_1912_00310_amd import Sim, sllg
    pinned = stream_shape or slab_shape
    if pinned:
        sllg.set_options(sllg.OPT_NO_TUNE)
    try:
        sim = Sim(wl["material"], wl["levels"], ckpt_every=ckpt)
    finally:
        if pinned:
            sllg.set_options(0)
    if stream_shape:
        sim.set_stream_shape(0, *[int(x) for x in stream_shape.split(",")])
    if slab_shape:
        sim.set_slab_shape(0, *[int(x) for x in slab_shape.split(",")])
    return sim


def dominant_kernel(sim, n_levels):
    """Kernel the library times (streamed if a level is streamed, else slab,
    else resident) and its family."""
    kernels = [sim.kernel_name(l) for l in range(n_levels)]
    fam = next((f for f in ("k_stream", "k_rows", "k_slab", "k_resident", "k_lanes", "k_demag")
                if any(k.startswith(f) for k in kernels)), "none")
    if fam == "k_rows" and any(k.startswith("k_stream") for k in kernels):
        fam = "k_stream"
    dom = next(k for k in kernels if k.startswith(fam)) if fam != "none" else "none"
    return dom, fam, kernels


def roofline(sim, wl, name, k_ms, k_n, k_cells):
    """Roofline object of the dominant kernel from its mean launch time."""
    levels = wl["levels"]
    dom, fam, kernels = dominant_kernel(sim, len(levels))
    if not (k_n > 0 and k_ms > 0):
        return None
    spl = 1
    mt = re.search(r"steps/launch (\d+)", dom)
    if mt:
        spl = int(mt.group(1))
    launch_ms = k_ms * spl            # a slab launch covers spl steps
    per_launch = k_cells * spl        # cell-updates per launch
    # steps one launch advances its levels (resident, lanes and demag
    # launches run many steps; a streamed launch one)
    dom_cells = sum(l["nx"] * l["ny"] * l["nz"] * l["n_real"] for l, k in zip(levels, kernels) if k == dom)
    steps_per_launch = per_launch / dom_cells if dom_cells else None
    has_axes = any(l.get("cone_deg", 0) > 0 for l in levels)
    bpc = BYTES_PER_CELL_UPDATE + (BYTES_AXES if has_axes else 0)
    fpc = FLOPS_PER_CELL_UPDATE
    if fam == "k_demag":
        # the magnetostatic field: a 3x3 tensor times m_j (9 FMA = 18 flops)
        # for every cell j, in both Heun stages
        fpc += 36 * max(l["nx"] * l["ny"] * l["nz"] for l in levels)
    s = launch_ms * 1e-3
    gbs = per_launch * bpc / s / 1e9
    tflops = per_launch * fpc / s / 1e12
    valu = per_launch * VALU_OPS_PER_CELL_UPDATE / s / 1e12
    traffic = measured_traffic(dom, name)
    # streamed kernels move the state through HBM every step (the HBM
    # roofline binds); slab and resident kernels keep it in LDS and are bound
    # by arithmetic and latency (the FP32 roofline)
    if fam in ("k_stream", "k_rows"):
        rl = {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
              "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": traffic}
    else:
        rl = {"bound": "alu", "achieved": round(tflops, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
              "frac": round(tflops / PEAK_FP32_TFLOPS, 4), "traffic": traffic}
    rl.update({
        "kernel": dom, "mean_launch_ms": launch_ms,
        "steps_per_launch": round(steps_per_launch, 2) if steps_per_launch else None,
        "launches_timed": k_n // spl if spl > 1 else k_n, "cell_updates_per_launch": per_launch,
        "bytes_per_cell_update": bpc, "algorithmic_bytes_per_launch": per_launch * bpc,
        "flops_per_cell_update": fpc,
        "hbm_GBps": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4),
        "fp32_TFLOPs": round(tflops, 3), "fp32_frac": round(tflops / PEAK_FP32_TFLOPS, 4),
        "valu_issue_frac": round(valu / PEAK_VALU_ISSUE_TOPS, 4),
    })
    return rl


def clean_stats(st):
    return {k: (None if isinstance(v, float) and math.isnan(v) else v) for k, v in st.items()}


def run_workload(name, steps, warmup, window=None, stream_shape=None, slab_shape=None, plain=False):
    """Time `steps` bench steps of one workload; returns a result dict."""
    import torch
    wl = workload(name)
    levels = wl["levels"]
    adjoint = name == "rod_b4_adjoint64"
    t_init = time.time()
    sim = open_sim(wl, wl.get("ckpt_every", 0) if adjoint else 0, stream_shape, slab_shape)
    torch.cuda.synchronize()
    t_init = time.time() - t_init
    params = [sim.level_params(l) for l in range(len(levels))]
    n_sweep = int(max(p["n_steps"] for p in params))
    if window is None and "window" in wl:
        window = wl["window"]["timed_steps"]
    window = min(window or n_sweep, n_sweep)
    cells_per_step = sum(sim.ncell(l) * levels[l]["n_real"] for l in range(len(levels)))
    t_split = {"forward": 0.0, "grad": 0.0}

    def one_step():
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
                log(f"  {done}/{n_sweep} Heun steps")
        elif window == n_sweep:
            sim.reset()
            sim.run_sweep()
        else:
            if sim.step(0) + window > n_sweep:
                sim.reset()
            sim.run_steps(window)
        if adjoint:
            sim.synchronize()
            t1 = time.perf_counter()
            sim.grad(0)          # synchronises
            t_split["forward"] += t1 - t
            t_split["grad"] += time.perf_counter() - t1
        for l in range(len(levels)):
            sim.loop(l, -1)      # synchronises and checks the status word

    if "window" in wl and window < n_sweep:
        sim.run_steps(wl["window"]["warmup_steps"])
    for i in range(warmup):
        one_step()
        log(f"{name}: warmup step {i + 1}/{warmup} done")
    sim.synchronize()
    t_split["forward"] = t_split["grad"] = 0.0
    # HIP events on the library's stream around the dominant kernel's launch
    # units (graph replays of 128 streamed steps, slab launches, or resident
    # launches)
    sim.set_timing(1)
    sim.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        one_step()
        log(f"{name}: timed step {i + 1}/{steps} done")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_n, k_cells = sim.kernel_time()
    sim.set_timing(0)
    dt = t1 - t0
    value = cells_per_step * window * steps / dt
    loops = sum(l["n_real"] for l in levels) * steps * window / n_sweep
    stats = {str(l): clean_stats(sim.loop(l, -1)[2]) for l in range(len(levels))}
    res = {
        "value": value, "unit": "cell-updates/s", "steps": steps, "warmup": warmup,
        "ms_per_step": dt / steps * 1e3, "loops_per_s": loops / dt, "init_s": round(t_init, 3),
        "config": {
            "workload": name,
            "levels": [f"{l['nx']}x{l['ny']}x{l['nz']} b={l['b']:g} x{l['n_real']}" for l in levels],
            "heun_steps_per_bench_step": window, "heun_steps_per_sweep": n_sweep,
            "dt_fs": [round(p["dt"] * 1e15, 3) for p in params],
            "alpha": [p["alpha"] for p in params],
            "plan": [int(p["plan"]) for p in params],
            "kernels": dominant_kernel(sim, len(levels))[2],
            "loop_accumulators": "f64",
        },
        "roofline": roofline(sim, wl, name, k_ms, k_n, k_cells),
        "loop": stats,
    }
    if adjoint:
        res["adjoint"] = {"forward_s_per_sweep": t_split["forward"] / steps,
                          "grad_s_per_sweep": t_split["grad"] / steps,
                          "grad_over_forward": t_split["grad"] / max(t_split["forward"], 1e-12)}
    sim.close()
    del sim
    if plain:
        res["batched_vs_plain"] = plain_leg(wl, dt / (steps * window))
    return res


def plain_leg(wl, batched_s_per_step, nsteps=2000):
    """The same instances stepped one realization at a time: a context per
    level holding a single realization (its own plan, tuned alike), timed
    over nsteps and scaled by the number of realizations.  Both forms run the
    same per-cell arithmetic, so their states are bit-identical."""
    import torch
    from paper_1912_00310_amd import Sim
    per_level = []
    plain = 0.0
    for lvd in wl["levels"]:
        one = dict(lvd, n_real=1)
        sim = Sim(wl["material"], [one])
        sim.run_steps(64)
        sim.synchronize()
        t = time.perf_counter()
        sim.run_steps(nsteps)
        sim.synchronize()
        s = (time.perf_counter() - t) / nsteps
        per_level.append({"grid": f"{lvd['nx']}x{lvd['ny']}x{lvd['nz']}", "us_per_step_one_realization": s * 1e6,
                          "kernel": sim.kernel_name(0)})
        plain += s * lvd["n_real"]
        sim.close()
    torch.cuda.synchronize()
    return {"plain_us_per_step": plain * 1e6, "batched_us_per_step": batched_s_per_step * 1e6,
            "speedup": plain / batched_s_per_step, "per_level": per_level}


def run_leg(name):
    """One leg of the bench line: a fixed amount of work per workload."""
    if name == "rod_b1_ens8":
        r = run_workload(name, steps=1, warmup=0)
    elif name == "multilevel_ens256":
        r = run_workload(name, steps=1, warmup=0, plain=True)
    elif name == "rod_b4_adjoint64":
        r = run_workload(name, steps=3, warmup=1)
    elif name == "block_b2_cone10_z1024":
        r = run_workload(name, steps=2, warmup=1)
    elif name in ("macrospin_sr2p5_ens256", "rod_b4_demag64"):
        r = run_workload(name, steps=2, warmup=1)
    else:
        raise ValueError(f"unknown leg {name}")
    r.pop("steps", None)
    r.pop("warmup", None)
    return r


# The source files a kernel's device code is compiled from (besides the
# shared per-cell header, the shared types and the build flags).
KERNEL_SOURCES = {
    "k_rows2": "sllg_rows2.hip", "k_rows": "sllg_rows.hip", "k_stream": "sllg_kernels.hip",
    "k_resident": "sllg_kernels.hip", "k_slab": "sllg_slab.hip", "k_slab2": "sllg_slab.hip",
    "k_lanes": "sllg_lanes.hip", "k_demag": "sllg_demag.hip", "k_adjoint": "sllg_adjoint.hip",
}


def source_digest(kernel):
    """SHA-256 over the sources of one kernel's device code: its own file,
    the per-cell header and the shared types (csrc/) and the build script
    (compiler flags), in that order."""
    fam = kernel.split("<")[0].split()[0]
    pkg = os.path.join(ROOT, "paper_1912_00310_amd")
    files = [os.path.join(pkg, "build_lib.py")] + [
        os.path.join(pkg, "csrc", n) for n in ("sllg_device.hpp", "sllg_types.hpp", KERNEL_SOURCES[fam])]
    h = hashlib.sha256()
    for path in files:
        with open(path, "rb") as f:
            h.update(os.path.basename(path).encode() + b"\0" + f.read())
    return h.hexdigest()


def kernel_instance(name):
    """'k_rows2<1024,1> tz 43' or 'k_rows2<1024,1,true>' -> 'k_rows2<1024,1'
    (template and its thread and cell counts; the axes flag follows the
    workload)."""
    n = name.split()[0].replace(" ", "")
    for flag in (",true>", ",false>"):
        n = n.replace(flag, ">")
    return n.rstrip(">")


def measured_traffic(kernel, workload_name):
    """HBM bytes per launch of the dominant kernel (as the library names it,
    e.g. 'k_rows2<1024,1> tz 43') from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by a plain copy of known size), or None
    when there is none, it was taken on another instantiation, or the kernel
    sources changed since."""
    path = os.path.join(ROOT, "profiles", f"{kernel.split('<')[0]}_{workload_name}_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if ":" in line:
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    try:
        if kv.get("source_sha256") != source_digest(kernel):
            return None
    except KeyError:
        return None
    if "<" in kernel and kernel_instance(kv.get("kernel", "")) != kernel_instance(kernel):
        return None
    try:
        return int(float(kv["hbm_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(name, seconds):
    """The FP64 oracle, unchanged, on the host cores over a bounded sample of
    the workload's largest level: one thread, then every thread OpenMP gives
    (over realizations, or over cells when there are fewer realizations than
    threads)."""
    import oracle
    from oracle import gk
    wl = workload(name)
    lvd = max(wl["levels"], key=lambda l: l["nx"] * l["ny"] * l["nz"] * l["n_real"])
    lv = gk.compile_level(wl["material"], lvd, wl["levels"].index(lvd))
    ncell = lv["nx"] * lv["ny"] * lv["nz"]
    u = oracle.make_axes(lv)
    all_threads = oracle.max_threads()
    legs = {}
    for threads in (1, all_threads):
        nreal = min(lvd["n_real"], threads)
        seeds = [lvd["seed_base"] + r for r in range(nreal)]
        # calibrate on a short run, then size the sample to about `seconds`
        probe = max(1, int(2e6 // (ncell * nreal)))
        t = time.perf_counter()
        oracle.run_batch(lv, seeds, probe, threads=threads, u=u)
        rate = ncell * nreal * probe / (time.perf_counter() - t)
        nsteps = max(1, min(lv["n_steps"], int(rate * seconds / (ncell * nreal))))
        t = time.perf_counter()
        oracle.run_batch(lv, seeds, nsteps, threads=threads, u=u)
        el = time.perf_counter() - t
        legs[threads] = dict(value=ncell * nreal * nsteps / el, nreal=nreal, nsteps=nsteps, seconds=round(el, 2))
        log(f"cpu baseline: {threads} thread(s) {legs[threads]['value']:.3e} cell-updates/s")
    top = legs[all_threads]
    par = "over realizations" if top["nreal"] >= all_threads or ncell < 65536 else "over cells"
    return {"value": top["value"], "unit": "cell-updates/s", "cores": all_threads, "kind": "oracle",
            "sample": f"{top['nreal']} realization(s) x {top['nsteps']} Heun steps of the "
                      f"{lv['nx']}x{lv['ny']}x{lv['nz']} grid of {name} (FP64 C oracle, OpenMP {par})",
            "seconds": top["seconds"], "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "one_thread": {"value": legs[1]["value"], "cores": 1,
                           "sample": f"{legs[1]['nreal']} realization(s) x {legs[1]['nsteps']} Heun steps",
                           "seconds": legs[1]["seconds"]}}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (every box here has one); "
                                   "--gpus must be 1", "n_gpus_requested": a.gpus}))
        sys.exit(2)
    import torch

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    wl = workload(a.workload)
    heavy = "window" not in wl and a.window is None
    steps = a.steps if a.steps is not None else (2 if heavy else 10)
    warmup = a.warmup if a.warmup is not None else 1
    multi = len(wl["levels"]) > 1 or wl["levels"][0]["n_real"] > 8
    head = run_workload(a.workload, steps, warmup, a.window, a.stream_shape, a.slab_shape, plain=multi)

    legs_arg = a.legs if a.legs is not None else ("all" if a.workload == HEADLINE else "none")
    names = LEGS if legs_arg == "all" else ([] if legs_arg == "none" else legs_arg.split(","))
    legs = {}
    for n in names:
        if n == a.workload:
            continue
        log(f"leg {n}")
        legs[n] = run_leg(n)

    cpu = None if a.no_cpu_baseline else cpu_baseline(a.workload, a.cpu_seconds)

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
        "value": head["value"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": head["config"],
        "loops_per_s": head["loops_per_s"],
        "init_s": head["init_s"],
        "roofline": head["roofline"],
        "cpu_baseline": cpu,
        "loop": head["loop"],
    }
    for k in ("adjoint", "batched_vs_plain"):
        if k in head:
            out[k] = head[k]
    if legs:
        out["legs"] = legs
    print(json.dumps(out))


if __name__ == "__main__":
    main()
