"""Write the oracle's whole-loop statistics used by the statistical GPU tests.

    python tests/golden/make_loop_stats.py [rod_b1_ens8|multilevel_ens256 ...]

Calls only the FP64 oracle (oracle/) on the seeded synthetic workloads of
sllg_workloads: every realization listed below is run over its full field
sweep from the all-+z state, and each loop is reduced to its area S (Oe of
the simulated field), its coercive field H_c (first zero crossing per branch,
linear interpolation) and its remanence; the ensemble's mean loop and one
standard error over realizations are stored beside them.  The output files
(loop_stats_<workload>.json in this folder) record the SHA-256 of the oracle
sources they were computed with.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import sllg_workloads as W  # noqa: E402
from oracle import gk  # noqa: E402

# realizations per level (the first k seeds of each level)
SUBSETS = {
    "rod_b1_ens8": [8],
    "multilevel_ens256": [8, 16, 32, 32],
}

# single-cell sweep-rate / damping scans (sllg_workloads.macrospin_pair):
# (T, [(SR Oe/ns, alpha), ...]), 32 realizations each
MACROSPIN = {
    "sharrock_T100": (100.0, [(0.075, 0.03), (0.25, 0.1), (0.75, 0.3), (2.5, 1.0), (7.5, 3.0), (25.0, 10.0),
                              (0.75, 0.1), (2.5, 0.1)]),
    "sharrock_T310": (310.0, [(0.075, 0.03), (0.25, 0.1), (0.75, 0.3), (2.5, 1.0), (7.5, 3.0), (25.0, 10.0)]),
}
MACROSPIN_REAL = 32


def oracle_digest():
    h = hashlib.sha256()
    for n in ("gk.py", "sllg_oracle.c"):
        with open(os.path.join(ROOT, "oracle", n), "rb") as f:
            h.update(n.encode() + b"\0" + f.read())
    return h.hexdigest()


def nan_to_none(x):
    return None if isinstance(x, float) and math.isnan(x) else x


def level_stats(wl, i, k, threads):
    lvd = wl["levels"][i]
    lv = gk.compile_level(wl["material"], lvd, i)
    seeds = [lvd["seed_base"] + r for r in range(k)]
    t = time.time()
    mbar, _ = oracle.run_batch(lv, seeds, lv["n_steps"], threads=threads)
    H = oracle.field_schedule_Oe(lv)
    st = oracle.ensemble_stats(lv, H, mbar)
    el = time.time() - t
    per = st["per_real"]
    return {
        "grid": [lv["nx"], lv["ny"], lv["nz"]], "b": lv["b"], "n_steps": lv["n_steps"],
        "seeds": seeds, "alpha": lv["alpha"], "dt": lv["dt"],
        "S": [p["S"] for p in per], "Hc": [nan_to_none(p["Hc"]) for p in per],
        "Hstar_desc": [nan_to_none(p["Hstar_desc"]) for p in per],
        "Hstar_asc": [nan_to_none(p["Hstar_asc"]) for p in per],
        "Mr": [nan_to_none(p["Mr"]) for p in per],
        "n_cross_desc": [int(p["n_cross_desc"]) for p in per],
        "n_cross_asc": [int(p["n_cross_asc"]) for p in per],
        "mean_loop": {k2: nan_to_none(st[k2]) for k2 in ("S_sim", "Hc", "Mr", "S_phys", "Hc_phys", "Mr_phys")},
        "S_se": nan_to_none(st["S_se"]), "Hc_se": nan_to_none(st["Hc_se"]),
        "S_mean_of_real": st["S_mean_of_real"], "Hc_mean_of_real": nan_to_none(st["Hc_mean_of_real"]),
        # the mean loop every 1000 steps, for plots and spot checks
        "mean_loop_every_1000": mbar.mean(axis=0)[::1000].tolist(),
        "oracle_seconds": round(el, 1),
    }


def streamed_stats(wl, k, threads):
    """As level_stats for one level, holding one realization's loop at a time
    (long single-cell sweeps): the realizations run in a thread pool (the C
    oracle releases the GIL) and the mean loop is accumulated."""
    from concurrent.futures import ThreadPoolExecutor
    lvd = wl["levels"][0]
    lv = gk.compile_level(wl["material"], lvd, 0)
    seeds = [lvd["seed_base"] + r for r in range(k)]
    t = time.time()
    H = oracle.field_schedule_Oe(lv)
    N = lv["nx"] * lv["ny"] * lv["nz"]
    total = np.zeros(lv["n_steps"] + 1)
    per = []

    def one(seed):
        _, mb = oracle.run(lv, seed, 0, lv["n_steps"], np.tile([0.0, 0.0, 1.0], (N, 1)))
        return seed, oracle.loop_stats(H, mb), mb

    with ThreadPoolExecutor(max_workers=max(1, threads)) as ex:
        for seed, st, mb in ex.map(one, seeds):
            per.append(st)
            total += mb
    mean = oracle.loop_stats(H, total / k)
    el = time.time() - t

    def se(a):
        a = [x for x in a if math.isfinite(x)]
        return float(np.std(a, ddof=1) / math.sqrt(len(a))) if len(a) > 1 else None

    S_r = [p["S"] for p in per]
    Hc_r = [p["Hc"] for p in per]
    return {
        "grid": [lv["nx"], lv["ny"], lv["nz"]], "b": lv["b"], "n_steps": lv["n_steps"], "seeds": seeds,
        "alpha": lv["alpha"], "dt": lv["dt"], "S": S_r, "Hc": [nan_to_none(x) for x in Hc_r],
        "n_cross_desc": [int(p["n_cross_desc"]) for p in per], "n_cross_asc": [int(p["n_cross_asc"]) for p in per],
        "mean_loop": {"S_sim": mean["S"], "Hc": nan_to_none(mean["Hc"]), "Mr": nan_to_none(mean["Mr"])},
        "S_se": se(S_r), "Hc_se": se(Hc_r), "oracle_seconds": round(el, 1),
    }


def main(names):
    threads = oracle.max_threads()
    for name in names:
        if name in MACROSPIN:
            T, pairs = MACROSPIN[name]
            out = {"_source": "FP64 oracle (oracle/), written by tests/golden/make_loop_stats.py",
                   "workload": name, "oracle_sha256": oracle_digest(), "threads": threads, "pairs": []}
            for sr, al in pairs:
                print(f"{name}: SR {sr} alpha {al}", flush=True)
                wl = W.macrospin_pair(sr, al, T_K=T, n_real=MACROSPIN_REAL)
                st = streamed_stats(wl, MACROSPIN_REAL, threads)
                st.update(SR=sr, T=T)
                out["pairs"].append(st)
                print(f"  done in {st['oracle_seconds']} s", flush=True)
            with open(os.path.join(HERE, f"loop_stats_{name}.json"), "w") as f:
                json.dump(out, f, indent=1)
            continue
        wl = W.workload(name)
        out = {"_source": "FP64 oracle (oracle/), written by tests/golden/make_loop_stats.py",
               "workload": name, "oracle_sha256": oracle_digest(), "threads": threads, "levels": []}
        for i, k in enumerate(SUBSETS[name]):
            print(f"{name} level {i}: {k} realizations", flush=True)
            out["levels"].append(level_stats(wl, i, k, threads))
            print(f"  done in {out['levels'][-1]['oracle_seconds']} s", flush=True)
        with open(os.path.join(HERE, f"loop_stats_{name}.json"), "w") as f:
            json.dump(out, f, indent=1)


if __name__ == "__main__":
    main(sys.argv[1:] or list(SUBSETS) + list(MACROSPIN))
