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


def main(names):
    threads = oracle.max_threads()
    for name in names:
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
    main(sys.argv[1:] or list(SUBSETS))
