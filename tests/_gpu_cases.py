"""Runs shared by the race and LDS-check tests and by their child processes.

A case is a small workload on one plan or tile kernel, stepped a few times
from its seeds in a fresh context; its result is a SHA-256 digest of the
states of every realization and of realization 0's loop ordinates (bit
patterns), with the kernel that ran.

As a script (the child process of a test):
    python tests/_gpu_cases.py LIB CASE [CASE ...]
loads the library LIB instead of the package's, runs each case and prints
one JSON line per case: {"case", "status" ("ok", "refused" or the error),
"digest", "kernel"}, after a line {"lib": <the library file mapped into the
process>}.  The child makes no cooperative launch (the slab plan is switched
off, also in the planner): one made in a child process after the parent had
made its own failed with hipErrorIllegalState.
"""
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import sllg_workloads as W  # noqa: E402

# name -> workload, level / material changes, plan or tile shape, steps,
# checkpoint interval
CASES = {
    # the streamed full-width-row kernel (kind 2) on the block's planes:
    # ragged z tiles (10 + 10 + 4), one and two cells per thread
    "rows2_block_slice_1024x1": dict(wl="block_b2_cone10", level=dict(nz=24), stream=(2, 1024, 1, 1, 10), steps=6),
    "rows2_block_slice_1024x2": dict(wl="block_b2_cone10", level=dict(nz=24), stream=(2, 1024, 2, 1, 8), steps=6),
    # ragged row windows and tiles at both grid ends, small grids (the second
    # one long enough for graph replays of 8 .. 128 launches)
    "rows2_ragged_512x2": dict(wl="block_b2_cone10", level=dict(nx=40, ny=36, nz=20), stream=(2, 512, 2, 1, 7),
                               steps=6),
    "rows2_ragged_256x1": dict(wl="block_b2_cone10", level=dict(nx=32, ny=50, nz=17), stream=(2, 256, 1, 1, 5),
                               steps=300),
    # one easy axis for all cells (no per-cell axes), two realizations,
    # checkpoints every 2 steps (the checkpoint path reads LDS too; a fast
    # sweep keeps the checkpoints of the whole sweep small)
    "rows2_uniform_axis_ckpt": dict(wl="block_b2_cone10", level=dict(nz=16, cone_deg=0.0, n_real=2),
                                    material=dict(sweep_Oe_per_ns=1e7), stream=(2, 768, 2, 1, 5), steps=6,
                                    ckpt=2),
    # whole x-y planes per tile (no ring rows): the b = 1 rod, 3 realizations
    "rows2_rod_b1": dict(wl="rod_b1_ens8", level=dict(n_real=3), stream=(2, 192, 1, 1, 16), steps=6),
    # the whole 128 x 128 x 512 block on the tuned tile kernel
    "rows2_block_full": dict(wl="block_b2_cone10", steps=3),
    # the other plans
    "stream_window_block_slice": dict(wl="block_b2_cone10", level=dict(nz=24), stream=(0, 64, 8, 1, 8), steps=6),
    "resident_rod_b4": dict(wl="rod_b4_adjoint64", level=dict(n_real=8), plan="PLAN_RESIDENT", steps=300),
    "slab_rod_b1": dict(wl="rod_b1_ens8", level=dict(n_real=2), slab=(1, 1024, 1, 2), steps=300),
    "lanes_macrospin": dict(wl="macrospin", steps=500),
    "demag_rod_b4": dict(wl="rod_b4_adjoint64", level=dict(n_real=4), material=dict(demag=True), steps=200),
}

LDS_CASES = [n for n in CASES if n.startswith("rows2_")]


def workload(c):
    if c["wl"] == "macrospin":
        wl = W.macrospin_pair(2.5, 1.0, T_K=310.0, n_real=64)
    else:
        wl = W.workload(c["wl"])
    wl["levels"][0].update(c.get("level", {}))
    wl["material"].update(c.get("material", {}))
    return wl


def pieces(steps):
    """The case's steps in three runs: 1, about a third, the rest."""
    a = max(1, steps // 3)
    return [1, a, steps - 1 - a]


def open_case(P, name):
    """A fresh context of the case, on its plan or tile shape."""
    c = CASES[name]
    wl = workload(c)
    sim = P.Sim(wl["material"], wl["levels"], ckpt_every=c.get("ckpt", 0))
    try:
        if "plan" in c:
            sim.set_plan(0, getattr(P, c["plan"]))
        if "stream" in c:
            sim.set_stream_shape(0, *c["stream"])
        if "slab" in c:
            sim.set_slab_shape(0, *c["slab"])
    except P.SllgError:
        sim.close()
        return None
    return sim


def run_case(P, name, split=False, resume=False):
    """(status, digest, kernel) of one case with the package's library; with
    split, the steps are run in three calls (pieces) instead of one; with
    resume, the first two pieces run in one context, whose snapshot a second
    context loads and continues."""
    c = CASES[name]
    wl = workload(c)
    if resume:
        first = open_case(P, name)
        if first is None:
            return "refused", None, None
        try:
            for k in pieces(c["steps"])[:2]:
                first.run_steps(k)
            snap = first.save_state()
        finally:
            first.close()
    sim = open_case(P, name)
    if sim is None:
        return "refused", None, None
    try:
        if resume:
            sim.load_state(snap)
            sim.run_steps(pieces(c["steps"])[2])
        else:
            for k in (pieces(c["steps"]) if split else [c["steps"]]):
                sim.run_steps(k)
        sim.synchronize()
        h = hashlib.sha256()
        for r in range(wl["levels"][0]["n_real"]):
            h.update(np.ascontiguousarray(sim.get_state(0, r)).tobytes())
        h.update(np.ascontiguousarray(sim.loop(0, 0)[1]).tobytes())
        return "ok", h.hexdigest(), sim.kernel_name(0)
    except P.SllgError as e:
        return str(e), None, None
    finally:
        sim.close()


def _mapped(path):
    with open("/proc/self/maps") as f:
        return any(line.rstrip().endswith(os.path.realpath(path)) for line in f)


if __name__ == "__main__":
    lib_path = os.path.realpath(sys.argv[1])
    import torch  # noqa: F401  (before the library)

    from paper_1912_00310_amd import sllg
    sllg.LIB_PATH = lib_path
    import paper_1912_00310_amd as P
    P.lib()
    sllg.set_options(sllg.OPT_NO_SLAB)
    print(json.dumps({"lib": lib_path if _mapped(lib_path) else None}), flush=True)
    for name in sys.argv[2:]:
        status, digest, kernel = run_case(P, name)
        print(json.dumps({"case": name, "status": status, "digest": digest, "kernel": kernel}), flush=True)
