"""Race and halo canaries of the GPU kernels (need a GPU):

  * LDS check: the debug library libsllg_ldscheck.so (built by build() with
    SLLG_LDS_CHECK) tags every LDS slot of the streamed full-width-row kernel
    with the plane it stands for and checks the tag of every slot it reads.
    A child process runs the kernel's tile configurations (ragged windows
    and z ranges, tiles at both grid ends, one and two cells per thread, per
    cell and uniform axes, checkpoints, the whole block) on it: no slot may
    be read before its plane's write, and the states must be bit-identical
    to the product library's.
  * Run twice: every plan and tile kernel, run twice from the same seeds in
    fresh contexts, gives bit-identical states and loop ordinates (a race
    between the threads of a kernel shows as a run-to-run difference).
  * Split runs: every case run in three calls (1 step, about a third, the
    rest) gives the bits of one call: the step index alone fixes the noise,
    and the launch units (graph replays, slab and resident launches) may be
    cut anywhere.
  * Resume: the first two pieces in one context, its snapshot
    (sllg_save_state) loaded into a fresh context (sllg_load_state), the
    rest there: the bits of the uninterrupted run, on every plan; a snapshot
    of another configuration or of the wrong size is refused.
  * Launch-blocking mode: a child process with every launch synchronous
    (HIP_LAUNCH_BLOCKING=1, kernels and copies serialised) gives the same
    bits as the normal asynchronous run, on every plan but the slab plan
    (child processes make no cooperative launch).
"""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import _gpu_cases as G

pytestmark = pytest.mark.gpu

ROOT = G.ROOT
DEBUG_LIB = os.path.join(ROOT, "paper_1912_00310_amd", "libsllg_ldscheck.so")
PRODUCT_LIB = os.path.join(ROOT, "paper_1912_00310_amd", "libsllg.so")


@pytest.fixture(scope="module")
def P():
    import torch
    assert torch.cuda.is_available()
    import paper_1912_00310_amd as P
    return P


@pytest.fixture(scope="module")
def reference(P):
    """Each case once with the product library, in this process."""
    return {name: G.run_case(P, name) for name in G.CASES}


def child(lib, names, env_extra=None, timeout=400):
    env = dict(os.environ)
    env.update(env_extra or {})
    print(f"child process: {os.path.basename(lib)} {' '.join(names)} {env_extra or ''}", flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "_gpu_cases.py"), lib, *names],
                       capture_output=True, text=True, env=env, timeout=timeout, cwd=ROOT)
    lines = [json.loads(l) for l in r.stdout.splitlines() if l.startswith("{")]
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-2000:])
    assert lines and lines[0].get("lib") == os.path.realpath(lib), lines[:1]
    return {l["case"]: l for l in lines[1:]}


def test_every_case_runs_on_the_product_library(reference):
    for name, (status, digest, kernel) in reference.items():
        assert status == "ok", (name, status)
        if name.startswith("rows2_"):
            assert kernel.startswith("k_rows2"), (name, kernel)
    assert reference["slab_rod_b1"][2].startswith("k_slab")
    assert reference["resident_rod_b4"][2].startswith("k_resident")
    assert reference["lanes_macrospin"][2].startswith("k_lanes")
    assert reference["demag_rod_b4"][2].startswith("k_demag")
    assert reference["stream_window_block_slice"][2].startswith("k_stream")


def test_lds_check_build_reads_no_stale_slot(reference):
    assert os.path.exists(DEBUG_LIB), "libsllg_ldscheck.so is missing: build() builds it"
    got = child(DEBUG_LIB, G.LDS_CASES)
    for name in G.LDS_CASES:
        g = got[name]
        print(name, g["kernel"], g["status"], flush=True)
        assert g["status"] == "ok", (name, g["status"])
        assert g["kernel"].startswith("k_rows2"), (name, g["kernel"])
        assert g["digest"] == reference[name][1], name


def test_run_twice_bit_identical(P, reference):
    for name in G.CASES:
        status, digest, kernel = G.run_case(P, name)
        print(name, kernel, flush=True)
        assert status == "ok", (name, status)
        assert digest == reference[name][1], name


def test_split_runs_bit_identical(P, reference):
    for name in G.CASES:
        assert sum(G.pieces(G.CASES[name]["steps"])) == G.CASES[name]["steps"]
        status, digest, kernel = G.run_case(P, name, split=True)
        print(name, kernel, G.pieces(G.CASES[name]["steps"]), flush=True)
        assert status == "ok", (name, status)
        assert digest == reference[name][1], name


def test_resume_from_snapshot_bit_identical(P, reference):
    for name in G.CASES:
        status, digest, kernel = G.run_case(P, name, resume=True)
        print(name, kernel, flush=True)
        assert status == "ok", (name, status)
        assert digest == reference[name][1], name


def test_resume_then_gradient_bit_identical(P):
    # the adjoint recomputes its segments from the checkpoints a snapshot
    # carries: the gradient after a resumed sweep is the uninterrupted one
    wl = G.workload(dict(wl="rod_b4_adjoint64", level=dict(n_real=4)))
    out = []
    for resume in (False, True):
        sim = P.Sim(wl["material"], wl["levels"], ckpt_every=256)
        if resume:
            sim.run_steps(15001)
            snap = sim.save_state()
            sim.close()
            sim = P.Sim(wl["material"], wl["levels"], ckpt_every=256)
            sim.load_state(snap)
        sim.run_sweep()
        ga, gh = sim.grad(0)
        out.append((sim.get_state(0, 3), sim.loop(0, -1)[1], ga, gh))
        sim.close()
    # (the coercive-field gradient is NaN when the mean loop of these 4
    # realizations misses a zero crossing on a branch; NaN matches NaN)
    assert np.isfinite(out[0][2]).all()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b, equal_nan=True)


def test_snapshot_of_another_configuration_is_refused(P):
    a = G.open_case(P, "resident_rod_b4")
    a.run_steps(10)
    snap = a.save_state()
    before = a.get_state(0, 0)
    with pytest.raises(P.SllgError):
        a.load_state(snap[:-8])          # wrong size
    bad = bytearray(snap)
    bad[0] ^= 0xFF
    with pytest.raises(P.SllgError):
        a.load_state(bytes(bad))         # not a snapshot
    assert (a.get_state(0, 0) == before).all()
    a.close()
    wl = G.workload(G.CASES["resident_rod_b4"])
    wl["levels"][0]["seed_base"] += 1    # same sizes, other seeds
    b = P.Sim(wl["material"], wl["levels"])
    with pytest.raises(P.SllgError):
        b.load_state(snap)
    assert b.step(0) == 0
    b.close()


def test_launch_blocking_mode_bit_identical(reference):
    names = ["rows2_block_slice_1024x1", "rows2_uniform_axis_ckpt", "stream_window_block_slice",
             "resident_rod_b4", "lanes_macrospin", "demag_rod_b4"]
    got = child(PRODUCT_LIB, names, {"HIP_LAUNCH_BLOCKING": "1", "AMD_SERIALIZE_KERNEL": "3",
                                     "AMD_SERIALIZE_COPY": "3"})
    for name in names:
        g = got[name]
        assert g["status"] == "ok", (name, g["status"])
        assert g["digest"] == reference[name][1], name
