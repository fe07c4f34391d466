"""sllg_init_static (the library's own static device workspace, no device
allocation) against sllg_init with a caller workspace: the same states bit
for bit and the same loops, on two calls in a row, the second with a smaller
input; a second live static context on the GPU and a workload beyond the
static workspace are refused."""
import numpy as np
import pytest

import sllg_workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_00310_amd as P
    P.lib()
    return P


def _workload_large():
    # a streamed level (28800 cells, axes in a cone) beside two resident ones
    wl = W.workload("block_b2_cone10")
    wl["material"]["sweep_Oe_per_ns"] = 4e4          # 1600 steps
    blk = dict(wl["levels"][0], nx=40, ny=36, nz=20, n_real=1)
    rod = dict(W.workload("rod_b4_single")["levels"][0], n_real=4, cone_deg=10.0, axis_seed=3)
    small = dict(rod, nx=1, ny=3, nz=7, b=8.0, n_real=3)
    wl["levels"] = [blk, rod, small]
    return wl


def _workload_small():
    wl = W.workload("rod_b4_single")
    wl["material"]["sweep_Oe_per_ns"] = 8e4          # 1000 steps
    wl["levels"][0].update(nx=1, ny=3, nz=7, b=8.0, n_real=2)
    return wl


def _run(P, wl, static):
    sim = P.Sim(wl["material"], wl["levels"], static_workspace=static)
    sim.run_sweep()
    out = []
    for l, lvd in enumerate(wl["levels"]):
        states = [sim.get_state(l, r) for r in range(lvd["n_real"])]
        H, m, st = sim.loop(l, -1)
        out.append((states, H, m, st, sim.kernel_name(l)))
    return sim, out


def _compare(a, b):
    for (sa, Ha, ma, sta, ka), (sb, Hb, mb, stb, kb) in zip(a, b):
        for x, y in zip(sa, sb):
            assert np.array_equal(x, y), (ka, kb)
        assert np.array_equal(Ha, Hb)
        # the loop ordinates differ only in how FP32 partial sums are grouped
        assert np.abs(ma - mb).max() < 1e-6, (ka, kb)
        assert sta["S_sim"] == pytest.approx(stb["S_sim"], rel=1e-6, abs=1e-6)
        assert sta["Mr_sim"] == pytest.approx(stb["Mr_sim"], abs=1e-6)


def test_static_workspace_matches_caller_workspace_twice(P):
    for wl in (_workload_large(), _workload_small()):
        ref, want = _run(P, wl, static=False)
        ref.close()
        sim, got = _run(P, wl, static=True)
        print("static context kernels:", [g[4] for g in got], flush=True)
        _compare(got, want)
        sim.close()


def test_one_live_static_context_per_gpu(P):
    wl = _workload_small()
    a = P.Sim(wl["material"], wl["levels"], static_workspace=True)
    with pytest.raises(P.SllgError) as e:
        P.Sim(wl["material"], wl["levels"], static_workspace=True)
    assert e.value.code == -4
    a.close()
    b = P.Sim(wl["material"], wl["levels"], static_workspace=True)
    b.close()


def test_workload_beyond_static_workspace_is_refused(P):
    wl = W.workload("rod_b1_ens8")                   # 4e6-step records of 8 realizations
    with pytest.raises(P.SllgError) as e:
        P.Sim(wl["material"], wl["levels"], static_workspace=True)
    assert e.value.code == -2 and "static workspace" in str(e.value)
