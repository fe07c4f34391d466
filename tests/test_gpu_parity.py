"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded Philox stream.

Tolerances
  * Philox words: bit-exact.
  * normals: the kernels use the hardware log2/sqrt/sin/cos (about 1 ulp);
    |xi_gpu - xi_oracle| <= 2e-5 absolute over the 5.77-sigma range.
  * trajectories: <= 1e-5 per component over the first 1000 steps (FP32 state
    vs FP64; the bar the method is held to).
  * loop ordinate (FP64 sum of FP32 values): <= 2e-6 absolute while the
    trajectories agree.
"""
import math

import numpy as np
import pytest

import sllg_workloads as W
from oracle import gk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def P(torch_cuda):
    import paper_1912_00310_amd as P
    P.lib()
    return P


def oracle_level(wl, i=0):
    return gk.compile_level(wl["material"], wl["levels"][i], i)


def gpu_state(sim, level=0, real=0):
    return sim.get_state(level, real).T.astype(np.float64)   # (N, 3)


# ---------------------------------------------------------------------------
def test_philox_words_bit_exact_and_normals(P, orc):
    rng = np.random.default_rng(1)
    n = 4096
    cells = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    steps = rng.integers(0, 2**40, n, dtype=np.uint64)
    for seed, level, tag in ((1, 0, 1), (0xDEADBEEF12345, 3, 1), (7, 255, 2)):
        raw, nrm = P.philox_probe(seed, level, tag, cells, steps)
        worst = 0.0
        for k in range(0, n, 7):
            want = orc.philox_cell(seed, level, tag, int(cells[k]), int(steps[k]))
            assert list(raw[k]) == want, (seed, level, tag, k)
            if tag == 1:
                xi = orc.normals(seed, level, int(cells[k]), int(steps[k]))
                worst = max(worst, max(abs(float(nrm[k, c]) - xi[c]) for c in range(3)))
        assert worst <= 2e-5, worst


def test_axes_match_oracle(P, orc):
    wl = W.workload("block_b2_cone10")
    wl["levels"][0].update(nx=16, ny=12, nz=10)
    sim = P.Sim(wl["material"], wl["levels"])
    u_gpu = sim.axes(0).T.astype(np.float64)
    u_ref = orc.make_axes(oracle_level(wl))
    assert np.abs(u_gpu - u_ref).max() < 2e-6
    ct = u_ref[:, 2]
    assert ct.min() >= math.cos(math.radians(10)) - 1e-12
    sim.close()


def _trajectory_check(P, orc, wl, nsteps, plan=None, every=1, tol=1e-5, check_loop=True, stream_shape=None):
    lv = oracle_level(wl)
    sim = P.Sim(wl["material"], wl["levels"])
    if plan is not None:
        sim.set_plan(0, plan)
    if stream_shape is not None:
        sim.set_stream_shape(0, *stream_shape)
    u = orc.make_axes(lv)
    N = lv["nx"] * lv["ny"] * lv["nz"]
    m_ref = np.tile([0.0, 0.0, 1.0], (N, 1))
    mbar_ref = [1.0]
    worst = 0.0
    n = 0
    while n < nsteps:
        k = min(every, nsteps - n)
        sim.run_steps(k)
        m_ref, mb = orc.run(lv, wl["levels"][0]["seed_base"], n, k, m_ref, u=u)
        mbar_ref.extend(mb[1:].tolist())
        n += k
        d = np.abs(gpu_state(sim) - m_ref).max()
        worst = max(worst, d)
        assert d <= tol, (n, d)
    if check_loop:
        _, mh, _ = sim.loop(0, 0)
        rec_every = wl["levels"][0].get("record_every", 1)
        ref = np.array(mbar_ref)[::rec_every]
        assert np.abs(mh - ref[:len(mh)]).max() <= 2e-6
    sim.close()
    return worst


def test_rod_b4_first_1000_steps_resident(P, orc):
    wl = W.workload("rod_b4_single")
    worst = _trajectory_check(P, orc, wl, 1000, plan=P.PLAN_RESIDENT, every=1)
    print("worst |dm| over 1000 steps (resident):", worst)


def test_rod_b4_first_1000_steps_stream(P, orc):
    wl = W.workload("rod_b4_single")
    worst = _trajectory_check(P, orc, wl, 1000, plan=P.PLAN_STREAM, every=10)
    print("worst |dm| over 1000 steps (stream):", worst)


def test_plans_bit_identical(P):
    wl = W.workload("rod_b4_single")
    out = []
    for plan in (P.PLAN_RESIDENT, P.PLAN_STREAM):
        sim = P.Sim(wl["material"], wl["levels"])
        sim.set_plan(0, plan)
        sim.run_steps(300)
        out.append(sim.get_state(0, 0))
        sim.close()
    assert np.array_equal(out[0], out[1])


def test_runs_are_deterministic(P):
    wl = W.workload("rod_b4_single")
    wl["levels"][0]["n_real"] = 4
    res = []
    for _ in range(2):
        sim = P.Sim(wl["material"], wl["levels"])
        sim.run_steps(500)
        res.append((sim.get_state(0, 3), sim.loop(0, -1)[1]))
        sim.close()
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])


@pytest.mark.parametrize("dims", [(40, 36, 20), (13, 7, 5), (1, 1, 9), (1, 1, 1), (70, 9, 3)])
def test_stream_ragged_tiles_with_cone(P, orc, dims):
    wl = W.workload("block_b2_cone10")
    wl["levels"][0].update(nx=dims[0], ny=dims[1], nz=dims[2])
    wl["material"]["sweep_Oe_per_ns"] = 1e5      # shorter sweep, faster field change
    _trajectory_check(P, orc, wl, 60, plan=P.PLAN_STREAM, every=20)


def test_resident_small_grids(P, orc):
    for dims in ((1, 1, 1), (3, 1, 1), (5, 4, 3)):
        wl = W.workload("rod_b4_single")
        wl["levels"][0].update(nx=dims[0], ny=dims[1], nz=dims[2])
        _trajectory_check(P, orc, wl, 200, plan=P.PLAN_RESIDENT, every=50)


# resident workgroups of every width: 2 chunks (4 cell waves + noise waves),
# 6 chunks (8 + noise waves), 16 chunks (16 waves, the folder owns a chunk,
# noise drawn inline), 18 chunks (two chunks per wave)
@pytest.mark.parametrize("dims", [(4, 4, 8), (6, 8, 8), (10, 10, 10), (8, 12, 12)])
def test_resident_workgroup_widths(P, orc, dims):
    wl = W.workload("block_b2_cone10")
    wl["levels"][0].update(nx=dims[0], ny=dims[1], nz=dims[2], n_real=2)
    wl["material"]["sweep_Oe_per_ns"] = 1e5
    _trajectory_check(P, orc, wl, 120, plan=P.PLAN_RESIDENT, every=40)
    out = []
    for plan in (P.PLAN_RESIDENT, P.PLAN_STREAM):
        sim = P.Sim(wl["material"], wl["levels"])
        sim.set_plan(0, plan)
        sim.run_steps(120)
        out.append((sim.get_state(0, 1), sim.loop(0, 1)[1], sim.kernel_name(0)))
        sim.close()
    assert np.array_equal(out[0][0], out[1][0]), out[0][2]
    assert np.abs(out[0][1] - out[1][1]).max() < 1e-6


def test_realizations_are_independent_streams(P, orc):
    wl = W.workload("rod_b4_single")
    wl["levels"][0]["n_real"] = 3
    wl["levels"][0]["seed_base"] = 11
    lv = oracle_level(wl)
    sim = P.Sim(wl["material"], wl["levels"])
    sim.run_steps(100)
    N = lv["nx"] * lv["ny"] * lv["nz"]
    for r in range(3):
        m_ref, _ = orc.run(lv, 11 + r, 0, 100, np.tile([0.0, 0.0, 1.0], (N, 1)))
        assert np.abs(gpu_state(sim, 0, r) - m_ref).max() < 1e-5
    sim.close()


# ---- persistent z-slab plan (workgroups of one realization exchange planes)



# (kind, threads, cells per thread, planes): kind 0 recomputes the halo
# predictor, kind 1 exchanges m' as well; None = the plan's default kernel
SLAB_SHAPES = [None, (0, 1024, 1, 2), (1, 1024, 1, 2), (1, 1024, 1, 1), (1, 384, 1, 2), (1, 192, 2, 2),
               (1, 768, 2, 3)]


def set_slab(P, sim, shape):
    if shape is None:
        sim.set_plan(0, P.PLAN_SLAB)
    else:
        sim.set_slab_shape(0, *shape)


@pytest.mark.parametrize("shape", SLAB_SHAPES)
def test_slab_plan_matches_oracle_and_other_plans(P, orc, shape):
    wl = W.workload("rod_b1_ens8")
    wl["levels"][0]["n_real"] = 2
    out = {}
    for plan in (P.PLAN_STREAM, P.PLAN_SLAB):
        sim = P.Sim(wl["material"], wl["levels"])
        if plan == P.PLAN_SLAB:
            set_slab(P, sim, shape)
        else:
            sim.set_plan(0, plan)
        sim.run_steps(300)
        out[plan] = (sim.get_state(0, 1), sim.loop(0, 1)[1])
        sim.close()
    assert np.array_equal(out[P.PLAN_STREAM][0], out[P.PLAN_SLAB][0])
    assert np.abs(out[P.PLAN_STREAM][1] - out[P.PLAN_SLAB][1]).max() < 1e-6
    lv = oracle_level(wl)
    N = lv["nx"] * lv["ny"] * lv["nz"]
    m_ref, mb = orc.run(lv, 2, 0, 300, np.tile([0.0, 0.0, 1.0], (N, 1)))
    assert np.abs(out[P.PLAN_SLAB][0].T - m_ref).max() < 1e-5
    assert np.abs(out[P.PLAN_SLAB][1] - mb).max() < 2e-6


@pytest.mark.parametrize("shape", [None, (1, 192, 2, 1), (1, 1024, 1, 2)])
@pytest.mark.parametrize("dims", [(5, 7, 11), (8, 24, 5), (3, 2, 4)])
def test_slab_plan_ragged(P, orc, dims, shape):
    wl = W.workload("block_b2_cone10")
    wl["levels"][0].update(nx=dims[0], ny=dims[1], nz=dims[2], n_real=2)
    wl["material"]["sweep_Oe_per_ns"] = 1e5
    lv = oracle_level(wl)
    sim = P.Sim(wl["material"], wl["levels"])
    set_slab(P, sim, shape)
    u = orc.make_axes(lv)
    N = lv["nx"] * lv["ny"] * lv["nz"]
    m_ref = [np.tile([0.0, 0.0, 1.0], (N, 1)) for _ in range(2)]
    for n in range(0, 150, 50):
        sim.run_steps(50)
        for r in range(2):
            m_ref[r], _ = orc.run(lv, 1 + r, n, 50, m_ref[r], u=u)
            assert np.abs(gpu_state(sim, 0, r) - m_ref[r]).max() < 1e-5, (dims, n, r)
    sim.close()


@pytest.mark.parametrize("shape", [None, (1, 192, 2, 1)])
def test_slab_plan_chunks_and_checkpoints(P, shape):
    # more steps than one slab launch holds, checkpoints written by the slab kernel
    wl = W.workload("rod_b4_adjoint64")
    wl["material"]["sweep_Oe_per_ns"] *= 20          # 2000 steps
    wl["levels"][0]["n_real"] = 2
    res = {}
    for plan in (P.PLAN_RESIDENT, P.PLAN_SLAB):
        sim = P.Sim(wl["material"], wl["levels"], ckpt_every=256)
        if plan == P.PLAN_SLAB:
            set_slab(P, sim, shape)
        else:
            sim.set_plan(0, plan)
        sim.run_sweep()
        res[plan] = (sim.get_state(0, 1), sim.grad(0))
        sim.close()
    assert np.array_equal(res[P.PLAN_RESIDENT][0], res[P.PLAN_SLAB][0])
    assert np.allclose(res[P.PLAN_RESIDENT][1][0], res[P.PLAN_SLAB][1][0], rtol=1e-5)


# ---- full-width streamed kernel with the z-columns in registers (kind 2)
ROWS2 = [(2, 1024, 2, 1), (2, 1024, 1, 1), (2, 768, 2, 1), (2, 512, 2, 1), (2, 256, 2, 1), (2, 192, 1, 1)]


@pytest.mark.parametrize("shape", ROWS2)
@pytest.mark.parametrize("dims,tz", [((40, 36, 20), 7), ((13, 7, 5), 2), ((1, 1, 9), 4), ((70, 9, 3), 1),
                                     ((96, 40, 6), 3)])
def test_rows2_ragged_tiles_with_cone(P, orc, shape, dims, tz):
    wl = W.workload("block_b2_cone10")
    wl["levels"][0].update(nx=dims[0], ny=dims[1], nz=dims[2])
    wl["material"]["sweep_Oe_per_ns"] = 1e5
    probe = P.Sim(wl["material"], wl["levels"])
    try:
        probe.set_stream_shape(0, *shape, tz)
    except P.SllgError:
        probe.close()
        pytest.skip("tiling does not fit this grid")
    probe.close()
    _trajectory_check(P, orc, wl, 60, every=20, stream_shape=(*shape, tz))


@pytest.mark.parametrize("cone", [10.0, 0.0])
def test_rows2_bit_identical_to_window_kernel(P, cone):
    # a 128 x 128 x 24 slice of the block, 20 steps: every streamed kernel
    # gives the same bits
    wl = W.workload("block_b2_cone10")
    wl["levels"][0].update(nz=24, cone_deg=cone)
    out = []
    for shape in [(0, 64, 8, 1, 8), (2, 1024, 2, 1, 8), (2, 512, 2, 1, 5), (2, 1024, 1, 1, 24)]:
        sim = P.Sim(wl["material"], wl["levels"])
        sim.set_stream_shape(0, *shape)
        sim.run_steps(20)
        out.append((sim.get_state(0, 0), sim.loop(0, 0)[1]))
        sim.close()
    for st, mh in out[1:]:
        assert np.array_equal(st, out[0][0])
        assert np.abs(mh - out[0][1]).max() < 1e-6


# ---- full-size workloads in the launch configuration the benchmark times
@pytest.mark.parametrize("cells,planes", [(1, 43), (2, 19)])
def test_block_full_size_bench_configuration(P, orc, cells, planes):
    # the 128 x 128 x 512 block on the two tile kernels the tuner picks
    # between for the benchmark (k_rows2<1024,1>, 43 planes per tile, and
    # k_rows2<1024,2>, 19 planes), three steps against the FP64 oracle over
    # all 8.4M cells
    wl = W.workload("block_b2_cone10")
    lv = oracle_level(wl)
    sim = P.Sim(wl["material"], wl["levels"])
    sim.set_stream_shape(0, 2, 1024, cells, 1, planes)
    assert sim.kernel_name(0).startswith(f"k_rows2<1024,{cells}> tz {planes}"), sim.kernel_name(0)
    sim.run_steps(3)
    N = lv["nx"] * lv["ny"] * lv["nz"]
    m_ref, mb = orc.run(lv, 1, 0, 3, np.tile([0.0, 0.0, 1.0], (N, 1)), u=orc.make_axes(lv))
    d = np.abs(gpu_state(sim) - m_ref).max()
    assert d <= 1e-5, d
    _, mh, _ = sim.loop(0, 0)
    assert np.abs(mh[:4] - mb).max() <= 2e-6
    sim.close()


def test_rod_ensemble_full_size_bench_configuration(P, orc):
    # the 8-realization b = 1 rod on the plan the tuner picks for the
    # benchmark (slab), 200 steps, the last realization against the oracle
    wl = W.workload("rod_b1_ens8")
    lv = oracle_level(wl)
    sim = P.Sim(wl["material"], wl["levels"])
    assert sim.kernel_name(0).startswith("k_slab"), sim.kernel_name(0)
    sim.run_steps(200)
    N = lv["nx"] * lv["ny"] * lv["nz"]
    m_ref, mb = orc.run(lv, 8, 0, 200, np.tile([0.0, 0.0, 1.0], (N, 1)))
    assert np.abs(gpu_state(sim, 0, 7) - m_ref).max() <= 1e-5
    _, mh, _ = sim.loop(0, 7)
    assert np.abs(mh[:201] - mb).max() <= 2e-6
    sim.close()
