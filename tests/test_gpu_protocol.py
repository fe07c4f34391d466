"""GPU parity on the paper's sweep-rate/damping protocol (Fig. 4 and the
single-cell limit of the cell-size discussion).

The protocol differs from the other workloads in four ways, each checked
here against the FP64 oracle: a cosine sweep (the GPU evaluates cos(2 pi s)
in FP64 every step), easy axes in a 5 degree cone, alpha set by the SR/alpha
rule (alpha = 0.1 SR / 0.25 Oe/ns), and a one-cell level whose cube has the
rod's volume (b = 10752^(1/3)).
"""
import math

import numpy as np
import pytest

import sllg_workloads as W
from oracle import gk

pytestmark = pytest.mark.gpu

PARAM_CHECK = ("zeta", "A", "K", "Ms", "a", "c_ex", "hk", "gamma1", "alpha", "sigma", "dt",
               "hscale", "cM", "hz_amp")


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1912_00310_amd as P
    P.lib()
    return P


def test_protocol_level_constants(P):
    wl = W.workload("rod_sine_sr250_ens100")
    sim = P.Sim(wl["material"], wl["levels"])
    for i, lvd in enumerate(wl["levels"]):
        lv = gk.compile_level(wl["material"], lvd, i)
        got = sim.level_params(i)
        for k in PARAM_CHECK:
            assert got[k] == pytest.approx(lv[k], rel=1e-12), (i, k)
        assert int(got["n_steps"]) == lv["n_steps"] == 1_600_000
        assert got["alpha"] == pytest.approx(100.0)
    # the single cell has the rod's volume
    a1 = sim.level_params(2)["a"]
    assert a1 ** 3 == pytest.approx(10752 * wl["material"]["a0_m"] ** 3, rel=1e-12)
    sim.close()


def test_protocol_levels_first_1000_steps(P, orc):
    # every level of the batched protocol, two realizations each, against the
    # oracle on the same Philox stream (level index in the counter)
    wl = W.workload("rod_sine_sr250_ens100")
    for lvd in wl["levels"]:
        lvd["n_real"] = 2
    sim = P.Sim(wl["material"], wl["levels"])
    lvs = [gk.compile_level(wl["material"], lvd, i) for i, lvd in enumerate(wl["levels"])]
    us = [orc.make_axes(lv) for lv in lvs]
    N = [lv["nx"] * lv["ny"] * lv["nz"] for lv in lvs]
    m_ref = {(i, r): np.tile([0.0, 0.0, 1.0], (N[i], 1)) for i in range(3) for r in range(2)}
    worst = 0.0
    for n in range(0, 1000, 250):
        sim.run_steps(250)
        for i in range(3):
            for r in range(2):
                m_ref[i, r], _ = orc.run(lvs[i], 1 + r, n, 250, m_ref[i, r], u=us[i])
                d = np.abs(sim.get_state(i, r).T.astype(np.float64) - m_ref[i, r]).max()
                worst = max(worst, d)
                assert d <= 1e-5, (i, r, n, d)
    # the cone: every easy axis within 5 degrees of z
    for i in range(3):
        assert us[i][:, 2].min() >= math.cos(math.radians(5.0)) - 1e-12
        assert np.abs(sim.axes(i).T - us[i]).max() < 2e-6
    print("worst |dm| over 1000 steps, three protocol levels:", worst)
    sim.close()


def cosine_switching_workload(n_real=16):
    """The b = 8 level of the protocol under a cosine sweep fast enough for a
    whole loop in 8e4 steps of 50 fs (alpha = 1 given directly)."""
    wl = W.workload("rod_sine_sr250_ens100")
    wl["material"].update(sweep_Oe_per_ns=500.0, sr_ref_Oe_per_ns=0.0)
    lv = dict(wl["levels"][1], alpha=1.0, dt_s=50e-15, n_real=n_real, record_every=1)
    wl["levels"] = [lv]
    return wl


def test_cosine_sweep_loop_matches_oracle(P, orc):
    wl = cosine_switching_workload(16)
    lv = gk.compile_level(wl["material"], wl["levels"][0], 0)
    seeds = [1 + r for r in range(16)]
    mbar, _ = orc.run_batch(lv, seeds, lv["n_steps"], u=orc.make_axes(lv))
    H = orc.field_schedule_Oe(lv)
    ref = orc.ensemble_stats(lv, H, mbar)
    sim = P.Sim(wl["material"], wl["levels"])
    sim.run_sweep()
    Hg, mg, st = sim.loop(0, -1)
    # the FP64 field schedule of the cosine sweep
    assert np.allclose(Hg, H, rtol=0, atol=1e-9)
    assert H[0] == pytest.approx(lv["hscale"] * 500.0)
    assert H[lv["n_steps"] // 2] == pytest.approx(-lv["hscale"] * 500.0)
    # whole-loop statistics within two standard errors, same crossings
    assert not math.isnan(ref["Hc"])
    for key, rkey, se in (("Hc_sim", "Hc", "Hc_se"), ("S_sim", "S_sim", "S_se")):
        s = math.sqrt(st[se] ** 2 + ref[se] ** 2)
        assert abs(st[key] - ref[rkey]) <= 2 * s, (key, st[key], ref[rkey], s)
    assert np.abs(mg[:1001] - mbar.mean(axis=0)[:1001]).max() < 1e-5
    sim.close()
