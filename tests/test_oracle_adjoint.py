"""Pins of the oracle's discrete adjoint: gradients of loop losses with
respect to the step constants and to (K, A, alpha, ms_scale) must equal
central finite differences of the FP64 forward run."""
import math

import numpy as np
import pytest

import sllg_workloads as W
from oracle import gk


def small_level(nsteps_period=400, **over):
    wl = W.workload("rod_b4_single")
    wl["material"]["sweep_Oe_per_ns"] = 2e4 * 40000 / nsteps_period
    lv = gk.compile_level(wl["material"], dict(wl["levels"][0], nx=2, ny=2, nz=3))
    lv.update(over)
    return lv


def loss(orc, lv, seeds, nsteps, w):
    mbar, _ = orc.run_batch(lv, seeds, nsteps)
    return w @ mbar.sum(axis=0)


CONSTS = ("c_ex", "hk", "gamma1", "alpha", "sigma")


def test_adjoint_raw_constants_vs_fd(orc):
    lv = small_level()
    nsteps = 300
    seeds = [1, 2]
    rng = np.random.default_rng(5)
    w = rng.normal(size=(2, nsteps + 1))
    g, _ = orc.adjoint_batch(lv, seeds, nsteps, w)
    for j, key in enumerate(CONSTS):
        h = 1e-4 * abs(lv[key])
        lp, lm = dict(lv), dict(lv)
        lp[key] += h
        lm[key] -= h
        fd = (loss(orc, lp, seeds, nsteps, w) - loss(orc, lm, seeds, nsteps, w)) / (2 * h)
        for l in range(2):
            assert g[l, j] == pytest.approx(fd[l], rel=1e-3, abs=1e-9 * abs(fd[l]).max()), (key, l)


def _params_to_level(base_wl, K, A, alpha, ms):
    """Level with the given simulated K, A, alpha and Ms multiplier."""
    wl = W.workload("rod_b4_single") if base_wl is None else base_wl
    mat = dict(wl["material"], ms_scale=ms)
    lvd = dict(wl["levels"][0], alpha=alpha)
    lv = gk.compile_level(mat, lvd)
    # replace K and A by the requested simulated values
    lv["K"], lv["A"] = K, A
    lv["hk"] = 2 * K / (gk.MU0 * lv["Ms"])
    lv["c_ex"] = 2 * A / (gk.MU0 * lv["Ms"] * lv["a"] ** 2)
    return lv


def test_chain_rule_to_material_parameters_vs_fd(orc):
    wl = W.workload("rod_b4_single")
    wl["material"]["sweep_Oe_per_ns"] = 2e4 * 100
    wl["levels"][0].update(nx=2, ny=2, nz=3)
    lv0 = gk.compile_level(wl["material"], wl["levels"][0])
    nsteps = lv0["n_steps"]
    seeds = [3, 4, 5]
    H = orc.field_schedule_Oe(lv0)
    mbar, _ = orc.run_batch(lv0, seeds, nsteps)
    w = orc.loss_weights(H, mbar.mean(axis=0), len(seeds))[:1]   # area only
    g, _ = orc.adjoint_batch(lv0, seeds, nsteps, w)
    dK, dA, dal, dms = gk.chain_rule(g[0], lv0)
    base = dict(K=lv0["K"], A=lv0["A"], alpha=lv0["alpha"], ms=1.0)
    for name, want in (("K", dK), ("A", dA), ("alpha", dal), ("ms", dms)):
        h = 1e-4 * base[name]
        vals = []
        for sgn in (1, -1):
            p = dict(base)
            p[name] += sgn * h
            lv = _params_to_level(wl, p["K"], p["A"], p["alpha"], p["ms"])
            if name == "ms":   # Ms scaling keeps the simulated K and A
                lv = _params_to_level(wl, base["K"], base["A"], base["alpha"], p["ms"])
            vals.append(loss(orc, lv, seeds, nsteps, w)[0])
        fd = (vals[0] - vals[1]) / (2 * h)
        assert want == pytest.approx(fd, rel=1e-3), name


def switching_workload():
    """b = 8 rod, alpha = 1, 50 fs, 500 Oe/ns: loops that reverse."""
    wl = W.workload("rod_b4_single")
    wl["material"].update(sweep_Oe_per_ns=500.0)
    wl["levels"][0].update(b=8, nx=1, ny=3, nz=7, alpha=1.0, dt_s=50e-15)
    return wl


def test_coercive_field_gradient_vs_fd(orc):
    wl = switching_workload()
    lv0 = gk.compile_level(wl["material"], wl["levels"][0])
    nsteps = lv0["n_steps"]
    seeds = list(range(1, 9))
    H = orc.field_schedule_Oe(lv0)
    mbar, _ = orc.run_batch(lv0, seeds, nsteps)
    st = orc.loop_stats(H, mbar.mean(axis=0))
    assert st["k_desc"] >= 0 and st["k_asc"] >= 0
    w = orc.loss_weights(H, mbar.mean(axis=0), len(seeds))
    g, _ = orc.adjoint_batch(lv0, seeds, nsteps, w)
    grads = gk.chain_rule(g[1], lv0)
    base = dict(K=lv0["K"], A=lv0["A"], alpha=lv0["alpha"], ms=1.0)

    def hc(p):
        lv = _params_to_level(wl, p["K"], p["A"], p["alpha"], p["ms"])
        mb, _ = orc.run_batch(lv, seeds, nsteps)
        return orc.loop_stats(H, mb.mean(axis=0))["Hc"]

    for (name, want) in zip(("K", "A", "alpha", "ms"), grads):
        h = 1e-4 * base[name]
        p1, p2 = dict(base), dict(base)
        p1[name] += h
        p2[name] -= h
        fd = (hc(p1) - hc(p2)) / (2 * h)
        assert want == pytest.approx(fd, rel=1e-3, abs=1e-6 * abs(st["Hc"]) / base[name]), name
