"""Pins of the oracle's coarse-graining rule (Eqs. 2-13) against numbers the
paper prints and against the exact solution of the RG flow."""
import json
import math
import os

import pytest

from oracle import gk

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.json")))


def v(key):
    return GOLD[key]["value"]


def test_heisenberg_tc_and_jeff():
    # J_eff = a0 A0 and Tc = 1.44 J_eff / k_B (material paragraph)
    a0 = v("a0_nm") * 1e-9
    assert a0 * v("A0_J_per_m") == pytest.approx(v("J_eff_J"), rel=1e-3)
    assert gk.heisenberg_tc(a0, v("A0_J_per_m")) == pytest.approx(v("Tc_K"), rel=1e-3)


def test_t_and_zeta_printed():
    t = 310.0 / v("Tc_K")
    assert t == pytest.approx(v("t"), abs=5e-5)
    for b, z in v("zeta").items():
        assert abs(gk.zeta(t, float(b)) - z) < 5e-5, b


def test_zeta_limits():
    # b = 1 leaves the system unchanged; b -> infinity tends to 1 - t
    assert gk.zeta(0.4, 1.0) == pytest.approx(1.0, abs=1e-15)
    assert gk.zeta(0.4, 1e12) == pytest.approx(0.6, abs=1e-9)


def test_rg_flow_matches_closed_form_exactly_without_h_g():
    # With h = g = 0 the flow of Eqs. (4)-(7) started at T*(0) = 2 pi t has
    # the exact solution zeta = t/b + 1 - t (the paper's analytic solution).
    for t in (0.1, 0.3613, 0.7):
        for b in (2.0, 4.0, 8.0, 22.0):
            _, _, _, z = gk.rg_flow(2 * math.pi * t, 0.0, 0.0, b)
            assert abs(z - gk.zeta(t, b)) < 1e-10, (t, b)


def test_rg_flow_close_to_closed_form_with_paper_h_g():
    # "practically indistinguishable" for g, h << 1 (text before Eq. 8)
    a0 = v("a0_nm") * 1e-9
    A0, Ms, K0 = v("A0_J_per_m"), v("Ms_A_per_m"), v("K0_J_per_m3")
    t = 310.0 / v("Tc_K")
    for H in (500.0, 1000.0):
        h0, g0 = gk.reduced_field_anisotropy(H, K0, Ms, A0, 1.0, a0)
        assert h0 < 1e-3 and g0 < 1e-3
        for b in (2.0, 4.0, 8.0, 22.0):
            _, _, _, z = gk.rg_flow(2 * math.pi * t, h0, g0, b)
            zc = gk.zeta(t, b)
            assert abs(z / zc - 1) < 1.5e-3, (H, b, z, zc)
            assert z >= zc  # h, g > 0 reduce F and so the decay of zeta


def test_rg_flow_h_doubles_per_octave():
    # dh/dl = 2h: h(b) = b^2 h(0)
    _, h, _, _ = gk.rg_flow(1.0, 1e-4, 0.0, 8.0)
    assert h == pytest.approx(64e-4, rel=1e-9)


def test_exchange_lengths_use_unscaled_ms():
    # l_ex,b = sqrt(2 zeta A0/(mu0 Ms^2)) with Ms NOT rescaled (paragraph after the areas)
    A0, Ms = v("A0_J_per_m"), v("Ms_A_per_m")
    assert gk.exchange_length(A0, Ms) * 1e9 == pytest.approx(v("l_ex0_nm"), abs=0.005)
    t = 310.0 / v("Tc_K")
    for b, l in v("l_exb_nm").items():
        z = gk.zeta(t, float(b))
        assert gk.exchange_length(z * A0, Ms) * 1e9 == pytest.approx(l, abs=0.006), b
    assert 8 * v("a0_nm") == pytest.approx(v("a8_nm"), abs=5e-4)


def test_cell_counts_and_rod_volume():
    nx, ny, nz = v("rod_cells_a0")
    for b, n in v("cells").items():
        b = int(b)
        assert (nx // b) * (ny // b) * (nz // b) == n
    assert abs((nx * ny * nz) ** (1 / 3) - 22) < 0.1  # geometric mean b = 22


def test_equivalent_temperature_limits():
    # Eq. (12): T(1) = T0; T(b) falls with b and T(b)*b*zeta = T0
    t0 = 310.0
    t = t0 / v("Tc_K")
    assert gk.equivalent_temperature(t0, 1.0, 1.0) == t0
    prev = t0
    for b in (2.0, 4.0, 8.0, 22.0):
        z = gk.zeta(t, b)
        Tb = gk.equivalent_temperature(t0, b, z)
        assert Tb < prev
        prev = Tb


def test_m_rescale_special_cases():
    # Eq. (13): delta = 1 reduces to Eq. (11) (factor zeta), delta = 0 to no rescale
    for z in (0.6551, 0.7290, 1.0):
        assert gk.loop_m_scale(1.0, z) == pytest.approx(z)
        assert gk.loop_m_scale(0.0, z) == 1.0
    assert gk.loop_m_scale(v("delta"), 1.0) == 1.0


def test_sr_alpha_rule():
    p = v("sr_alpha_pair")
    assert p["SR_Oe_per_ns"] / p["alpha"] == pytest.approx(p["ratio"])
    assert gk.alpha_sweep_scaled(p["alpha"], 1000.0, p["SR_Oe_per_ns"]) == pytest.approx(400.0)
    # the ratio is what is preserved
    a = gk.alpha_sweep_scaled(0.1, 2.5, 0.25)
    assert 2.5 / a == pytest.approx(p["ratio"])


def test_compile_level_rod_b4():
    import sllg_workloads as W
    wl = W.workload("rod_b4_single")
    lv = gk.compile_level(wl["material"], wl["levels"][0])
    t = 310.0 / 858.0
    z = gk.zeta(t, 4.0)
    assert lv["zeta"] == z
    assert lv["A"] == pytest.approx(z * 0.98e-11)
    assert lv["K"] == pytest.approx(z ** 3 * 1e4)
    assert lv["Ms"] == 480e3                       # not rescaled with b
    assert lv["n_steps"] == 40000                  # 4000 Oe of sweep at 2e4 Oe/ns, 5 fs
    assert lv["hscale"] == z and lv["cM"] == pytest.approx(1 - 0.511 * (1 - z))
    # H_K in Oe for K(4): 2K/(mu0 Ms) / (1000/4pi)
    assert lv["hk"] / gk.OE_TO_APM == pytest.approx(2 * z ** 3 * 1e4 / (gk.MU0 * 480e3) / gk.OE_TO_APM)


def test_dt_rule_gives_paper_steps():
    # 1 fs at b = 1 (Fig. 2 caption) and at least 5x larger for b >= 2
    import sllg_workloads as W
    m = dict(W.BASE_MATERIAL, scale_AK=True)
    for b, want in ((1, 1e-15), (2, 5e-15), (4, 5e-15), (8, 5e-15)):
        lvd = dict(nx=1, ny=1, nz=1, b=b, alpha=0.1, dt_s=0.0)
        assert gk.compile_level(m, lvd)["dt"] == pytest.approx(want), b
