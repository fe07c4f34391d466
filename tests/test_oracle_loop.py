"""Pins of the oracle's loop analytics (area, coercive field, remanence) on
loops whose values are known in closed form, and of the loss weights used
by the adjoint against finite differences of those analytics."""
import math

import numpy as np
import pytest


def triangle(Hm, n):
    """H_k for a +Hm -> -Hm -> +Hm triangle with n segments (n % 4 == 0)."""
    k = np.arange(n + 1)
    s = k / n
    return np.where(2 * k <= n, Hm * (1 - 4 * s), Hm * (4 * s - 3))


def parallelogram(H, Hc, w):
    """Piecewise-linear loop: +1 -> -1 ramp of half-width w centred on -Hc on
    the falling branch, mirrored on the rising branch."""
    n = len(H) - 1
    m = np.empty_like(H)
    for k, h in enumerate(H):
        centre = -Hc if 2 * k <= n else Hc
        sgn = 1.0 if 2 * k <= n else -1.0
        m[k] = np.clip((h - centre) / w, -1, 1) if sgn > 0 else np.clip((h - centre) / w, -1, 1)
    return m


def test_parallelogram_area_hc_mr(orc):
    Hm, n = 1000.0, 400          # 10 Oe per segment
    H = triangle(Hm, n)
    Hc, w = 300.0, 50.0          # kinks land on grid points
    m = parallelogram(H, Hc, w)
    st = orc.loop_stats(H, m)
    assert st["S"] == pytest.approx(4 * Hc, rel=1e-12)      # width 2Hc, height 2
    assert st["Hstar_desc"] == pytest.approx(-Hc, rel=1e-12)
    assert st["Hstar_asc"] == pytest.approx(Hc, rel=1e-12)
    assert st["Hc"] == pytest.approx(Hc, rel=1e-12)
    assert st["Mr"] == pytest.approx(1.0)
    assert st["n_cross_desc"] == 1 and st["n_cross_asc"] == 1


def test_area_sign_and_reversal(orc):
    H = triangle(1000.0, 400)
    m = parallelogram(H, 300.0, 50.0)
    # a loop traversed the other way round has negative area
    st = orc.loop_stats(H[::-1].copy(), m[::-1].copy())
    assert st["S"] == pytest.approx(-1200.0, rel=1e-12)


def test_no_crossing_gives_nan(orc):
    H = triangle(1000.0, 400)
    m = 0.9 + 0.05 * np.cos(np.linspace(0, 2 * np.pi, len(H)))
    st = orc.loop_stats(H, m)
    assert math.isnan(st["Hc"]) and st["k_desc"] == -1 and st["k_asc"] == -1
    assert st["n_cross_desc"] == 0


def test_first_crossing_is_selected(orc):
    H = triangle(1000.0, 400)
    m = parallelogram(H, 300.0, 50.0)
    # a noisy dip below zero early on the falling branch
    k0 = 30
    m[k0] = -0.2
    st = orc.loop_stats(H, m)
    assert st["k_desc"] == k0 - 1
    assert st["n_cross_desc"] == 3
    want = H[k0 - 1] - m[k0 - 1] * (H[k0] - H[k0 - 1]) / (m[k0] - m[k0 - 1])
    assert st["Hstar_desc"] == pytest.approx(want)


def test_loss_weights_match_finite_differences(orc):
    H = triangle(1000.0, 200)
    rng = np.random.default_rng(0)
    m = parallelogram(H, 300.0, 60.0) + 0.01 * rng.normal(size=len(H))
    w = orc.loss_weights(H, m, n_real=1)
    h = 1e-7
    for k in range(len(H)):
        mp, mm = m.copy(), m.copy()
        mp[k] += h
        mm[k] -= h
        sp, sm = orc.loop_stats(H, mp), orc.loop_stats(H, mm)
        assert (sp["S"] - sm["S"]) / (2 * h) == pytest.approx(w[0, k], rel=1e-5, abs=1e-4)
        if sp["k_desc"] == sm["k_desc"] and sp["k_asc"] == sm["k_asc"]:
            assert (sp["Hc"] - sm["Hc"]) / (2 * h) == pytest.approx(w[1, k], rel=1e-5, abs=1e-5)
    assert np.count_nonzero(w[1]) == 4
    # weights are per realization of an n_real ensemble
    assert np.allclose(orc.loss_weights(H, m, n_real=4), w / 4)
