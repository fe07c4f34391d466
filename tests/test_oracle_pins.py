"""Pins of the oracle parts that the physics tests do not reach on their own:
the Philox4x32 constants, the distribution of the per-cell easy axes in a
cone (the "5 degree dispersion" of the material paragraph), and the standard
errors of the ensemble statistics (one standard error, Fig. 2 caption)."""
import json
import math
import os
import statistics
from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy import stats

from oracle import gk
import sllg_workloads as W

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "philox4x32_constants.json")))


# ---------------------------------------------------------------------------
# Philox4x32-10
# ---------------------------------------------------------------------------

def _weyl(x: Decimal, bits: int) -> int:
    return int((x - 1) * (Decimal(2) ** bits))


def test_philox_weyl_constants_from_their_definition():
    # The key increments are the fractional parts of the golden ratio and of
    # sqrt(3) in fixed point (SC'11); 40 digits are ample for 64 bits.
    getcontext().prec = 40
    phi = (1 + Decimal(5).sqrt()) / 2
    r3 = Decimal(3).sqrt()
    assert _weyl(phi, 32) == int(GOLD["weyl"][0], 16)
    assert _weyl(r3, 32) == int(GOLD["weyl"][1], 16)
    # the same definition gives the 64-bit increments that numpy's
    # Philox4x64 uses (the oracle matches numpy bit for bit elsewhere)
    assert _weyl(phi, 64) == 0x9E3779B97F4A7C15
    assert _weyl(r3, 64) == 0xBB67AE8584CAA73B


def _philox4x32_10_ref(ctr, key):
    """Philox4x32-10 from the SC'11 description: each round computes the two
    products M0*c0 and M1*c2 as 64-bit numbers; the new words are
    (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0)); the key
    is bumped by the Weyl increments between rounds."""
    M0, M1 = (int(x, 16) for x in GOLD["multipliers"])
    W0, W1 = (int(x, 16) for x in GOLD["weyl"])
    c = [int(x) & 0xFFFFFFFF for x in ctr]
    k0, k1 = (int(x) & 0xFFFFFFFF for x in key)
    for _ in range(GOLD["rounds"]):
        p0, p1 = M0 * c[0], M1 * c[2]
        c = [((p1 >> 32) ^ c[1] ^ k0) & 0xFFFFFFFF, p1 & 0xFFFFFFFF,
             ((p0 >> 32) ^ c[3] ^ k1) & 0xFFFFFFFF, p0 & 0xFFFFFFFF]
        k0, k1 = (k0 + W0) & 0xFFFFFFFF, (k1 + W1) & 0xFFFFFFFF
    return c


def test_philox4x32_uses_the_published_constants(orc):
    rng = np.random.default_rng(2024)
    cases = [([0, 0, 0, 0], [0, 0]), ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2)]
    cases += [(list(rng.integers(0, 2**32, 4, dtype=np.uint64)),
               list(rng.integers(0, 2**32, 2, dtype=np.uint64))) for _ in range(300)]
    for ctr, key in cases:
        assert orc.philox4x32_10(ctr, key) == _philox4x32_10_ref(ctr, key), (ctr, key)


# ---------------------------------------------------------------------------
# Per-cell easy axes in a cone
# ---------------------------------------------------------------------------

def _cone_level(axis, cone_deg=10.0, dims=(100, 100, 4), seed=7):
    mat = dict(W.BASE_MATERIAL, easy_axis=tuple(axis))
    lvl = dict(nx=dims[0], ny=dims[1], nz=dims[2], b=2.0, n_real=1, seed_base=1,
               alpha=0.05, dt_s=5e-15, cone_deg=cone_deg, axis_seed=seed,
               record_every=1)
    lv = gk.compile_level(mat, lvl, 0)
    # compile_level keeps the axis as given; the oracle normalises it
    return lv


def _frame(e):
    e = np.asarray(e, float) / np.linalg.norm(e)
    t = np.array([1.0, 0.0, 0.0]) if abs(e[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = t - e * (t @ e)
    e1 /= np.linalg.norm(e1)
    return e, e1, np.cross(e, e1)


@pytest.mark.parametrize("axis", [(0.0, 0.0, 1.0), (1.0, 2.0, 2.0), (0.0, -1.0, 0.0),
                                  (0.0, 0.0, -1.0)])
def test_cone_axes_are_uniform_on_the_spherical_cap(orc, axis):
    # A uniform distribution on a spherical cap of half-angle theta_max about
    # the axis e has (1 - cos theta) uniform on [0, 1 - cos theta_max] and an
    # azimuth about e uniform on the circle (Archimedes' hat-box theorem);
    # its mean vector is e (1 + cos theta_max)/2.
    lv = _cone_level(axis)
    u = orc.make_axes(lv)
    n = len(u)
    assert n == 40000
    assert np.allclose(np.linalg.norm(u, axis=1), 1.0, atol=1e-14)
    e, e1, e2 = _frame(axis)
    cmin = math.cos(math.radians(10.0))
    c = u @ e
    assert c.min() >= cmin - 1e-14
    x = (1.0 - c) / (1.0 - cmin)
    assert stats.kstest(x, "uniform").pvalue > 1e-3
    psi = np.arctan2(u @ e2, u @ e1)
    assert stats.kstest((psi + math.pi) / (2 * math.pi), "uniform").pvalue > 1e-3
    mean = u.mean(axis=0)
    se = u.std(axis=0) / math.sqrt(n)
    want = e * (1.0 + cmin) / 2.0
    assert np.all(np.abs(mean - want) < 5 * se + 1e-15), (mean, want, se)


def test_cone_axes_a_theta_uniform_cap_would_fail_the_pin():
    # the statistic above separates the two readings of a "uniform cone" at
    # this sample size: theta uniform on [0, theta_max] is far from it
    rng = np.random.default_rng(5)
    th = rng.uniform(0.0, math.radians(10.0), 40000)
    cmin = math.cos(math.radians(10.0))
    assert stats.kstest((1 - np.cos(th)) / (1 - cmin), "uniform").pvalue < 1e-10


def test_cone_axes_depend_on_seed_and_level_only(orc):
    a = orc.make_axes(_cone_level((0, 0, 1), dims=(8, 8, 8), seed=3))
    b = orc.make_axes(_cone_level((0, 0, 1), dims=(8, 8, 8), seed=3))
    c = orc.make_axes(_cone_level((0, 0, 1), dims=(8, 8, 8), seed=4))
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert orc.make_axes(_cone_level((0, 0, 1), cone_deg=0.0)) is None


# ---------------------------------------------------------------------------
# Ensemble statistics
# ---------------------------------------------------------------------------

def _triangle(Hm, n):
    k = np.arange(n + 1)
    s = k / n
    return np.where(2 * k <= n, Hm * (1 - 4 * s), Hm * (4 * s - 3))


def _square_ramp_loop(H, Hc, w):
    # +1 -> -1 ramp of half-width w centred on -Hc while H falls, mirrored
    # while it rises: area 4 Hc, coercive field Hc
    n = len(H) - 1
    centre = np.where(2 * np.arange(n + 1) <= n, -Hc, Hc)
    return np.clip((H - centre) / w, -1.0, 1.0)


def test_ensemble_standard_errors(orc):
    # one standard error = sample standard deviation / sqrt(R) over the
    # realizations' areas and coercive fields (Fig. 2 caption); the area of
    # the mean loop is the mean of the areas (the trapezoid is linear in m)
    H = _triangle(1000.0, 800)
    hcs = [150.0, 200.0, 250.0, 300.0, 375.0]
    mbar = np.array([_square_ramp_loop(H, hc, 25.0) for hc in hcs])
    lv = dict(hscale=0.8, cM=0.9)
    st = orc.ensemble_stats(lv, H, mbar)
    areas = [4 * hc for hc in hcs]
    assert st["S_sim"] == pytest.approx(statistics.mean(areas), rel=1e-12)
    assert st["S_se"] == pytest.approx(statistics.stdev(areas) / math.sqrt(5), rel=1e-12)
    assert st["Hc_se"] == pytest.approx(statistics.stdev(hcs) / math.sqrt(5), rel=1e-12)
    assert st["Hc_mean_of_real"] == pytest.approx(statistics.mean(hcs), rel=1e-12)
    # physical units: H / hscale and m * cM (Eqs. 10, 13)
    assert st["S_phys"] == pytest.approx(st["S_sim"] * 0.9 / 0.8, rel=1e-12)
    assert st["Hc_phys"] == pytest.approx(st["Hc"] / 0.8, rel=1e-12)
    assert st["Mr_phys"] == pytest.approx(st["Mr"] * 0.9, rel=1e-12)
    # a single realization has no standard error
    one = orc.ensemble_stats(lv, H, mbar[:1])
    assert math.isnan(one["S_se"]) and math.isnan(one["Hc_se"])


def test_oracle_threads_do_not_change_results(orc):
    # cell loops spread over threads when there are fewer realizations than
    # threads: every cell is still computed the same way
    lv = _cone_level((0, 0, 1), dims=(64, 32, 40))
    a, fa = orc.run_batch(lv, [1, 2], 20, threads=1, want_final=True)
    b, fb = orc.run_batch(lv, [1, 2], 20, threads=4, want_final=True)
    c, fc = orc.run_batch(lv, [1, 2], 20, threads=2, want_final=True)
    assert np.array_equal(a, b) and np.array_equal(fa, fb)
    assert np.array_equal(a, c) and np.array_equal(fa, fc)
