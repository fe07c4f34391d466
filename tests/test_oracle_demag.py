"""Pins of the oracle's magnetostatic field (beyond the paper, which folds
shape anisotropy into K and leaves magnetostatics open): the demagnetising
tensor N of two uniformly magnetised cubes (Newell, Williams, Dunlop 1993)
against what fixes it independently of its closed form, and the field
-Ms sum_j N(r_i - r_j) m_j against its energy."""
import itertools
import math

import numpy as np
import pytest

import sllg_workloads as W
from oracle import gk


def tensor(t):
    xx, yy, zz, xy, xz, yz = t
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def test_self_term_of_a_cube(orc):
    # a uniformly magnetised cube: N = I/3 (symmetry and trace 1)
    t = orc.newell(0, 0, 0)
    assert np.allclose(t[:3], 1 / 3, rtol=0, atol=1e-13)
    assert np.allclose(t[3:], 0, atol=1e-13)


@pytest.mark.parametrize("r", [(1, 0, 0), (1, 1, 0), (1, 1, 1), (2, 1, 0), (3, -2, 1), (5, 3, 2), (0, 7, -4)])
def test_trace_symmetry_and_parity(orc, r):
    # outside the source the field is curl- and divergence-free: trace 0;
    # N(-r) = N(r); exchanging axes exchanges components
    N = tensor(orc.newell(*r))
    assert abs(np.trace(N)) < 1e-12
    assert np.allclose(tensor(orc.newell(*[-c for c in r])), N, atol=1e-14)
    X, Y, Z = r
    P = tensor(orc.newell(Y, X, Z))          # x <-> y
    swap = np.array([[0, 1, 0], [1, 0, 0], [0, 0, 1]])
    assert np.allclose(swap @ N @ swap, P, atol=1e-14)


@pytest.mark.parametrize("r", [(20, 7, 3), (0, 0, 25), (15, -15, 10)])
def test_far_field_is_a_point_dipole(orc, r):
    # far apart, a cube acts as a point dipole of moment M V (V = 1):
    # H = (3 rhat (rhat . m) - m)/(4 pi r^3), so N = -(3 rhat rhat^T - I)/(4 pi r^3);
    # the correction for cubes is of relative order (1/r)^4
    v = np.array(r, float)
    d = np.linalg.norm(v)
    rh = v / d
    want = -(3 * np.outer(rh, rh) - np.eye(3)) / (4 * math.pi * d ** 3)
    got = tensor(orc.newell(*r))
    assert np.abs(got - want).max() < 2e-4 * np.abs(want).max() + 1e-15


def _point_dipole_sum(r, s):
    """Mean over s^3 points of cube i of the dipole field of s^3 point moments
    filling cube j (each 1/s^3 of the unit moment): a brute-force N."""
    g = (np.arange(s) + 0.5) / s - 0.5
    P = np.array(list(itertools.product(g, g, g)))
    N = np.zeros((3, 3))
    for p in P:
        # field at the target point p of the sources at r + P
        v = p - (np.array(r, float) + P)
        dist = np.linalg.norm(v, axis=1)
        rh = v / dist[:, None]
        # N = -(3 rhat rhat^T - I) / (4 pi d^3), summed over sources and averaged
        N += -(3 * np.einsum("ki,kj->ij", rh / dist[:, None] ** 1.5, rh / dist[:, None] ** 1.5)
               - np.eye(3) * np.sum(1 / dist ** 3)) / (4 * math.pi)
    return N / len(P) / len(P)


def test_against_brute_force_point_dipoles(orc):
    # two cubes two edges apart (plus one sideways): the tensor as a double
    # sum of point dipoles, Richardson-extrapolated in the subdivision
    r = (2, 1, 0)
    n8 = _point_dipole_sum(r, 8)
    n16 = _point_dipole_sum(r, 16)
    extrap = n16 + (n16 - n8) / 3.0       # error ~ 1/s^2
    got = tensor(orc.newell(*r))
    assert np.abs(got - extrap).max() < 2e-4 * np.abs(got).max(), (got, extrap)


def _level(dims, demag=True, **over):
    wl = W.workload("rod_b4_single")
    mat = dict(wl["material"], demag=demag)
    lvd = dict(wl["levels"][0], nx=dims[0], ny=dims[1], nz=dims[2])
    lv = gk.compile_level(mat, lvd, 0)
    lv.update(over)
    return lv


@pytest.mark.parametrize("dims", [(3, 3, 3), (2, 2, 6), (4, 1, 2), (2, 6, 14)])
def test_uniform_prism_sum_rule(orc, dims):
    # a uniformly magnetised prism built of cubes: the cell average of
    # sum_j N(r_i - r_j) is the prism's demagnetising tensor, whose trace is
    # 1; a cube of cubes has N = I/3 by symmetry; a square cross-section has
    # N_xx = N_yy; longer axes have smaller factors
    T = orc.demag_tensor(_level(dims))
    nx, ny, nz = dims
    tot = np.zeros(6)
    for i in itertools.product(range(nx), range(ny), range(nz)):
        for j in itertools.product(range(nx), range(ny), range(nz)):
            dx, dy, dz = (i[0] - j[0], i[1] - j[1], i[2] - j[2])
            tot += T[dz + nz - 1, dy + ny - 1, dx + nx - 1]
    Np = tot / (nx * ny * nz)
    assert abs(Np[:3].sum() - 1) < 1e-12
    assert np.allclose(Np[3:], 0, atol=1e-13)
    if nx == ny == nz:
        assert np.allclose(Np[:3], 1 / 3, atol=1e-12)
    order = np.argsort(dims)
    assert Np[order[0]] >= Np[order[1]] - 1e-12 and Np[order[1]] >= Np[order[2]] - 1e-12


def test_demag_field_is_minus_energy_gradient(orc):
    lv = _level((3, 2, 4), c_ex=0.0, hk=0.0)
    N = 24
    m = W.seeded_unit_vectors(N, 5)
    H = orc.effective_field(lv, m, 0.0, None)
    h = 1e-6
    for i in range(N):
        for c in range(3):
            mp, mm = m.copy(), m.copy()
            mp[i, c] += h
            mm[i, c] -= h
            g = (orc.energy(lv, mp, 0.0) - orc.energy(lv, mm, 0.0)) / (2 * h)
            assert -g == pytest.approx(H[i, c], rel=1e-6, abs=1e-7 * lv["demag_ms"])
    # uniform magnetisation: the field is -Ms N_prism m on average
    mu = np.tile([0.0, 0.0, 1.0], (N, 1))
    Hu = orc.effective_field(lv, mu, 0.0, None)
    assert np.all(Hu[:, 2] < 0)


def test_energy_non_increasing_with_demag(orc):
    lv = _level((2, 3, 5), sigma=0.0, wave=2, hz_amp=-100 * gk.OE_TO_APM)
    m = W.seeded_unit_vectors(30, 9)
    e0 = orc.energy(lv, m, lv["hz_amp"])
    e_prev = e0
    for n in range(1500):
        m = orc.heun_step(lv, 1, n, m)
        e = orc.energy(lv, m, lv["hz_amp"])
        assert e <= e_prev + 1e-12 * abs(e_prev), n
        e_prev = e
    assert e < e0


def test_without_demag_flag_nothing_changes(orc):
    a = _level((2, 3, 4), demag=False)
    b = dict(a, demag_ms=0.0)
    m = W.seeded_unit_vectors(24, 2)
    assert np.array_equal(orc.effective_field(a, m, 10.0, None), orc.effective_field(b, m, 10.0, None))
    assert a["demag_ms"] == 0.0 and _level((2, 3, 4))["demag_ms"] == a["Ms"]


def test_adjoint_refuses_demag(orc):
    lv = _level((1, 1, 2))
    lv["n_period"] = lv["n_steps"] = 10
    with pytest.raises(AssertionError):
        orc.adjoint_batch(lv, [1], 10, np.ones((1, 11)))
