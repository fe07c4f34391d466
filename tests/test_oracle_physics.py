"""Pins of the oracle's integrator against textbook physics: Stoner-Wohlfarth
switching, Larmor precession, the damped closed form of Eq. (1), |m| = 1,
monotone energy at T = 0, the field as the energy gradient, Boltzmann
(Langevin) equilibrium, and uniform-state invariance of the exchange term."""
import math

import numpy as np
import pytest
from scipy import integrate

import sllg_workloads as W
from oracle import gk

OE = gk.OE_TO_APM


def single_cell(hk=0.0, alpha=0.0, hz=0.0, sigma=0.0, dt=1e-15, axis=(0, 0, 1),
                nx=1, ny=1, nz=1, c_ex=0.0, wave=2, n_period=1):
    return dict(nx=nx, ny=ny, nz=nz, level_tag=0, c_ex=c_ex, hk=hk,
                gamma1=gk.GAMMA0 / (1 + alpha * alpha), alpha=alpha, sigma=sigma,
                dt=dt, hz_amp=hz, n_period=n_period, wave=wave, axis=tuple(axis),
                cone_deg=0.0, axis_seed=0)


def run1(orc, lv, m0, nsteps, seed=1):
    m, mbar = orc.run(lv, seed, 0, nsteps, np.array(m0, dtype=float).reshape(-1, 3))
    return m, mbar


HK_B1 = 2 * 1e4 / (gk.MU0 * 480e3)     # A/m, H_K at b = 1


@pytest.mark.parametrize("eps,switch", [(0.02, True), (-0.02, False)])
def test_stoner_wohlfarth_aligned(orc, eps, switch):
    # axis z, field along -z: the +z state loses stability at |H| = H_K
    lv = single_cell(hk=HK_B1, alpha=1.0, hz=-(1 + eps) * HK_B1, dt=2e-12)
    th = 1e-3
    m, _ = run1(orc, lv, [math.sin(th), 0, math.cos(th)], 150000)
    assert (m[0, 2] < -0.99) if switch else (m[0, 2] > 0.99)


def test_stoner_wohlfarth_antiparallel_is_fixed_point(orc):
    lv = single_cell(hk=HK_B1, alpha=1.0, hz=-2 * HK_B1, dt=2e-12)
    m, _ = run1(orc, lv, [0, 0, 1], 20000)
    assert m[0, 2] == 1.0


@pytest.mark.parametrize("psi_deg", [10.0, 30.0, 45.0])
def test_stoner_wohlfarth_astroid(orc, psi_deg):
    psi = math.radians(psi_deg)
    h_sw = (math.cos(psi) ** (2 / 3) + math.sin(psi) ** (2 / 3)) ** -1.5
    ax = (math.sin(psi), 0.0, math.cos(psi))
    for eps, switch in ((0.01, True), (-0.01, False)):
        lv = single_cell(hk=HK_B1, alpha=1.0, hz=-(1 + eps) * h_sw * HK_B1,
                         dt=2e-12, axis=ax)
        m, _ = run1(orc, lv, ax, 60000)
        along = float(np.dot(m[0], ax))
        assert (along < 0) if switch else (along > 0), (psi_deg, eps, along)


def test_larmor_frequency(orc):
    H = 1000 * OE
    th0 = math.radians(30)
    lv = single_cell(hz=H, dt=1e-15)
    period = 2 * math.pi / (gk.GAMMA0 * H)
    assert period == pytest.approx(357.0e-12, rel=2e-4)
    n = 100000
    m, _ = run1(orc, lv, [math.sin(th0), 0, math.cos(th0)], n)
    phi = math.atan2(m[0, 1], m[0, 0])
    want = math.remainder(gk.GAMMA0 * H * n * 1e-15, 2 * math.pi)
    assert abs(math.remainder(phi - want, 2 * math.pi)) < 1e-6
    assert m[0, 2] == pytest.approx(math.cos(th0), abs=1e-12)


def _compiled_single_cell(alpha, H_Oe, T_K=0.0, K0=0.0, A0=0.0, b=1.0, dt_s=1e-15,
                          nx=1, ny=1, nz=1):
    """A level compiled by gk.compile_level (not built by hand): constant
    applied field H_Oe along z, no field scaling, exchange and anisotropy as
    given.  The physics pins below then test compile_level's gamma1, sigma
    and dt together with the integrator."""
    mat = dict(W.BASE_MATERIAL, A0=A0, K0=K0, T_K=T_K, Hmax_Oe=H_Oe,
               sweep_Oe_per_ns=1.0, wave="constant", scale_AK=True, scale_H=False)
    lvl = dict(nx=nx, ny=ny, nz=nz, b=b, n_real=1, seed_base=1, alpha=alpha,
               dt_s=dt_s, cone_deg=0.0, axis_seed=0, record_every=1)
    return gk.compile_level(mat, lvl, 0)


# gamma0 = mu0 gamma_e from the printed gamma_e (text under Eq. 1) and the
# classical mu0; written out here so that the pins do not reuse gk's constant.
_GAMMA0_PRINTED = 4e-7 * math.pi * 1.76e11


def test_damped_closed_form(orc):
    # Eq. (1) in Gilbert form dm/dt = -gamma0 m x H + alpha m x dm/dt has,
    # for a static field H along z, the textbook solution in which m
    # precesses at omega = gamma0 H/(1 + alpha^2) while its polar angle
    # relaxes as tan(theta/2) = tan(theta0/2) exp(-alpha omega t).  The
    # level comes from gk.compile_level, so this pins its gamma1, the sign of
    # the damping term and the integrator.
    H_Oe, alpha = 1000.0, 0.1
    H = H_Oe * 1000 / (4 * math.pi)
    lv = _compiled_single_cell(alpha, H_Oe)
    assert lv["sigma"] == 0.0 and lv["hk"] == 0.0 and lv["c_ex"] == 0.0
    omega = _GAMMA0_PRINTED * H / (1 + alpha ** 2)
    th0, n, dt = math.radians(150), 200000, lv["dt"]
    assert dt == 1e-15
    m, _ = run1(orc, lv, [math.sin(th0), 0, math.cos(th0)], n)
    t = n * dt
    th = 2 * math.atan(math.tan(th0 / 2) * math.exp(-alpha * omega * t))
    phi = math.remainder(omega * t, 2 * math.pi)
    assert math.acos(m[0, 2]) == pytest.approx(th, abs=1e-8)
    assert abs(math.remainder(math.atan2(m[0, 1], m[0, 0]) - phi, 2 * math.pi)) < 1e-8


def test_larmor_from_compiled_level(orc):
    # alpha = 0: compile_level gives sigma = 0 and gamma1 = gamma0, so m
    # precesses at the Larmor frequency gamma0 H (period 357.0 ps at 1000 Oe)
    lv = _compiled_single_cell(0.0, 1000.0, T_K=310.0)
    assert lv["sigma"] == 0.0
    H = 1000.0 * 1000 / (4 * math.pi)
    th0, n = math.radians(40), 50000
    m, _ = run1(orc, lv, [math.sin(th0), 0, math.cos(th0)], n)
    phi = math.atan2(m[0, 1], m[0, 0])
    want = math.remainder(_GAMMA0_PRINTED * H * n * lv["dt"], 2 * math.pi)
    assert abs(math.remainder(phi - want, 2 * math.pi)) < 1e-6


def rod_b4_level(**over):
    wl = W.workload("rod_b4_single")
    lv = gk.compile_level(wl["material"], wl["levels"][0])
    lv.update(over)
    return lv


def test_unit_norm_every_step(orc):
    lv = rod_b4_level()
    m = np.tile([0.0, 0.0, 1.0], (lv["nx"] * lv["ny"] * lv["nz"], 1))
    for n in range(50):
        m = orc.heun_step(lv, 1, n, m)
        assert np.max(np.abs(np.linalg.norm(m, axis=1) - 1)) < 4e-16


def test_field_is_minus_energy_gradient(orc):
    lv = rod_b4_level(nx=3, ny=2, nz=4)
    N = 24
    m = W.seeded_unit_vectors(N, 3)
    ax = W.seeded_unit_vectors(N, 4)
    hz = -300 * OE
    H = orc.effective_field(lv, m, hz, None, u=ax)
    h = 1e-6
    for i in range(N):
        for c in range(3):
            mp, mm = m.copy(), m.copy()
            mp[i, c] += h
            mm[i, c] -= h
            g = (orc.energy(lv, mp, hz, u=ax) - orc.energy(lv, mm, hz, u=ax)) / (2 * h)
            assert -g == pytest.approx(H[i, c], rel=1e-6, abs=1e-6 * lv["c_ex"])


def test_energy_constants_match_continuum(orc):
    # mu0 Ms V (c_ex/2) = A a  (exchange energy A a sum |m_i - m_j|^2)
    # mu0 Ms V (hk/2)   = K V  (uniaxial energy K V (m.u)^2)
    lv = rod_b4_level()
    assert gk.MU0 * lv["Ms"] * lv["V"] * lv["c_ex"] / 2 == pytest.approx(lv["A"] * lv["a"])
    assert gk.MU0 * lv["Ms"] * lv["V"] * lv["hk"] / 2 == pytest.approx(lv["K"] * lv["V"])


def test_energy_non_increasing_at_zero_temperature(orc):
    lv = rod_b4_level(sigma=0.0, wave=2, hz_amp=-200 * OE)
    m = W.seeded_unit_vectors(lv["nx"] * lv["ny"] * lv["nz"], 11)
    e_prev = orc.energy(lv, m, lv["hz_amp"])
    for n in range(3000):
        m = orc.heun_step(lv, 1, n, m)
        e = orc.energy(lv, m, lv["hz_amp"])
        assert e <= e_prev + 1e-12 * abs(e_prev), n
        e_prev = e
    assert e < orc.energy(lv, W.seeded_unit_vectors(lv["nx"] * lv["ny"] * lv["nz"], 11), lv["hz_amp"])


def test_uniform_state_is_single_cell_bit_for_bit(orc):
    lv = rod_b4_level(sigma=0.0)
    one = dict(lv, nx=1, ny=1, nz=1)
    m0 = np.array([math.sin(0.3), 0.1, math.cos(0.3)])
    m0 /= np.linalg.norm(m0)
    N = lv["nx"] * lv["ny"] * lv["nz"]
    mg, _ = orc.run(lv, 1, 0, 400, np.tile(m0, (N, 1)))
    ms, _ = orc.run(one, 1, 0, 400, m0.reshape(1, 3))
    assert np.array_equal(mg, np.tile(ms[0], (N, 1)))


def test_triangle_schedule(orc):
    lv = rod_b4_level()
    N, A = lv["n_period"], lv["hz_amp"]
    assert orc.applied_field(lv, 0) == A
    assert orc.applied_field(lv, N // 4) == 0.0
    assert orc.applied_field(lv, N // 2) == -A
    assert orc.applied_field(lv, 3 * N // 4) == 0.0
    assert orc.applied_field(lv, N) == A
    H = orc.field_schedule_Oe(lv)
    d = np.diff(H)
    assert np.allclose(np.abs(d), 4 * lv["Hmax_Oe"] * lv["hscale"] / N, rtol=1e-9)


def test_cosine_schedule(orc):
    # the paper's sinusoidal field (protocol paragraph) started at +Hmax:
    # extremes and zeros at the quarter periods, symmetric about the half
    # period, and the mean |dH/dt| over a cycle equal to the sweep rate
    # SR = 4 Hmax f (Hmax, SR as the workload gives them)
    wl = W.workload("rod_sine_sr250_ens100")
    lv = gk.compile_level(wl["material"], wl["levels"][0], 0)
    N, A = lv["n_period"], lv["hz_amp"]
    assert orc.applied_field(lv, 0) == pytest.approx(A, rel=1e-15)
    assert orc.applied_field(lv, N // 2) == pytest.approx(-A, rel=1e-15)
    assert abs(orc.applied_field(lv, N // 4)) < 1e-9 * A
    assert abs(orc.applied_field(lv, 3 * N // 4)) < 1e-9 * A
    for n in (1, 12345, N // 3, N // 2 - 7):
        assert orc.applied_field(lv, n) == pytest.approx(orc.applied_field(lv, N - n), rel=1e-12, abs=1e-9)
    H = orc.field_schedule_Oe(lv)
    assert len(H) == N + 1
    mean_rate = np.abs(np.diff(H)).sum() / (N * lv["dt"]) / 1e9          # Oe/ns
    assert mean_rate == pytest.approx(wl["material"]["sweep_Oe_per_ns"] * lv["hscale"], rel=1e-9)


def _langevin(x):
    return 1 / math.tanh(x) - 1 / x


@pytest.mark.parametrize("with_k", [False, True])
def test_boltzmann_equilibrium(orc, with_k):
    # Independent spins (no exchange), b = 8 cell, T = 310 K, H = 1000 Oe.
    # Brown's thermal field must give <m_z> = L(xi) and <m_x^2> = L(xi)/xi
    # (K = 0) or the Boltzmann quadrature with the uniaxial term.  The level
    # (sigma, gamma1, dt, H_K) comes from gk.compile_level; the expected
    # values use only printed inputs (a0, Ms, K0, zeta(8), T) and the
    # Boltzmann weight, so a wrong thermal-field variance, cell volume or
    # anisotropy constant in compile_level fails here.
    T, b, H_Oe = 310.0, 8.0, 1000.0
    lv = _compiled_single_cell(1.0, H_Oe, T_K=T, K0=1e4 if with_k else 0.0,
                               b=b, dt_s=50e-15, nx=32, ny=32)
    assert lv["c_ex"] == 0.0
    H = H_Oe * 1000 / (4 * math.pi)
    V = (b * 0.839e-9) ** 3
    Ms = 480e3
    K = 0.6839 ** 3 * 1e4 if with_k else 0.0       # printed zeta(8), Eq. (9)
    xi = 4e-7 * math.pi * Ms * V * H / (1.380649e-23 * T)
    kv = K * V / (1.380649e-23 * T)
    assert xi == pytest.approx(3.391, abs=2e-3)
    w = lambda c: math.exp(xi * c + kv * c * c)
    Z = integrate.quad(w, -1, 1)[0]
    mz_want = integrate.quad(lambda c: c * w(c), -1, 1)[0] / Z
    mx2_want = 0.5 * (1 - integrate.quad(lambda c: c * c * w(c), -1, 1)[0] / Z)
    if not with_k:
        assert mz_want == pytest.approx(_langevin(xi), rel=1e-9)
        assert mx2_want == pytest.approx(_langevin(xi) / xi, rel=1e-9)
    seeds = list(range(1, 17))
    nsteps = 12000
    mbar, mf = orc.run_batch(lv, seeds, nsteps, want_final=True)
    # samples: final snapshot of 16 x 1024 independent spins
    mz = mf[:, :, 2].ravel()
    mx2 = (mf[:, :, 0] ** 2).ravel()
    se_z = mz.std() / math.sqrt(mz.size)
    se_x = mx2.std() / math.sqrt(mx2.size)
    assert abs(mz.mean() - mz_want) < 3.5 * se_z, (mz.mean(), mz_want, se_z)
    assert abs(mx2.mean() - mx2_want) < 3.5 * se_x, (mx2.mean(), mx2_want, se_x)
    # time average of the loop ordinate over the second half agrees as well
    late = mbar[:, nsteps // 2:].mean()
    assert abs(late - mz_want) < 0.01
