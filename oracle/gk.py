"""FP64 oracle, parameter side: the modified Grinstein-Koch rule and the
per-level constants of the stochastic LLG step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import this
module; only tests/, the smoke check and the benchmark's CPU-baseline leg do.

Everything here is plain Python floats (IEEE double).  Citations name the
paper's equations (Behbahani, Plumer, Saika-Voivod, arXiv:1912.00310).
"""
from __future__ import annotations

import math

# Physical constants.  mu0 is the classical 4*pi*1e-7 (consistent with the
# 1000/4pi Oe -> A/m factor of Eq. 3); gamma_e is the value printed under
# Eq. (1); k_B is the SI-exact value.
MU0 = 4.0e-7 * math.pi
KB = 1.380649e-23
GAMMA_E = 1.76e11                 # rad/(s T), text under Eq. (1)
GAMMA0 = MU0 * GAMMA_E            # m/(A s)
OE_TO_APM = 1000.0 / (4.0 * math.pi)   # 1 Oe in A/m, Eq. (3)


# ---------------------------------------------------------------------------
# Coarse-graining rule (Eqs. 2-13)
# ---------------------------------------------------------------------------

def zeta(t: float, b: float) -> float:
    """Closed-form magnetisation factor zeta(b) = t/b + 1 - t, t = T/Tc
    (text after Eq. 11)."""
    return t / b + 1.0 - t


def heisenberg_tc(a0: float, A0: float) -> float:
    """Tc = 1.44 J_eff / k_B with J_eff = a0*A0 (material paragraph)."""
    return 1.44 * a0 * A0 / KB


def reduced_temperature(T: float, A: float, b: float, a0: float) -> float:
    """Eq. (2): T* = k_B T Lambda / A with Lambda = 2 pi/(b a0)."""
    lam = 2.0 * math.pi / (b * a0)
    return KB * T * lam / A


def reduced_field_anisotropy(H_Oe: float, K: float, Ms: float, A: float,
                             b: float, a0: float):
    """Eq. (3): h = mu0 Ms H/(A Lambda^2) * 1000/4pi (H in Oe),
    g = K/(A Lambda^2)."""
    lam = 2.0 * math.pi / (b * a0)
    h = MU0 * Ms * H_Oe / (A * lam * lam) * (1000.0 / (4.0 * math.pi))
    g = K / (A * lam * lam)
    return h, g


def rg_F(Ts: float, h: float, g: float) -> float:
    """Eq. (5): F = T*/(2 pi (1 + h + g))."""
    return Ts / (2.0 * math.pi * (1.0 + h + g))


def rg_flow(Ts0: float, h0: float, g0: float, b: float, n_steps: int = 4000):
    """Integrate the flow of Eqs. (4) together with the exponent of Eq. (7)
    from l = 0 to l = ln b with classical fourth-order Runge-Kutta.

    State y = (T*, h, g, I) with dI/dl = F, so zeta(l) = exp(-I) (Eqs. 6-7).
    Returns (T*, h, g, zeta) at l = ln b.
    """
    def rhs(y):
        Ts, h, g, _ = y
        F = rg_F(Ts, h, g)
        return ((-1.0 + F) * Ts, 2.0 * h, (2.0 - 2.0 * F) * g, F)

    l_end = math.log(b)
    if l_end == 0.0:
        return Ts0, h0, g0, 1.0
    dl = l_end / n_steps
    y = (Ts0, h0, g0, 0.0)
    for _ in range(n_steps):
        k1 = rhs(y)
        k2 = rhs(tuple(y[i] + 0.5 * dl * k1[i] for i in range(4)))
        k3 = rhs(tuple(y[i] + 0.5 * dl * k2[i] for i in range(4)))
        k4 = rhs(tuple(y[i] + dl * k3[i] for i in range(4)))
        y = tuple(y[i] + dl / 6.0 * (k1[i] + 2 * k2[i] + 2 * k3[i] + k4[i])
                  for i in range(4))
    return y[0], y[1], y[2], math.exp(-y[3])


def equivalent_temperature(T0: float, b: float, z: float) -> float:
    """Eq. (12): T(b) = T0/(b zeta(b, T0))."""
    return T0 / (b * z)


def exchange_length(A: float, Ms: float) -> float:
    """l_ex = sqrt(2A/(mu0 Ms^2)) (paragraph after the loop areas)."""
    return math.sqrt(2.0 * A / (MU0 * Ms * Ms))


def loop_m_scale(delta: float, z: float) -> float:
    """Eq. (13) solved for the factor applied to the simulated loop:
    M0 = (delta*zeta + 1 - delta) M(b)."""
    return 1.0 - delta * (1.0 - z)


def alpha_sweep_scaled(alpha_ref: float, sr: float, sr_ref: float) -> float:
    """SR/alpha invariance (Sharrock argument, Eq. 14 and Fig. 4):
    keep SR/alpha fixed, alpha_sim = alpha_ref * SR/SR_ref."""
    return alpha_ref * sr / sr_ref


# ---------------------------------------------------------------------------
# Per-level constants of the step
# ---------------------------------------------------------------------------

def dt_rule(c_ex: float, hk: float, hz_amp: float, alpha: float) -> float:
    """Default time step when none is given: the largest whole femtosecond
    not above 0.15 sqrt(1+alpha^2)/(gamma0 (12 c_ex + H_K + H_max)), capped
    at 5 fs (the paper uses 1 fs at b=1 and says larger cells allow at least
    five times more, Fig. 4 discussion)."""
    bound = 0.15 * math.sqrt(1.0 + alpha * alpha) / (
        GAMMA0 * (12.0 * c_ex + hk + hz_amp))
    fs = math.floor(bound / 1e-15)
    return max(1, min(5, fs)) * 1e-15


def compile_level(material: dict, level: dict, level_index: int = 0) -> dict:
    """All FP64 constants one level needs.

    Applies Eqs. (8)-(10) and (13) with the closed-form zeta, the Brown
    thermal-field variance for Eq. (1) and the SR/alpha rule.
    """
    m = material
    Tc = m["Tc_K"] if m.get("Tc_K", 0.0) > 0.0 else heisenberg_tc(m["a0_m"], m["A0"])
    t = m["T_K"] / Tc
    b = float(level["b"])
    z = zeta(t, b)
    A = z * m["A0"] if m["scale_AK"] else m["A0"]
    K = z ** 3 * m["K0"] if m["scale_AK"] else m["K0"]
    hscale = z if m["scale_H"] else 1.0
    cM = loop_m_scale(m["delta"], z) if m["scale_H"] else 1.0
    Ms = m["ms_scale"] * m["Ms0"]
    a = b * m["a0_m"]
    V = a ** 3
    if m.get("sr_ref_Oe_per_ns", 0.0) > 0.0:
        alpha = alpha_sweep_scaled(m["alpha_ref"], m["sweep_Oe_per_ns"],
                                   m["sr_ref_Oe_per_ns"])
    else:
        alpha = level["alpha"]
    c_ex = 2.0 * A / (MU0 * Ms * a * a)
    hk = 2.0 * K / (MU0 * Ms)
    hz_amp = hscale * m["Hmax_Oe"] * OE_TO_APM
    dt = level["dt_s"] if level.get("dt_s", 0.0) > 0.0 else dt_rule(c_ex, hk, hz_amp, alpha)
    gamma1 = GAMMA0 / (1.0 + alpha * alpha)
    sigma = math.sqrt(2.0 * alpha * KB * m["T_K"] / (GAMMA0 * MU0 * Ms * V * dt))
    period = 4.0 * m["Hmax_Oe"] / (m["sweep_Oe_per_ns"] * 1e9)
    n_period = int(round(period / dt))
    return dict(
        nx=level["nx"], ny=level["ny"], nz=level["nz"], level_tag=level_index,
        b=b, t=t, zeta=z, A=A, K=K, Ms=Ms, a=a, V=V, alpha=alpha, dt=dt,
        c_ex=c_ex, hk=hk, gamma1=gamma1, sigma=sigma, hz_amp=hz_amp,
        hscale=hscale, cM=cM, n_period=n_period,
        n_steps=n_period * int(m.get("n_cycles", 1)),
        wave={"triangle": 0, "cosine": 1, "constant": 2}[m.get("wave", "triangle")],
        axis=tuple(m["easy_axis"]), cone_deg=level.get("cone_deg", 0.0),
        axis_seed=level.get("axis_seed", 0),
        Hmax_Oe=m["Hmax_Oe"], T=m["T_K"], Ms0=m["Ms0"],
        # magnetostatics (beyond the paper): the field -Ms N m of the cells
        demag_ms=Ms if m.get("demag", False) else 0.0,
    )


def chain_rule(g5, lv: dict):
    """Map gradients with respect to the step constants
    (c_ex, H_K, gamma1, alpha as it multiplies the damping term, sigma)
    onto the level parameters (K, A, alpha, ms_scale).

    c_ex = 2A/(mu0 Ms a^2), H_K = 2K/(mu0 Ms), gamma1 = gamma0/(1+alpha^2),
    sigma = sqrt(2 alpha kB T/(gamma0 mu0 Ms V dt)), Ms = ms_scale*Ms0.
    """
    g_cex, g_hk, g_g1, g_al, g_sig = g5
    al = lv["alpha"]
    dK = g_hk * lv["hk"] / lv["K"]
    dA = g_cex * lv["c_ex"] / lv["A"]
    dg1_dal = -2.0 * al * GAMMA0 / (1.0 + al * al) ** 2
    dsig_dal = lv["sigma"] / (2.0 * al) if al > 0.0 else 0.0
    dal = g_al + g_g1 * dg1_dal + g_sig * dsig_dal
    Ms = lv["Ms"]
    dMs = -g_cex * lv["c_ex"] / Ms - g_hk * lv["hk"] / Ms - g_sig * lv["sigma"] / (2.0 * Ms)
    dms = dMs * lv["Ms0"]
    return dK, dA, dal, dms
