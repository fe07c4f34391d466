"""Synthetic workloads for the stochastic-LLG hysteresis-loop path.

This module only *describes* inputs: the base material, the field sweep and the
per-level grid / realization / seed settings of the workloads below.  It
holds none of the method's arithmetic (no coarse-graining rule, no field, no
integrator) so that both the FP64 oracle and the HIP path can read it without
sharing any computation.

Every workload is a magnetite rod (or block) built from cubic cells of edge
b*a0.  The paper's rod is 8a0 x 24a0 x 56a0 with a0 = 0.839 nm (material
paragraph, Fig. 1); coarse-graining by b gives (8/b) x (24/b) x (56/b) cells.
Base parameters: Ms = 480 kA/m, A0 = 0.98e-11 J/m, K0 = 10 kJ/m^3 along z,
T = 310 K, Tc = 858 K, delta = 0.511 (Eq. 13).  Every sweep starts at +Hmax
with every moment along +z.

Names
-----
rod_b4_single      2x6x14 rod, b=4, one realization, seed 1, 4e4 steps of 5 fs
rod_b1_ens8        8x24x56 rod, b=1, 8 seeds, 4e6 steps of 1 fs
multilevel_ens256  256 realizations at each of b=1,2,4,8 (1024 instances)
block_b2_cone10    128x128x512 block, b=2, per-cell axes in a 10 degree cone
rod_b4_adjoint64   64 realizations of the 2x6x14 b=4 rod, checkpoints every 256
rod_sine_sr250_ens100
                   the paper's sweep-rate/damping protocol (Fig. 4): Hmax = 500
                   Oe, a cosine sweep at 250 Oe/ns, easy axes in a 5 degree
                   cone, alpha = 0.1 SR/(0.25 Oe/ns) = 100, 100 realizations at
                   b = 4 (2x6x14), b = 8 (1x3x7) and the single-cell limit
                   (1x1x1, b = 10752^(1/3) so that the cell has the rod's
                   volume), 5 fs steps
rod_sine_sr2p5_ens100
                   the same rod levels at 2.5 Oe/ns with alpha = 0.1 (the
                   conditions of the cell-size figure, Fig. 2) and alpha = 1
                   (SR/alpha = 2.5 Oe/ns, Fig. 4), 100 realizations each,
                   1.6e8 steps of 5 fs: the comparison with the printed areas
"""
from __future__ import annotations

import copy

# Base (b = 1) material and protocol, SI unless noted.
BASE_MATERIAL = dict(
    a0_m=0.839e-9,          # cubic unit-cell edge (material paragraph)
    Ms0=480e3,              # A/m, bulk magnetite
    A0=0.98e-11,            # J/m exchange stiffness
    K0=1.0e4,               # J/m^3 uniaxial anisotropy
    T_K=310.0,              # K
    Tc_K=858.0,             # K, printed Heisenberg Tc
    delta=0.511,            # Eq. (13) weight
    easy_axis=(0.0, 0.0, 1.0),
    Hmax_Oe=1000.0,
    sweep_Oe_per_ns=2.0e4,
    wave="triangle",
    n_cycles=1,
    scale_AK=True,          # apply Eqs. (8)-(9)
    scale_H=True,           # apply Eq. (10) to the applied field
    ms_scale=1.0,
    sr_ref_Oe_per_ns=0.0,   # >0 switches on alpha = alpha_ref*SR/SR_ref
    alpha_ref=0.0,
    demag=False,            # magnetostatic field of the cells (beyond the paper)
)


def _level(nx, ny, nz, b, alpha, dt_s, n_real=1, seed_base=1, cone_deg=0.0,
           axis_seed=0, record_every=1):
    return dict(nx=nx, ny=ny, nz=nz, b=float(b), n_real=n_real,
                seed_base=seed_base, alpha=alpha, dt_s=dt_s,
                cone_deg=cone_deg, axis_seed=axis_seed,
                record_every=record_every)


def _rod_dims(b):
    return (8 // b, 24 // b, 56 // b)


WORKLOADS = {
    "rod_b4_single": dict(
        material=dict(BASE_MATERIAL, Hmax_Oe=1000.0, sweep_Oe_per_ns=2.0e4),
        levels=[_level(*_rod_dims(4), b=4, alpha=0.1, dt_s=5e-15,
                       n_real=1, seed_base=1)],
        ckpt_every=0,
    ),
    "rod_b1_ens8": dict(
        material=dict(BASE_MATERIAL, Hmax_Oe=1000.0, sweep_Oe_per_ns=1.0e3,
                      scale_AK=False, scale_H=False),
        levels=[_level(*_rod_dims(1), b=1, alpha=0.1, dt_s=1e-15,
                       n_real=8, seed_base=1)],
        ckpt_every=0,
    ),
    "multilevel_ens256": dict(
        material=dict(BASE_MATERIAL, Hmax_Oe=1000.0, sweep_Oe_per_ns=1.0e3,
                      sr_ref_Oe_per_ns=0.25, alpha_ref=0.1),
        levels=[_level(*_rod_dims(b), b=b, alpha=0.1, dt_s=5e-15,
                       n_real=256, seed_base=1, record_every=100)
                for b in (1, 2, 4, 8)],
        ckpt_every=0,
    ),
    "block_b2_cone10": dict(
        material=dict(BASE_MATERIAL, Hmax_Oe=800.0, sweep_Oe_per_ns=100.0),
        levels=[_level(128, 128, 512, b=2, alpha=0.05, dt_s=5e-15,
                       n_real=1, seed_base=1, cone_deg=10.0, axis_seed=7,
                       record_every=1)],
        ckpt_every=0,
        window=dict(warmup_steps=200, timed_steps=2000),
    ),
    "rod_b4_adjoint64": dict(
        material=dict(BASE_MATERIAL, Hmax_Oe=1000.0, sweep_Oe_per_ns=2.0e4),
        levels=[_level(*_rod_dims(4), b=4, alpha=0.1, dt_s=5e-15,
                       n_real=64, seed_base=1)],
        ckpt_every=256,
    ),
}


# Single-cell limit of the rod: one cube with the rod's volume 10752 a0^3.
B_SINGLE_CELL = 10752.0 ** (1.0 / 3.0)

WORKLOADS["rod_sine_sr250_ens100"] = dict(
    material=dict(BASE_MATERIAL, Hmax_Oe=500.0, sweep_Oe_per_ns=250.0, wave="cosine",
                  sr_ref_Oe_per_ns=0.25, alpha_ref=0.1),
    levels=[_level(*dims, b=b, alpha=0.1, dt_s=5e-15, n_real=100, seed_base=1,
                   cone_deg=5.0, axis_seed=11, record_every=100)
            for dims, b in (((2, 6, 14), 4), ((1, 3, 7), 8), ((1, 1, 1), B_SINGLE_CELL))],
    ckpt_every=0,
)


WORKLOADS["rod_sine_sr2p5_ens100"] = dict(
    material=dict(BASE_MATERIAL, Hmax_Oe=500.0, sweep_Oe_per_ns=2.5, wave="cosine"),
    levels=[_level(*dims, b=b, alpha=alpha, dt_s=5e-15, n_real=100, seed_base=1,
                   cone_deg=5.0, axis_seed=11, record_every=1000)
            for alpha in (0.1, 1.0)
            for dims, b in (((2, 6, 14), 4), ((1, 3, 7), 8), ((1, 1, 1), B_SINGLE_CELL))],
    ckpt_every=0,
)


def workload(name: str) -> dict:
    """A deep copy of one named workload (material dict, level list, extras)."""
    return copy.deepcopy(WORKLOADS[name])


def shrink(wl: dict, *, n_real=None, sweep_scale=None, dims=None) -> dict:
    """A smaller copy of a workload for fast tests.

    ``sweep_scale`` multiplies the sweep rate (fewer steps per cycle);
    ``dims`` replaces every level's grid; ``n_real`` caps realizations.
    """
    w = copy.deepcopy(wl)
    if sweep_scale is not None:
        w["material"]["sweep_Oe_per_ns"] *= sweep_scale
    for lv in w["levels"]:
        if n_real is not None:
            lv["n_real"] = min(lv["n_real"], n_real)
        if dims is not None:
            lv["nx"], lv["ny"], lv["nz"] = dims
    return w


def seeded_unit_vectors(n: int, seed: int):
    """Seeded random unit vectors (n, 3), float64, for initial states in tests.

    Uses numpy's PCG64 stream; this is an input generator only.
    """
    import numpy as np
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v


def macrospin_pair(sr_Oe_per_ns: float, alpha: float, T_K: float = 310.0, n_real: int = 256,
                   dt_s: float = 1e-12, n_points: int = 4000, seed_base: int = 1,
                   Hmax_Oe: float = 500.0, wave: str = "cosine") -> dict:
    """The single-macrospin limit of the rod (one cubic cell with the rod's
    volume, b = 10752^(1/3), easy axis along z, no cone) under the paper's
    cosine sweep of +-Hmax at sweep rate SR with damping alpha: one point of
    a sweep-rate / damping scan (Sharrock's law, Eq. 14).  Time steps of
    1 ps resolve the precession at the largest field (about 0.014 rad per
    step); the loop keeps about n_points recorded points (the area and the
    per-realization crossings use every step)."""
    period_steps = 4.0 * Hmax_Oe / (sr_Oe_per_ns * 1e9) / dt_s
    rec = max(1, int(period_steps // n_points))
    return dict(
        material=dict(BASE_MATERIAL, T_K=T_K, Hmax_Oe=Hmax_Oe, sweep_Oe_per_ns=sr_Oe_per_ns, wave=wave),
        levels=[_level(1, 1, 1, b=B_SINGLE_CELL, alpha=alpha, dt_s=dt_s, n_real=n_real,
                       seed_base=seed_base, record_every=rec)],
        ckpt_every=0,
    )
