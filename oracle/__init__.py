"""FP64 CPU oracle for the stochastic-LLG hysteresis-loop path.

TEST INFRASTRUCTURE ONLY: the plain, slow reference that the HIP library is
checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it.  It shares no code with the
product package ``paper_1912_00310_amd`` and never imports it.

Layers
------
``gk``              the coarse-graining rule and per-level constants (Python)
``sllg_oracle.c``   Philox, Box-Muller, the Heun step, loop analytics and the
                    adjoint, in plain C (FP64), reached here through ctypes.

Parity status: every C entry point is pinned by ``tests/test_oracle_*.py``
(closed forms, paper numbers, textbook limits, numpy's Philox4x64 for the
round structure).  Whole finite-temperature loops have no printed reference in
the paper under the same protocol; those are checked only statistically.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

from . import gk

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sllg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP) into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class Level(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("level_tag", C.c_int32),
        ("c_ex", C.c_double), ("hk", C.c_double), ("gamma1", C.c_double),
        ("alpha", C.c_double), ("sigma", C.c_double), ("dt", C.c_double),
        ("hz_amp", C.c_double), ("n_period", C.c_int64), ("wave", C.c_int32),
        ("axis", C.c_double * 3), ("cone_deg", C.c_double),
        ("axis_seed", C.c_uint64), ("demag_ms", C.c_double),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.POINTER
        dp, u32p, u64p = P(C.c_double), P(C.c_uint32), P(C.c_uint64)
        lp = P(Level)
        sig = {
            "orc_philox4x32_10": (None, [u32p, u32p, u32p]),
            "orc_philox4x64_10": (None, [u64p, u64p, u64p]),
            "orc_philox_cell": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, u32p]),
            "orc_uniforms": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, dp]),
            "orc_normals": (None, [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, dp]),
            "orc_make_axes": (None, [lp, dp]),
            "orc_applied_field": (C.c_double, [lp, C.c_int64]),
            "orc_effective_field": (None, [lp, dp, dp, C.c_double, dp, dp]),
            "orc_heun_step": (C.c_int, [lp, dp, C.c_uint64, C.c_int64, dp, dp]),
            "orc_energy": (C.c_double, [lp, dp, dp, C.c_double]),
            "orc_run": (C.c_int, [lp, dp, C.c_uint64, C.c_int64, C.c_int64, dp, dp]),
            "orc_run_batch": (C.c_int, [lp, dp, u64p, C.c_int32, C.c_int64, dp, dp, C.c_int32]),
            "orc_max_threads": (C.c_int, []),
            "orc_newell": (None, [C.c_int, C.c_int, C.c_int, dp]),
            "orc_demag_tensor": (None, [lp, dp]),
            "orc_loop_stats": (None, [dp, dp, C.c_int64, dp]),
            "orc_adjoint": (C.c_int, [lp, dp, C.c_uint64, C.c_int64, dp, C.c_int32, dp, dp]),
            "orc_adjoint_batch": (C.c_int, [lp, dp, u64p, C.c_int32, C.c_int64, dp, C.c_int32, dp, dp, C.c_int32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _dp(a):
    return None if a is None else a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# Low-level wrappers
# ---------------------------------------------------------------------------

def level_struct(lv: dict) -> Level:
    """ctypes description of one compiled level (a dict from gk.compile_level
    or any dict carrying the same keys)."""
    s = Level()
    s.nx, s.ny, s.nz = int(lv["nx"]), int(lv["ny"]), int(lv["nz"])
    s.level_tag = int(lv.get("level_tag", 0))
    s.c_ex, s.hk, s.gamma1 = lv["c_ex"], lv["hk"], lv["gamma1"]
    s.alpha, s.sigma, s.dt = lv["alpha"], lv["sigma"], lv["dt"]
    s.hz_amp = lv["hz_amp"]
    s.n_period = int(lv["n_period"])
    s.wave = int(lv.get("wave", 0))
    ax = lv.get("axis", (0.0, 0.0, 1.0))
    s.axis[0], s.axis[1], s.axis[2] = ax
    s.cone_deg = lv.get("cone_deg", 0.0)
    s.axis_seed = int(lv.get("axis_seed", 0))
    s.demag_ms = float(lv.get("demag_ms", 0.0))
    return s


def philox4x32_10(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [o[i] for i in range(4)]


def philox4x64_10(ctr, key):
    M = (1 << 64) - 1
    c = (C.c_uint64 * 4)(*[int(x) & M for x in ctr])
    k = (C.c_uint64 * 2)(*[int(x) & M for x in key])
    o = (C.c_uint64 * 4)()
    lib().orc_philox4x64_10(c, k, o)
    return [o[i] for i in range(4)]


def philox_cell(seed, level, tag, cell, step):
    o = (C.c_uint32 * 4)()
    lib().orc_philox_cell(seed, level, tag, cell, step, o)
    return [o[i] for i in range(4)]


def uniforms(seed, level, tag, cell, step):
    o = (C.c_double * 4)()
    lib().orc_uniforms(seed, level, tag, cell, step, o)
    return [o[i] for i in range(4)]


def normals(seed, level, cell, step):
    o = (C.c_double * 3)()
    lib().orc_normals(seed, level, cell, step, o)
    return [o[i] for i in range(3)]


def ncell(lv):
    return int(lv["nx"]) * int(lv["ny"]) * int(lv["nz"])


def make_axes(lv):
    """(N,3) per-cell easy axes, or None when the level uses one axis."""
    if lv.get("cone_deg", 0.0) <= 0.0:
        return None
    u = np.zeros((ncell(lv), 3))
    s = level_struct(lv)
    lib().orc_make_axes(C.byref(s), _dp(u))
    return u


def newell(X, Y, Z):
    """Demagnetising tensor (xx, yy, zz, xy, xz, yz) between two unit cubes
    whose centres are (X, Y, Z) cell edges apart (Newell et al. 1993)."""
    o = (C.c_double * 6)()
    lib().orc_newell(int(X), int(Y), int(Z), o)
    return np.array(list(o))


def demag_tensor(lv):
    """(2nz-1, 2ny-1, 2nx-1, 6) table of the tensor over every cell offset."""
    s = level_struct(lv)
    shape = (2 * int(lv["nz"]) - 1, 2 * int(lv["ny"]) - 1, 2 * int(lv["nx"]) - 1, 6)
    T = np.zeros(shape)
    lib().orc_demag_tensor(C.byref(s), _dp(T))
    return T


def applied_field(lv, n):
    """Applied field along z at step n, A/m."""
    s = level_struct(lv)
    return lib().orc_applied_field(C.byref(s), int(n))


def field_schedule_Oe(lv, nsteps=None):
    """Simulated applied field H_n (Oe) for n = 0..nsteps."""
    s = level_struct(lv)
    n_all = int(lv["n_steps"] if nsteps is None else nsteps)
    f = lib().orc_applied_field
    return np.array([f(C.byref(s), n) for n in range(n_all + 1)]) / gk.OE_TO_APM


def effective_field(lv, m, hz, hth=None, u=None):
    s = level_struct(lv)
    m = _f64(m)
    H = np.zeros_like(m)
    lib().orc_effective_field(C.byref(s), _dp(u), _dp(m), float(hz),
                              _dp(None if hth is None else _f64(hth)), _dp(H))
    return H


def heun_step(lv, seed, n, m, u=None):
    s = level_struct(lv)
    m = _f64(m)
    out = np.zeros_like(m)
    rc = lib().orc_heun_step(C.byref(s), _dp(u), int(seed), int(n), _dp(m), _dp(out))
    assert rc == 0
    return out


def energy(lv, m, hz, u=None):
    """Reduced energy E/(mu0 Ms V) in A/m for a constant field hz (A/m)."""
    s = level_struct(lv)
    return lib().orc_energy(C.byref(s), _dp(u), _dp(_f64(m)), float(hz))


def run(lv, seed, n0, nsteps, m, u=None):
    """Advance one realization nsteps from step n0; returns (m, mbar)."""
    s = level_struct(lv)
    m = _f64(m).copy()
    mbar = np.zeros(int(nsteps) + 1)
    rc = lib().orc_run(C.byref(s), _dp(u), int(seed), int(n0), int(nsteps), _dp(m), _dp(mbar))
    assert rc == 0
    return m, mbar


def run_batch(lv, seeds, nsteps, threads=0, want_final=False, u=None):
    """Realizations from the all-+z state.  Returns (mbar[R, nsteps+1],
    m_final[R, N, 3] or None)."""
    s = level_struct(lv)
    seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
    R = len(seeds)
    mbar = np.zeros((R, int(nsteps) + 1))
    mf = np.zeros((R, ncell(lv), 3)) if want_final else None
    if u is None:
        u = make_axes(lv)
    rc = lib().orc_run_batch(C.byref(s), _dp(u), seeds.ctypes.data_as(C.POINTER(C.c_uint64)),
                             R, int(nsteps), _dp(mbar), _dp(mf), int(threads))
    assert rc == 0
    return mbar, mf


def max_threads():
    return lib().orc_max_threads()


STAT_KEYS = ("S", "Hstar_desc", "Hstar_asc", "Hc", "Mr", "n_cross_desc",
             "n_cross_asc", "k_desc", "k_asc", "m0_desc", "m0_asc")


def loop_stats(H, m):
    """Area, coercive field, remanence of one loop (see sllg_oracle.c)."""
    H, m = _f64(H), _f64(m)
    out = np.zeros(11)
    lib().orc_loop_stats(_dp(H), _dp(m), len(H), _dp(out))
    return dict(zip(STAT_KEYS, out.tolist()))


def adjoint_batch(lv, seeds, nsteps, w, threads=0, u=None):
    """Gradients of L_l = sum_n w[l, n] * mbar_n (summed over realizations)
    with respect to (c_ex, hk, gamma1, alpha, sigma).  Returns (g[nloss, 5],
    mbar[R, nsteps+1])."""
    s = level_struct(lv)
    seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
    w = _f64(np.atleast_2d(w))
    nloss = w.shape[0]
    assert w.shape[1] == nsteps + 1
    g = np.zeros((nloss, 5))
    mbar = np.zeros((len(seeds), int(nsteps) + 1))
    rc = lib().orc_adjoint_batch(C.byref(s), _dp(u), seeds.ctypes.data_as(C.POINTER(C.c_uint64)),
                                 len(seeds), int(nsteps), _dp(w), nloss, _dp(g), _dp(mbar),
                                 int(threads))
    assert rc == 0
    return g, mbar


# ---------------------------------------------------------------------------
# Loop post-processing and loss weights
# ---------------------------------------------------------------------------

def ensemble_stats(lv, H_Oe, mbar):
    """Statistics of the realizations' loops (rows of mbar) and of their mean.

    Returns the mean-loop S, H_c, M_r (simulation units, Oe), their physical
    values (H/zeta-type factor hscale and the Eq. 13 factor cM), and one
    standard error over realizations for S and H_c."""
    mbar = np.atleast_2d(mbar)
    R = mbar.shape[0]
    mean = mbar.mean(axis=0)
    st = loop_stats(H_Oe, mean)
    per = [loop_stats(H_Oe, row) for row in mbar]
    S_r = np.array([p["S"] for p in per])
    Hc_r = np.array([p["Hc"] for p in per])
    Hc_ok = Hc_r[np.isfinite(Hc_r)]
    se = lambda a: float(np.std(a, ddof=1) / math.sqrt(len(a))) if len(a) > 1 else float("nan")
    hs, cM = lv.get("hscale", 1.0), lv.get("cM", 1.0)
    return dict(
        S_sim=st["S"], Hc=st["Hc"], Mr=st["Mr"],
        S_phys=st["S"] * cM / hs, Hc_phys=st["Hc"] / hs, Mr_phys=st["Mr"] * cM,
        S_mean_of_real=float(S_r.mean()), S_se=se(S_r),
        Hc_mean_of_real=float(Hc_ok.mean()) if len(Hc_ok) else float("nan"),
        Hc_se=se(Hc_ok), n_real=R, mean_loop=st, per_real=per,
    )


def loss_weights(H_Oe, mbar_mean, n_real):
    """Weights w[2, N+1] such that, for every realization r,
    dL/dmbar_{r,n} = w[l, n]:  l = 0 the mean loop area (trapezoid),
    l = 1 the coercive field of the mean loop (first crossing per branch,
    linear interpolation).  Both in simulation units (Oe)."""
    H = _f64(H_Oe)
    n = len(H)
    w = np.zeros((2, n))
    # area: S = -sum_k (m_k + m_{k+1})/2 (H_{k+1} - H_k)
    for k in range(n - 1):
        dH = H[k + 1] - H[k]
        w[0, k] += -0.5 * dH
        w[0, k + 1] += -0.5 * dH
    st = loop_stats(H, mbar_mean)
    m = _f64(mbar_mean)
    for key, sgn in (("k_desc", -0.5), ("k_asc", 0.5)):
        k = int(st[key])
        if k < 0:
            continue
        dH = H[k + 1] - H[k]
        D = m[k + 1] - m[k]
        w[1, k] += sgn * (-dH * m[k + 1] / (D * D))
        w[1, k + 1] += sgn * (dH * m[k] / (D * D))
    return w / float(n_real)
