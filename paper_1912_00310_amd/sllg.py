"""Python binding of the C ABI in include/sllg.h (argument marshalling only).

PyTorch provides the device workspace and the HIP stream; every step of the
path runs in the gfx950 kernels of libsllg.so.  The library must have been
built (``paper_1912_00310_amd.build_lib.build()``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsllg.so")

SLLG_OK = 0
ERRORS = {-1: "SLLG_E_INVAL", -2: "SLLG_E_WORKSPACE", -3: "SLLG_E_CAPACITY",
          -4: "SLLG_E_STATE", -5: "SLLG_E_HIP", -6: "SLLG_E_NUMERIC"}
WAVES = {"triangle": 0, "cosine": 1, "constant": 2}
PLAN_AUTO, PLAN_RESIDENT, PLAN_STREAM, PLAN_SLAB, PLAN_LANES, PLAN_DEMAG = 0, 1, 2, 3, 4, 5
OPT_NO_TUNE, OPT_NO_SLAB, OPT_NO_GRAPH, OPT_VERBOSE = 1, 2, 4, 8


class SllgError(RuntimeError):
    def __init__(self, fn, code, msg):
        super().__init__(f"{fn} -> {ERRORS.get(code, code)}: {msg}")
        self.code = code


class Material(C.Structure):
    _fields_ = [
        ("a0_m", C.c_double), ("Ms0", C.c_double), ("A0", C.c_double), ("K0", C.c_double),
        ("T_K", C.c_double), ("Tc_K", C.c_double), ("delta", C.c_double),
        ("easy_axis", C.c_double * 3), ("Hmax_Oe", C.c_double), ("sweep_Oe_per_ns", C.c_double),
        ("wave", C.c_int32), ("n_cycles", C.c_int32), ("scale_AK", C.c_int32),
        ("scale_H", C.c_int32), ("ms_scale", C.c_double), ("sr_ref_Oe_per_ns", C.c_double),
        ("alpha_ref", C.c_double), ("demag", C.c_int32),
    ]


class Level(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("b", C.c_double),
        ("n_real", C.c_int32), ("seed_base", C.c_uint64), ("alpha", C.c_double),
        ("dt_s", C.c_double), ("cone_deg", C.c_double), ("axis_seed", C.c_uint64),
        ("record_every", C.c_int32),
    ]


class LoopStats(C.Structure):
    _fields_ = [
        ("S_sim", C.c_double), ("S_phys", C.c_double), ("Hc_desc", C.c_double),
        ("Hc_asc", C.c_double), ("Hc_sim", C.c_double), ("Hc_phys", C.c_double),
        ("Mr_sim", C.c_double), ("Mr_phys", C.c_double), ("S_se", C.c_double),
        ("Hc_se", C.c_double), ("n_cross_desc", C.c_int32), ("n_cross_asc", C.c_int32),
        ("n_real", C.c_int32),
    ]


_lib = None


def lib():
    """The loaded libsllg.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "paper_1912_00310_amd.build_lib.build()")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        vp = C.c_void_p
        sig = {
            "sllg_workspace_bytes": (C.c_size_t, [P(Material), P(Level), C.c_int32, C.c_int32]),
            "sllg_init": (C.c_int, [P(Material), P(Level), C.c_int32, C.c_int32, vp, C.c_size_t, vp, P(vp)]),
            "sllg_run_sweep": (C.c_int, [vp]),
            "sllg_run_steps": (C.c_int, [vp, C.c_int64]),
            "sllg_reset": (C.c_int, [vp]),
            "sllg_loop": (C.c_int, [vp, C.c_int32, C.c_int32, P(C.c_double), P(C.c_double), C.c_int64,
                                    P(C.c_int64), P(LoopStats)]),
            "sllg_grad": (C.c_int, [vp, C.c_int32, P(C.c_double), P(C.c_double)]),
            "sllg_last_error": (C.c_char_p, []),
            "sllg_free": (None, [vp]),
            "sllg_level_params": (C.c_int, [vp, C.c_int32, P(C.c_double)]),
            "sllg_level_step": (C.c_int64, [vp, C.c_int32]),
            "sllg_level_kernel": (C.c_int, [vp, C.c_int32, C.c_char_p, C.c_int32]),
            "sllg_get_state": (C.c_int, [vp, C.c_int32, C.c_int32, P(C.c_float)]),
            "sllg_set_state": (C.c_int, [vp, C.c_int32, C.c_int32, P(C.c_float)]),
            "sllg_set_plan": (C.c_int, [vp, C.c_int32, C.c_int32]),
            "sllg_save_state": (C.c_int, [vp, vp, C.c_size_t, P(C.c_size_t)]),
            "sllg_load_state": (C.c_int, [vp, vp, C.c_size_t]),
            "sllg_set_slab_shape": (C.c_int, [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
            "sllg_set_stream_shape": (C.c_int, [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                                C.c_int32]),
            "sllg_philox_probe": (C.c_int, [C.c_uint64, C.c_uint32, C.c_uint32, P(C.c_uint32),
                                            P(C.c_uint64), C.c_int32, P(C.c_uint32), P(C.c_float), vp, vp]),
            "sllg_get_axes": (C.c_int, [vp, C.c_int32, P(C.c_float)]),
            "sllg_set_timing": (C.c_int, [vp, C.c_int32]),
            "sllg_kernel_time": (C.c_int, [vp, P(C.c_double), P(C.c_int64), P(C.c_int64)]),
            "sllg_sync": (C.c_int, [vp]),
            "sllg_init_static": (C.c_int, [P(Material), P(Level), C.c_int32, C.c_int32, vp, P(vp)]),
            "sllg_set_options": (C.c_int, [C.c_int32]),
            "sllg_set_spin_limit": (C.c_int, [vp, C.c_uint32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    """Names the header declares (for the symbol test)."""
    return [n for n in (
        "sllg_workspace_bytes", "sllg_init", "sllg_run_sweep", "sllg_run_steps", "sllg_reset",
        "sllg_loop", "sllg_grad", "sllg_last_error", "sllg_free", "sllg_level_params",
        "sllg_level_step", "sllg_level_kernel", "sllg_get_state", "sllg_set_state", "sllg_set_plan",
        "sllg_set_slab_shape", "sllg_set_stream_shape",
        "sllg_philox_probe", "sllg_get_axes", "sllg_set_timing", "sllg_kernel_time",
        "sllg_sync", "sllg_set_options", "sllg_set_spin_limit", "sllg_init_static", "sllg_save_state",
        "sllg_load_state")]


def _check(fn, rc):
    if rc != SLLG_OK:
        raise SllgError(fn, rc, lib().sllg_last_error().decode())


def material_struct(m: dict) -> Material:
    s = Material()
    s.a0_m, s.Ms0, s.A0, s.K0 = m["a0_m"], m["Ms0"], m["A0"], m["K0"]
    s.T_K, s.Tc_K, s.delta = m["T_K"], m.get("Tc_K", 858.0), m.get("delta", 0.511)
    ax = m.get("easy_axis", (0.0, 0.0, 1.0))
    s.easy_axis[0], s.easy_axis[1], s.easy_axis[2] = ax
    s.Hmax_Oe, s.sweep_Oe_per_ns = m["Hmax_Oe"], m["sweep_Oe_per_ns"]
    w = m.get("wave", "triangle")
    s.wave = WAVES[w] if isinstance(w, str) else int(w)
    s.n_cycles = int(m.get("n_cycles", 1))
    s.scale_AK, s.scale_H = int(bool(m.get("scale_AK", True))), int(bool(m.get("scale_H", True)))
    s.ms_scale = m.get("ms_scale", 1.0)
    s.sr_ref_Oe_per_ns, s.alpha_ref = m.get("sr_ref_Oe_per_ns", 0.0), m.get("alpha_ref", 0.0)
    s.demag = int(bool(m.get("demag", False)))
    return s


def levels_struct(levels) -> C.Array:
    arr = (Level * len(levels))()
    for s, l in zip(arr, levels):
        s.nx, s.ny, s.nz, s.b = int(l["nx"]), int(l["ny"]), int(l["nz"]), float(l["b"])
        s.n_real, s.seed_base = int(l.get("n_real", 1)), int(l.get("seed_base", 1))
        s.alpha, s.dt_s = float(l.get("alpha", 0.1)), float(l.get("dt_s", 0.0))
        s.cone_deg, s.axis_seed = float(l.get("cone_deg", 0.0)), int(l.get("axis_seed", 0))
        s.record_every = int(l.get("record_every", 1))
    return arr


PARAM_KEYS = ("zeta", "A", "K", "Ms", "a", "c_ex", "hk", "gamma1", "alpha", "sigma", "dt",
              "hscale", "cM", "n_steps", "hz_amp", "plan")


class Sim:
    """One context: levels x realizations of the stochastic LLG loop on one GPU."""

    def __init__(self, material: dict, levels, ckpt_every: int = 0, device="cuda:0", stream=None,
                 static_workspace: bool = False):
        """static_workspace=True: sllg_init_static (the library's own device
        array; no device memory is allocated by this object)."""
        import torch
        self._torch = torch
        self.device = torch.device(device)
        self.mat = material_struct(material)
        self.lv = levels_struct(levels)
        self.n_levels = len(levels)
        L = lib()
        if static_workspace:
            with torch.cuda.device(self.device):
                self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
                self.ws = None
                ctx = C.c_void_p()
                _check("sllg_init_static", L.sllg_init_static(C.byref(self.mat), self.lv, self.n_levels,
                                                              int(ckpt_every), C.c_void_p(self.stream.cuda_stream),
                                                              C.byref(ctx)))
            self.ctx = ctx
            self.ckpt_every = ckpt_every
            return
        nbytes = L.sllg_workspace_bytes(C.byref(self.mat), self.lv, self.n_levels, int(ckpt_every))
        if nbytes == 0:
            raise SllgError("sllg_workspace_bytes", -1, L.sllg_last_error().decode())
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        base = self.ws.data_ptr()
        self._ws_ptr = (base + 255) & ~255
        ctx = C.c_void_p()
        _check("sllg_init", L.sllg_init(C.byref(self.mat), self.lv, self.n_levels, int(ckpt_every),
                                        C.c_void_p(self._ws_ptr), nbytes,
                                        C.c_void_p(self.stream.cuda_stream), C.byref(ctx)))
        self.ctx = ctx
        self.ckpt_every = ckpt_every

    # -- lifecycle -----------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            lib().sllg_free(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- running -------------------------------------------------------------
    def run_sweep(self):
        _check("sllg_run_sweep", lib().sllg_run_sweep(self.ctx))

    def run_steps(self, n: int):
        _check("sllg_run_steps", lib().sllg_run_steps(self.ctx, int(n)))

    def reset(self):
        _check("sllg_reset", lib().sllg_reset(self.ctx))

    def synchronize(self):
        """Wait for the stream and raise if a kernel reported a failure."""
        _check("sllg_sync", lib().sllg_sync(self.ctx))

    def set_spin_limit(self, polls: int):
        """Polls of one slab exchange word before the wait gives up."""
        _check("sllg_set_spin_limit", lib().sllg_set_spin_limit(self.ctx, int(polls)))

    # -- results -------------------------------------------------------------
    def loop(self, level: int = 0, real: int = -1):
        """(H_Oe, mH, stats) of one realization or of the ensemble mean."""
        n = C.c_int64()
        _check("sllg_loop", lib().sllg_loop(self.ctx, level, real, None, None, 0, C.byref(n), None))
        H = np.zeros(n.value)
        m = np.zeros(n.value)
        st = LoopStats()
        _check("sllg_loop", lib().sllg_loop(self.ctx, level, real,
                                            H.ctypes.data_as(C.POINTER(C.c_double)),
                                            m.ctypes.data_as(C.POINTER(C.c_double)), n.value,
                                            C.byref(n), C.byref(st)))
        stats = {k: getattr(st, k) for k, _ in LoopStats._fields_}
        return H, m, stats

    def grad(self, level: int = 0):
        """d(S_sim, Hc_sim)/d(K, A, alpha, ms_scale) of the ensemble-mean loop."""
        ga = (C.c_double * 4)()
        gh = (C.c_double * 4)()
        _check("sllg_grad", lib().sllg_grad(self.ctx, level, ga, gh))
        return np.array(list(ga)), np.array(list(gh))

    def level_params(self, level: int = 0) -> dict:
        out = (C.c_double * 16)()
        _check("sllg_level_params", lib().sllg_level_params(self.ctx, level, out))
        return dict(zip(PARAM_KEYS, list(out)))

    def kernel_name(self, level: int = 0) -> str:
        """Kernel (template shape and tiling) that steps the level."""
        buf = C.create_string_buffer(96)
        _check("sllg_level_kernel", lib().sllg_level_kernel(self.ctx, level, buf, 96))
        return buf.value.decode()

    def step(self, level: int = 0) -> int:
        return int(lib().sllg_level_step(self.ctx, level))

    def ncell(self, level: int = 0) -> int:
        l = self.lv[level]
        return l.nx * l.ny * l.nz

    def get_state(self, level: int = 0, real: int = 0) -> np.ndarray:
        """(3, ncell) float32 magnetisation planes."""
        out = np.zeros(3 * self.ncell(level), dtype=np.float32)
        _check("sllg_get_state", lib().sllg_get_state(self.ctx, level, real,
                                                      out.ctypes.data_as(C.POINTER(C.c_float))))
        return out.reshape(3, -1)

    def set_state(self, m, level: int = 0, real: int = 0):
        a = np.ascontiguousarray(np.asarray(m, dtype=np.float32).reshape(3, -1))
        _check("sllg_set_state", lib().sllg_set_state(self.ctx, level, real,
                                                      a.ctypes.data_as(C.POINTER(C.c_float))))

    def save_state(self) -> bytes:
        """Snapshot of everything the sweep carries from step to step (step
        indices, magnetisation, loop accumulators and records, checkpoints)."""
        need = C.c_size_t()
        _check("sllg_save_state", lib().sllg_save_state(self.ctx, None, 0, C.byref(need)))
        buf = C.create_string_buffer(need.value)
        _check("sllg_save_state", lib().sllg_save_state(self.ctx, buf, need.value, C.byref(need)))
        return buf.raw

    def load_state(self, snap: bytes):
        """Continue from a snapshot of a context of the same configuration."""
        _check("sllg_load_state", lib().sllg_load_state(self.ctx, snap, len(snap)))

    def set_plan(self, level: int, plan: int):
        _check("sllg_set_plan", lib().sllg_set_plan(self.ctx, level, plan))

    def set_slab_shape(self, level: int, kind: int, threads: int, cells_per_thread: int, planes: int):
        """Slab plan with a given kernel (kind 0: halo recompute, 1: m' exchange) and thickness."""
        _check("sllg_set_slab_shape", lib().sllg_set_slab_shape(self.ctx, level, kind, threads,
                                                                cells_per_thread, planes))

    def set_stream_shape(self, level: int, kind: int, a: int, b: int, c: int, planes: int):
        """Streamed plan with a given tile kernel (kind 0: x-y window <a,b,c>, 1: rows <a,b>, 2: rows2 <a,b>)."""
        _check("sllg_set_stream_shape", lib().sllg_set_stream_shape(self.ctx, level, kind, a, b, c, planes))

    def axes(self, level: int = 0) -> np.ndarray:
        out = np.zeros(3 * self.ncell(level), dtype=np.float32)
        _check("sllg_get_axes", lib().sllg_get_axes(self.ctx, level,
                                                    out.ctypes.data_as(C.POINTER(C.c_float))))
        return out.reshape(3, -1)

    def set_timing(self, every: int):
        """Bracket every ``every``-th launch of the dominant kernel with events (0: off)."""
        _check("sllg_set_timing", lib().sllg_set_timing(self.ctx, int(every)))

    def kernel_time(self):
        """(mean ms per launch of the dominant kernel, launches, cell-updates per launch)."""
        ms = C.c_double()
        nl = C.c_int64()
        cells = C.c_int64()
        _check("sllg_kernel_time", lib().sllg_kernel_time(self.ctx, C.byref(ms), C.byref(nl), C.byref(cells)))
        return ms.value, nl.value, cells.value


def set_options(flags: int):
    """Process-wide OPT_* flags for contexts created afterwards."""
    _check("sllg_set_options", lib().sllg_set_options(int(flags)))


def philox_probe(seed, level, tag, cells, steps, device="cuda:0"):
    """Device Philox words (n, 4) uint32 and normals (n, 3) float32."""
    import torch
    cells = np.ascontiguousarray(cells, dtype=np.uint32)
    steps = np.ascontiguousarray(steps, dtype=np.uint64)
    n = len(cells)
    raw = np.zeros((n, 4), dtype=np.uint32)
    nrm = np.zeros((n, 3), dtype=np.float32)
    scratch = torch.empty(48 * n + 1024, dtype=torch.uint8, device=device)
    ptr = (scratch.data_ptr() + 255) & ~255
    stream = torch.cuda.current_stream(torch.device(device)).cuda_stream
    _check("sllg_philox_probe", lib().sllg_philox_probe(
        int(seed), int(level), int(tag), cells.ctypes.data_as(C.POINTER(C.c_uint32)),
        steps.ctypes.data_as(C.POINTER(C.c_uint64)), n,
        raw.ctypes.data_as(C.POINTER(C.c_uint32)), nrm.ctypes.data_as(C.POINTER(C.c_float)),
        C.c_void_p(ptr), C.c_void_p(stream)))
    return raw, nrm


# ---------------------------------------------------------------------------
# torch.autograd interface to sllg_grad
# ---------------------------------------------------------------------------
def _loop_function():
    import torch

    class SllgLoop(torch.autograd.Function):
        """(S_sim, Hc_sim) of the ensemble-mean loop of one level as a
        function of its simulated K, A (J/m^3, J/m), its damping alpha and the
        Ms multiplier ms_scale (0-d float64 tensors).

        The forward runs one sweep of every realization of ``level`` under
        ``material`` with those four values substituted (K and A are taken as
        the simulated values, so the coarse-graining rule is not applied to
        them again; the field and loop scales of the level stay as the rule
        gives them) and keeps the context; the first backward calls
        sllg_grad, the discrete adjoint under the same noise, which gives the
        gradients of both outputs, and frees it.  Hc_sim is NaN
        when a branch of the mean loop never crosses zero; its gradient is
        then NaN too.
        """

        @staticmethod
        def forward(ctx, K, A, alpha, ms_scale, material, level, ckpt_every=256, info=None):
            mat = dict(material, K0=float(K), A0=float(A), ms_scale=float(ms_scale), scale_AK=False,
                       sr_ref_Oe_per_ns=0.0)
            # the adjoint weights every step of the loop: record every step
            lvd = dict(level, alpha=float(alpha), record_every=1)
            sim = Sim(mat, [lvd], ckpt_every=ckpt_every)
            sim.run_sweep()
            st = sim.loop(0, -1)[2]
            if info is not None:
                # the whole statistics record and the level's loop scales
                info.update(st)
                p = sim.level_params(0)
                info.update(hscale=p["hscale"], cM=p["cM"], zeta=p["zeta"])
            ctx.sim = sim
            return (torch.tensor(st["S_sim"], dtype=torch.float64),
                    torch.tensor(st["Hc_sim"], dtype=torch.float64))

        @staticmethod
        def backward(ctx, gS, gHc):
            # one adjoint sweep gives both rows; a second backward (the other
            # output) reuses them
            if getattr(ctx, "rows", None) is None:
                ctx.rows = ctx.sim.grad(0)
                ctx.sim.close()
                ctx.sim = None
            ga, gh = ctx.rows
            g = gS.double() * torch.tensor(ga, dtype=torch.float64)
            if float(gHc) != 0.0:
                g = g + gHc.double() * torch.tensor(gh, dtype=torch.float64)
            return g[0], g[1], g[2], g[3], None, None, None, None

    return SllgLoop


_SLLG_LOOP = None


def loop_area_hc(K, A, alpha, ms_scale, material: dict, level: dict, ckpt_every: int = 256,
                 info: dict | None = None):
    """(S_sim, Hc_sim) = SllgLoop.apply(K, A, alpha, ms_scale, ...): the
    differentiable loop of one level (see SllgLoop).  ``info``, if given, is
    filled with the loop's statistics (sllg_loop) and the level's scales
    hscale (zeta of Eq. 10), cM (Eq. 13 factor) and zeta."""
    global _SLLG_LOOP
    if _SLLG_LOOP is None:
        _SLLG_LOOP = _loop_function()
    return _SLLG_LOOP.apply(K, A, alpha, ms_scale, material, level, ckpt_every, info)
