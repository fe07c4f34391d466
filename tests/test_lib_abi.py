"""CPU checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects bad arguments before touching a GPU."""
import ctypes as C
import os
import re

import pytest

import sllg_workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "sllg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sllg_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def L():
    from paper_1912_00310_amd import sllg
    if not os.path.exists(sllg.LIB_PATH):
        from paper_1912_00310_amd import build_lib
        build_lib.build()
    return sllg


def test_every_declared_symbol_is_exported(L):
    names = header_functions()
    assert len(names) >= 15
    lib = C.CDLL(L.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.exported_symbols()) == names


def test_debug_library_exports_the_same_symbols(L):
    # the LDS-check build (tests only) has the product library's C ABI
    from paper_1912_00310_amd import build_debug
    if not os.path.exists(build_debug.LIB):
        build_debug.build()
    lib = C.CDLL(build_debug.LIB)
    for n in header_functions():
        assert hasattr(lib, n), n


def test_snapshot_calls_reject_null_arguments(L):
    # argument checks come before any device access
    need = C.c_size_t(7)
    assert L.lib().sllg_save_state(None, None, 0, C.byref(need)) == -1
    assert L.lib().sllg_load_state(None, b"x", 1) == -1
    assert L.lib().sllg_last_error()


def test_workspace_bytes_sizes(L):
    wl = W.workload("rod_b4_single")
    m = L.material_struct(wl["material"])
    lv = L.levels_struct(wl["levels"])
    n0 = L.lib().sllg_workspace_bytes(C.byref(m), lv, 1, 0)
    n1 = L.lib().sllg_workspace_bytes(C.byref(m), lv, 1, 256)
    assert n0 > 0 and n1 > n0
    # state (2 x 3 x 168 floats) and the loop record (4e4+1 doubles) are inside
    assert n0 > 2 * 3 * 168 * 4 + 40001 * 8


@pytest.mark.parametrize("field,value", [("nx", 0), ("b", 0.5), ("n_real", 0), ("dt_s", -1.0),
                                         ("record_every", 0), ("cone_deg", 95.0)])
def test_invalid_levels_rejected(L, field, value):
    wl = W.workload("rod_b4_single")
    wl["levels"][0][field] = value
    m = L.material_struct(wl["material"])
    lv = L.levels_struct(wl["levels"])
    assert L.lib().sllg_workspace_bytes(C.byref(m), lv, 1, 0) == 0
    ctx = C.c_void_p()
    rc = L.lib().sllg_init(C.byref(m), lv, 1, 0, None, 0, None, C.byref(ctx))
    assert rc == -1 and not ctx.value
    assert L.lib().sllg_last_error()


@pytest.mark.parametrize("field,value", [("Ms0", 0.0), ("T_K", -1.0), ("sweep_Oe_per_ns", 0.0),
                                         ("ms_scale", 0.0), ("n_cycles", 0)])
def test_invalid_material_rejected(L, field, value):
    wl = W.workload("rod_b4_single")
    wl["material"][field] = value
    m = L.material_struct(wl["material"])
    lv = L.levels_struct(wl["levels"])
    ctx = C.c_void_p()
    rc = L.lib().sllg_init(C.byref(m), lv, 1, 0, None, 0, None, C.byref(ctx))
    assert rc == -1


def test_workspace_errors(L):
    wl = W.workload("rod_b4_single")
    m = L.material_struct(wl["material"])
    lv = L.levels_struct(wl["levels"])
    ctx = C.c_void_p()
    assert L.lib().sllg_init(C.byref(m), lv, 1, 0, None, 10, None, C.byref(ctx)) == -2
    assert L.lib().sllg_init(C.byref(m), lv, 1, -1, None, 10, None, C.byref(ctx)) == -1
    # misaligned pointer (never dereferenced: rejected first)
    assert L.lib().sllg_init(C.byref(m), lv, 1, 0, C.c_void_p(8), 1 << 30, None, C.byref(ctx)) == -2
    # too small
    assert L.lib().sllg_init(C.byref(m), lv, 1, 0, C.c_void_p(1 << 20), 1024, None, C.byref(ctx)) == -2


def test_null_context_calls(L):
    lib = L.lib()
    assert lib.sllg_run_sweep(None) == -1
    assert lib.sllg_run_steps(None, 1) == -1
    assert lib.sllg_level_step(None, 0) == -1
    lib.sllg_free(None)


def test_options_and_null_contexts_rejected(L):
    lib = L.lib()
    assert lib.sllg_set_options(16) == -1
    assert lib.sllg_set_options(0) == 0
    assert lib.sllg_sync(None) == -1
    assert lib.sllg_set_spin_limit(None, 0) == -1


def test_demag_level_size_limit(L):
    wl = W.workload("rod_b4_single")
    wl["material"]["demag"] = True
    wl["levels"][0].update(nx=8, ny=8, nz=17)       # 1088 cells
    m = L.material_struct(wl["material"])
    lv = L.levels_struct(wl["levels"])
    assert L.lib().sllg_workspace_bytes(C.byref(m), lv, 1, 0) == 0
    assert b"1024 cells" in L.lib().sllg_last_error()
    wl["levels"][0].update(nz=16)                   # 1024 cells
    lv = L.levels_struct(wl["levels"])
    assert L.lib().sllg_workspace_bytes(C.byref(m), lv, 1, 0) > 0
