"""The C ABI library loads and exports every function include/tron.h declares (no GPU
needed: nothing here launches work), and the host-side helpers behave."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = "".join(open(os.path.join(ROOT, "include", h)).read() for h in sorted(os.listdir(os.path.join(ROOT, "include")))
                  if h.endswith(".h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("tron_batch_create", "tron_batch_solve", "tron_batch_destroy", "admm_step"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2106_14995_amd import tron
    L = tron.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_host_helpers():
    from paper_2106_14995_amd import tron
    assert tron.param_size(tron.QP4, 8) == 36 + 8 + 1
    assert tron.param_size(tron.QP4, 128) == 128 * 129 // 2 + 129
    assert tron.param_size(tron.BR6, 6) == 36
    assert tron.param_size(tron.BR6, 5) == -1
    assert tron.param_size(tron.HS45M, 4) == 0
    assert tron.param_size(tron.HS45M, 128) == 0
    assert tron.param_size(tron.BR8L, 8) == 40
    assert tron.param_size(tron.BR8L, 6) == -1
    o = tron.options()
    assert o.gtol == 1e-6 and o.max_iter == 500 and o.cg_rtol == 0.1 and o.flags == 0
    a = tron.AlOptions()
    tron.lib().tron_default_al_options(C.byref(a))
    assert (a.ctol, a.outer_max, a.rho_growth, a.decrease, a.rho_max) == (1e-6, 50, 10.0, 0.25, 1e6)


def test_default_plan_spec_matches_the_binding():
    from paper_2106_14995_amd import tron
    spec = tron.PlanSpec()
    tron.lib().tron_default_plan_spec(C.byref(spec))
    mine = tron.plan_spec()
    assert spec.lane_max_n == mine.lane_max_n and spec.streams == mine.streams
    assert spec.lane_block == mine.lane_block == 64
    assert spec.pool_waves == mine.pool_waves == 12
    assert spec.lane_group == mine.lane_group == 0 and spec.group16 == mine.group16 == 0
    assert spec.wave_global == mine.wave_global == 0
    assert list(spec.edges[:spec.nedges]) == list(tron.DEFAULT_EDGES) == list(mine.edges[:mine.nedges])


def test_design_calls_reject_bad_arguments_before_touching_the_device():
    from paper_2106_14995_amd import tron
    L = tron.lib()
    assert L.tron_design_chol(7, 1, 4, None, None, None, None) == 1    # unknown variant
    assert L.tron_design_chol(4, 1, 4, None, None, None, None) == 1    # one past the last
    assert L.tron_design_chol(tron.CHOL_BLOCKED_MFMA, 0, 64, None, None, None, None) == 0  # valid, empty
    assert L.tron_design_chol(tron.CHOL_BLOCKED_MFMA, 1, 4, None, None, None, None) == 1  # null pointers
    assert L.tron_design_chol(0, 1, 65, None, None, None, None) == 1   # n above 64
    assert L.tron_design_chol(0, 1, 4, None, None, None, None) == 1    # null pointers
    assert L.tron_design_chol(0, 0, 4, None, None, None, None) == 0    # empty batch
    assert L.tron_design_trsv(0, 1, 4, None, None, None, 0, None) == 1  # reps < 1
    assert L.tron_design_trsv(4, 1, 4, None, None, None, 1, None) == 1  # unknown variant
    assert L.tron_design_fma_peak(1, 1, None, None) == 1                # null sink
    assert L.tron_design_fma_peak(0, 1, None, None) == 1                # no workgroup
    assert L.tron_design_fma_peak(1, 0, None, None) == 1                # no iteration


def test_al_solve_rejects_bad_arguments_before_touching_the_device():
    from paper_2106_14995_amd import tron
    L = tron.lib()
    null = [None] * 10
    assert L.tron_al_solve(None, None, *null, None) == 1


def test_create_rejects_bad_arguments_before_touching_the_device():
    from paper_2106_14995_amd import tron
    h = C.c_void_p()
    L = tron.lib()
    assert L.tron_batch_create(None, 0, 1, None, 4, None, None) == 1
    assert L.tron_batch_create(C.byref(h), 7, 1, None, 4, None, None) == 1
    assert L.tron_batch_create(C.byref(h), tron.BR6, 1, None, 5, None, None) == 1
    assert L.tron_batch_create(C.byref(h), tron.QP4, -1, None, 4, None, None) == 1
    assert b"invalid" in L.tron_last_error() or len(L.tron_last_error()) > 0


def declared_arities():
    src = "".join(open(os.path.join(ROOT, "include", h)).read() for h in sorted(os.listdir(os.path.join(ROOT, "include")))
                  if h.endswith(".h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    out = {}
    for name, params in re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(([^;{]*?)\)\s*;",
                                   src, flags=re.M | re.S):
        params = params.strip()
        out[name] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_binding_declares_every_call_with_the_header_arity():
    """Every declared call has ctypes argument types in the binding, as many as the header
    declares: an undeclared call would pass 64-bit pointers and sizes as C ints."""
    from paper_2106_14995_amd import tron
    L = tron.lib()
    ar = declared_arities()
    assert set(ar) == set(declared_functions())
    bad = {n: (k, getattr(L, n).argtypes) for n, k in ar.items()
           if getattr(L, n).argtypes is None or len(getattr(L, n).argtypes) != k}
    assert not bad, bad
