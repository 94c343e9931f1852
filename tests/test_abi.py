"""The C ABI library (CPU only: no compute calls).

libfmm2d.so must load and export every function include/fmm2d.h declares;
argument validation that happens before any device work, and the order rule
p(eps), must behave as documented."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "fmm2d.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?\**\s*\b(fmm_[a-z_0-9]+)\s*\(",
                       src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def F():
    from paper_1204_3105_amd import fmm
    return fmm


def test_library_exports_every_declared_symbol(F):
    names = declared_functions()
    assert len(names) >= 14, names
    lib = C.CDLL(F.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert set(F.EXPORTED) == set(names)


def test_order_rule_matches_separation_ratios(F):
    # p = ceil(ln eps / ln q) - 1 with q = 1/(2 sqrt2 - 1), 0.524434, 1/(sqrt7 - 1)
    assert [F.order_for_eps(t, 1e-6) for t in ("quad", "sept", "tri")] == [22, 21, 27]
    assert [F.order_for_eps(t, 1e-10) for t in ("quad", "sept", "tri")] == [38, 35, 46]
    assert [F.order_for_eps(t, 1e-4) for t in ("quad", "sept", "tri")] == [15, 14, 18]
    assert F.order_for_eps("quad", 0.0) == -1
    assert F.order_for_eps("quad", 0.7) == -1


def test_options_default_and_validation(F):
    lib = F.lib()
    o = F.Options()
    assert lib.fmm_options_default(C.byref(o)) == 0
    assert o.struct_size == C.sizeof(F.Options) and o.leaf_size == 64
    assert o.lmax == -1 and o.p == -1 and o.precision == 0
    plan = C.c_void_p()
    pts = (C.c_double * 4)(0.1, 0.2, 0.3, 0.4)
    # bad tiling, negative count, null array, bad eps: rejected before any device call
    assert lib.fmm_plan(7, pts, 2, pts, 2, 1e-6, C.byref(o), C.byref(plan)) == 1
    assert b"tiling" in lib.fmm_last_error()
    assert lib.fmm_plan(0, pts, -1, pts, 2, 1e-6, C.byref(o), C.byref(plan)) == 1
    assert lib.fmm_plan(0, None, 2, pts, 2, 1e-6, C.byref(o), C.byref(plan)) == 1
    assert lib.fmm_plan(0, pts, 2, pts, 2, 0.0, C.byref(o), C.byref(plan)) == 1
    assert lib.fmm_plan(0, pts, 2, pts, 2, 0.6, C.byref(o), C.byref(plan)) == 1
    o.struct_size = 3
    assert lib.fmm_plan(0, pts, 2, pts, 2, 1e-6, C.byref(o), C.byref(plan)) == 1
    assert lib.fmm_eval(None, None, None) == 1
    assert lib.fmm_eval_field(None, None, None, None) == 1
    lib.fmm_plan_destroy(None)


def test_server_option_validation(F):
    lib = F.lib()
    s = C.c_void_p()
    o = F.ServerOptions()
    o.struct_size = C.sizeof(F.ServerOptions)
    o.hbm_budget_bytes = 0
    o.max_inflight = 4
    assert lib.fmm_server_create(C.byref(o), C.byref(s)) == 1
    o.hbm_budget_bytes = 1 << 20
    o.max_inflight = 0
    assert lib.fmm_server_create(C.byref(o), C.byref(s)) == 1


def test_direct_validation(F):
    lib = F.lib()
    o = F.Options()
    assert lib.fmm_options_default(C.byref(o)) == 0
    pts = (C.c_double * 4)(0.1, 0.2, 0.3, 0.4)
    u = (C.c_double * 2)(1.0, -1.0)
    phi = (C.c_double * 4)()
    # negative sizes, null arrays, a bad options struct: rejected before any device call
    assert lib.fmm_direct(pts, -1, pts, 2, u, phi, C.byref(o)) == 1
    assert lib.fmm_direct(pts, 2, pts, -2, u, phi, C.byref(o)) == 1
    assert lib.fmm_direct(None, 2, pts, 2, u, phi, C.byref(o)) == 1
    assert lib.fmm_direct(pts, 2, pts, 2, None, phi, C.byref(o)) == 1
    assert lib.fmm_direct(pts, 2, None, 2, u, phi, C.byref(o)) == 1
    assert lib.fmm_direct(pts, 2, pts, 2, u, None, C.byref(o)) == 1
    assert b"null" in lib.fmm_last_error()
    bad = (C.c_double * 4)(0.1, float("nan"), 0.3, 0.4)
    assert lib.fmm_direct(bad, 2, pts, 2, u, phi, None) == 1
    assert b"finite" in lib.fmm_last_error()
    assert lib.fmm_direct(pts, 2, bad, 2, u, phi, None) == 1
    o2 = F.Options()
    lib.fmm_options_default(C.byref(o2))
    o2.struct_size = 3
    assert lib.fmm_direct(pts, 2, pts, 2, u, phi, C.byref(o2)) == 1
    # no targets: nothing to do, no device needed
    assert lib.fmm_direct(pts, 2, None, 0, u, None, None) == 0


def test_depth_rule_option(F):
    lib = F.lib()
    o = F.Options()
    assert lib.fmm_options_default(C.byref(o)) == 0
    assert o.depth_rule == 0
    o.depth_rule = 5
    plan = C.c_void_p()
    pts = (C.c_double * 4)(0.1, 0.2, 0.3, 0.4)
    assert lib.fmm_plan(0, pts, 2, pts, 2, 1e-6, C.byref(o), C.byref(plan)) == 1
    assert b"depth" in lib.fmm_last_error()


def test_near_stream_option(F):
    lib = F.lib()
    o = F.Options()
    assert lib.fmm_options_default(C.byref(o)) == 0
    assert o.near_stream == 0
    assert C.sizeof(o) == o.struct_size
    o.near_stream = 2
    plan = C.c_void_p()
    pts = (C.c_double * 4)(0.1, 0.2, 0.3, 0.4)
    assert lib.fmm_plan(0, pts, 2, pts, 2, 1e-6, C.byref(o), C.byref(plan)) == 1
    assert b"near_stream" in lib.fmm_last_error()
