"""The C interface: the library loads, exports what include/hfmm.h declares, and
rejects bad arguments on the host before touching the device."""
import ctypes
import os
import re

import pytest

import paper_1703_09136_amd as hf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "hfmm.h")).read()
    return sorted(set(re.findall(r"\b(hfmm_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert sorted(hf.EXPORTS) == declared_functions()


def test_library_exports_every_declared_symbol():
    lib = hf.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_default_options_and_status_strings():
    o = hf.default_options()
    assert o.struct_size == ctypes.sizeof(hf.Options)
    assert o.leaf_size == 64 and o.interface_refine == 1
    lib = hf.load()
    for s in range(7):
        assert lib.hfmm_status_string(s)


def _plan(lib, layers, k, ifs, n, tol, opts=None, points=1):
    h = ctypes.c_void_p()
    kk = (ctypes.c_double * len(k))(*k)
    ii = (ctypes.c_double * max(1, len(ifs)))(*(ifs or [0.0]))
    o = opts if opts is not None else hf.default_options()
    st = lib.hfmm_plan(ctypes.byref(h), layers, kk, ii, n, ctypes.c_void_p(points), tol, ctypes.byref(o), None)
    return st, h


@pytest.mark.parametrize("case,expected", [
    (dict(layers=4), 3),
    (dict(layers=1), 1),
    (dict(layers=1, opts=dict(impedance=-1.0)), 1),
    (dict(layers=1, opts=dict(impedance=float("inf"))), 1),
    (dict(opts=dict(impedance=1.0)), 1),
    (dict(n=0), 1),
    (dict(tol=1e-16), 1),
    (dict(tol=0.5), 1),
    (dict(k=(5.0, -1.0)), 3),
    (dict(k=(5.0, 3.0)), 3),
    (dict(k=(5.0, float("nan"))), 3),
    (dict(layers=3, k=(5.0, 6.0, 7.0), ifs=(0.0, 0.5)), 1),
    (dict(points=0), 1),
    (dict(opts=dict(leaf_size=0)), 1),
    (dict(opts=dict(precision=7)), 3),
    (dict(opts=dict(max_level=1)), 1),
    (dict(opts=dict(top_level=1)), 1),
    (dict(opts=dict(top_level=31)), 1),
    (dict(opts=dict(leaf_kb=0.1)), 1),
    (dict(opts=dict(self_term=5)), 1),
    (dict(opts=dict(order=-1)), 1),
    (dict(opts=dict(order=256)), 1),
    (dict(opts=dict(max_nrhs=-1)), 1),
    (dict(opts=dict(deterministic=2)), 1),
    (dict(opts=dict(precision=3)), 3),
])
def test_plan_rejects_bad_arguments(case, expected):
    lib = hf.load()
    layers = case.get("layers", 2)
    k = case.get("k", (5.0, 6.0, 7.0)[:max(2, min(layers, 3))] if layers in (2, 3) else (5.0, 6.0))
    ifs = case.get("ifs", (0.0, -0.5)[:max(1, layers - 1)] if layers in (2, 3) else (0.0,))
    opts = hf.default_options(**case.get("opts", {}))
    st, h = _plan(lib, layers, k, ifs, case.get("n", 10), case.get("tol", 1e-8), opts, case.get("points", 1))
    assert st == expected, lib.hfmm_last_error_message()
    assert not h.value
    assert lib.hfmm_last_error_message()


def test_null_plan_calls_fail_cleanly():
    lib = hf.load()
    assert lib.hfmm_apply(None, None, None, 1, None) == 1
    assert lib.hfmm_apply_adjoint(None, None, None, 1, None, None, None) == 1
    info = hf.Info()
    assert lib.hfmm_plan_info(None, ctypes.byref(info)) == 1
    lib.hfmm_destroy(None)


def test_allocator_must_come_with_free():
    lib = hf.load()
    o = hf.default_options()
    o.alloc = hf._TORCH_ALLOC
    st, h = _plan(lib, 2, (5.0, 6.0), (0.0,), 10, 1e-8, o)
    assert st == 1 and not h.value
    assert "alloc" in lib.hfmm_last_error_message().decode()


def test_tree_build_rejects_bad_arguments():
    lib = hf.load()
    h = ctypes.c_void_p()
    k = (ctypes.c_double * 1)(5.0)
    ifs = (ctypes.c_double * 1)(0.0)
    pts = ctypes.c_void_p(1)  # never dereferenced: every case fails on the host first

    def build(out=ctypes.byref(h), n=10, points=pts, builder=0, **opts):
        o = hf.default_options(**opts)
        return lib.hfmm_tree_build(out, k, ifs, n, points, ctypes.byref(o), builder, None)

    assert build(out=None) == 1
    assert build(n=0) == 1
    assert build(points=None) == 1
    assert build(builder=2) == 1
    assert build(leaf_size=0) == 1
    assert build(max_level=1) == 1
    assert build(leaf_kb=0.1) == 1
    assert not h.value
    counts = (ctypes.c_int64 * 8)()
    assert lib.hfmm_tree_counts(None, counts) == 1
    assert lib.hfmm_tree_copy(None, None, None, None, None, None, None, None, None, None) == 1
    lib.hfmm_tree_destroy(None)
