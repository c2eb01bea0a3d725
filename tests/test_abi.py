"""CPU checks of the C ABI: the library loads, exports every function that
include/fmm.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_2511_15269_amd import _lib as L

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "fmm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fmm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_api():
    names = declared_functions()
    for want in ("fmm_plan_create", "fmm_evaluate", "fmm_plan_destroy", "fmm_last_error",
                 "fmm_abi_version", "fmm_plan_get_info", "fmm_plan_get_tree", "fmm_plan_get_lists"):
        assert want in names


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_abi_version():
    assert L.lib().fmm_abi_version() == 1


def _create(**kw):
    prm = L.FmmParams(p=8, leaf_max=128, splits=2, theta=0.7, max_depth=16,
                      precision=L.FMM_FP64, tie_refine=0, max_rhs=1)
    n = kw.pop("n", 1000)
    for k, v in kw.items():
        setattr(prm, k, v)
    out = ctypes.c_void_p(12345)
    # a dummy, never dereferenced position pointer: argument checks come first
    st = L.lib().fmm_plan_create(ctypes.c_void_p(0x1000), n, ctypes.byref(prm), None, ctypes.byref(out))
    return st, out


@pytest.mark.parametrize("kw,code", [
    (dict(p=0), L.FMM_EINVAL), (dict(p=11), L.FMM_ENOTSUP), (dict(splits=0), L.FMM_EINVAL),
    (dict(splits=4), L.FMM_EINVAL), (dict(leaf_max=3), L.FMM_EINVAL), (dict(theta=0.0), L.FMM_EINVAL),
    (dict(theta=1.0), L.FMM_EINVAL), (dict(theta=float("nan")), L.FMM_EINVAL),
    (dict(max_depth=-1), L.FMM_EINVAL), (dict(max_depth=17), L.FMM_EINVAL),
    (dict(precision=2), L.FMM_EINVAL), (dict(tie_refine=2), L.FMM_EINVAL),
    (dict(max_rhs=0), L.FMM_EINVAL), (dict(n=0), L.FMM_EINVAL), (dict(n=1 << 31), L.FMM_EINVAL)])
def test_bad_parameters_are_rejected_and_out_is_untouched(kw, code):
    st, out = _create(**kw)
    assert st == code
    assert out.value == 12345
    assert L.lib().fmm_last_error().decode() != ""


def test_null_arguments():
    lib = L.lib()
    prm = L.FmmParams(p=8, leaf_max=128, splits=2, theta=0.7, max_depth=16, precision=0,
                      tie_refine=0, max_rhs=1)
    out = ctypes.c_void_p()
    assert lib.fmm_plan_create(None, 10, ctypes.byref(prm), None, ctypes.byref(out)) == L.FMM_EINVAL
    assert lib.fmm_plan_create(ctypes.c_void_p(0x1000), 10, None, None, ctypes.byref(out)) == L.FMM_EINVAL
    assert lib.fmm_plan_create(ctypes.c_void_p(0x1000), 10, ctypes.byref(prm), None, None) == L.FMM_EINVAL
    assert lib.fmm_evaluate(None, None, 1, None, None, None) == L.FMM_EINVAL
    assert lib.fmm_plan_get_info(None, None) == L.FMM_EINVAL
    assert lib.fmm_plan_destroy(None) == L.FMM_OK


@pytest.mark.parametrize("offsets,nprob", [
    ([0], 0),                 # no problem
    ([1, 10], 1),             # offsets[0] != 0
    ([0, 10, 10], 2),         # an empty problem
    ([0, 10, 5], 2),          # decreasing
    ([0, 1 << 31], 1),        # total too large
])
def test_multi_plan_bad_offsets(offsets, nprob):
    lib = L.lib()
    prm = L.FmmParams(p=8, leaf_max=128, splits=2, theta=0.7, max_depth=16, precision=0,
                      tie_refine=0, max_rhs=1)
    off = (ctypes.c_int64 * len(offsets))(*offsets)
    out = ctypes.c_void_p(777)
    st = lib.fmm_multi_plan_create(ctypes.c_void_p(0x1000), off, nprob, ctypes.byref(prm), None,
                                   ctypes.byref(out))
    assert st == L.FMM_EINVAL
    assert out.value == 777
    assert lib.fmm_last_error().decode() != ""


def test_graph_null_arguments():
    lib = L.lib()
    out = ctypes.c_void_p(5)
    assert lib.fmm_graph_create(None, 0, None, 1, None, None, ctypes.byref(out)) == L.FMM_EINVAL
    assert out.value == 5
    assert lib.fmm_graph_launch(None, None) == L.FMM_EINVAL
    assert lib.fmm_graph_destroy(None) == L.FMM_OK
    assert lib.fmm_multi_plan_create(None, None, 1, None, None, ctypes.byref(out)) == L.FMM_EINVAL


def test_autotune_null_arguments():
    lib = L.lib()
    assert lib.fmm_plan_autotune(None, None, None, None, None) == L.FMM_EINVAL
