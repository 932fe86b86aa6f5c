"""CPU checks of the C ABI: the library loads and exports every symbol that
include/ils.h declares, argument errors are reported without a GPU call, and
the Python structs match the C layouts."""
import ctypes as C
import os
import re

import pytest

import paper_2203_15340_amd as ils

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ils.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ils_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = ils.load_library()
    names = declared_functions()
    assert "ils_sp_solve" in names and "ils_rk_solve" in names and "ils_rgs_solve" in names
    for name in names:
        assert hasattr(L, name), name
    assert sorted(ils.EXPORTS) == names


def test_struct_layouts():
    # ils_opts: 8 + 4*4 + 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8 bytes, ils_info: 4+4+8*5
    assert C.sizeof(ils.Opts) == 88
    assert C.sizeof(ils._Info) == 48
    assert C.sizeof(ils._TuneEntry) == 48  # 2 int32, 2 int64, 2 int32, 1 double, 2 int32
    o = ils.Opts()
    ils.load_library().ils_opts_default(C.byref(o))
    assert o.tol == 1e-6 and o.max_outer == 20000 and o.stop_rule == ils.STOP_RR
    assert o.form == ils.FORM_PAPER and o.precision == ils.PREC_FP64


def test_status_strings():
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert ils.status_string(code)
    assert ils.status_string(-2).startswith("A1^T A1")


def test_null_handle_is_an_argument_error():
    L = ils.load_library()
    o = ils.Opts()
    L.ils_opts_default(C.byref(o))
    info = ils._Info()
    rc = L.ils_sp_solve(None, 10, 2, 5, None, 12, None, None, None, C.byref(o), C.byref(info))
    assert rc == ils.ERR_ARG and info.status == ils.ERR_ARG
    for fn in ("ils_rk_solve", "ils_rgs_solve"):
        assert getattr(L, fn)(None, 10, 2, 5, None, 12, None, None, None, C.byref(o), C.byref(info)) == ils.ERR_ARG
    assert L.ils_destroy(None) == ils.ERR_ARG


def test_create_without_gpu_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert ils.load_library().ils_create(C.byref(h), 0, None) != ils.OK
    with pytest.raises(ils.ILSError):
        ils.handle()
