"""CPU-side checks of the C ABI: the library loads, exports every function
include/qm.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import pytest

import paper_0901_0638_amd as qm
from paper_0901_0638_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions(name="qm.h"):
    src = open(os.path.join(ROOT, "include", name)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qm_[a-z_0-9]+)\s*\(", src)))


def all_header_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            names += header_functions(h)
    return sorted(set(names))


def test_header_declares_the_bound_functions():
    assert header_functions("qm.h") == sorted(_lib.SIGNATURES)
    assert header_functions("qm_debug.h") == sorted(_lib.DEBUG_SIGNATURES)


def test_library_exports_every_symbol():
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for name in all_header_functions():
        assert hasattr(lib, name), name


def test_request_layout():
    """qm_request as include/qm.h declares it: 88 bytes, the hyperbolic
    parameters after user_tag."""
    r = _lib.qm_request
    assert ctypes.sizeof(r) == 88
    assert r.user_tag.offset == 48 and r.alpha.offset == 56 and r.mu.offset == 80
    assert qm.QM_EXP_TO_HYPERBOLIC == 4 and qm.QM_EXP_TO_VG == 5


def test_status_strings():
    lib = _lib.load()
    for s, name in [(0, b"QM_OK"), (1, b"QM_PENDING"), (-1, b"QM_E_INVAL"), (-2, b"QM_E_DTYPE"),
                    (-3, b"QM_E_NOMEM"), (-4, b"QM_E_HIP"), (-5, b"QM_E_CLOSED"), (-6, b"QM_E_TICKET")]:
        assert lib.qm_status_string(s) == name


def test_null_context_rejected_without_device_work():
    lib = _lib.load()
    p = ctypes.c_void_p(0x1000)
    assert lib.qm_normal_quantile(None, p, p, 10, qm.QM_F64, qm.QM_PLAIN, None) == qm.QM_E_INVAL
    assert b"context" in lib.qm_last_error()
    assert lib.qm_recycle_student_t(None, p, p, 10, qm.QM_F64, qm.QM_PLAIN, 4.0, None) == qm.QM_E_INVAL
    assert lib.qm_recycle_exp_to_normal(None, p, p, 10, qm.QM_F64, qm.QM_PLAIN, None) == qm.QM_E_INVAL
    assert lib.qm_recycle_exp_to_hyperbolic(None, p, p, 10, qm.QM_F64, qm.QM_PLAIN, 1.0, 0.0, 1.0, 0.0,
                                            None) == qm.QM_E_INVAL
    lp = ctypes.c_double()
    assert lib.qm_hyperbolic_masses(None, 1.0, 0.0, 1.0, ctypes.byref(lp), None) == qm.QM_E_INVAL
    assert lib.qm_init(0, 0, None) == qm.QM_E_INVAL
    lib.qm_shutdown(None)


def test_init_without_gpu_reports_error():
    """In a container without a GPU qm_init must fail cleanly."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = _lib.load()
    h = ctypes.c_void_p()
    st = lib.qm_init(0, 0, ctypes.byref(h))
    assert st in (qm.QM_E_HIP, qm.QM_E_INVAL)
    assert not h.value
