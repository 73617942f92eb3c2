"""ctypes binding of libqm.so (include/qm.h), argument marshalling only.

Every function here forwards to the C ABI of the same name; all arithmetic
runs in the library's HIP kernels.  Tensors are used only for their device
pointers and the current HIP stream.  If libqm.so has not been built the
import fails loudly: there is no CPU fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqm.so")

QM_OK = 0
QM_PENDING = 1
QM_E_INVAL = -1
QM_E_DTYPE = -2
QM_E_NOMEM = -3
QM_E_HIP = -4
QM_E_CLOSED = -5
QM_E_TICKET = -6

QM_BATCH_NOALLOC_MAX_REQUESTS = 4096

QM_F32 = 0
QM_F64 = 1

QM_PLAIN = 0
QM_F32_REFINE = 1
QM_PAPER = 2
QM_PAPER_T2 = 3

QM_NORMAL_QUANTILE = 0
QM_STUDENT_T = 1
QM_EXP_TO_NORMAL = 2
QM_UNIFORM = 3
QM_EXP_TO_HYPERBOLIC = 4
QM_EXP_TO_VG = 5


class qm_request(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_uint32),
        ("dtype", ctypes.c_uint32),
        ("mode", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("nu", ctypes.c_double),
        ("d_in", ctypes.c_void_p),
        ("d_out", ctypes.c_void_p),
        ("n", ctypes.c_uint64),
        ("user_tag", ctypes.c_uint64),
        ("alpha", ctypes.c_double),
        ("beta", ctypes.c_double),
        ("delta", ctypes.c_double),
        ("mu", ctypes.c_double),
    ]


class qm_serving_counters(ctypes.Structure):
    _fields_ = [(name, ctypes.c_uint64) for name in (
        "submitted", "completed", "failed", "queued", "in_flight_requests", "in_flight_bytes",
        "in_flight_bytes_high_water", "budget_bytes", "tickets_kept")]


# name -> (restype, argtypes), exactly the declarations of include/qm.h
_vp, _u64, _i, _d = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int, ctypes.c_double
_st = ctypes.c_int32
SIGNATURES = {
    "qm_init": (_st, [_i, _u64, ctypes.POINTER(_vp)]),
    "qm_shutdown": (None, [_vp]),
    "qm_normal_quantile": (_st, [_vp, _vp, _vp, _u64, _i, _i, _vp]),
    "qm_recycle_student_t": (_st, [_vp, _vp, _vp, _u64, _i, _i, _d, _vp]),
    "qm_recycle_exp_to_normal": (_st, [_vp, _vp, _vp, _u64, _i, _i, _vp]),
    "qm_recycle_exp_to_hyperbolic": (_st, [_vp, _vp, _vp, _u64, _i, _i, _d, _d, _d, _d, _vp]),
    "qm_hyperbolic_masses": (_st, [_vp, _d, _d, _d, ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    "qm_recycle_exp_to_vg": (_st, [_vp, _vp, _vp, _u64, _i, _i, _d, _d, _d, _d, _vp]),
    "qm_vg_masses": (_st, [_vp, _d, _d, _d, ctypes.POINTER(_d), ctypes.POINTER(_d)]),
    "qm_generate": (_st, [_vp, _u64, _u64, _u64, _vp, _u64, _i, _i, _i, _vp]),
    "qm_generate_student_t": (_st, [_vp, _u64, _u64, _u64, _vp, _u64, _i, _i, _d, _vp]),
    "qm_generate_hyperbolic": (_st, [_vp, _u64, _u64, _u64, _vp, _u64, _i, _i, _d, _d, _d, _d, _vp]),
    "qm_generate_vg": (_st, [_vp, _u64, _u64, _u64, _vp, _u64, _i, _i, _d, _d, _d, _d, _vp]),
    "qm_run_batch": (_st, [_vp, ctypes.POINTER(qm_request), _u64, _vp]),
    "qm_run_batch_noalloc": (_st, [_vp, ctypes.POINTER(qm_request), _u64, _vp]),
    "qm_submit": (_st, [_vp, ctypes.POINTER(qm_request), ctypes.POINTER(_u64)]),
    "qm_poll": (_st, [_vp, _u64]),
    "qm_poll_times": (_st, [_vp, _u64, ctypes.POINTER(_u64), ctypes.POINTER(_u64)]),
    "qm_serving_stats": (_st, [_vp, ctypes.POINTER(qm_serving_counters)]),
    "qm_serving_latencies": (_u64, [_vp, ctypes.POINTER(_u64), _u64]),
    "qm_status_string": (ctypes.c_char_p, [_st]),
    "qm_last_error": (ctypes.c_char_p, []),
}

# include/qm_debug.h: host-only diagnostics of the table builders
DEBUG_SIGNATURES = {
    "qm_debug_student_dense": (ctypes.c_int, [_d, ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.c_int]),
    "qm_debug_student_table": (ctypes.c_int, [_d, _vp, ctypes.POINTER(_d), ctypes.c_int]),
    "qm_debug_hyperbolic_dense": (ctypes.c_int, [_d, _d, _d, ctypes.POINTER(_d), ctypes.POINTER(_d), ctypes.c_int]),
    "qm_debug_hyperbolic_table": (ctypes.c_int, [_d, _d, _d, _vp, ctypes.POINTER(_d), ctypes.c_int]),
    "qm_debug_vg_table": (ctypes.c_int, [_d, _d, _d, _vp, ctypes.POINTER(_d), ctypes.c_int]),
}

_lib = None


def load():
    """Load libqm.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libqm.so not built at %s (run python -m paper_0901_0638_amd.build)" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in list(SIGNATURES.items()) + list(DEBUG_SIGNATURES.items()):
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class QMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (load().qm_status_string(status).decode(), msg))
        self.status = status


def check(status):
    if status < 0:
        raise QMError(status, load().qm_last_error().decode())
    return status
