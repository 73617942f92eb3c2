"""MI355X-native quantile mechanics (Shaw, Luu & Brickman, "Quantile Mechanics II").

Thin Python binding of libqm.so.  The functions carry the C ABI's names and
forward torch device tensors (pointers + current HIP stream) to it; every
step of the maps runs in the library's HIP kernels.

    ctx = Context(device=0)
    qm_normal_quantile(ctx, u, w)                 # w = Phi^{-1}(u)
    qm_recycle_student_t(ctx, z, t, nu=4.0)       # t = F_nu^{-1}(Phi(z))
    qm_recycle_exp_to_normal(ctx, x, z)           # z = sign(x) Phi^{-1}(1 - e^{-|x|}/2)
    qm_recycle_exp_to_hyperbolic(ctx, v, x, alpha, beta, delta)   # x = F_hyp^{-1}(F0(v))
    qm_generate(ctx, seed, stream, first, w, QM_NORMAL_QUANTILE)   # w = Phi^{-1}(Philox uniforms)
"""
import ctypes

from ._lib import (  # noqa: F401
    QM_E_CLOSED, QM_E_DTYPE, QM_E_HIP, QM_E_INVAL, QM_E_NOMEM, QM_E_TICKET, QM_EXP_TO_NORMAL, QM_F32,
    QM_F32_REFINE, QM_F64, QM_NORMAL_QUANTILE, QM_OK, QM_PAPER, QM_PAPER_T2, QM_PENDING, QM_PLAIN, QM_STUDENT_T, QM_UNIFORM, QMError,
    QM_EXP_TO_HYPERBOLIC, QM_EXP_TO_VG, QM_BATCH_NOALLOC_MAX_REQUESTS,
    check, load, qm_request, qm_serving_counters,
)

_DTYPES = {"torch.float64": QM_F64, "torch.float32": QM_F32}


class Context:
    """Owns a qm_ctx (Student t and hyperbolic tables, serving state) on one HIP device."""

    def __init__(self, device=0, hbm_budget_bytes=0):
        lib = load()
        h = ctypes.c_void_p()
        check(lib.qm_init(int(device), int(hbm_budget_bytes), ctypes.byref(h)))
        self._h = h
        self.device = device

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("context already shut down")
        return self._h

    def close(self):
        if self._h is not None:
            load().qm_shutdown(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dtype_of(t):
    try:
        return _DTYPES[str(t.dtype)]
    except KeyError:
        raise TypeError("expected a float32 or float64 tensor, got %s" % t.dtype)


def _stream(stream, t):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _io(inp, out):
    if inp.device.type != "cuda" or out.device.type != "cuda":
        raise ValueError("tensors must be on a HIP device")
    if not (inp.is_contiguous() and out.is_contiguous()):
        raise ValueError("tensors must be contiguous")
    if inp.numel() != out.numel() or inp.dtype != out.dtype:
        raise ValueError("input and output must have the same size and dtype")
    return ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()), inp.numel(), _dtype_of(inp)


def qm_normal_quantile(ctx, u, w, mode=QM_PLAIN, stream=None):
    """w = Phi^{-1}(u) on the device (FP64: PLAIN/PAPER/PAPER_T2; FP32: PLAIN/F32_REFINE/PAPER)."""
    pi, po, n, dt = _io(u, w)
    check(load().qm_normal_quantile(ctx.handle, pi, po, n, dt, mode, _stream(stream, u)))


def qm_generate(ctx, seed, stream_id, first, out, kind=QM_NORMAL_QUANTILE, mode=None, stream=None):
    """out[i] = map of the open uniform of element first + i of the Philox4x32-10
    stream with key (seed, stream_id): kind QM_UNIFORM (u itself) or
    QM_NORMAL_QUANTILE (Phi^{-1}(u); FP64 PLAIN/PAPER, FP32 F32_REFINE/PLAIN/PAPER)."""
    if out.device.type != "cuda" or not out.is_contiguous():
        raise ValueError("output must be a contiguous tensor on a HIP device")
    dt = _dtype_of(out)
    if mode is None:
        mode = QM_F32_REFINE if (dt == QM_F32 and kind == QM_NORMAL_QUANTILE) else QM_PLAIN
    check(load().qm_generate(ctx.handle, int(seed), int(stream_id), int(first), ctypes.c_void_p(out.data_ptr()),
                             out.numel(), int(kind), dt, int(mode), _stream(stream, out)))


def qm_generate_student_t(ctx, seed, stream_id, first, out, nu, mode=None, stream=None):
    """Student t samples of a Philox stream: the t map of qm_generate's normals, fused."""
    dt = _dtype_of(out)
    if mode is None:
        mode = QM_PLAIN if dt == QM_F64 else QM_F32_REFINE
    check(load().qm_generate_student_t(ctx.handle, int(seed), int(stream_id), int(first), ctypes.c_void_p(out.data_ptr()),
                                       out.numel(), dt, int(mode), float(nu), _stream(stream, out)))


def qm_generate_hyperbolic(ctx, seed, stream_id, first, out, alpha, beta, delta, mu=0.0, mode=None, stream=None):
    """Hyperbolic samples of a Philox stream: each uniform's two-sided exponential base sample, mapped, fused."""
    dt = _dtype_of(out)
    if mode is None:
        mode = QM_PLAIN if dt == QM_F64 else QM_F32_REFINE
    check(load().qm_generate_hyperbolic(ctx.handle, int(seed), int(stream_id), int(first),
                                        ctypes.c_void_p(out.data_ptr()), out.numel(), dt, int(mode), float(alpha),
                                        float(beta), float(delta), float(mu), _stream(stream, out)))


def qm_generate_vg(ctx, seed, stream_id, first, out, lam, alpha, beta, mu=0.0, mode=None, stream=None):
    """Variance-gamma samples (lambda in [1, 8]) of a Philox stream through the two-sided exponential base, fused."""
    dt = _dtype_of(out)
    if mode is None:
        mode = QM_PLAIN if dt == QM_F64 else QM_F32_REFINE
    check(load().qm_generate_vg(ctx.handle, int(seed), int(stream_id), int(first), ctypes.c_void_p(out.data_ptr()),
                                out.numel(), dt, int(mode), float(lam), float(alpha), float(beta), float(mu),
                                _stream(stream, out)))


def qm_recycle_student_t(ctx, z, t, nu, mode=None, stream=None):
    """t = F_nu^{-1}(Phi(z)) (FP64 PLAIN or FP32 F32_REFINE)."""
    pi, po, n, dt = _io(z, t)
    if mode is None:
        mode = QM_PLAIN if dt == QM_F64 else QM_F32_REFINE
    check(load().qm_recycle_student_t(ctx.handle, pi, po, n, dt, mode, float(nu), _stream(stream, z)))


def qm_recycle_exp_to_normal(ctx, x, z, mode=None, stream=None):
    """z = sign(x) Phi^{-1}(1 - e^{-|x|}/2) (FP64 PLAIN/PAPER or FP32 F32_REFINE/PLAIN)."""
    pi, po, n, dt = _io(x, z)
    if mode is None:
        mode = QM_PLAIN if dt == QM_F64 else QM_F32_REFINE
    check(load().qm_recycle_exp_to_normal(ctx.handle, pi, po, n, dt, mode, _stream(stream, x)))


def qm_recycle_exp_to_hyperbolic(ctx, v, x, alpha, beta, delta, mu=0.0, mode=None, stream=None):
    """x = mu + F^{-1}(F0(v)), two-sided exponential base -> hyperbolic (FP64 PLAIN or FP32 F32_REFINE)."""
    pi, po, n, dt = _io(v, x)
    if mode is None:
        mode = QM_PLAIN if dt == QM_F64 else QM_F32_REFINE
    check(load().qm_recycle_exp_to_hyperbolic(ctx.handle, pi, po, n, dt, mode, float(alpha), float(beta),
                                              float(delta), float(mu), _stream(stream, v)))


def qm_hyperbolic_masses(ctx, alpha, beta, delta):
    """(log p+, log p-) of the hyperbolic target: the base's masses on each side."""
    lp, lm = ctypes.c_double(), ctypes.c_double()
    check(load().qm_hyperbolic_masses(ctx.handle, float(alpha), float(beta), float(delta), ctypes.byref(lp),
                                      ctypes.byref(lm)))
    return lp.value, lm.value


def qm_recycle_exp_to_vg(ctx, v, x, lam, alpha, beta, mu=0.0, mode=None, stream=None):
    """x = mu + F^{-1}(F0(v)), two-sided exponential base -> variance-gamma, lambda in [1, 8] (Section 8.2)."""
    pi, po, n, dt = _io(v, x)
    if mode is None:
        mode = QM_PLAIN if dt == QM_F64 else QM_F32_REFINE
    check(load().qm_recycle_exp_to_vg(ctx.handle, pi, po, n, dt, mode, float(lam), float(alpha), float(beta),
                                      float(mu), _stream(stream, v)))


def qm_vg_masses(ctx, lam, alpha, beta):
    """(log p+, log p-) of the variance-gamma target."""
    lp, lm = ctypes.c_double(), ctypes.c_double()
    check(load().qm_vg_masses(ctx.handle, float(lam), float(alpha), float(beta), ctypes.byref(lp), ctypes.byref(lm)))
    return lp.value, lm.value


def make_request(kind, inp, out, mode=None, nu=0.0, user_tag=0, hyperbolic=(0.0, 0.0, 0.0), mu=0.0):
    """qm_request for qm_run_batch / qm_submit from a pair of device tensors
    (`hyperbolic` = (alpha, beta, delta) and `mu` for QM_EXP_TO_HYPERBOLIC)."""
    pi, po, n, dt = _io(inp, out)
    if mode is None:
        mode = QM_PLAIN if dt == QM_F64 else QM_F32_REFINE
    a, b, d = (float(x) for x in hyperbolic)
    return qm_request(kind, dt, mode, 0, float(nu), pi.value, po.value, n, user_tag, a, b, d, float(mu))


def qm_run_batch(ctx, reqs, stream=None, device_tensor=None):
    """Run a list of qm_request as one persistent launch."""
    arr = (qm_request * len(reqs))(*reqs)
    s = ctypes.c_void_p(int(stream)) if stream is not None else _stream(None, device_tensor) if device_tensor is not None else ctypes.c_void_p(0)
    check(load().qm_run_batch(ctx.handle, arr, len(reqs), s))


def qm_run_batch_noalloc(ctx, reqs, stream=None, device_tensor=None):
    """qm_run_batch through the allocation-free entry point (tables must
    already be in the context)."""
    arr = (qm_request * len(reqs))(*reqs)
    s = ctypes.c_void_p(int(stream)) if stream is not None else _stream(None, device_tensor) if device_tensor is not None else ctypes.c_void_p(0)
    check(load().qm_run_batch_noalloc(ctx.handle, arr, len(reqs), s))


def qm_submit(ctx, req):
    """Enqueue one request in the serving loop; returns its ticket."""
    ticket = ctypes.c_uint64()
    check(load().qm_submit(ctx.handle, ctypes.byref(req), ctypes.byref(ticket)))
    return ticket.value


def qm_poll(ctx, ticket):
    """QM_OK when complete, QM_PENDING before; raises on errors."""
    return check(load().qm_poll(ctx.handle, int(ticket)))


def qm_poll_times(ctx, ticket):
    """(status, submit_ns, done_ns) of a ticket; times on the monotonic
    clock (time.monotonic_ns), done_ns only with QM_OK; raises on errors."""
    a, b = ctypes.c_uint64(), ctypes.c_uint64()
    st = check(load().qm_poll_times(ctx.handle, int(ticket), ctypes.byref(a), ctypes.byref(b)))
    return st, a.value, (b.value if st == QM_OK else None)


def qm_serving_latencies(ctx, cap=1 << 20):
    """Submit -> completion latencies (ns) of the most recent completed
    requests, oldest first."""
    buf = (ctypes.c_uint64 * cap)()
    n = load().qm_serving_latencies(ctx.handle, buf, cap)
    return [buf[i] for i in range(min(n, cap))]


def qm_serving_stats_of(ctx):
    """The serving loop's counters as a dict (qm_serving_stats)."""
    st = qm_serving_counters()
    check(load().qm_serving_stats(ctx.handle, ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in qm_serving_counters._fields_}


class TCells(ctypes.Structure):
    """Layout of qm::TCells (csrc/qm_table.h): one cell approximation of R(y) = t/z."""
    _fields_ = [("h", ctypes.c_double), ("inv_h", ctypes.c_double), ("y_max", ctypes.c_double),
                ("y_lds", ctypes.c_double), ("centre_offset", ctypes.c_double), ("max_rel_err", ctypes.c_double),
                ("ncell", ctypes.c_int32), ("nlds", ctypes.c_int32), ("degree", ctypes.c_int32),
                ("stride", ctypes.c_int32), ("coef_offset", ctypes.c_uint64)]


class TTableHeader(ctypes.Structure):
    """Layout of qm::TTableHeader (csrc/qm_table.h)."""
    _fields_ = [("nu", ctypes.c_double), ("log_K", ctypes.c_double), ("tail_a", ctypes.c_double * 4),
                ("identity", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("f64", TCells), ("f32", TCells)]


def debug_student_dense(nu, z):
    """Host-side dense RODE solution Q(z) used to build the t tables (qm_debug.h)."""
    import numpy as np
    z = np.ascontiguousarray(z, dtype=np.float64)
    q = np.empty_like(z)
    dp = ctypes.POINTER(ctypes.c_double)
    r = load().qm_debug_student_dense(float(nu), z.ctypes.data_as(dp), q.ctypes.data_as(dp), z.size)
    if r != 0:
        raise ValueError("dense solution unavailable for nu=%r" % nu)
    return q


def debug_student_table(nu, which="f64"):
    """(header, cells, coefficients[ncell, stride]) of the host-built table;
    `which` selects the cell approximation for FP64 ("f64") or FP32 ("f32")
    outputs."""
    import numpy as np
    h = TTableHeader()
    lib = load()
    dp = ctypes.POINTER(ctypes.c_double)
    n = lib.qm_debug_student_table(float(nu), ctypes.byref(h), None, 0)
    if n < 0:
        raise ValueError("table build failed for nu=%r" % nu)
    c = getattr(h, which)
    block = np.empty(max(n, 0), np.float64)
    if n > 0:
        lib.qm_debug_student_table(float(nu), None, block.ctypes.data_as(dp), n)
    coef = block[c.coef_offset:c.coef_offset + c.ncell * c.stride].reshape(c.ncell, c.stride)
    return h, c, coef


class HypSide(ctypes.Structure):
    """Layout of qm::HypSide (csrc/qm_hyp_table.h): the cells of one side of the hyperbolic map."""
    _fields_ = [("v0", ctypes.c_double), ("inv_v0", ctypes.c_double), ("v_top", ctypes.c_double),
                ("far_c0", ctypes.c_double), ("far_c1", ctypes.c_double), ("far_c2", ctypes.c_double),
                ("far_clog", ctypes.c_double),
                ("max_rel_err", ctypes.c_double), ("noct", ctypes.c_int32), ("ncell", ctypes.c_int32),
                ("degree", ctypes.c_int32), ("origin", ctypes.c_int32), ("coef_offset", ctypes.c_uint64)]


class HypTableHeader(ctypes.Structure):
    """Layout of qm::HypTableHeader (csrc/qm_hyp_table.h)."""
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("delta", ctypes.c_double),
                ("log_p_plus", ctypes.c_double), ("log_p_minus", ctypes.c_double),
                ("right", HypSide), ("left", HypSide), ("right32", HypSide), ("left32", HypSide)]


HYP_DEGREE = 11       # FP64-output cells
HYP_DEGREE_F32 = 7    # FP32-output cells
HYP_SUB = 8


def debug_hyperbolic_dense(alpha, beta, delta, v):
    """Host-side solution Q(v) that the hyperbolic tables are fitted to (qm_debug.h)."""
    import numpy as np
    v = np.ascontiguousarray(v, dtype=np.float64)
    q = np.empty_like(v)
    dp = ctypes.POINTER(ctypes.c_double)
    r = load().qm_debug_hyperbolic_dense(float(alpha), float(beta), float(delta), v.ctypes.data_as(dp),
                                         q.ctypes.data_as(dp), v.size)
    if r != 0:
        raise ValueError("dense solution unavailable for %r" % ((alpha, beta, delta),))
    return q


def _debug_base_table(fn, args, which):
    import numpy as np
    h = HypTableHeader()
    dp = ctypes.POINTER(ctypes.c_double)
    n = fn(*[float(a) for a in args], ctypes.byref(h), None, 0)
    if n < 0:
        raise ValueError("table build failed for %r" % (args,))
    block = np.empty(n, np.float64)
    fn(*[float(a) for a in args], None, block.ctypes.data_as(dp), n)
    sides = (h.right, h.left) if which == "f64" else (h.right32, h.left32)
    rows = [block[s.coef_offset:s.coef_offset + s.ncell * (s.degree + 1)].reshape(s.ncell, s.degree + 1)
            for s in sides]
    return h, rows[0], rows[1]


def debug_vg_table(lam, alpha, beta, which="f64"):
    """(header, right rows, left rows) of the host-built variance-gamma table (lambda in [1, 8])."""
    return _debug_base_table(load().qm_debug_vg_table, (lam, alpha, beta), which)


def debug_hyperbolic_table(alpha, beta, delta, which="f64"):
    """(header, right rows[ncell, degree+1], left rows) of the host-built table;
    `which` selects the cells for FP64 ("f64") or FP32 ("f32") outputs.  The
    header's `right`/`left` fields describe the FP64 cells, `right32`/`left32`
    the FP32 ones."""
    import numpy as np
    h = HypTableHeader()
    lib = load()
    dp = ctypes.POINTER(ctypes.c_double)
    n = lib.qm_debug_hyperbolic_table(float(alpha), float(beta), float(delta), ctypes.byref(h), None, 0)
    if n < 0:
        raise ValueError("table build failed for %r" % ((alpha, beta, delta),))
    block = np.empty(n, np.float64)
    lib.qm_debug_hyperbolic_table(float(alpha), float(beta), float(delta), None, block.ctypes.data_as(dp), n)
    sides = (h.right, h.left) if which == "f64" else (h.right32, h.left32)
    rows = [block[s.coef_offset:s.coef_offset + s.ncell * (s.degree + 1)].reshape(s.ncell, s.degree + 1)
            for s in sides]
    return h, rows[0], rows[1]
