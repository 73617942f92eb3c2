"""Slow CPU reference ("the oracle") for the quantile-mechanics hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  The product library never imports,
links or runs it, and it shares no code with the product; both sides only
share the seeded input generator in ``qm_inputs``.

Functions (all FP64 results, plain definitions solved in x87 extended
precision, see oracle.c):

  norm_quantile(u)        w(u) = Phi^{-1}(u)                  (Section 1, eq. 1)
  exp_to_normal(x)        sign(x) Phi^{-1}(1 - e^{-|x|}/2)     (Section 6)
  student_t_map(z, nu)    F_nu^{-1}(Phi(z))                    (Sections 1, 3.1)
  betainc(a, b, x)        regularized incomplete beta I_x(a,b) (used by the t map)
  hyperbolic_map(v, alpha, beta, delta)
                          F^{-1}(F0(v)), two-sided exponential base -> hyperbolic
                          target (Section 8.1; hyperbolic.c)
  hyperbolic_masses(...)  (log p+, log p-, log C) of the hyperbolic target
  hyperbolic_log_tail(x, ...)  log(1 - F(x)) for x >= 0, log F(x) for x < 0
  vg_map(v, lam, alpha, beta)  F^{-1}(F0(v)), the same base -> variance-gamma
                          target with integer lambda (Section 8.2; vg.c)
  vg_masses(...), vg_log_tail(x, ...)  as for the hyperbolic target
  vgr_map(v, lam, alpha, beta)  the same map for real lambda >= 1, by the
                          Bessel-integral form of the masses (vg_real.c)
  vgr_masses(...), vgr_log_tail(x, ...), vgr_central_mass(x, ...)
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, f) for f in ("oracle.c", "hyperbolic.c", "vg.c", "vg_real.c")]
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=True):
    """Compile liboracle.so with gcc (no fast-math: the oracle needs IEEE semantics)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    cmd = ["gcc", "-O2", "-Wall", "-shared", "-fPIC", "-o", _LIB + ".tmp"] + _SRC + ["-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    dp = ctypes.POINTER(ctypes.c_double)
    for name in ("oracle_norm_quantile", "oracle_exp_to_normal"):
        f = getattr(lib, name)
        f.argtypes = [dp, dp, ctypes.c_size_t, ctypes.c_int]
        f.restype = ctypes.c_int
    lib.oracle_student_t_map.argtypes = [dp, dp, ctypes.c_size_t, ctypes.c_double, ctypes.c_int]
    lib.oracle_student_t_map.restype = ctypes.c_int
    lib.oracle_betainc.argtypes = [ctypes.c_double] * 3
    lib.oracle_betainc.restype = ctypes.c_double
    for name in ("oracle_norm_quantile1", "oracle_exp_to_normal1"):
        f = getattr(lib, name)
        f.argtypes = [ctypes.c_double]
        f.restype = ctypes.c_double
    lib.oracle_student_t_map1.argtypes = [ctypes.c_double, ctypes.c_double]
    lib.oracle_student_t_map1.restype = ctypes.c_double
    d = ctypes.c_double
    lib.oracle_hyperbolic_map.argtypes = [dp, dp, ctypes.c_size_t, d, d, d, ctypes.c_int]
    lib.oracle_hyperbolic_map.restype = ctypes.c_int
    lib.oracle_hyperbolic_masses.argtypes = [d, d, d, dp, dp, dp]
    lib.oracle_hyperbolic_masses.restype = ctypes.c_int
    lib.oracle_hyperbolic_log_tail.argtypes = [d, d, d, d]
    lib.oracle_hyperbolic_log_tail.restype = d
    lib.oracle_vg_map.argtypes = [dp, dp, ctypes.c_size_t, d, d, d, ctypes.c_int]
    lib.oracle_vg_map.restype = ctypes.c_int
    lib.oracle_vg_masses.argtypes = [d, d, d, dp, dp]
    lib.oracle_vg_masses.restype = ctypes.c_int
    lib.oracle_vg_log_tail.argtypes = [d, d, d, d]
    lib.oracle_vg_log_tail.restype = d
    lib.oracle_vgr_map.argtypes = [dp, dp, ctypes.c_size_t, d, d, d, ctypes.c_int]
    lib.oracle_vgr_map.restype = ctypes.c_int
    lib.oracle_vgr_masses.argtypes = [d, d, d, dp, dp]
    lib.oracle_vgr_masses.restype = ctypes.c_int
    for name in ("oracle_vgr_log_tail", "oracle_vgr_central_mass"):
        f = getattr(lib, name)
        f.argtypes = [d, d, d, d]
        f.restype = d
    for name in ("oracle_vgr_log_upper_gamma", "oracle_vgr_log_lower_gamma"):
        f = getattr(lib, name)
        f.argtypes = [d, d]
        f.restype = d
    _lib = lib
    return lib


def _as_f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def norm_quantile(u, threads=0):
    """Phi^{-1}(u) element-wise (FP64 in/out).  threads<=0: all cores."""
    u = _as_f64(u)
    out = np.empty_like(u)
    _load().oracle_norm_quantile(_ptr(u), _ptr(out), u.size, threads)
    return out


def exp_to_normal(x, threads=0):
    """sign(x) Phi^{-1}(1 - exp(-|x|)/2) element-wise."""
    x = _as_f64(x)
    out = np.empty_like(x)
    _load().oracle_exp_to_normal(_ptr(x), _ptr(out), x.size, threads)
    return out


def student_t_map(z, nu, threads=0):
    """F_nu^{-1}(Phi(z)) element-wise for real nu > 0 (nu = inf: identity)."""
    z = _as_f64(z)
    out = np.empty_like(z)
    _load().oracle_student_t_map(_ptr(z), _ptr(out), z.size, float(nu), threads)
    return out


def betainc(a, b, x):
    """Regularized incomplete beta I_x(a, b) (scalar)."""
    return _load().oracle_betainc(float(a), float(b), float(x))


def threads_used(threads=0):
    """Number of threads the array drivers use for a given request."""
    return threads if threads > 0 else (os.cpu_count() or 1)


def hyperbolic_map(v, alpha, beta, delta, threads=0):
    """x = F^{-1}(F0(v)): two-sided exponential base -> hyperbolic target (Section 8.1)."""
    v = _as_f64(v)
    out = np.empty_like(v)
    _load().oracle_hyperbolic_map(_ptr(v), _ptr(out), v.size, float(alpha), float(beta), float(delta),
                                  threads_used(threads))
    return out


def hyperbolic_masses(alpha, beta, delta):
    """(log p+, log p-, log C) of the hyperbolic density with these parameters."""
    a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    if _load().oracle_hyperbolic_masses(float(alpha), float(beta), float(delta), ctypes.byref(a), ctypes.byref(b),
                                        ctypes.byref(c)) != 0:
        raise ValueError("invalid hyperbolic parameters")
    return a.value, b.value, c.value


def hyperbolic_log_tail(x, alpha, beta, delta):
    """log(1 - F(x)) for x >= 0, log F(x) for x < 0."""
    return _load().oracle_hyperbolic_log_tail(float(x), float(alpha), float(beta), float(delta))


def vg_map(v, lam, alpha, beta, threads=0):
    """x = F^{-1}(F0(v)): two-sided exponential base -> variance-gamma target, integer lambda (Section 8.2)."""
    v = _as_f64(v)
    out = np.empty_like(v)
    _load().oracle_vg_map(_ptr(v), _ptr(out), v.size, float(lam), float(alpha), float(beta), threads_used(threads))
    return out


def vg_masses(lam, alpha, beta):
    """(log p+, log p-) of the variance-gamma density with these parameters."""
    a, b = ctypes.c_double(), ctypes.c_double()
    if _load().oracle_vg_masses(float(lam), float(alpha), float(beta), ctypes.byref(a), ctypes.byref(b)) != 0:
        raise ValueError("invalid variance-gamma parameters")
    return a.value, b.value


def vg_log_tail(x, lam, alpha, beta):
    """log(1 - F(x)) for x >= 0, log F(x) for x < 0."""
    return _load().oracle_vg_log_tail(float(x), float(lam), float(alpha), float(beta))


def vgr_map(v, lam, alpha, beta, threads=0):
    """x = F^{-1}(F0(v)): two-sided exponential base -> variance-gamma target, real lambda >= 1 (Section 8.2)."""
    v = _as_f64(v)
    out = np.empty_like(v)
    _load().oracle_vgr_map(_ptr(v), _ptr(out), v.size, float(lam), float(alpha), float(beta), threads_used(threads))
    return out


def vgr_masses(lam, alpha, beta):
    """(log p+, log p-) of the variance-gamma density, real lambda (Bessel-integral form)."""
    a, b = ctypes.c_double(), ctypes.c_double()
    if _load().oracle_vgr_masses(float(lam), float(alpha), float(beta), ctypes.byref(a), ctypes.byref(b)) != 0:
        raise ValueError("invalid variance-gamma parameters")
    return a.value, b.value


def vgr_log_tail(x, lam, alpha, beta):
    """log(1 - F(x)) for x >= 0, log F(x) for x < 0, real lambda."""
    return _load().oracle_vgr_log_tail(float(x), float(lam), float(alpha), float(beta))


def vgr_central_mass(x, lam, alpha, beta):
    """int_0^|x| f on the side of x, real lambda."""
    return _load().oracle_vgr_central_mass(float(x), float(lam), float(alpha), float(beta))


def vgr_log_upper_gamma(a, y):
    return _load().oracle_vgr_log_upper_gamma(float(a), float(y))


def vgr_log_lower_gamma(a, y):
    return _load().oracle_vgr_log_lower_gamma(float(a), float(y))
