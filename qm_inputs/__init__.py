"""Seeded synthetic inputs shared by the tests, the oracle checks and the benchmark.

Holds none of the quantile method's arithmetic: only a counter-based
generator (Philox4x32-10, SC'11) and the transforms that define the workload
arrays.  Each element depends only on (seed, stream, index), so the oracle can
regenerate any sampled element without the full array.

Workloads (sizes and seeds as used by the tests and the benchmark):

  uniform53      u = (k + 1/2) 2^-53, k the top 53 bits of a Philox word pair
                 (rounded to nearest: a tie to even for k >= 2^52, and 1.0
                 for k = 2^53 - 1)
  uniform23      u = (k + 1/2) 2^-23 in FP32, k the top 23 bits of a word
                 (exact, 0 < u < 1)
  mixture        90% open uniform, 10% tail t log-uniform in [lo, 1e-2],
                 mirrored to 1 - t with probability 1/2
  normals        Box-Muller pairs from two open uniforms
  exponentials   -log(u) of an open uniform
  two_sided_exponentials
                 log(u/p-)/rate_minus for u < p-, else
                 -log((1-u)/(1-p-))/rate_plus: the two-sided exponential
                 with mass p- below 0, drawn from one open uniform u
                 (1 - u is exact for u = (k + 1/2) 2^-53)
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qm_inputs.c")
_LIB = os.path.join(_HERE, "libqm_inputs.so")
_lib = None


def build(force=True):
    if not force and os.path.exists(_LIB):
        return _LIB
    cmd = ["gcc", "-O2", "-Wall", "-shared", "-fPIC", "-o", _LIB + ".tmp", _SRC, "-lm", "-lpthread"]
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
    u64, sz, ci, cd = ctypes.c_uint64, ctypes.c_size_t, ctypes.c_int, ctypes.c_double
    vp = ctypes.c_void_p
    lib.qmi_philox4x32_10.argtypes = [vp, vp, vp]
    lib.qmi_philox4x32_10.restype = None
    for name in ("qmi_uniform53", "qmi_uniform23", "qmi_normals", "qmi_exponentials"):
        f = getattr(lib, name)
        f.argtypes = [u64, u64, vp, sz, ci]
        f.restype = ci
    for name in ("qmi_u53_of_bits", "qmi_u23_of_words"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, sz]
        f.restype = None
    for name in ("qmi_mixture_f64", "qmi_mixture_f32"):
        f = getattr(lib, name)
        f.argtypes = [u64, u64, cd, cd, vp, sz, ci]
        f.restype = ci
    _lib = lib
    return lib


def philox4x32_10(counter, key):
    """One Philox4x32-10 block: counter (4 x u32), key (2 x u32) -> 4 x u32."""
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    _load().qmi_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def u53_of_bits(bits):
    """The FP64 open-uniform formula (k + 1/2) 2^-53 of the top 53 bits k of
    each 64-bit value."""
    b = np.ascontiguousarray(bits, dtype=np.uint64)
    out = np.empty(b.size, np.float64)
    _load().qmi_u53_of_bits(b.ctypes.data, out.ctypes.data, b.size)
    return out


def u23_of_words(words):
    """The FP32 open-uniform formula (k + 1/2) 2^-23 of the top 23 bits k of
    each 32-bit word."""
    w = np.ascontiguousarray(words, dtype=np.uint32)
    out = np.empty(w.size, np.float32)
    _load().qmi_u23_of_words(w.ctypes.data, out.ctypes.data, w.size)
    return out


def uniform53(seed, stream, n, threads=0, out=None):
    out = np.empty(n, np.float64) if out is None else out
    _load().qmi_uniform53(seed, stream, out.ctypes.data, n, threads)
    return out


def uniform23(seed, stream, n, threads=0, out=None):
    out = np.empty(n, np.float32) if out is None else out
    _load().qmi_uniform23(seed, stream, out.ctypes.data, n, threads)
    return out


def mixture(seed, stream, n, dtype=np.float64, p_tail=0.1, tail_lo=None, threads=0, out=None):
    """Bulk/tail mixture; tail_lo defaults to 1e-300 (f64) or 1e-37 (f32)."""
    dtype = np.dtype(dtype)
    if tail_lo is None:
        tail_lo = 1e-300 if dtype == np.float64 else 1e-37
    out = np.empty(n, dtype) if out is None else out
    f = _load().qmi_mixture_f64 if dtype == np.float64 else _load().qmi_mixture_f32
    f(seed, stream, p_tail, tail_lo, out.ctypes.data, n, threads)
    return out


def normals(seed, stream, n, threads=0, out=None):
    out = np.empty(n, np.float64) if out is None else out
    _load().qmi_normals(seed, stream, out.ctypes.data, n, threads)
    return out


def exponentials(seed, stream, n, threads=0, out=None):
    out = np.empty(n, np.float64) if out is None else out
    _load().qmi_exponentials(seed, stream, out.ctypes.data, n, threads)
    return out


def two_sided_exponentials(seed, stream, n, rate_plus, rate_minus, p_minus, threads=0):
    """Two-sided exponential samples (mass p_minus below 0), one uniform each."""
    u = uniform53(seed, stream, n, threads)
    neg = u < p_minus
    v = np.empty(n, np.float64)
    v[neg] = np.log(u[neg] / p_minus) / rate_minus
    v[~neg] = -np.log((1.0 - u[~neg]) / (1.0 - p_minus)) / rate_plus
    return v


# Workload definitions (seeds and streams fixed here so every user agrees).
def uniforms_2e20():
    """Plain FP64 quantile workload: 2^20 open uniforms, seed 0."""
    return uniform53(0, 0, 1 << 20)


def mixture_f64(n=1 << 28, threads=0):
    """FP64 mixture workload: 10% tail log-uniform in [1e-300, 1e-2], seed 1."""
    return mixture(1, 0, n, np.float64, 0.1, 1e-300, threads)


def mixture_f32(n=1 << 28, threads=0):
    """FP32 mixture workload: 10% tail log-uniform in [1e-37, 1e-2], seed 1."""
    return mixture(1, 0, n, np.float32, 0.1, 1e-37, threads)


def recycle_normals(n=1 << 26, threads=0):
    """Box-Muller normals for the Student t map, seed 2 stream 0."""
    return normals(2, 0, n, threads)


def recycle_exponentials(n=1 << 26, threads=0):
    """Exp(1) samples for the exponential -> normal map, seed 2 stream 1."""
    return exponentials(2, 1, n, threads)


HYPERBOLIC_PARAMS = (1.0, 0.0, 1.0)   # (alpha, beta, delta) of the Section 8.1 illustration


def recycle_two_sided(n, alpha, beta, p_minus, threads=0):
    """Base samples for the exponential -> hyperbolic map: rates alpha -+ beta,
    mass p_minus below 0, seed 2 stream 2."""
    return two_sided_exponentials(2, 2, n, alpha - beta, alpha + beta, p_minus, threads)


# Batched / serving request mix: per request r, three parameter uniforms from
# streams 100-102 of the seed; inputs of request r from stream 1000 + r.
MIX = (("nq_f32_refine", 0.4), ("nq_f64", 0.2), ("student_f64", 0.3), ("exp_f64", 0.1))


def request_mix(seed, count, log2_lo, log2_hi):
    """List of dicts {kind, n, nu, stream} for a heterogeneous batch:
    sizes log-uniform in [2^log2_lo, 2^log2_hi], kinds 40% quantile
    FP32+refine, 20% quantile FP64, 30% Student t FP64 with nu uniform-integer
    in [1, 50], 10% exponential -> normal FP64."""
    us = uniform53(seed, 100, count)
    uk = uniform53(seed, 101, count)
    un = uniform53(seed, 102, count)
    out = []
    for r in range(count):
        n = int(2.0 ** (log2_lo + (log2_hi - log2_lo) * us[r]))
        acc, kind = 0.0, MIX[-1][0]
        for name, p in MIX:
            acc += p
            if uk[r] < acc:
                kind = name
                break
        out.append({"kind": kind, "n": n, "nu": float(1 + int(50 * un[r])), "stream": 1000 + r})
    return out


def request_input(seed, req):
    """The input array of one request of request_mix."""
    k, n, s = req["kind"], req["n"], req["stream"]
    if k == "nq_f32_refine":
        return uniform23(seed, s, n)
    if k == "nq_f64":
        return uniform53(seed, s, n)
    if k == "student_f64":
        return normals(seed, s, n)
    return exponentials(seed, s, n)
