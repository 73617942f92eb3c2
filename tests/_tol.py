"""Tolerance rule for comparing a GPU result with the oracle (FP64 reference).

Pass iff |got - ref| <= rtol * max(|ref|, 1e-3): relative error away from
zero, absolute error rtol * 1e-3 near it.  Equal infinities pass, NaN
matches NaN, and +0 equals -0.  rtol is 2e-15 for FP64 outputs and 2e-7 for
FP32 outputs.
"""
import numpy as np

RTOL_F64 = 2e-15
RTOL_F32 = 2e-7
ABS_FLOOR = 1e-3


def compare(got, ref, rtol):
    """Returns (ok_mask, report dict)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    both_nan = np.isnan(got) & np.isnan(ref)
    same_inf = np.isinf(ref) & (got == ref)
    finite = np.isfinite(ref) & np.isfinite(got)
    err = np.zeros_like(ref)
    err[finite] = np.abs(got[finite] - ref[finite])
    scale = np.maximum(np.abs(ref), ABS_FLOOR)
    ok = both_nan | same_inf | (finite & (err <= rtol * scale))
    big = finite & (np.abs(ref) >= ABS_FLOOR)
    small = finite & (np.abs(ref) < ABS_FLOOR)
    rep = {
        "n": int(ref.size),
        "fails": int((~ok).sum()),
        "max_rel": float(np.max(err[big] / np.abs(ref[big]))) if big.any() else 0.0,
        "max_abs_small": float(np.max(err[small])) if small.any() else 0.0,
        "specials": int((~np.isfinite(ref)).sum()),
    }
    if rep["fails"]:
        i = int(np.flatnonzero(~ok)[0])
        rep["first_fail"] = (i, float(got[i]), float(ref[i]))
    return ok, rep


def assert_close(got, ref, rtol, what=""):
    ok, rep = compare(got, ref, rtol)
    assert rep["fails"] == 0, "%s: %r" % (what, rep)
    return rep


def as_f32_output(ref):
    """An FP64 reference for FP32 outputs: a magnitude that rounds beyond
    FLT_MAX is +-inf in FP32, as the output itself must then be."""
    r = np.asarray(ref, dtype=np.float64)
    with np.errstate(over="ignore"):
        r32 = r.astype(np.float32)
    return np.where(np.isinf(r32) & np.isfinite(r), r32.astype(np.float64), r)
