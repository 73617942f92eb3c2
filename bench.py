#!/usr/bin/env python3
"""Benchmark of the quantile-mechanics hot path on one MI355X.

Default workload (one "step"): the Gaussian quantile on 2^28 samples, once in
FP64 (plain, 2e-15) and once in FP32 + FP64 refine (2e-7): u is 90% open
uniform, 10% tail stratum log-uniform in [1e-300, 1e-2] (FP64) or
[1e-37, 1e-2] (FP32), mirrored to 1-u with probability 1/2, seed 1.  Inputs
are resident in HBM before the timed region.  value = samples of both passes
/ wall time of the timed steps.  The JSON line also carries, outside the
timed region, the normal -> Student t map (2^26 normals, nu in
{1,2,3,4,5,10,30}) and exponential -> normal (2^26) rates, the roofline of
the dominant kernel (FP64 quantile: 16 algorithmic bytes per sample, timed
per launch with HIP events on its stream) and the CPU oracle on a bounded
sample.

    --workload batch   4096 mixed requests (sizes log-uniform 2^10..2^22,
                       40% quantile FP32+refine, 20% quantile FP64, 30%
                       Student t nu in 1..50, 10% exp -> normal), seed 3:
                       one persistent launch vs one launch per request.
    --workload serve   Poisson arrivals at swept rates, sizes 2^12..2^24,
                       same mix, HBM budget 64 GB: p50/p99 latency and
                       Gsamples/s, vs the same trace as sequential launches.
"""
import argparse
import json
import math
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gsamples/s Φ^{-1} & t-recycle (FP64 vs FP32+refine) at stated max err; p50/p99"
HBM_PEAK_GBS = 8000.0
T_NUS = (1, 2, 3, 4, 5, 10, 30)


QUANTILE_SOURCES = ("qm_kernels.hip", "qm_hybrid.hpp", "qm_device.hpp", "qm_coeffs.h", "qm_paper_coeffs.h")
HYPERBOLIC_SOURCES = ("qm_hyp.hip", "qm_hyp_device.hpp", "qm_hyp_table.h", "qm_device.hpp")


def kernel_source_hash(files=QUANTILE_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_0901_0638_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_figure(profile, key, files=QUANTILE_SOURCES):
    """A figure ("<key>: <number>") from a committed rocprofv3 summary under
    profiles/, or None if the kernel sources changed since it was taken (the
    summary records their hash) or the figure is absent."""
    import re
    path = os.path.join(ROOT, "profiles", profile)
    try:
        text = open(path).read()
    except OSError:
        return None
    m = re.search(r"Kernel source hash: `([0-9a-f]+)`", text)
    t = re.search(r"^%s: ([0-9.]+)" % re.escape(key), text, flags=re.M)
    if not m or not t or m.group(1) != kernel_source_hash(files):
        return None
    v = float(t.group(1))
    return int(v) if v == int(v) else v


def counted_traffic(profile="quantile_mixture_2e28_hbm_counters.md", kernel="k_hybrid<double>",
                    files=QUANTILE_SOURCES):
    """HBM bytes per launch of a kernel from its committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary, or None if the kernel sources changed
    since those counters were taken."""
    v = profile_figure(profile, "traffic_bytes_per_launch %s" % kernel, files)
    return None if v is None else int(v)


def profiler_avg_ms(profile, kernel, files=QUANTILE_SOURCES):
    """The profiler's average duration of a kernel (ms) from a committed
    kernel-trace summary, or None if the sources changed since."""
    us = profile_figure(profile, "profiler_avg_us %s" % kernel, files)
    return None if us is None else round(us / 1e3, 4)


# VALU issue peak of MI355X: 256 CUs x 4 SIMDs, one wave64 instruction per
# SIMD every 4 cycles (16 lanes per cycle; FP64 FMA is full rate), 2.4 GHz
VALU_PEAK_WAVE_INSTS_S = 256 * 4 * 2.4e9 / 4


def valu_fraction(profile, kernel, avg_ms, files=QUANTILE_SOURCES):
    """Wave-level VALU instructions per launch (SQ_INSTS_VALU, committed
    counters) over the launch's measured duration, as a fraction of the
    issue peak; None without current counters."""
    insts = profile_figure(profile, "valu_insts_per_launch %s" % kernel, files)
    if insts is None or not avg_ms:
        return None
    return {"insts_per_launch": int(insts), "frac": round(insts / (avg_ms * 1e-3) / VALU_PEAK_WAVE_INSTS_S, 4),
            "peak_wave_insts_per_s": VALU_PEAK_WAVE_INSTS_S}


def error_report(got, ref, rtol):
    """Measured error of outputs against oracle values (FP64): the largest
    relative error where |ref| >= 1e-3, the largest absolute error below,
    and the count outside the tolerance rtol * max(|ref|, 1e-3) (equal
    infinities and NaN = NaN pass)."""
    import numpy as np
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    fin = np.isfinite(ref) & np.isfinite(got)
    err = np.abs(np.where(fin, got, 0.0) - np.where(fin, ref, 0.0))
    big = fin & (np.abs(ref) >= 1e-3)
    small = fin & (np.abs(ref) < 1e-3)
    special_ok = (~np.isfinite(ref)) & ((got == ref) | (np.isnan(got) & np.isnan(ref)))
    ok = special_ok | (fin & (err <= rtol * np.maximum(np.abs(ref), 1e-3)))
    return {"checked": int(ref.size),
            "max_rel_err": float(np.max(err[big] / np.abs(ref[big]))) if big.any() else 0.0,
            "max_abs_err_near_0": float(np.max(err[small])) if small.any() else 0.0,
            "specials_matched": int(special_ok.sum()), "outside_tolerance": int((~ok).sum()), "tolerance": rtol}


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(math.ceil(p / 100.0 * len(xs))) - 1))
    return xs[k]


def timed_launches(torch, stream, fn, reps, scrub=None):
    """Per-launch durations (ms) with HIP events on the launch stream, after
    one untimed call (the first launch of a kernel also loads its code).
    scrub, if given, runs untimed on the same stream before every timed
    launch (a copy larger than the 256 MB last-level cache, so that no
    launch finds the previous one's data there)."""
    fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        if scrub is not None:
            scrub()
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


# ---------------------------------------------------------------------------
def per_launch(torch, stream, fns, reps):
    """Per-launch durations (ms) of several calls interleaved as in a step,
    reps rounds, HIP events on the launch stream around each call."""
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in fns]
          for _ in range(reps)]
    torch.cuda.synchronize()
    for row in ev:
        for (a, b), fn in zip(row, fns):
            a.record(stream)
            fn()
            b.record(stream)
    torch.cuda.synchronize()
    return [[row[j][0].elapsed_time(row[j][1]) for row in ev] for j in range(len(fns))]


def sample_indices(n, u=None, seed=7):
    """A stratified sample of output indices for the accuracy check: 2^18
    random ones, the last 300, and (given the inputs) every outer element
    |u - 1/2| > 0.45 among the first 2^22."""
    import numpy as np
    rng = np.random.default_rng(seed)
    parts = [rng.integers(0, n, 1 << 18), np.arange(max(0, n - 300), n)]
    if u is not None:
        head = np.asarray(u[: 1 << 22], dtype=np.float64)
        parts.append(np.flatnonzero(np.abs(head - 0.5) > 0.45))
    return np.unique(np.concatenate(parts))


def gather(torch, t, idx):
    return t[torch.from_numpy(idx).to(t.device)].cpu().numpy()


def run_quantile(args, torch, qm, qi):
    n = args.n
    t0 = time.time()
    h64 = qi.mixture_f64(n)
    h32 = qi.mixture_f32(n)
    u64 = torch.from_numpy(h64).cuda()
    u32 = torch.from_numpy(h32).cuda()
    w64 = torch.empty_like(u64)
    w32 = torch.empty_like(u32)
    torch.cuda.synchronize()
    print("inputs ready in %.1f s" % (time.time() - t0), file=sys.stderr, flush=True)

    ctx = qm.Context(0)
    stream = torch.cuda.current_stream()
    f64 = lambda: qm.qm_normal_quantile(ctx, u64, w64, qm.QM_PLAIN)          # noqa: E731
    f32 = lambda: qm.qm_normal_quantile(ctx, u32, w32, qm.QM_F32_REFINE)     # noqa: E731

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        f64()
        if ev is not None:
            ev[1].record(stream)
        f32()
        if ev is not None:
            ev[2].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.copy_calibration:
        # a plain copy of known size: 2^28 doubles read + written (4 GiB)
        w64.copy_(u64)
        torch.cuda.synchronize()

    events = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        step(events[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    print("timed %d steps in %.3f s" % (args.steps, wall), file=sys.stderr, flush=True)

    d64 = [e[0].elapsed_time(e[1]) for e in events]  # ms
    d32 = [e[1].elapsed_time(e[2]) for e in events]
    avg64 = sum(d64) / len(d64)
    avg32 = sum(d32) / len(d32)
    print("per-step ms FP64: %s" % " ".join("%.3f" % d for d in d64), file=sys.stderr)
    print("per-step ms FP32: %s" % " ".join("%.3f" % d for d in d32), file=sys.stderr, flush=True)
    # latency percentiles over more launches than the timed steps, outside
    # the timed region (same interleaving)
    p64, p32 = per_launch(torch, stream, [f64, f32], args.pct_reps) if args.pct_reps > 0 else (d64, d32)
    bytes64 = 16.0 * n
    achieved = bytes64 / (avg64 * 1e-3) / 1e9
    prof_stats = "quantile_mixture_2e28_kernel_stats.md"
    prof_counters = "quantile_mixture_2e28_hbm_counters.md"
    full = n == (1 << 28)
    result = {
        "metric": METRIC,
        "value": round(2.0 * n * args.steps / wall / 1e9, 3),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "gaussian-quantile 2^28 mixture (90% uniform, 10% log-uniform tail to 1e-300 "
                               "FP64 / 1e-37 FP32, mirrored p=1/2), seed 1; FP64 plain + FP32+FP64-refine",
                   "n_per_pass": n, "passes_per_step": 2},
        "fp64": {"gsamples_s": round(n / (avg64 * 1e-3) / 1e9, 2), "avg_ms": round(avg64, 4),
                 "p50_ms": percentile(p64, 50), "p99_ms": percentile(p64, 99), "percentile_launches": len(p64),
                 "tolerance": 2e-15},
        "fp32_refine": {"gsamples_s": round(n / (avg32 * 1e-3) / 1e9, 2), "avg_ms": round(avg32, 4),
                        "p50_ms": percentile(p32, 50), "p99_ms": percentile(p32, 99),
                        "percentile_launches": len(p32), "gbs": round(8.0 * n / (avg32 * 1e-3) / 1e9, 1),
                        "tolerance": 2e-7},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": counted_traffic(prof_counters) if full else None,
                     "kernel": "qm::k_hybrid<double, 4, qm::HybridNQ64> (FP64 quantile: central piece, "
                               "outer elements gathered per wave)",
                     "algorithmic_bytes_per_launch": bytes64, "avg_launch_ms": round(avg64, 4),
                     "profiler_avg_launch_ms": profiler_avg_ms(prof_stats, "k_hybrid<double>") if full else None},
        "valu": {"k_hybrid<double>": valu_fraction(prof_counters, "k_hybrid<double>", avg64) if full else None,
                 "k_hybrid<float>": valu_fraction(prof_counters, "k_hybrid<float>", avg32) if full else None},
    }
    # outputs kept on the host for the accuracy check against the oracle
    acc = {}
    if not args.no_extra:
        # context for the roofline: a plain device copy of the same bytes
        # (2^28 doubles read and written), timed the same way, outside the
        # timed region
        ds = timed_launches(torch, stream, lambda: w64.copy_(u64), 10)
        avg = sum(ds) / len(ds)
        result["roofline"]["device_copy_same_bytes_gbs"] = round(bytes64 / (avg * 1e-3) / 1e9, 1)
        forms = fp64_forms(torch, qm, ctx, stream, u64, w64, acc)
        # restore the FP64 outputs the copy and the forms overwrote (kept for the accuracy check)
        f64()
    if not args.no_cpu:
        torch.cuda.synchronize()
        mm = min(args.cpu_sample, n)
        acc["fp64"] = (h64[:mm], w64[:mm].cpu().numpy(), "norm_quantile", 2e-15)
        idx = sample_indices(n, h32)
        acc["fp32_refine"] = (h32[idx], gather(torch, w32, idx), "norm_quantile", 2e-7)
    del u64, u32, w64, w32
    torch.cuda.empty_cache()

    if not args.no_extra:
        result["extra"] = secondary_maps(args, torch, qm, qi, ctx, stream, n, acc)
        result["extra"]["fp64_forms"] = forms
        if args.serve_extra:
            result["extra"]["serving"] = serve_rates(torch, qm, args.serve_extra_count, args.serve_extra_rates)

    if not args.no_cpu:
        result["cpu_baseline"], errors = oracle_leg(args, acc, h64)
        result["fp64"].update(errors.pop("fp64"))
        result["fp32_refine"].update(errors.pop("fp32_refine"))
        if "extra" in result:
            result["extra"]["measured_error"] = errors
    ctx.close()
    return result


def fp64_forms(torch, qm, ctx, stream, u64, w64, acc, reps=10):
    """The FP64 hybrid beside the paper's own FP64 forms -- the branchless
    (13,13) rational (Appendix B) and the T2 hybrid with its whole-wave vote
    (Appendix C) -- on the mixture and on open uniforms of the same size (the
    input the paper times), outside the timed region.  The T2 form's outputs
    on the uniforms are kept at sampled indices for the accuracy check."""
    n = u64.numel()
    uu = torch.empty_like(u64)
    qm.qm_generate(ctx, 2, 0, 0, uu, qm.QM_UNIFORM)
    forms = {}
    scrub_in = torch.empty(1 << 26, dtype=torch.float64, device="cuda")
    scrub_out = torch.empty_like(scrub_in)
    scrub = lambda: scrub_out.copy_(scrub_in)     # noqa: E731
    for name, inp in (("mixture", u64), ("uniforms", uu)):
        forms[name] = {}
        for form, mode in (("hybrid", qm.QM_PLAIN), ("paper_branchless", qm.QM_PAPER),
                           ("paper_t2_vote", qm.QM_PAPER_T2)):
            ds = timed_launches(torch, stream, lambda: qm.qm_normal_quantile(ctx, inp, w64, mode), reps, scrub)
            avg = sum(ds) / len(ds)
            forms[name][form] = {"gsamples_s": round(n / (avg * 1e-3) / 1e9, 2), "avg_ms": round(avg, 4),
                                 "p50_ms": percentile(ds, 50)}
    torch.cuda.synchronize()
    idx = sample_indices(n, None, 9)
    acc["fp64_paper_t2 uniforms"] = (gather(torch, uu, idx), gather(torch, w64, idx), "norm_quantile", 2e-15)
    del uu, scrub_in, scrub_out
    torch.cuda.empty_cache()
    return forms


def secondary_maps(args, torch, qm, qi, ctx, stream, n, acc):
    """Rates of the other maps, outside the timed region, and their outputs
    at sampled indices for the accuracy check."""
    import numpy as np
    m = 1 << 26
    zh = qi.recycle_normals(m)
    xh = qi.recycle_exponentials(m)
    z = torch.from_numpy(zh).cuda()
    x = torch.from_numpy(xh).cuda()
    o = torch.empty_like(z)
    reps = 10
    # every timed launch below starts with none of its data in the 256 MB
    # last-level cache (back-to-back launches over 2^26 elements would
    # otherwise find part of their input there)
    scrub_in = torch.empty(1 << 26, dtype=torch.float64, device="cuda")
    scrub_out = torch.empty_like(scrub_in)
    scrub = lambda: scrub_out.copy_(scrub_in)     # noqa: E731
    rng = np.random.default_rng(3)
    zidx = np.unique(np.concatenate([rng.integers(0, m, 1 << 12), np.flatnonzero(np.abs(zh[: 1 << 22]) > 4.0)]))
    extra = {"student_t_f64": {}, "n": m}
    for nu in T_NUS:
        qm.qm_recycle_student_t(ctx, z, o, nu)  # builds and caches the table
        ds = timed_launches(torch, stream, lambda nu=nu: qm.qm_recycle_student_t(ctx, z, o, nu), reps, scrub)
        avg = sum(ds) / len(ds)
        extra["student_t_f64"][str(nu)] = {"gsamples_s": round(m / (avg * 1e-3) / 1e9, 2),
                                           "gbs": round(16.0 * m / (avg * 1e-3) / 1e9, 1),
                                           "p50_ms": percentile(ds, 50), "p99_ms": percentile(ds, 99)}
        acc["student_t_f64 nu=%g" % nu] = (zh[zidx], gather(torch, o, zidx), ("student_t_map", nu), 2e-15)
    ds = timed_launches(torch, stream, lambda: qm.qm_recycle_exp_to_normal(ctx, x, o), reps, scrub)
    avg = sum(ds) / len(ds)
    extra["exp_to_normal_f64"] = {"gsamples_s": round(m / (avg * 1e-3) / 1e9, 2),
                                  "gbs": round(16.0 * m / (avg * 1e-3) / 1e9, 1),
                                  "p50_ms": percentile(ds, 50), "p99_ms": percentile(ds, 99)}
    xidx = sample_indices(m, None, 5)
    acc["exp_to_normal_f64"] = (xh[xidx], gather(torch, o, xidx), "exp_to_normal", 2e-15)
    x32 = x.float()
    o32 = torch.empty_like(x32)
    ds = timed_launches(torch, stream, lambda: qm.qm_recycle_exp_to_normal(ctx, x32, o32), reps, scrub)
    avg = sum(ds) / len(ds)
    extra["exp_to_normal_f32_refine"] = {"gsamples_s": round(m / (avg * 1e-3) / 1e9, 2),
                                         "gbs": round(8.0 * m / (avg * 1e-3) / 1e9, 1)}
    acc["exp_to_normal_f32_refine"] = (xh[xidx].astype(np.float32), gather(torch, o32, xidx), "exp_to_normal", 2e-7)
    del x32, o32
    z32 = z.float()
    o32 = torch.empty_like(z32)
    extra["student_t_f32_refine"] = {}
    for nu in (1.0, 4.0, 30.0):
        ds = timed_launches(torch, stream, lambda nu=nu: qm.qm_recycle_student_t(ctx, z32, o32, nu), reps, scrub)
        avg = sum(ds) / len(ds)
        extra["student_t_f32_refine"][str(nu)] = {"gsamples_s": round(m / (avg * 1e-3) / 1e9, 2),
                                                  "gbs": round(8.0 * m / (avg * 1e-3) / 1e9, 1)}
        acc["student_t_f32_refine nu=%g" % nu] = (zh[zidx].astype(np.float32), gather(torch, o32, zidx),
                                                  ("student_t_map", nu), 2e-7)
    # exponential -> hyperbolic (Section 8.1), base samples with the target's masses
    extra["exp_to_hyperbolic_f64"] = {}
    extra["exp_to_hyperbolic_f32"] = {}
    for hp in (qi.HYPERBOLIC_PARAMS, (1.0, 0.5, 1.0)):
        tb = time.perf_counter()
        lp, lm = qm.qm_hyperbolic_masses(ctx, *hp)   # builds and caches the table
        tb = time.perf_counter() - tb
        hv = torch.from_numpy(qi.recycle_two_sided(m, hp[0], hp[1], math.exp(lm))).cuda()
        ds = timed_launches(torch, stream, lambda: qm.qm_recycle_exp_to_hyperbolic(ctx, hv, o, *hp), reps, scrub)
        avg = sum(ds) / len(ds)
        key = "a%g_b%g_d%g" % hp
        extra["exp_to_hyperbolic_f64"][key] = {"gsamples_s": round(m / (avg * 1e-3) / 1e9, 2),
                                              "gbs": round(16.0 * m / (avg * 1e-3) / 1e9, 1),
                                              "p50_ms": percentile(ds, 50), "p99_ms": percentile(ds, 99),
                                              "table_build_s": round(tb, 3)}
        hv32 = hv.float()
        ds = timed_launches(torch, stream, lambda: qm.qm_recycle_exp_to_hyperbolic(ctx, hv32, o32, *hp), reps, scrub)
        avg = sum(ds) / len(ds)
        extra["exp_to_hyperbolic_f32"][key] = {"gsamples_s": round(m / (avg * 1e-3) / 1e9, 2),
                                              "gbs": round(8.0 * m / (avg * 1e-3) / 1e9, 1)}
        del hv, hv32
    # exponential -> variance-gamma (Section 8.2)
    extra["exp_to_vg_f64"] = {}
    for vp in ((2, 1.0, 0.0), (3, 2.0, -1.0)):
        tb = time.perf_counter()
        lp, lm = qm.qm_vg_masses(ctx, *vp)
        tb = time.perf_counter() - tb
        vv = torch.from_numpy(qi.two_sided_exponentials(2, 3, m, vp[1] - vp[2], vp[1] + vp[2], math.exp(lm))).cuda()
        ds = timed_launches(torch, stream, lambda: qm.qm_recycle_exp_to_vg(ctx, vv, o, *vp), reps, scrub)
        avg = sum(ds) / len(ds)
        extra["exp_to_vg_f64"]["l%g_a%g_b%g" % vp] = {"gsamples_s": round(m / (avg * 1e-3) / 1e9, 2),
                                                      "gbs": round(16.0 * m / (avg * 1e-3) / 1e9, 1),
                                                      "table_build_s": round(tb, 3)}
        del vv
    del z, x, o, z32, o32
    torch.cuda.empty_cache()
    # fused Philox generation + quantile (write-only), vs generation alone
    g64 = torch.empty(n, dtype=torch.float64, device="cuda")
    g32 = torch.empty(n, dtype=torch.float32, device="cuda")
    fused = {"n": n}
    for name, buf, kind in (("uniform_f64", g64, qm.QM_UNIFORM), ("quantile_f64", g64, qm.QM_NORMAL_QUANTILE),
                            ("uniform_f32", g32, qm.QM_UNIFORM),
                            ("quantile_f32_refine", g32, qm.QM_NORMAL_QUANTILE)):
        ds = timed_launches(torch, stream, lambda buf=buf, kind=kind: qm.qm_generate(ctx, 1, 0, 0, buf, kind), reps, scrub)
        avg = sum(ds) / len(ds)
        fused[name] = {"gsamples_s": round(n / (avg * 1e-3) / 1e9, 2),
                       "gbs": round(buf.element_size() * n / (avg * 1e-3) / 1e9, 1),
                       "p50_ms": percentile(ds, 50), "p99_ms": percentile(ds, 99)}
    # fused chains: Philox -> normal -> Student t (nu = 4), Philox -> base -> hyperbolic (1, 0, 1)
    for name, buf, fn in (
            ("student_t_f64_nu4", g64, lambda: qm.qm_generate_student_t(ctx, 1, 0, 0, g64, 4.0)),
            ("student_t_f32_nu4", g32, lambda: qm.qm_generate_student_t(ctx, 1, 0, 0, g32, 4.0)),
            ("hyperbolic_f64", g64, lambda: qm.qm_generate_hyperbolic(ctx, 1, 0, 0, g64, *qi.HYPERBOLIC_PARAMS)),
            ("hyperbolic_f32", g32, lambda: qm.qm_generate_hyperbolic(ctx, 1, 0, 0, g32, *qi.HYPERBOLIC_PARAMS))):
        ds = timed_launches(torch, stream, fn, reps, scrub)
        avg = sum(ds) / len(ds)
        fused[name] = {"gsamples_s": round(n / (avg * 1e-3) / 1e9, 2),
                       "gbs": round(buf.element_size() * n / (avg * 1e-3) / 1e9, 1),
                       "p50_ms": percentile(ds, 50), "p99_ms": percentile(ds, 99)}
    extra["generate_fused"] = fused
    del g64, g32
    torch.cuda.empty_cache()
    return extra


def oracle_leg(args, acc, h64):
    """The CPU oracle: timed on a bounded sample of the FP64 workload (the
    CPU baseline), and, with the same outputs and on stratified samples of
    the other results, the measured error of every result."""
    import oracle
    mm = min(args.cpu_sample, h64.size)
    threads = oracle.threads_used(0)
    c0 = time.perf_counter()
    ref64 = oracle.norm_quantile(h64[:mm], threads)
    cdt = time.perf_counter() - c0
    base = {"value": round(mm / cdt / 1e9, 6), "unit": "Gsamples/s", "cores": threads, "kind": "oracle",
            "sample": "first %d elements of the FP64 mixture workload, FP64 quantile, %.1f s wall on %d threads "
                      "(%s)" % (mm, cdt, threads, cpu_model())}
    m1 = min(1 << 20, h64.size)                 # the same oracle on one thread, a smaller sample
    c0 = time.perf_counter()
    oracle.norm_quantile(h64[:m1], 1)
    c1 = time.perf_counter() - c0
    base["one_thread"] = {"value": round(m1 / c1 / 1e9, 6), "unit": "Gsamples/s",
                          "sample": "first %d elements, %.1f s wall on 1 thread" % (m1, c1)}
    errors = {}
    for name, (x, got, fn, rtol) in acc.items():
        if name == "fp64":
            ref = ref64
        elif isinstance(fn, tuple):
            ref = getattr(oracle, fn[0])(x.astype("float64"), fn[1])
        else:
            ref = getattr(oracle, fn)(x.astype("float64"))
        if got.dtype.itemsize == 4:
            import numpy as np
            with np.errstate(over="ignore"):
                r32 = ref.astype(np.float32)
            ref = np.where(np.isinf(r32) & np.isfinite(ref), r32.astype(np.float64), ref)
        rep = error_report(got, ref, rtol)
        rep["sample"] = ("every element of the first %d" % mm) if name == "fp64" else "stratified (%d)" % x.size
        errors[name] = rep
    return base, errors


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


# ---------------------------------------------------------------------------
def make_requests(qm, qi, torch, seed, count, lo, hi):
    """Device inputs and outputs for a request mix (inputs generated per request)."""
    kinds = {"nq_f32_refine": (qm.QM_NORMAL_QUANTILE, qm.QM_F32, qm.QM_F32_REFINE),
             "nq_f64": (qm.QM_NORMAL_QUANTILE, qm.QM_F64, qm.QM_PLAIN),
             "student_f64": (qm.QM_STUDENT_T, qm.QM_F64, qm.QM_PLAIN),
             "exp_f64": (qm.QM_EXP_TO_NORMAL, qm.QM_F64, qm.QM_PLAIN)}
    spec = qi.request_mix(seed, count, lo, hi)
    reqs, keep = [], []
    for r in spec:
        x = torch.from_numpy(qi.request_input(seed, r)).cuda()
        y = torch.empty_like(x)
        kind, dt, mode = kinds[r["kind"]]
        reqs.append(qm.qm_request(kind, dt, mode, 0, r["nu"], x.data_ptr(), y.data_ptr(), x.numel(), 0))
        keep.append((x, y))
    return spec, reqs, keep


def single_call(qm, ctx, r, stream_ptr):
    lib = qm.load()
    import ctypes
    s = ctypes.c_void_p(stream_ptr)
    if r.kind == qm.QM_NORMAL_QUANTILE:
        st = lib.qm_normal_quantile(ctx.handle, r.d_in, r.d_out, r.n, r.dtype, r.mode, s)
    elif r.kind == qm.QM_STUDENT_T:
        st = lib.qm_recycle_student_t(ctx.handle, r.d_in, r.d_out, r.n, r.dtype, r.mode, r.nu, s)
    else:
        st = lib.qm_recycle_exp_to_normal(ctx.handle, r.d_in, r.d_out, r.n, r.dtype, r.mode, s)
    qm.check(st)


def run_batch(args, torch, qm, qi):
    t0 = time.time()
    spec, reqs, keep = make_requests(qm, qi, torch, 3, args.batch_count, 10, 22)
    total = sum(r.n for r in reqs)
    print("batch inputs ready in %.1f s (%d requests, %d elements)" % (time.time() - t0, len(reqs), total),
          file=sys.stderr, flush=True)
    ctx = qm.Context(0)
    stream = torch.cuda.current_stream()
    sp = stream.cuda_stream
    qm.qm_run_batch(ctx, reqs, stream=sp)       # builds the nu tables
    for r in reqs:
        single_call(qm, ctx, r, sp)
    for _ in range(args.warmup):                # past the clock ramp (about 30 ms of work)
        qm.qm_run_batch(ctx, reqs, stream=sp)
    torch.cuda.synchronize()
    db = timed_launches(torch, stream, lambda: qm.qm_run_batch(ctx, reqs, stream=sp), args.steps)

    def seq():
        for r in reqs:
            single_call(qm, ctx, r, sp)
    ds = timed_launches(torch, stream, seq, max(2, args.steps // 4))
    ab, aseq = sum(db) / len(db), sum(ds) / len(ds)
    nbytes = sum(r.n * (4 if r.dtype == qm.QM_F32 else 8) * 2 for r in reqs)
    ctx.close()
    return {"metric": "Gsamples/s batched heterogeneous launch", "value": round(total / (ab * 1e-3) / 1e9, 3),
            "unit": "Gsamples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "higher_is_better": True,
            "dtype": "f64+f32", "data": "synthetic",
            "config": {"workload": "batch: %d requests, sizes log-uniform 2^10..2^22, mix 40/20/30/10, seed 3"
                                   % len(reqs), "elements": total, "bytes": nbytes},
            "batch": {"p50_ms": percentile(db, 50), "p99_ms": percentile(db, 99),
                      "gbs": round(nbytes / (ab * 1e-3) / 1e9, 1)},
            "sequential_launches": {"gsamples_s": round(total / (aseq * 1e-3) / 1e9, 3),
                                    "p50_ms": percentile(ds, 50)},
            "speedup_vs_sequential": round(aseq / ab, 3)}


SERVE_KINDS = {"nq_f32_refine": ("QM_NORMAL_QUANTILE", "QM_F32", "QM_F32_REFINE", 4),
               "nq_f64": ("QM_NORMAL_QUANTILE", "QM_F64", "QM_PLAIN", 8),
               "student_f64": ("QM_STUDENT_T", "QM_F64", "QM_PLAIN", 8),
               "exp_f64": ("QM_EXP_TO_NORMAL", "QM_F64", "QM_PLAIN", 8)}


def serving_trace(torch, qm, qi, seed, count):
    """Requests of the serving workload (sizes 2^12..2^24, mix 40/20/30/10,
    nu uniform in 1..50), each with its own inputs: request r's input is
    drawn on the device from Philox stream 1000 + r of `seed` (uniforms as
    the input generator defines them; normals as Phi^{-1} of such uniforms;
    exponentials as -log of them), so no two requests share data and the
    total far exceeds the caches.  Returns (qm_request list, keep-alive
    tensors, spec)."""
    spec = qi.request_mix(seed, count, 12, 24)
    ctx = qm.Context(0)
    reqs, keep = [], []
    for i, r in enumerate(spec):
        kind, dt, mode, es = SERVE_KINDS[r["kind"]]
        tdt = torch.float32 if es == 4 else torch.float64
        x = torch.empty(r["n"], dtype=tdt, device="cuda")
        gen_kind = qm.QM_NORMAL_QUANTILE if r["kind"] == "student_f64" else qm.QM_UNIFORM
        qm.qm_generate(ctx, seed, 1000 + i, 0, x, gen_kind, qm.QM_PLAIN)
        if r["kind"] == "exp_f64":
            x.log_().neg_()
        y = torch.empty_like(x)
        reqs.append(qm.qm_request(getattr(qm, kind), getattr(qm, dt), getattr(qm, mode), 0, r["nu"],
                                  x.data_ptr(), y.data_ptr(), r["n"], i))
        keep.append((x, y))
    torch.cuda.synchronize()
    ctx.close()
    return reqs, keep, spec


def serve_rates(torch, qm, count, rates, seed=5, budget=64 << 30):
    """Open-loop Poisson arrivals through qm_submit at each rate (0 = all at
    once): latency of each request from its scheduled arrival to the
    scheduler's observation of its completion (qm_poll_times, monotonic
    clock), p50/p99/max, delivered Gsamples/s, and the in-flight
    high-water mark; then the same trace as sequential single launches."""
    import ctypes

    import numpy as np

    import qm_inputs as qi
    reqs, keep, spec = serving_trace(torch, qm, qi, seed, count)
    total = sum(r.n for r in reqs)
    nus = sorted({r.nu for r in reqs if r.kind == qm.QM_STUDENT_T})
    lib = qm.load()
    rng = np.random.default_rng(seed)
    out = []
    for rate in rates:
        ctx = qm.Context(0, hbm_budget_bytes=budget)
        z = torch.zeros(1, dtype=torch.float64, device="cuda")
        for nu in nus:                       # tables built before the clock starts
            qm.qm_recycle_student_t(ctx, z[:0], z[:0], nu)
        # one request through the loop before the clock starts: the first
        # submit starts the scheduler (thread, streams, events) and the first
        # batch launch loads the kernel's code
        wu = torch.full((4096,), 0.25, dtype=torch.float64, device="cuda")
        wo = torch.empty_like(wu)
        torch.cuda.synchronize()
        wt = qm.qm_submit(ctx, qm.make_request(qm.QM_NORMAL_QUANTILE, wu, wo))
        while qm.qm_poll(ctx, wt) == qm.QM_PENDING:
            time.sleep(0.0002)
        torch.cuda.synchronize()
        arrivals = np.cumsum(rng.exponential(1.0 / rate, count)) if rate > 0 else np.zeros(count)
        tickets = [0] * count
        t0_ns = time.monotonic_ns()
        tk = ctypes.c_uint64()
        lag = 0.0
        for i in range(count):
            due = t0_ns + int(arrivals[i] * 1e9)
            while time.monotonic_ns() < due:
                pass
            lag = max(lag, (time.monotonic_ns() - due) / 1e6)
            qm.check(lib.qm_submit(ctx.handle, ctypes.byref(reqs[i]), ctypes.byref(tk)))
            tickets[i] = tk.value
        done_ns = [None] * count
        while any(d is None for d in done_ns):
            for i in range(count):
                if done_ns[i] is None:
                    st, _, d = qm.qm_poll_times(ctx, tickets[i])
                    if st == qm.QM_OK:
                        done_ns[i] = d
            time.sleep(0.0002)
        wall = (max(done_ns) - t0_ns) / 1e9
        lat_ms = [(done_ns[i] - (t0_ns + int(arrivals[i] * 1e9))) / 1e6 for i in range(count)]
        stats = qm.qm_serving_stats_of(ctx)
        ctx.close()
        row = {"rate_req_s": rate if rate > 0 else "burst", "requests": count, "elements": total,
               "wall_s": round(wall, 4), "gsamples_s": round(total / wall / 1e9, 3),
               "offered_gsamples_s": round(total / arrivals[-1] / 1e9, 3) if rate > 0 else None,
               "p50_ms": round(percentile(lat_ms, 50), 4), "p99_ms": round(percentile(lat_ms, 99), 4),
               "max_ms": round(max(lat_ms), 4), "max_submit_lag_ms": round(lag, 4),
               "in_flight_high_water_bytes": stats["in_flight_bytes_high_water"]}
        out.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
    # the same trace as sequential single launches on one stream
    ctx = qm.Context(0)
    z = torch.zeros(1, dtype=torch.float64, device="cuda")
    for nu in nus:
        qm.qm_recycle_student_t(ctx, z[:0], z[:0], nu)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        single_call(qm, ctx, r, stream.cuda_stream)
    torch.cuda.synchronize()
    seq_wall = time.perf_counter() - t0
    ctx.close()
    del keep
    torch.cuda.empty_cache()
    return {"config": "Poisson arrivals, %d requests per rate, sizes log-uniform 2^12..2^24, mix 40/20/30/10, "
                      "distinct inputs per request, HBM budget %d GB, seed %d; latency from scheduled arrival"
                      % (count, budget >> 30, seed),
            "rates": out,
            "sequential_launches": {"wall_s": round(seq_wall, 4), "gsamples_s": round(total / seq_wall / 1e9, 3)}}


def run_serve(args, torch, qm, qi):
    """Open-loop Poisson arrivals through qm_submit/qm_poll at swept rates."""
    r = serve_rates(torch, qm, args.serve_count, args.rates)
    return {"metric": "serving p50/p99 latency and Gsamples/s (continuous batching)",
            "value": max(x["gsamples_s"] for x in r["rates"]),
            "unit": "Gsamples/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64+f32", "data": "synthetic",
            "config": {"workload": "serving: " + r["config"]},
            "rates": r["rates"], "sequential_launches": r["sequential_launches"]}


# ---------------------------------------------------------------------------
def run_hyperbolic(args, torch, qm, qi):
    """Exponential -> hyperbolic (Section 8.1): 2^26 base samples of the
    Section 8.1 illustration (alpha = delta = 1, beta = 0), FP64 then FP32
    in/out per step, inputs resident in HBM."""
    hp = qi.HYPERBOLIC_PARAMS
    n = 1 << 26
    t0 = time.time()
    ctx = qm.Context(0)
    tb = time.perf_counter()
    lp, lm = qm.qm_hyperbolic_masses(ctx, *hp)       # builds and caches the table
    tb = time.perf_counter() - tb
    v64 = torch.from_numpy(qi.recycle_two_sided(n, hp[0], hp[1], math.exp(lm))).cuda()
    v32 = v64.float()
    x64 = torch.empty_like(v64)
    x32 = torch.empty_like(v32)
    torch.cuda.synchronize()
    print("hyperbolic inputs ready in %.1f s (table %.2f s)" % (time.time() - t0, tb), file=sys.stderr, flush=True)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        qm.qm_recycle_exp_to_hyperbolic(ctx, v64, x64, *hp)
        qm.qm_recycle_exp_to_hyperbolic(ctx, v32, x32, *hp)
    torch.cuda.synchronize()
    if args.copy_calibration:
        x64.copy_(v64)      # a plain copy of 2^26 doubles (512 MiB read + written), for counter scaling
        torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t_start = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        qm.qm_recycle_exp_to_hyperbolic(ctx, v64, x64, *hp)
        ev[k][1].record(stream)
        qm.qm_recycle_exp_to_hyperbolic(ctx, v32, x32, *hp)
        ev[k][2].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    d64 = [e[0].elapsed_time(e[1]) for e in ev]
    d32 = [e[1].elapsed_time(e[2]) for e in ev]
    avg64, avg32 = sum(d64) / len(d64), sum(d32) / len(d32)
    achieved = 16.0 * n / (avg64 * 1e-3) / 1e9
    # outputs for the measured error, outside the timed region: the first
    # 2^13 base samples and the 256 largest |v| among the first 2^22
    sidx = torch.cat([torch.arange(1 << 13, device=v64.device), torch.topk(v64[:1 << 22].abs(), 256).indices])
    samp = {"fp64": (v64[sidx].cpu().numpy(), x64[sidx].cpu().numpy(), 2e-15),
            "fp32": (v32[sidx].cpu().numpy(), x32[sidx].cpu().numpy(), 2e-7)}
    result = {
        "metric": "Gsamples/s exponential->hyperbolic recycling (FP64 + FP32 in/out)",
        "value": round(2.0 * n * args.steps / wall / 1e9, 3),
        "unit": "Gsamples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "exp->hyperbolic, 2^26 two-sided exponential base samples of (alpha, beta, delta) = "
                               "(1, 0, 1), seed 2 stream 2; FP64 then FP32 in/out",
                   "n_per_pass": n, "passes_per_step": 2, "table_build_s": round(tb, 3)},
        "fp64": {"gsamples_s": round(n / (avg64 * 1e-3) / 1e9, 2), "avg_ms": round(avg64, 4),
                 "p50_ms": percentile(d64, 50), "p99_ms": percentile(d64, 99), "tolerance": 2e-15},
        "fp32": {"gsamples_s": round(n / (avg32 * 1e-3) / 1e9, 2), "avg_ms": round(avg32, 4),
                 "p50_ms": percentile(d32, 50),
                 "p99_ms": percentile(d32, 99), "gbs": round(8.0 * n / (avg32 * 1e-3) / 1e9, 1),
                 "tolerance": 2e-7},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": counted_traffic("hyperbolic_exp_2e26_hbm_counters.md", "k_hyperbolic<double>",
                                                HYPERBOLIC_SOURCES),
                     "kernel": "qm::k_hyperbolic<double, true, 4, 11> (16 workgroups/CU x 4 vectors, wave-contiguous tiles)",
                     "algorithmic_bytes_per_launch": 16.0 * n, "avg_launch_ms": round(avg64, 4),
                     "profiler_avg_launch_ms": profiler_avg_ms("hyperbolic_exp_2e26_kernel_stats.md",
                                                               "k_hyperbolic<double>", HYPERBOLIC_SOURCES)},
        "valu": {"k_hyperbolic<double>": valu_fraction("hyperbolic_exp_2e26_hbm_counters.md", "k_hyperbolic<double>",
                                                       avg64, HYPERBOLIC_SOURCES),
                 "k_hyperbolic<float>": valu_fraction("hyperbolic_exp_2e26_hbm_counters.md", "k_hyperbolic<float>",
                                                      avg32, HYPERBOLIC_SOURCES)},
    }
    # context for the roofline: a plain device copy of the same bytes, timed
    # the same way, outside the timed region
    ds = timed_launches(torch, stream, lambda: x64.copy_(v64), 10)
    result["roofline"]["device_copy_same_bytes_gbs"] = round(16.0 * n / (sum(ds) / len(ds) * 1e-3) / 1e9, 1)
    del v32, x32, x64
    if not args.no_cpu:
        import oracle
        threads = oracle.threads_used(0)
        for key, (vin, got, rtol) in samp.items():
            c0 = time.perf_counter()
            ref = oracle.hyperbolic_map(vin.astype("float64"), *hp, threads=threads)
            cdt = time.perf_counter() - c0
            rep = error_report(got, ref, rtol)
            rep["sample"] = "first 8192 base samples and the 256 largest |v| among the first 2^22"
            result[key]["measured_error"] = rep
            if key == "fp64":
                mm = vin.size
                result["cpu_baseline"] = {"value": round(mm / cdt / 1e9, 9), "unit": "Gsamples/s", "cores": threads,
                                          "kind": "oracle",
                                          "sample": "%d base samples (the measured-error sample), FP64 map, %.1f s "
                                                    "wall on %d threads (%s)" % (mm, cdt, threads, cpu_model())}
    ctx.close()
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps before the timed ones (default: 60 quantile steps, 240 hyperbolic "
                         "steps, about 80 ms of work: the clocks settle over the first 30 ms of a run)")
    ap.add_argument("--workload", choices=["quantile", "batch", "serve", "hyperbolic"], default="quantile")
    ap.add_argument("--n", type=int, default=1 << 28, help="samples per pass (quantile workload)")
    ap.add_argument("--cpu-sample", type=int, default=1 << 28, help="oracle sample size (elements)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the secondary maps")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of the FP64 input (for HBM counter scaling; "
                         "quantile and hyperbolic workloads)")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--serve-count", type=int, default=2000)
    ap.add_argument("--rates", type=float, nargs="+", default=[1000, 2000, 5000, 10000, 20000, 50000, 100000, 0],
                    help="arrival rates in requests/s; 0 = burst (all requests at once)")
    ap.add_argument("--pct-reps", type=int, default=64,
                    help="extra launches per kernel for the p50/p99 latencies (outside the timed region)")
    ap.add_argument("--serve-extra", type=int, default=1,
                    help="quantile workload: also run a bounded serving trace (0 = skip)")
    ap.add_argument("--serve-extra-count", type=int, default=500)
    ap.add_argument("--serve-extra-rates", type=float, nargs="+", default=[10000, 50000])
    args = ap.parse_args()
    if args.warmup is None:
        args.warmup = {"quantile": 60, "hyperbolic": 240, "batch": 10}.get(args.workload, 1)
    if args.gpus != 1:
        print("bench.py measures one GPU only: the maps are elementwise and shard into contiguous ranges "
              "without communication, so --gpus %d is not run." % args.gpus, file=sys.stderr)
        return 2

    import torch

    import paper_0901_0638_amd as qm
    import qm_inputs as qi

    if args.workload == "batch":
        result = run_batch(args, torch, qm, qi)
    elif args.workload == "serve":
        result = run_serve(args, torch, qm, qi)
    elif args.workload == "hyperbolic":
        result = run_hyperbolic(args, torch, qm, qi)
    else:
        result = run_quantile(args, torch, qm, qi)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
