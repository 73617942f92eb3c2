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


def counted_traffic(profile="quantile_mixture_2e28_hbm_counters.md", kernel="k_hybrid<double>",
                    files=QUANTILE_SOURCES):
    """HBM bytes per launch of a kernel from its committed rocprofv3
    FETCH_SIZE/WRITE_SIZE summary, or None if the kernel sources changed
    since those counters were taken."""
    import re
    path = os.path.join(ROOT, "profiles", profile)
    try:
        text = open(path).read()
    except OSError:
        return None
    m = re.search(r"Kernel source hash: `([0-9a-f]+)`", text)
    t = re.search(r"traffic_bytes_per_launch %s: ([0-9]+)" % re.escape(kernel), text)
    if not m or not t or m.group(1) != kernel_source_hash(files):
        return None
    return int(t.group(1))


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(math.ceil(p / 100.0 * len(xs))) - 1))
    return xs[k]


def timed_launches(torch, stream, fn, reps):
    """Per-launch durations (ms) with HIP events on the launch stream, after
    one untimed call (the first launch of a kernel also loads its code)."""
    fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


# ---------------------------------------------------------------------------
def run_quantile(args, torch, qm, qi):
    n = args.n
    t0 = time.time()
    u64 = torch.from_numpy(qi.mixture_f64(n)).cuda()
    u32 = torch.from_numpy(qi.mixture_f32(n)).cuda()
    w64 = torch.empty_like(u64)
    w32 = torch.empty_like(u32)
    torch.cuda.synchronize()
    print("inputs ready in %.1f s" % (time.time() - t0), file=sys.stderr, flush=True)

    ctx = qm.Context(0)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        qm.qm_normal_quantile(ctx, u64, w64, qm.QM_PLAIN)
        if ev is not None:
            ev[1].record(stream)
        qm.qm_normal_quantile(ctx, u32, w32, qm.QM_F32_REFINE)
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
    bytes64 = 16.0 * n
    achieved = bytes64 / (avg64 * 1e-3) / 1e9
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
        "fp64": {"gsamples_s": round(n / (avg64 * 1e-3) / 1e9, 2), "p50_ms": percentile(d64, 50),
                 "p99_ms": percentile(d64, 99), "max_rel_err_bound": 2e-15},
        "fp32_refine": {"gsamples_s": round(n / (avg32 * 1e-3) / 1e9, 2), "p50_ms": percentile(d32, 50),
                        "p99_ms": percentile(d32, 99), "gbs": round(8.0 * n / (avg32 * 1e-3) / 1e9, 1),
                        "max_rel_err_bound": 2e-7},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": counted_traffic() if n == (1 << 28) else None,
                     "kernel": "qm::k_hybrid<double, 4, qm::HybridNQ64> (FP64 quantile: central piece, "
                               "outer elements gathered per wave; 64 workgroups/CU x 4 vectors)",
                     "algorithmic_bytes_per_launch": bytes64, "avg_launch_ms": round(avg64, 4)},
    }
    if not args.no_extra:
        # context for the roofline: a plain device copy of the same bytes
        # (2^28 doubles read and written), timed the same way, outside the
        # timed region
        ds = timed_launches(torch, stream, lambda: w64.copy_(u64), 10)
        avg = sum(ds) / len(ds)
        result["roofline"]["device_copy_same_bytes_gbs"] = round(bytes64 / (avg * 1e-3) / 1e9, 1)
    del u64, u32, w64, w32
    torch.cuda.empty_cache()

    if not args.no_extra:
        # secondary maps, outside the timed region (normals / Exp(1), seed 2)
        m = 1 << 26
        z = torch.from_numpy(qi.recycle_normals(m)).cuda()
        x = torch.from_numpy(qi.recycle_exponentials(m)).cuda()
        o = torch.empty_like(z)
        extra = {"student_t_f64": {}, "n": m}
        for nu in T_NUS:
            qm.qm_recycle_student_t(ctx, z, o, nu)  # builds and caches the table
            ds = timed_launches(torch, stream, lambda nu=nu: qm.qm_recycle_student_t(ctx, z, o, nu), 10)
            avg = sum(ds) / len(ds)
            extra["student_t_f64"][str(nu)] = {"gsamples_s": round(m / (avg * 1e-3) / 1e9, 2),
                                               "gbs": round(16.0 * m / (avg * 1e-3) / 1e9, 1),
                                               "p50_ms": percentile(ds, 50), "p99_ms": percentile(ds, 99)}
        ds = timed_launches(torch, stream, lambda: qm.qm_recycle_exp_to_normal(ctx, x, o), 10)
        avg = sum(ds) / len(ds)
        extra["exp_to_normal_f64"] = {"gsamples_s": round(m / (avg * 1e-3) / 1e9, 2),
                                      "gbs": round(16.0 * m / (avg * 1e-3) / 1e9, 1),
                                      "p50_ms": percentile(ds, 50), "p99_ms": percentile(ds, 99)}
        z32 = z.float()
        o32 = torch.empty_like(z32)
        extra["student_t_f32_refine"] = {}
        for nu in (1.0, 4.0, 30.0):
            ds = timed_launches(torch, stream, lambda nu=nu: qm.qm_recycle_student_t(ctx, z32, o32, nu), 10)
            avg = sum(ds) / len(ds)
            extra["student_t_f32_refine"][str(nu)] = {"gsamples_s": round(m / (avg * 1e-3) / 1e9, 2),
                                                      "gbs": round(8.0 * m / (avg * 1e-3) / 1e9, 1)}
        # exponential -> hyperbolic (Section 8.1), base samples with the target's masses
        extra["exp_to_hyperbolic_f64"] = {}
        extra["exp_to_hyperbolic_f32"] = {}
        for hp in (qi.HYPERBOLIC_PARAMS, (1.0, 0.5, 1.0)):
            tb = time.perf_counter()
            lp, lm = qm.qm_hyperbolic_masses(ctx, *hp)   # builds and caches the table
            tb = time.perf_counter() - tb
            hv = torch.from_numpy(qi.recycle_two_sided(m, hp[0], hp[1], math.exp(lm))).cuda()
            ds = timed_launches(torch, stream, lambda: qm.qm_recycle_exp_to_hyperbolic(ctx, hv, o, *hp), 10)
            avg = sum(ds) / len(ds)
            key = "a%g_b%g_d%g" % hp
            extra["exp_to_hyperbolic_f64"][key] = {"gsamples_s": round(m / (avg * 1e-3) / 1e9, 2),
                                                  "gbs": round(16.0 * m / (avg * 1e-3) / 1e9, 1),
                                                  "p50_ms": percentile(ds, 50), "p99_ms": percentile(ds, 99),
                                                  "table_build_s": round(tb, 3)}
            hv32 = hv.float()
            ds = timed_launches(torch, stream, lambda: qm.qm_recycle_exp_to_hyperbolic(ctx, hv32, o32, *hp), 10)
            avg = sum(ds) / len(ds)
            extra["exp_to_hyperbolic_f32"][key] = {"gsamples_s": round(m / (avg * 1e-3) / 1e9, 2),
                                                  "gbs": round(8.0 * m / (avg * 1e-3) / 1e9, 1)}
            del hv, hv32
        # exponential -> variance-gamma, integer lambda (Section 8.2)
        extra["exp_to_vg_f64"] = {}
        for vp in ((2, 1.0, 0.0), (3, 2.0, -1.0)):
            tb = time.perf_counter()
            lp, lm = qm.qm_vg_masses(ctx, *vp)
            tb = time.perf_counter() - tb
            vv = torch.from_numpy(qi.two_sided_exponentials(2, 3, m, vp[1] - vp[2], vp[1] + vp[2], math.exp(lm))).cuda()
            ds = timed_launches(torch, stream, lambda: qm.qm_recycle_exp_to_vg(ctx, vv, o, *vp), 10)
            avg = sum(ds) / len(ds)
            extra["exp_to_vg_f64"]["l%d_a%g_b%g" % vp] = {"gsamples_s": round(m / (avg * 1e-3) / 1e9, 2),
                                                          "gbs": round(16.0 * m / (avg * 1e-3) / 1e9, 1),
                                                          "table_build_s": round(tb, 3)}
            del vv
        # fused Philox generation + quantile (write-only), vs generation alone
        g64 = torch.empty(n, dtype=torch.float64, device="cuda")
        g32 = torch.empty(n, dtype=torch.float32, device="cuda")
        fused = {"n": n}
        for name, buf, kind in (("uniform_f64", g64, qm.QM_UNIFORM), ("quantile_f64", g64, qm.QM_NORMAL_QUANTILE),
                                ("uniform_f32", g32, qm.QM_UNIFORM),
                                ("quantile_f32_refine", g32, qm.QM_NORMAL_QUANTILE)):
            ds = timed_launches(torch, stream, lambda buf=buf, kind=kind: qm.qm_generate(ctx, 1, 0, 0, buf, kind), 10)
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
            ds = timed_launches(torch, stream, fn, 10)
            avg = sum(ds) / len(ds)
            fused[name] = {"gsamples_s": round(n / (avg * 1e-3) / 1e9, 2),
                           "gbs": round(buf.element_size() * n / (avg * 1e-3) / 1e9, 1),
                           "p50_ms": percentile(ds, 50), "p99_ms": percentile(ds, 99)}
        extra["generate_fused"] = fused
        del g64, g32
        result["extra"] = extra
        del z, x, o, z32, o32
        torch.cuda.empty_cache()

    if not args.no_cpu:
        import oracle
        mm = args.cpu_sample
        us = qi.mixture_f64(mm)
        threads = oracle.threads_used(0)
        c0 = time.perf_counter()
        oracle.norm_quantile(us, threads)
        cdt = time.perf_counter() - c0
        result["cpu_baseline"] = {"value": round(mm / cdt / 1e9, 6), "unit": "Gsamples/s", "cores": threads,
                                  "kind": "oracle",
                                  "sample": "first %d elements of the FP64 mixture workload, FP64 quantile, "
                                            "%.1f s wall on %d threads (%s)" % (mm, cdt, threads, cpu_model())}
    ctx.close()
    return result


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
            "unit": "Gsamples/s", "n_gpus": 1, "steps": args.steps, "warmup": 1, "higher_is_better": True,
            "dtype": "f64+f32", "data": "synthetic",
            "config": {"workload": "batch: %d requests, sizes log-uniform 2^10..2^22, mix 40/20/30/10, seed 3"
                                   % len(reqs), "elements": total, "bytes": nbytes},
            "batch": {"p50_ms": percentile(db, 50), "p99_ms": percentile(db, 99),
                      "gbs": round(nbytes / (ab * 1e-3) / 1e9, 1)},
            "sequential_launches": {"gsamples_s": round(total / (aseq * 1e-3) / 1e9, 3),
                                    "p50_ms": percentile(ds, 50)},
            "speedup_vs_sequential": round(aseq / ab, 3)}


def run_serve(args, torch, qm, qi):
    """Open-loop Poisson arrivals through qm_submit/qm_poll at swept rates."""
    import numpy as np
    seed = 5
    count = args.serve_count
    spec = qi.request_mix(seed, count, 12, 24)
    pools = {}
    maxn = 1 << 24
    # shared read-only input pools, one per kind (the content is workload-shaped)
    pools["nq_f32_refine"] = torch.from_numpy(qi.uniform24(seed, 1, maxn)).cuda()
    pools["nq_f64"] = torch.from_numpy(qi.uniform53(seed, 2, maxn)).cuda()
    pools["student_f64"] = torch.from_numpy(qi.normals(seed, 3, maxn)).cuda()
    pools["exp_f64"] = torch.from_numpy(qi.exponentials(seed, 4, maxn)).cuda()
    budget = 64 << 30
    out_ring_bytes = 40 << 30
    out_ring = torch.empty(out_ring_bytes // 8, dtype=torch.float64, device="cuda")
    kinds = {"nq_f32_refine": (qm.QM_NORMAL_QUANTILE, qm.QM_F32, qm.QM_F32_REFINE, 4),
             "nq_f64": (qm.QM_NORMAL_QUANTILE, qm.QM_F64, qm.QM_PLAIN, 8),
             "student_f64": (qm.QM_STUDENT_T, qm.QM_F64, qm.QM_PLAIN, 8),
             "exp_f64": (qm.QM_EXP_TO_NORMAL, qm.QM_F64, qm.QM_PLAIN, 8)}
    reqs = []
    off = 0
    base = out_ring.data_ptr()
    for r in spec:
        kind, dt, mode, es = kinds[r["kind"]]
        nbytes = r["n"] * es
        if off + nbytes > out_ring_bytes:
            off = 0
        reqs.append(qm.qm_request(kind, dt, mode, 0, r["nu"], pools[r["kind"]].data_ptr(), base + off, r["n"], 0))
        off += (nbytes + 255) // 256 * 256
    total = sum(r.n for r in reqs)
    rng = np.random.default_rng(seed)
    results = []
    warm = qm.Context(0, hbm_budget_bytes=budget)
    for nu in range(1, 51):                  # warm the table builder's cache path
        qm.qm_recycle_student_t(warm, pools["student_f64"][:1024], out_ring[:1024], float(nu))
    warm.close()
    for rate in args.rates:
        ctx = qm.Context(0, hbm_budget_bytes=budget)
        for nu in range(1, 51):
            qm.qm_recycle_student_t(ctx, pools["student_f64"][:1024], out_ring[:1024], float(nu))
        torch.cuda.synchronize()
        if rate > 0:
            arrivals = np.cumsum(rng.exponential(1.0 / rate, count))
        else:                                # burst: everything arrives at once (capacity)
            arrivals = np.zeros(count)
        tickets = [None] * count
        lib = qm.load()
        import ctypes

        def submitter():
            t0 = time.perf_counter()
            for i in range(count):
                while time.perf_counter() - t0 < arrivals[i]:
                    pass
                tk = ctypes.c_uint64()
                qm.check(lib.qm_submit(ctx.handle, ctypes.byref(reqs[i]), ctypes.byref(tk)))
                tickets[i] = tk.value

        th = threading.Thread(target=submitter)
        t_start = time.perf_counter()
        th.start()
        th.join()
        done = 0
        while done < count:
            done = sum(1 for t in tickets if lib.qm_poll(ctx.handle, t) == qm.QM_OK)
            if done < count:
                time.sleep(0.0005)
        wall = time.perf_counter() - t_start
        lat = qm.qm_serving_latencies(ctx)
        ctx.close()
        lat_ms = [x / 1e6 for x in lat]
        results.append({"rate_req_s": rate if rate > 0 else "burst", "requests": count, "elements": total,
                        "wall_s": round(wall, 4), "gsamples_s": round(total / wall / 1e9, 3),
                        "offered_gsamples_s": round(total / arrivals[-1] / 1e9, 3) if rate > 0 else None,
                        "p50_ms": round(percentile(lat_ms, 50), 4), "p99_ms": round(percentile(lat_ms, 99), 4),
                        "max_ms": round(max(lat_ms), 4)})
        print(json.dumps(results[-1]), file=sys.stderr, flush=True)
    # the same trace as sequential launches, one request at a time on one stream
    ctx = qm.Context(0)
    for nu in range(1, 51):                  # tables built before timing
        qm.qm_recycle_student_t(ctx, pools["student_f64"][:1024], out_ring[:1024], float(nu))
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for r in reqs:
        single_call(qm, ctx, r, stream.cuda_stream)
    torch.cuda.synchronize()
    seq_wall = time.perf_counter() - t0
    ctx.close()
    return {"metric": "serving p50/p99 latency and Gsamples/s (continuous batching)",
            "value": max(r["gsamples_s"] for r in results),
            "unit": "Gsamples/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64+f32", "data": "synthetic",
            "config": {"workload": "serving: Poisson arrivals, %d requests per rate, sizes log-uniform 2^12..2^24, "
                                   "mix 40/20/30/10, HBM budget 64 GB, seed 5" % count},
            "rates": results,
            "sequential_launches": {"wall_s": round(seq_wall, 4), "gsamples_s": round(total / seq_wall / 1e9, 3)}}


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
    result = {
        "metric": "Gsamples/s exponential->hyperbolic recycling (FP64 + FP32 in/out)",
        "value": round(2.0 * n * args.steps / wall / 1e9, 3),
        "unit": "Gsamples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "exp->hyperbolic, 2^26 two-sided exponential base samples of (alpha, beta, delta) = "
                               "(1, 0, 1), seed 2 stream 2; FP64 then FP32 in/out",
                   "n_per_pass": n, "passes_per_step": 2, "table_build_s": round(tb, 3)},
        "fp64": {"gsamples_s": round(n / (avg64 * 1e-3) / 1e9, 2), "p50_ms": percentile(d64, 50),
                 "p99_ms": percentile(d64, 99), "max_rel_err_bound": 2e-15},
        "fp32": {"gsamples_s": round(n / (avg32 * 1e-3) / 1e9, 2), "p50_ms": percentile(d32, 50),
                 "p99_ms": percentile(d32, 99), "gbs": round(8.0 * n / (avg32 * 1e-3) / 1e9, 1),
                 "max_rel_err_bound": 2e-7},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": counted_traffic("hyperbolic_exp_2e26_hbm_counters.md", "k_hyperbolic<double>",
                                                HYPERBOLIC_SOURCES),
                     "kernel": "qm::k_hyperbolic<double, true, 4, 11> (8 workgroups/CU x 4 vectors)",
                     "algorithmic_bytes_per_launch": 16.0 * n, "avg_launch_ms": round(avg64, 4)},
    }
    # context for the roofline: a plain device copy of the same bytes, timed
    # the same way, outside the timed region
    ds = timed_launches(torch, stream, lambda: x64.copy_(v64), 10)
    result["roofline"]["device_copy_same_bytes_gbs"] = round(16.0 * n / (sum(ds) / len(ds) * 1e-3) / 1e9, 1)
    del v32, x32, x64
    if not args.no_cpu:
        import oracle
        mm = 1 << 13
        vs = v64[:mm].cpu().numpy()
        threads = oracle.threads_used(0)
        c0 = time.perf_counter()
        oracle.hyperbolic_map(vs, *hp, threads=threads)
        cdt = time.perf_counter() - c0
        result["cpu_baseline"] = {"value": round(mm / cdt / 1e9, 9), "unit": "Gsamples/s", "cores": threads,
                                  "kind": "oracle",
                                  "sample": "first %d base samples, FP64 map, %.1f s wall on %d threads (%s)"
                                            % (mm, cdt, threads, cpu_model())}
    ctx.close()
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
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
    args = ap.parse_args()
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
