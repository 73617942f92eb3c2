#!/usr/bin/env python3
"""Benchmark of the quantile-mechanics hot path on one MI355X.

Workload (one "step"): the Gaussian quantile on 2^28 samples, once in FP64
(plain, 2e-15) and once in FP32 + FP64 refine (2e-7): u is 90% open uniform,
10% tail stratum log-uniform in [1e-300, 1e-2] (FP64) or [1e-37, 1e-2]
(FP32), mirrored to 1-u with probability 1/2, seed 1.  Inputs are resident in
HBM before the timed region.  value = samples of both passes / wall time of
the timed steps.

Prints one JSON line (see the keys below), with the roofline of the dominant
kernel (FP64 quantile: 16 algorithmic bytes per sample, timed per launch by
HIP events on its stream) and the CPU oracle's rate on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gsamples/s Φ^{-1} & t-recycle (FP64 vs FP32+refine) at stated max err; p50/p99"
HBM_PEAK_GBS = 8000.0


def percentile(xs, p):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(p / 100.0 * (len(xs) - 1)))))
    return xs[k]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1 << 28, help="samples per pass")
    ap.add_argument("--cpu-sample", type=int, default=1 << 23, help="oracle sample size (elements)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain device copy of the FP64 input (for HBM counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the hot path is elementwise and shards without "
              "communication, so --gpus %d is not run (see DESIGN.md)." % args.gpus, file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_0901_0638_amd as qm
    import qm_inputs as qi

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

    d64 = [e[0].elapsed_time(e[1]) for e in events]  # ms
    d32 = [e[1].elapsed_time(e[2]) for e in events]
    ms_step = wall * 1e3 / args.steps
    value = 2.0 * n * args.steps / wall / 1e9

    avg64 = sum(d64) / len(d64)
    bytes64 = 16.0 * n
    achieved = bytes64 / (avg64 * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                "kernel": "k_map<double, VECTOR, 2, OpNQ64Plain> (FP64 quantile)",
                "algorithmic_bytes_per_launch": bytes64, "avg_launch_ms": round(avg64, 4)}

    result = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gsamples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
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
        "fp32_refine": {"gsamples_s": round(n / (sum(d32) / len(d32) * 1e-3) / 1e9, 2),
                        "p50_ms": percentile(d32, 50), "p99_ms": percentile(d32, 99),
                        "gbs": round(8.0 * n / (sum(d32) / len(d32) * 1e-3) / 1e9, 1), "max_rel_err_bound": 2e-7},
        "roofline": roofline,
    }

    if not args.no_cpu:
        import oracle
        m = args.cpu_sample
        us = qi.mixture_f64(m)
        threads = oracle.threads_used(0)
        c0 = time.perf_counter()
        oracle.norm_quantile(us, threads)
        cdt = time.perf_counter() - c0
        result["cpu_baseline"] = {"value": round(m / cdt / 1e9, 6), "unit": "Gsamples/s", "cores": threads,
                                  "kind": "oracle", "sample": "first %d elements of the FP64 mixture workload, "
                                  "FP64 quantile, %.1f s wall on %d threads" % (m, cdt, threads)}
    print(json.dumps(result))
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
