"""Benchmark: subset-terms/s of one 56x56 hafnian on one MI355X.

A step is one complete hafnian of the 56x56 complex Gaussian symmetric matrix
(seed 5601): all 2^28 subset terms (gather, Hessenberg reduction,
characteristic polynomial, power traces, series) and the signed double-double
sum, with the matrix already resident in device memory.  The printed JSON line
carries the throughput, the roofline position of the dominant kernel (the
per-subset coefficient kernel, timed with HIP events on its own stream inside
the timed region) and the CPU oracle timed on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 56] [--kind haf|lhaf]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6          # MI355X vector FP64: 256 CU x 128 flop/clk x 2.4 GHz


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(A, n, loops, seconds_target=15.0):
    """The CPU oracle (long double, explicit-power route) on a uniform random
    sample of subsets of the same matrix, scaled to subset-terms/s."""
    import numpy as np

    import oracle
    N = n // 2
    threads = os.cpu_count() or 1
    rng = np.random.default_rng(12345)
    probe = rng.integers(1, 1 << N, size=8 * threads, dtype=np.int64).astype(np.uint32)
    t0 = time.time()
    oracle.formula_masks(A, probe, loops=loops, prec="ld", threads=threads)
    dt = max(time.time() - t0, 1e-3)
    count = int(max(8 * threads, min(2_000_000, len(probe) * seconds_target / dt)))
    masks = rng.integers(1, 1 << N, size=count, dtype=np.int64).astype(np.uint32)
    t0 = time.time()
    oracle.formula_masks(A, masks, loops=loops, prec="ld", threads=threads)
    dt = time.time() - t0
    return {"value": count / dt, "unit": "subset-terms/s", "cores": threads, "kind": "oracle",
            "sample": "%d uniformly random subsets of the %dx%d matrix (%s), long double, %.1f s" % (
                count, n, n, "lhaf" if loops else "haf", dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=56)
    ap.add_argument("--kind", choices=["haf", "lhaf"], default="haf")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--kernel-path", type=int, default=0)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(each GPU would own a share of the subset ranks; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1805_12498_amd as hg
    from gen import inputs as gi

    n, kind = args.n, (hg.KIND_LHAF if args.kind == "lhaf" else hg.KIND_HAF)
    seed = {56: gi.SEED_N56, 40: gi.SEED_N40, 16: gi.SEED_N16}.get(n, 5600 + n)
    A = gi.gaussian_symmetric(n, seed)
    torch.cuda.init()
    dA = torch.from_numpy(A).cuda()
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    hg.set_kernel_path(args.kernel_path)
    log("device:", hg.device_info())

    def step():
        hg.haf_dev(dA.data_ptr(), n, n, out.data_ptr(), stream.cuda_stream, kind=kind, x2=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    hg.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = hg.profile_read()
    hg.profile_enable(False)
    res = out.cpu().numpy()
    log("result:", complex(res[0] + res[1], res[2] + res[3]))

    secs = t1 - t0
    terms = float((1 << (n // 2)) * args.steps)
    achieved = prof["coef_model_flops"] / (prof["coef_ms"] * 1e-3) / 1e12 if prof["coef_ms"] > 0 else 0.0
    per_launch_ms = prof["coef_ms"] / max(prof["coef_launches"], 1)
    log("coefficient kernel: %d launches, %.3f ms total, %.4f ms/launch, %.3g model flops, series %.3f ms" % (
        prof["coef_launches"], prof["coef_ms"], per_launch_ms, prof["coef_model_flops"], prof["series_ms"]))
    line = {
        "metric": "subset-terms/s",
        "value": terms / secs,
        "unit": "subset-terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": secs / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s of a %dx%d complex Gaussian symmetric matrix A=(G+G^T)/2, seed %d, "
                               "2^%d subset terms per step" % (args.kind, n, n, seed, n // 2),
                   "n": n, "kind": args.kind, "subsets_per_step": 1 << (n // 2)},
        "roofline": {
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_FP64_TFLOPS,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": None,
            "kernel": "coefficient kernel (per-subset Hessenberg + characteristic polynomial)",
            "model": "(44/3) s^3 flops per subset of size s (+ 8 (N-1) s^2 for loop hafnians)",
            "launches": prof["coef_launches"],
            "avg_launch_ms": per_launch_ms,
            "share_of_step": prof["coef_ms"] * 1e-3 / secs,
        },
        "fp64_model_tflops_step": prof["coef_model_flops"] / secs / 1e12,
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(A, n, kind == hg.KIND_LHAF, args.cpu_seconds)
        line["cpu_baseline"]["gpu_over_cpu"] = line["value"] / line["cpu_baseline"]["value"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
