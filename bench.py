"""Benchmark: subset-terms/s of one 56x56 hafnian on one MI355X, plus the
batched and serving throughput against the plain one-hafnian-per-call path.

A step is one complete hafnian of the 56x56 complex Gaussian symmetric matrix
(seed 5601): all 2^28 subset terms (gather, Hessenberg reduction,
characteristic polynomial, power traces, series) and the signed double-double
sum, with the matrix already resident in device memory.  The printed JSON line
carries the throughput, the roofline position of the dominant kernel (the
per-subset coefficient kernel, timed with HIP events on its own stream inside
the timed region), the CPU oracle timed on a bounded sample, and two extra
objects measured after the timed steps:

  batched  4096 GBS-style loop hafnians, n in [8, 32] (seed 4096), one batched
           call (after the autotuner) versus 4096 single-matrix calls on one
           stream; haf/s of each and whether every result agrees bitwise;
  serving  a Poisson stream of haf / lhaf requests, n in [12, 44] with
           geometric skew (seed 2027), replayed open-loop through the
           continuous-batching server and through the plain server (one
           request at a time), at a rate set from the plain server's measured
           capacity; p50 / p99 latency (completion minus arrival) and haf/s.

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

# Counter figures of the coefficient kernel at n = 56 (haf), valid only while the
# kernel's sources are the ones the counters were taken on (sha256 below):
#  * HBM bytes per launch, from rocprofv3 FETCH_SIZE and WRITE_SIZE runs calibrated
#    against a 1 GiB device copy (profiles/coef_kernel_n56_haf_hbm_traffic.md);
#  * FP64 flops per step as the SQ counters count them, 64 x (ADD_F64 + MUL_F64 +
#    TRANS_F64 + 2 FMA_F64) wave instructions, which ignore the exec mask
#    (profiles/coef_kernel_n56_haf_sq_counters.md).
COUNTER_SOURCES = ("paper_1805_12498_amd/csrc/haf_coef_reg.hpp", "paper_1805_12498_amd/csrc/haf_kernels_reg.hip",
                   "paper_1805_12498_amd/csrc/haf_common.hpp")
COUNTER_SHA256 = "f9ce639779121b2f3215a01f5ce5d825a3eec39f9b9c92442ec4843992a64f5c"
TRAFFIC_N56_HAF_BYTES_PER_LAUNCH = 9.251e8
COUNTER_N56_HAF_FP64_FLOPS_PER_STEP = 2.042e14


def counters_valid(n, kind):
    import hashlib
    if n != 56 or kind != "haf":
        return False
    h = hashlib.sha256()
    for f in COUNTER_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest() == COUNTER_SHA256


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(A, n, loops, seconds_target=15.0):
    """The CPU oracle's formula route (explicit matrix powers) instantiated on double,
    on a uniform random sample of subsets of the same matrix, scaled to subset-terms/s."""
    import numpy as np

    import oracle
    N = n // 2
    threads = os.cpu_count() or 1
    rng = np.random.default_rng(12345)
    probe = rng.integers(1, 1 << N, size=64 * threads, dtype=np.int64).astype(np.uint32)
    t0 = time.time()
    oracle.formula_masks(A, probe, loops=loops, prec="d", threads=threads)
    dt = max(time.time() - t0, 1e-3)
    count = int(max(64 * threads, min(20_000_000, len(probe) * seconds_target / dt)))
    masks = rng.integers(1, 1 << N, size=count, dtype=np.int64).astype(np.uint32)
    t0 = time.time()
    oracle.formula_masks(A, masks, loops=loops, prec="d", threads=threads)
    dt = time.time() - t0
    return {"value": count / dt, "unit": "subset-terms/s", "cores": threads, "kind": "oracle",
            "cpu": cpu_model(),
            "sample": "%d uniformly random subsets of the %dx%d matrix (%s), the oracle's formula route "
                      "(explicit matrix powers) in double, %.1f s on %d threads" % (
                          count, n, n, "lhaf" if loops else "haf", dt, threads)}


def gold_values():
    path = os.path.join(ROOT, "tests", "golden", "oracle_values.json")
    return json.load(open(path)) if os.path.exists(path) else {}


def gold_hp(g, name):
    import oracle
    v = g[name]["value"]
    return oracle.HighPrec((v["re"][0], v["re"][1], v["im"][0], v["im"][1]))


def bench_configs(hg, gi):
    """Timing and relative error of every configuration besides the headline one."""
    import numpy as np
    import torch

    g = gold_values()
    st = torch.cuda.current_stream()
    out = {}
    dout = torch.zeros(4, dtype=torch.float64, device="cuda")

    def timed(fn, reps):
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return np.array(ts)

    def result():
        r = dout.cpu().numpy()
        return complex(r[0] + r[1], r[2] + r[3])

    # C1: one 16x16 hafnian per call, latency distribution of the plain path
    A = gi.gaussian_symmetric(16, gi.SEED_N16)
    dA = torch.from_numpy(A).cuda()
    fn = lambda: hg.haf_dev(dA.data_ptr(), 16, 16, dout.data_ptr(), st.cuda_stream, kind=0, x2=True)  # noqa: E731
    timed(fn, 20)
    ts = timed(fn, 1000)
    c1 = {"workload": "haf of the 16x16 Gaussian matrix, seed 1601, 2^8 subsets, one call at a time",
          "p10_ms": float(np.percentile(ts, 10) * 1e3), "p50_ms": float(np.median(ts) * 1e3),
          "p90_ms": float(np.percentile(ts, 90) * 1e3), "calls": len(ts)}
    if "n16_haf" in g:
        c1["relerr"] = gold_hp(g, "n16_haf").relerr(result())
        c1["relerr_vs"] = "oracle formula route in binary128"
    out["C1_n16_haf"] = c1
    log("C1:", c1)

    # C2: 40x40, haf and lhaf, double and per-term double-double
    A = gi.gaussian_symmetric(40, gi.SEED_N40)
    dA = torch.from_numpy(A).cuda()
    for kind, name in ((0, "haf"), (1, "lhaf")):
        fn = lambda: hg.haf_dev(dA.data_ptr(), 40, 40, dout.data_ptr(), st.cuda_stream, kind=kind, x2=True)  # noqa: E731
        timed(fn, 2)
        ts = timed(fn, 30)
        c2 = {"workload": "%s of the 40x40 Gaussian matrix, seed 4001, 2^20 subsets" % name,
              "ms_median": float(np.median(ts) * 1e3), "subset_terms_per_s": (1 << 20) / float(np.median(ts))}
        key = "n40_" + name
        if key in g:
            c2["relerr"] = gold_hp(g, key).relerr(result())
            c2["kappa"] = g[key]["kappa"]
            c2["relerr_vs"] = "oracle formula route in double-double"
        fdd = lambda: hg.haf_dev_dd(dA.data_ptr(), 40, 40, dout.data_ptr(), st.cuda_stream, kind=kind)  # noqa: E731
        ts = timed(fdd, 3)
        c2["dd_mode_ms_median"] = float(np.median(ts) * 1e3)
        if key in g:
            import oracle
            r = dout.cpu().numpy()
            c2["dd_mode_relerr"] = gold_hp(g, key).relerr_hp(oracle.HighPrec(tuple(float(x) for x in r)))
        out["C2_n40_" + name] = c2
        log("C2 %s:" % name, c2)

    # C3b: the 56-vertex 0/1 graph, double path and the exact modular path
    G = gi.random_graph(56, 0.5, gi.SEED_N56_GRAPH)
    dA = torch.from_numpy(G.astype(np.complex128)).cuda()
    fn = lambda: hg.haf_dev(dA.data_ptr(), 56, 56, dout.data_ptr(), st.cuda_stream, kind=0, x2=True)  # noqa: E731
    ts = timed(fn, 1)
    c3b = {"workload": "haf of the 56-vertex 0/1 graph G(56, 1/2), seed 5602, 2^28 subsets",
           "ms": float(ts[0] * 1e3), "subset_terms_per_s": (1 << 28) / float(ts[0])}
    got = result()
    t0 = time.perf_counter()
    exact = hg.haf_exact(G, 0)
    c3b["exact_path_s"] = time.perf_counter() - t0
    c3b["exact_path_value"] = str(exact)
    if "n56_graph_exact" in g:
        ref = int(g["n56_graph_exact"]["exact"])
        c3b["exact_path_equals_oracle"] = exact == ref
        c3b["relerr"] = abs(complex(got) - ref) / ref
        c3b["relerr_vs"] = "the oracle's exact count (sum over F_p for four 31-bit primes, CRT, and a check prime)"
    else:
        c3b["relerr_vs_exact_path"] = abs(complex(got) - exact) / abs(exact)
    out["C3b_n56_graph"] = c3b
    log("C3b:", c3b)
    return out


def bench_batched(hg, gi, count=4096):
    """One batched call over the GBS-style batch versus the plain path, one call per matrix."""
    import numpy as np
    import torch

    mats = gi.gbs_batch(count, seed=gi.SEED_BATCH)
    flat, offs, sizes = gi.pack(mats)
    kinds = np.ones(count, dtype=np.uint8)
    dA = torch.from_numpy(flat).cuda()
    out_b = torch.zeros(count, dtype=torch.complex128, device="cuda")
    out_p = torch.zeros(count, dtype=torch.complex128, device="cuda")
    stream = torch.cuda.current_stream()
    cfg, tune_ms = hg.batched_tune(dA.data_ptr(), offs, sizes, kinds, out_b.data_ptr(), stream.cuda_stream)
    log("batched autotuner:", cfg, "%.1f ms" % tune_ms)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hg.batched_dev(dA.data_ptr(), offs, sizes, kinds, out_b.data_ptr(), stream.cuda_stream)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    base = dA.data_ptr()
    for t in range(min(count, 64)):       # warm the single-matrix path's workspaces
        hg.haf_dev(base + 16 * int(offs[t]), int(sizes[t]), int(sizes[t]), out_p.data_ptr() + 16 * t,
                   stream.cuda_stream, kind=1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(count):
        hg.haf_dev(base + 16 * int(offs[t]), int(sizes[t]), int(sizes[t]), out_p.data_ptr() + 16 * t,
                   stream.cuda_stream, kind=1)
    torch.cuda.synchronize()
    t_p = time.perf_counter() - t0
    same = bool(torch.equal(torch.view_as_real(out_b), torch.view_as_real(out_p)))
    terms = int(sum(1 << (int(n) // 2) for n in sizes))
    return {"workload": "%d loop hafnians of GBS-style submatrices, n in [8, 32] (mean %.1f), seed %d"
                        % (count, float(np.mean(sizes)), gi.SEED_BATCH),
            "haf_per_s": count / t_b, "ms": t_b * 1e3, "subset_terms_per_s": terms / t_b,
            "plain_haf_per_s": count / t_p, "plain_ms": t_p * 1e3, "speedup_vs_plain": t_p / t_b,
            "bitwise_equal_to_plain": same, "tuned_config": cfg}


def replay(hg, trace, t_offset, **cfg):
    """Open-loop replay: submit each request at its arrival time; latency = done - arrival."""
    import numpy as np

    srv = hg.Server(**cfg)
    try:
        start = hg.now() + t_offset
        arrival = {}
        results = []
        for t_arr, kind, A in trace:
            target = start + t_arr
            while True:
                now = hg.now()
                if now >= target:
                    break
                if target - now > 2e-3:
                    time.sleep(min(target - now - 1e-3, 0.05))
                results.extend(srv.poll(4096))
            arrival[srv.submit(A, kind)] = target
        srv.drain()
        results.extend(srv.poll(len(trace) + 10))
        end = hg.now()
    finally:
        srv.close()
    lat = np.array([r.t_done - arrival[r.ticket] for r in results])
    assert all(r.status == 0 for r in results) and len(results) == len(trace)
    span = end - start
    # latency histogram: counts per power-of-two bucket of milliseconds, [2^(k-1), 2^k) for key 2^k
    edges = 2.0 ** np.arange(-6, 12)
    counts = np.histogram(lat * 1e3, bins=np.concatenate(([0.0], edges, [np.inf])))[0]
    hist = {("<%g" % e if k < len(edges) else ">=%g" % edges[-1]): int(c)
            for k, (e, c) in enumerate(zip(list(edges) + [np.inf], counts)) if c}
    return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3), "haf_per_s": len(trace) / span, "requests": len(trace),
            "seconds": span, "latency_ms_histogram": hist}


def bench_serving(hg, gi, min_requests=10000):
    """Capacities of the plain and the continuous server (closed loop), then two open-loop
    Poisson streams replayed through both: Q1 = half the plain server's capacity (both
    stable) and Q2 = 0.8 of the continuous server's capacity (the plain server saturates)."""
    probe = gi.serving_trace(600, qps=1e9, seed=gi.SEED_SERVE + 1)
    plain_cap = replay(hg, probe, 0.0, continuous=0)["haf_per_s"]
    cont_cap = replay(hg, probe, 0.0, continuous=1)["haf_per_s"]
    points = {}
    for name, qps in (("Q1", 0.5 * plain_cap), ("Q2", 0.8 * cont_cap)):
        trace = gi.serving_trace(min_requests, qps=qps, seed=gi.SEED_SERVE)
        cont = replay(hg, trace, 0.05, continuous=1)
        plain = replay(hg, trace, 0.05, continuous=0)
        points[name] = {"qps": qps, "continuous": cont, "plain": plain}
        log("serving %s at %.0f req/s: continuous p50/p99 %.2f/%.2f ms (%.0f haf/s), plain %.2f/%.2f ms (%.0f haf/s)"
            % (name, qps, cont["p50_ms"], cont["p99_ms"], cont["haf_per_s"], plain["p50_ms"], plain["p99_ms"],
               plain["haf_per_s"]))
    return {"workload": "Poisson arrivals, haf/lhaf 50/50, n = 12 + 2j with P(j) ~ 0.7^j up to 44, "
                        "GBS-style submatrices, seed %d, %d requests per point" % (gi.SEED_SERVE, min_requests),
            "capacity_haf_per_s": {"continuous": cont_cap, "plain": plain_cap}, **points}


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
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-configs", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=10000)
    ap.add_argument("--jsonl", default=None,
                    help="append the result line, with run metadata, to this JSON-lines file")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(each GPU would own a share of the subset ranks)", file=sys.stderr)
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
            "traffic": TRAFFIC_N56_HAF_BYTES_PER_LAUNCH if counters_valid(n, args.kind) else None,
            "traffic_unit": "bytes per launch",
            "kernel": "coefficient kernel (per-subset Hessenberg + characteristic polynomial)",
            "model": "(44/3) s^3 flops per subset of size s (+ 8 (N-1) s^2 for loop hafnians)",
            "launches": prof["coef_launches"],
            "avg_launch_ms": per_launch_ms,
            "share_of_step": prof["coef_ms"] * 1e-3 / secs,
        },
        "fp64_model_tflops_step": prof["coef_model_flops"] / secs / 1e12,
        "fp64_counter": ({"flops_per_step": COUNTER_N56_HAF_FP64_FLOPS_PER_STEP,
                          "tflops": COUNTER_N56_HAF_FP64_FLOPS_PER_STEP / (secs / args.steps) / 1e12,
                          "frac_of_peak": COUNTER_N56_HAF_FP64_FLOPS_PER_STEP / (secs / args.steps) / 1e12
                          / PEAK_FP64_TFLOPS,
                          "note": "SQ_INSTS_VALU_{ADD,MUL,TRANS,FMA}_F64 wave instructions x 64 lanes (exec mask "
                                  "ignored), per step, from the profile of this kernel source"}
                         if counters_valid(n, args.kind) else None),
        "cpu_baseline": None,
    }
    if not args.no_configs:
        line["configs"] = bench_configs(hg, gi)
    if not args.no_batched:
        line["batched"] = bench_batched(hg, gi)
    if not args.no_serving:
        line["serving"] = bench_serving(hg, gi, args.serve_requests)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(A, n, kind == hg.KIND_LHAF, args.cpu_seconds)
        line["cpu_baseline"]["gpu_over_cpu"] = line["value"] / line["cpu_baseline"]["value"]
    print(json.dumps(line), flush=True)
    if args.jsonl:
        append_jsonl(args.jsonl, line, A, hg, vars(args))


def append_jsonl(path, line, A, hg, args):
    """One record per run: the result line plus when, where and on what it ran."""
    import hashlib
    import platform
    import subprocess
    rec = dict(line)
    rec["run"] = {
        "utc": time.strftime("%Y-%m-%dT%H:%M:%SZ", time.gmtime()),
        "args": args,
        "input_sha256": hashlib.sha256(A.tobytes()).hexdigest(),
        "device": hg.device_info(),
        "host": {"cpu": cpu_model(), "threads": os.cpu_count(), "python": platform.python_version()},
    }
    try:
        rec["run"]["commit"] = subprocess.run(["git", "rev-parse", "HEAD"], cwd=ROOT, capture_output=True,
                                              text=True, timeout=10).stdout.strip() or None
    except (OSError, subprocess.SubprocessError):
        rec["run"]["commit"] = None
    with open(path, "a") as f:
        f.write(json.dumps(rec) + "\n")


if __name__ == "__main__":
    main()
