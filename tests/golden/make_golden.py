"""Write the stored oracle values the GPU parity tests compare against.

Calls only ``oracle`` and ``gen`` (never the GPU library).  Usage:

    python tests/golden/make_golden.py [name ...]

Each entry of ``oracle_values.json`` records the workload, the value as
(hi, lo) doubles per component, kappa = sum_Z |f(Z)| / |value| where the
formula route was used, the oracle route and precision, wall time and the host.
"""
from __future__ import annotations

import json
import os
import platform
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from gen import inputs as gi  # noqa: E402

OUT = os.path.join(HERE, "oracle_values.json")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def hp_dict(r):
    return {"re": [r.re_hi, r.re_lo], "im": [r.im_hi, r.im_lo]}


def formula_entry(A, loops, prec, what):
    t0 = time.time()
    r, kappa = oracle.formula(A, loops, prec=prec, want_kappa=True)
    return {"what": what, "route": "formula/explicit powers", "prec": prec, "value": hp_dict(r),
            "kappa": kappa, "seconds": time.time() - t0}


def ryser_entry(W, prec, what):
    t0 = time.time()
    r = oracle.ryser(W, prec=prec)
    return {"what": what, "route": "ryser (bipartite identity)", "prec": prec, "value": hp_dict(r),
            "seconds": time.time() - t0}


def exact_entry(A, loops, what, nprimes):
    # Many more threads than cores: the static split of the mask range gives the
    # ranges with high leading bits larger subsets, so fine ranges balance the load.
    # The sum mod p is exact, so the thread count does not change the value.
    threads = 8 * (os.cpu_count() or 1)
    v, sec = oracle.exact_int(A, loops, nprimes=nprimes, threads=threads)
    return {"what": what, "route": "formula over F_p + CRT", "primes": nprimes + 1, "exact": str(v),
            "seconds": sec, "threads": threads}


JOBS = {
    "n16_haf": lambda: formula_entry(gi.gaussian_symmetric(16, gi.SEED_N16), False, "q",
                                     "haf, 16x16 Gaussian symmetric, seed 1601"),
    "n16_lhaf": lambda: formula_entry(gi.gaussian_symmetric(16, gi.SEED_N16), True, "q",
                                      "lhaf, 16x16 Gaussian symmetric, seed 1601"),
    "n40_haf": lambda: formula_entry(gi.gaussian_symmetric(40, gi.SEED_N40), False, "dd",
                                     "haf, 40x40 Gaussian symmetric, seed 4001"),
    "n40_lhaf": lambda: formula_entry(gi.gaussian_symmetric(40, gi.SEED_N40), True, "dd",
                                      "lhaf, 40x40 Gaussian symmetric, seed 4001"),
    "n40_haf_ld": lambda: formula_entry(gi.gaussian_symmetric(40, gi.SEED_N40), False, "ld",
                                        "haf, 40x40 Gaussian symmetric, seed 4001 (long double cross-check)"),
    "n56_bipartite": lambda: ryser_entry(gi.gaussian_square(28, gi.SEED_N56_BIPARTITE), "dd",
                                         "haf([[0,W],[W^T,0]]) = per(W), W 28x28 Gaussian, seed 5603"),
    "n56_graph_exact": lambda: exact_entry(gi.random_graph(56, 0.5, gi.SEED_N56_GRAPH), False,
                                           "haf, 56x56 0/1 adjacency of G(56, 1/2), seed 5602", 4),
}


def main(names):
    data = {}
    if os.path.exists(OUT):
        data = json.load(open(OUT))
    for name in names or [k for k in JOBS if k != "n56_graph_exact"]:
        print("computing", name, flush=True)
        e = JOBS[name]()
        e["host"] = {"cpu": cpu_model(), "threads": os.cpu_count()}
        data[name] = e
        # re-read so concurrent runs for different names do not drop each other's entries
        cur = json.load(open(OUT)) if os.path.exists(OUT) else {}
        cur[name] = e
        with open(OUT + ".tmp", "w") as f:
            json.dump(cur, f, indent=1, sort_keys=True)
        os.replace(OUT + ".tmp", OUT)
        print(name, json.dumps(e), flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
