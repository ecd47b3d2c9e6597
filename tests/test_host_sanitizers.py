"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The host side of every source (no device code) is built with the sanitizers and
loaded, with the sanitizer runtime preloaded, into a child Python process that
drives the host-only logic through the ordinary binding: the batched planner on
many random batches, the batched configuration and its checks, the autotune
cache loader, the server configuration from the environment, and the argument
and value checks of the entry points (which reject before any device work).
Any sanitizer report ends the child with an error.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r'''
import os, sys
import numpy as np
sys.path.insert(0, os.environ["HAF_ROOT"])
import paper_1805_12498_amd._native as nat
lib = nat.load(os.environ["HAF_ASAN_LIB"])          # the sanitized build, before anything loads the other
assert lib._name == os.environ["HAF_ASAN_LIB"], lib._name
import paper_1805_12498_amd as hg
HafError = nat.HafError

rng = np.random.default_rng(2024)
plans = 0
for trial in range(300):
    count = int(rng.integers(0, 200))
    sizes = rng.integers(0, 65, size=count).astype(np.int32)
    kinds = rng.integers(0, 2, size=count).astype(np.uint8)
    if trial % 3 == 0:
        hg.set_batched_config(table=int(rng.integers(0, 2)), span=int(rng.integers(1, 65)),
                              streams=int(rng.integers(1, 5)), grouped=int(rng.integers(0, 2)),
                              coef_budget_mb=int(rng.choice([64, 256, 8192])))
    launches, chunks = hg.batched_plan(sizes, kinds)
    plans += 1
for bad in (dict(table=2), dict(span=0), dict(span=65), dict(streams=0), dict(streams=9), dict(grouped=3),
            dict(coef_budget_mb=1)):
    cfg = dict(table=0, span=4, streams=4, grouped=1, coef_budget_mb=8192)
    cfg.update(bad)
    try:
        hg.set_batched_config(**cfg)
        raise SystemExit("accepted %r" % bad)
    except HafError:
        pass
try:
    hg.batched_plan(np.array([66], np.int32), np.array([0], np.uint8))
    raise SystemExit("accepted n = 66")
except HafError:
    pass

os.environ.pop("HAF_AUTOTUNE_CACHE", None)
try:
    hg.batched_load_cache()
    raise SystemExit("cache loader without its variable")
except HafError:
    pass

for v in ("1", "64K", "3M", "1G", "", "x", "-5"):
    os.environ["HAF_ARENA_BYTES"] = v
    c = nat.ServerConfig()
    lib.haf_server_default_config(nat.ctypes.byref(c))
    assert c.arena_bytes > 0

A = np.ones((6, 6), complex)
B = A.copy(); B[0, 1] = 2.0
C = A.copy(); C[2, 2] = np.nan
for M, kind in ((B, 0), (C, 1), (np.ones((65, 65), complex), 0)):
    try:
        hg.haf_host(M, kind)
        raise SystemExit("accepted a bad matrix")
    except HafError:
        pass
print("host paths ok", plans, flush=True)
'''


@pytest.fixture(scope="module")
def sanitized_lib(tmp_path_factory):
    sys.path.insert(0, ROOT)
    from paper_1805_12498_amd import build
    rt = build.asan_runtime()
    if not rt:
        pytest.skip("no AddressSanitizer runtime next to the compiler")
    lib = build.build_host_sanitized(str(tmp_path_factory.mktemp("host_asan")))
    return lib, rt


def test_host_code_clean_under_sanitizers(sanitized_lib):
    lib, rt = sanitized_lib
    env = dict(os.environ, LD_PRELOAD=rt, HAF_ASAN_LIB=lib, HAF_ROOT=ROOT,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    p = subprocess.run([sys.executable, "-c", CHILD], capture_output=True, text=True, timeout=600, env=env)
    assert p.returncode == 0, (p.stdout[-2000:], p.stderr[-4000:])
    assert "AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr, p.stderr[-4000:]
    assert "host paths ok 300" in p.stdout
