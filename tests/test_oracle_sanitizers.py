"""The oracle's C under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

oracle/haf_oracle.c is compiled with gcc -fsanitize=address,undefined together
with a small driver (tests/oracle_sanitizer_driver.c) that calls every exported
routine: brute force (complex and integer), the formula in all four precisions
with and without loops, single terms, mask lists, Ryser, and the sums over F_p.
The run must end cleanly (any sanitizer report aborts it) and print the same
values as the ordinary build of the oracle on the same inputs and thread counts.
"""
import ctypes
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest

import oracle
from gen import inputs as gi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DRIVER = os.path.join(ROOT, "tests", "oracle_sanitizer_driver.c")
SOURCE = os.path.join(ROOT, "oracle", "haf_oracle.c")

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")


@pytest.fixture(scope="module")
def sanitized(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("asan") / "oracle_asan")
    cmd = ["gcc", "-O1", "-g", "-std=gnu11", "-fopenmp", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I" + os.path.join(ROOT, "oracle"), "-o", exe, DRIVER, SOURCE, "-lquadmath", "-lm"]
    subprocess.run(cmd, check=True, cwd=os.path.join(ROOT, "oracle"), capture_output=True, text=True)
    return exe


def inputs():
    A = np.ascontiguousarray(gi.gaussian_symmetric(10, 71))
    G = np.ascontiguousarray(gi.random_graph(12, 0.5, 72).real.astype(np.int64))
    G[np.arange(12), np.arange(12)] = np.arange(12) % 3        # integer loop weights
    W = np.ascontiguousarray(gi.gaussian_square(6, 73))
    return A, G, W


def write_input(path, A, G, W):
    with open(path, "wb") as f:
        f.write(struct.pack("<i", A.shape[0]) + A.astype(np.complex128).tobytes())
        f.write(struct.pack("<i", G.shape[0]) + G.astype(np.int64).tobytes())
        f.write(struct.pack("<i", W.shape[0]) + W.astype(np.complex128).tobytes())


def reference_lines(A, G, W):
    """The same calls on the ordinary build, printed the same way."""
    lib = oracle._load()
    dp = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))  # noqa: E731
    ip = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))  # noqa: E731
    up = lambda x: x.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))  # noqa: E731
    n, g, k = A.shape[0], G.shape[0], W.shape[0]
    N = n // 2
    f4 = lambda tag, a, b, r: "%s %d %d %s" % (tag, a, b, " ".join("%.17g" % v for v in r))  # noqa: E731
    out = []
    r = np.zeros(4)
    ab = np.zeros(1)
    for loops in (0, 1):
        assert lib.orc_brute(dp(A), n, loops, dp(r)) == 0
        out.append(f4("brute", loops, 0, r))
        for prec in range(4):
            assert lib.orc_formula_range(dp(A), n, loops, prec, ctypes.c_uint64(1), ctypes.c_uint64(1 << N), 2,
                                         dp(r), dp(ab)) == 0
            out.append(f4("formula", loops, prec, r))
            out.append("absum %d %d %.17g" % (loops, prec, ab[0]))
            assert lib.orc_term(dp(A), n, loops, prec, ctypes.c_uint32((1 << N) - 1 - 2), dp(r)) == 0
            out.append(f4("term", loops, prec, r))
        masks = np.array([1, 3, 6, (1 << N) - 1, 5], dtype=np.uint32)
        assert lib.orc_formula_masks(dp(A), n, loops, 1, masks.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
                                     ctypes.c_int64(5), 2, dp(r)) == 0
        out.append(f4("masks", loops, 1, r))
        bi = np.zeros(2, dtype=np.uint64)
        assert lib.orc_brute_int(ip(G), g, loops, up(bi)) == 0
        out.append("brute_int %d %d %d" % (loops, int(bi[0]), int(bi[1])))
        v = np.zeros(1, dtype=np.uint64)
        assert lib.orc_modp(ip(G), g, loops, ctypes.c_uint64(2147483647), 2, up(v)) == 0
        out.append("modp %d %d" % (loops, int(v[0])))
        assert lib.orc_modp_term(ip(G), g, loops, ctypes.c_uint64(2147483629), ctypes.c_uint32(5), up(v)) == 0
        out.append("modp_term %d %d" % (loops, int(v[0])))
    for prec in range(4):
        assert lib.orc_ryser(dp(W), k, prec, 2, dp(r)) == 0
        out.append(f4("ryser", prec, 0, r))
    return out


def test_oracle_clean_under_sanitizers(sanitized, tmp_path):
    A, G, W = inputs()
    path = str(tmp_path / "input.bin")
    write_input(path, A, G, W)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    p = subprocess.run([sanitized, path], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0, p.stderr[-3000:]
    assert "Sanitizer" not in p.stderr and "runtime error" not in p.stderr, p.stderr[-3000:]
    got = p.stdout.strip().splitlines()
    want = reference_lines(A, G, W)
    assert got == want


def test_sanitizers_catch_a_planted_overrun(tmp_path):
    """The harness itself works: an out-of-bounds read in a copy of the driver is reported."""
    src = tmp_path / "bad.c"
    src.write_text("#include <stdlib.h>\nint main(void) { int* p = malloc(4 * sizeof(int)); int s = p[4];"
                   " free(p); return s == 12345; }\n")
    exe = str(tmp_path / "bad")
    subprocess.run(["gcc", "-O0", "-g", "-fsanitize=address", "-o", exe, str(src)], check=True)
    p = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert p.returncode != 0 and "heap-buffer-overflow" in p.stderr
