"""GPU tests of the exact integer path (haf_exact_i64, haf_modp_c) through the C ABI.

The subset sum of Sec. 3.2 runs modulo primes below 2^25 on the GPU and the
integer comes back by Chinese remaindering on the host.  Checks, all exact:
  * residues bit for bit against the oracle's own sum over F_p (its Gaussian
    elimination, polynomial recurrence, Newton and series over the field) for
    random integer matrices with negative entries, both kinds, odd n;
  * exact values against brute-force matching enumeration (128-bit integers);
  * closed forms at sizes far beyond double precision: (n-1)!! for K_n, T(n)
    for lhaf(J_n), (n/2)! for complete bipartite graphs, rank-1 integer
    matrices, and the 7 x 8 grid (56 vertices, Kasteleyn's product formula),
    whose 2^28-term sum cancels by a factor of about 7e18, far out of reach of
    a complex-double chain;
  * the 56-vertex random graph of edge probability 1/2 (seed 5602) against the
    oracle's exact count, when it has been computed and stored;
  * errors.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
from gen import inputs as gi
from oracle import closed_forms as cf

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")))


def is_prime(p):
    if p < 2:
        return False
    d = 2
    while d * d <= p:
        if p % d == 0:
            return False
        d += 1
    return True


def primes_below(limit, k):
    out, p = [], limit - 1
    while len(out) < k:
        if is_prime(p):
            out.append(p)
        p -= 1
    return out


PRIMES = primes_below(1 << 25, 3) + [40009, 104729]


@pytest.fixture(scope="module")
def hg():
    import paper_1805_12498_amd as hg
    hg.load()
    return hg


def rand_int_sym(n, seed, lo=-3, hi=3):
    rng = np.random.default_rng(seed)
    A = rng.integers(lo, hi + 1, (n, n))
    return np.triu(A) + np.triu(A, 1).T


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 10, 13, 16, 20, 24])
@pytest.mark.parametrize("kind", [0, 1])
def test_residues_vs_oracle(hg, n, kind):
    A = rand_int_sym(n, 100 * n + kind)
    got = hg.haf_modp(A, PRIMES, kind)
    if n % 2 and kind == 0:
        assert got == [0] * len(PRIMES)
        return
    B = A
    if n % 2:
        B = np.zeros((n + 1, n + 1), dtype=np.int64)
        B[:n, :n] = A
        B[n, n] = 1
    ref = [oracle.modp(B, p, bool(kind)) for p in PRIMES]
    assert got == ref, (n, kind, got, ref)


@pytest.mark.parametrize("n", [0, 1, 2, 5, 6, 9, 12, 15, 18, 20])
@pytest.mark.parametrize("kind", [0, 1])
def test_exact_vs_brute_force(hg, n, kind):
    A = rand_int_sym(n, 300 + 2 * n + kind, -5, 5)
    got = hg.haf_exact(A, kind)
    ref = 1 if n == 0 else oracle.brute_int(A, bool(kind))
    assert got == ref, (n, kind, got, ref)


@pytest.mark.parametrize("n", [24, 32, 40])
def test_exact_closed_forms(hg, n):
    J = np.ones((n, n), dtype=np.int64)
    assert hg.haf_exact(J - np.eye(n, dtype=np.int64), 0) == cf.haf_complete(n)
    assert hg.haf_exact(J, 1) == cf.telephone(n)
    assert hg.haf_exact(J[:n - 1, :n - 1], 1) == cf.telephone(n - 1)        # odd n: padded
    assert hg.haf_exact(gi.complete_bipartite(n).real.astype(np.int64), 0) == math.factorial(n // 2)
    v = np.arange(1, n + 1, dtype=np.int64) % 7 - 3
    v[v == 0] = 2
    R = np.outer(v, v)
    assert hg.haf_exact(R, 0) == cf.double_factorial(n - 1) * math.prod(int(x) for x in v)


def test_grid_7x8_exact(hg):
    """Perfect matchings of the 7 x 8 grid (56 vertices, 2^28 subsets): Kasteleyn's count."""
    G = gi.grid_graph(7, 8).real.astype(np.int64)
    assert hg.haf_exact(G, 0) == cf.grid_perfect_matchings(7, 8)


def test_random_graph_n56_exact(hg):
    """The 56-vertex 0/1 graph, edge probability 1/2, seed 5602: the exact matching count
    against the oracle's (its own sum over four 31-bit primes plus a check prime, CRT; the
    product of the four bounds the count of any 56-vertex graph, 55!! < 2^123)."""
    if "n56_graph_exact" not in GOLD:
        pytest.skip("the oracle's exact count of G(56, 1/2) seed 5602 is not stored yet")
    G = gi.random_graph(56, 0.5, gi.SEED_N56_GRAPH).real.astype(np.int64)
    assert hg.haf_exact(G, 0) == int(GOLD["n56_graph_exact"]["exact"])


def test_exact_errors(hg):
    from paper_1805_12498_amd._native import HafError
    A = rand_int_sym(6, 1)
    B = A.copy()
    B[0, 1] += 1
    with pytest.raises(HafError, match="NOT_SYMMETRIC"):
        hg.haf_exact(B, 0)
    with pytest.raises(HafError, match="INVALID_ARG"):
        hg.haf_modp(A, [33554432], 0)                      # 2^25: not a prime below 2^25
    with pytest.raises(HafError, match="INVALID_ARG"):
        hg.haf_modp(A, [7], 0)                             # p <= n + 1
    with pytest.raises(HafError, match="INVALID_ARG"):
        hg.haf_modp(A, [40009, 40011], 0)                  # 40011 = 3 x 13337
    with pytest.raises(HafError, match="TOO_LARGE"):
        hg.haf_exact(rand_int_sym(16, 2) * (1 << 40), 0)   # bound beyond ten primes
    with pytest.raises(HafError, match="TOO_LARGE"):
        hg.haf_exact(np.ones((66, 66), dtype=np.int64), 0)
    # a diagonal is ignored by haf and needs no symmetry partner
    D = rand_int_sym(8, 3)
    D2 = D.copy()
    np.fill_diagonal(D2, 1000)
    assert hg.haf_exact(D, 0) == hg.haf_exact(D2, 0) == oracle.brute_int(D, False)
