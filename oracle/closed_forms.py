"""Closed-form and combinatorial values used to pin the oracle (test infrastructure).

Every value here is exact (Python integers) and independent of the subset-sum
formula.
"""
from __future__ import annotations

import itertools
import math


def double_factorial(k: int) -> int:
    """k!! with (-1)!! = 0!! = 1."""
    r = 1
    while k > 1:
        r *= k
        k -= 2
    return r


def haf_complete(n: int) -> int:
    """Perfect matchings of K_n: (n-1)!! for even n (Sec. 2, Eq. haf1), 0 for odd n."""
    return 0 if n % 2 else double_factorial(n - 1)


def telephone(n: int) -> int:
    """T(n) = number of matchings of K_n = |SPM(n)| (Sec. 2, Eq. haf2): T(n) = T(n-1) + (n-1) T(n-2)."""
    a, b = 1, 1
    if n == 0:
        return 1
    for k in range(2, n + 1):
        a, b = b, b + (k - 1) * a
    return b


def telephone_appendix_sum(n: int) -> int:
    """App. A's printed binomial sum, kept only to document that it does not give T(n)."""
    return sum(double_factorial(n - 1) // max(double_factorial(j - 1), 1) * math.comb(n // 2, j)
               for j in range(0, n // 2 + 1))


def haf_complete_bipartite(n: int) -> int:
    """per(J_{n/2}) = (n/2)! (Sec. 4, graph family 2; the text's (n/2)!, not the caption's n!)."""
    return math.factorial(n // 2)


def fibonacci(k: int) -> int:
    a, b = 0, 1
    for _ in range(k):
        a, b = b, a + b
    return a


def path_matchings(n: int) -> int:
    """All matchings of the path P_n (Hosoya index) = F(n+1); equals lhaf with unit loops (Sec. 2, end)."""
    return fibonacci(n + 1)


def path_perfect_matchings(n: int) -> int:
    return 1 if n % 2 == 0 else 0


def grid_perfect_matchings(a: int, b: int) -> int:
    """Perfect matchings of the a x b grid graph (domino tilings), exact, by a
    transfer matrix over column profiles: a column state is the set of cells of
    the current column already covered by horizontal dominoes from the left."""
    if (a * b) % 2:
        return 0
    full = (1 << a) - 1
    ways = {0: 1}
    for _col in range(b):
        nxt = {}
        for state, w in ways.items():
            # fill the current column: cells in `state` are taken; others get a
            # vertical domino (with the cell below) or a horizontal one (to the right)
            def fill(i, cur, out):
                if i == a:
                    nxt[out] = nxt.get(out, 0) + w
                    return
                if cur >> i & 1:
                    fill(i + 1, cur, out)
                    return
                fill(i + 1, cur | (1 << i), out | (1 << i))          # horizontal
                if i + 1 < a and not (cur >> (i + 1) & 1):
                    fill(i + 2, cur | (3 << i), out)                 # vertical
            fill(0, state, 0)
        ways = nxt
    return ways.get(0, 0)


def grid_kasteleyn(a: int, b: int) -> float:
    """Kasteleyn's product for domino tilings of an a x b rectangle (float, cross-check)."""
    prod = 1.0
    for j in range(1, math.ceil(a / 2) + 1):
        for k in range(1, math.ceil(b / 2) + 1):
            prod *= 4 * math.cos(math.pi * j / (a + 1)) ** 2 + 4 * math.cos(math.pi * k / (b + 1)) ** 2
    return prod


def enumerate_perfect_matchings(n: int):
    """All perfect matchings of {0..n-1} as lists of pairs (tiny n only)."""
    def rec(rest):
        if not rest:
            yield []
            return
        i = rest[0]
        for t in range(1, len(rest)):
            j = rest[t]
            for m in rec(rest[1:t] + rest[t + 1:]):
                yield [(i, j)] + m
    yield from rec(list(range(n)))


def enumerate_single_pair_matchings(n: int):
    """All single-pair matchings (pairs and loops) of {0..n-1} (tiny n only)."""
    def rec(rest):
        if not rest:
            yield []
            return
        i = rest[0]
        for m in rec(rest[1:]):
            yield [(i, i)] + m
        for t in range(1, len(rest)):
            j = rest[t]
            for m in rec(rest[1:t] + rest[t + 1:]):
                yield [(i, j)] + m
    yield from rec(list(range(n)))


def haf_by_enumeration(A, loops: bool = False):
    """Sum over explicitly listed (single-pair) perfect matchings; Python arithmetic."""
    n = len(A)
    it = enumerate_single_pair_matchings(n) if loops else enumerate_perfect_matchings(n)
    tot = 0
    for m in it:
        p = 1
        for i, j in m:
            p = p * A[i][j]
        tot = tot + p
    return tot


def all_pairings_count(n: int) -> int:
    return sum(1 for _ in itertools.islice(enumerate_perfect_matchings(n), 10 ** 7))
