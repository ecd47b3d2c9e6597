"""Pins for the CPU oracle: it is checked against facts the paper and the
mathematics fix, never against itself or the GPU library.

Each pin is chosen so that a plausible slip in the oracle (a dropped term, a
wrong sign or index, a transposed operand, a wrong loop term) fails one of them.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf
from gen import inputs as gi

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def rand_sym(n, seed, scale=0.7):
    rng = np.random.default_rng(seed)
    G = rng.normal(0, scale, (n, n)) + 1j * rng.normal(0, scale, (n, n))
    return (G + G.T) / 2


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


# ---------------------------------------------------------------- definitions
def test_worked_examples_n4():
    """Sec. 2: haf of a 4x4 matrix has the 3 terms of Eq. hafB; lhaf the 10 terms of SPM(4)."""
    g = json.load(open(os.path.join(GOLD, "worked_examples.json")))
    assert len(g["haf4"]) == 3 and len(g["lhaf4"]) == 10
    for seed in range(5):
        B = rand_sym(4, seed)
        h = sum(np.prod([B[i, j] for i, j in m]) for m in g["haf4"])
        l = sum(np.prod([B[i, j] for i, j in m]) for m in g["lhaf4"])
        assert rel(oracle.brute(B).value, h) < 1e-14
        assert rel(oracle.brute(B, True).value, l) < 1e-14
        assert rel(oracle.formula(B, prec="ld").value, h) < 1e-14
        assert rel(oracle.formula(B, True, prec="ld").value, l) < 1e-14


def test_lhaf_n2_by_hand():
    g = json.load(open(os.path.join(GOLD, "worked_examples.json")))["lhaf2_hand"]
    A = np.array(g["A"])
    assert oracle.brute_int(A, True) == g["value"]
    assert abs(oracle.formula(A, True, prec="q").value - g["value"]) < 1e-15
    assert oracle.exact_int(A, True)[0] == g["value"]


def test_printed_loop_term_literal_reading_fails():
    """The loop term read literally as v (X B)^(k-1) v^T / 2 with B = X A_Z gives
    b + (a^2 + c^2)/2 at n = 2, not b + a c; the oracle's reading d^T B^(k-1) X d
    (zero-diagonal B) gives the definition's value."""
    a, b, c = 2.0, 3.0, 5.0
    literal = b + (a * a + c * c) / 2          # k = 1 term of p is tr(B)/2 = b; loop term v v^T / 2
    assert literal != b + a * c
    A = np.array([[a, b], [b, c]])
    assert abs(oracle.formula(A, True).value - (b + a * c)) < 1e-15


@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 6, 7, 8])
def test_brute_vs_explicit_enumeration(n):
    """The table-based brute force against an explicit list of (single-pair) matchings."""
    A = rand_sym(n, 100 + n)
    L = [[complex(A[i, j]) for j in range(n)] for i in range(n)]
    assert rel(oracle.brute(A).value, cf.haf_by_enumeration(L)) < 1e-13 or n % 2 == 1
    if n % 2 == 1:
        assert oracle.brute(A).value == 0
    assert rel(oracle.brute(A, True).value, cf.haf_by_enumeration(L, True)) < 1e-13


def test_matching_counts():
    """(n-1)!! perfect matchings (Eq. haf1) and T(n) single-pair matchings (Eq. haf2)."""
    for n in range(0, 11):
        assert sum(1 for _ in cf.enumerate_single_pair_matchings(n)) == cf.telephone(n)
        if n % 2 == 0:
            assert sum(1 for _ in cf.enumerate_perfect_matchings(n)) == cf.haf_complete(n)
    assert cf.telephone(4) == 10  # the 10 elements listed in SPM(4)


def test_appendix_binomial_sum_is_not_T():
    """App. A's printed sum gives 12 at n = 4, but SPM(4) has 10 elements; the
    recurrence T(n) = T(n-1) + (n-1) T(n-2) is used instead."""
    assert cf.telephone_appendix_sum(4) == 12
    assert cf.telephone(4) == 10


# ---------------------------------------------------------------- formula vs definition
@pytest.mark.parametrize("n", [2, 4, 6, 8, 10, 12, 14])
@pytest.mark.parametrize("loops", [False, True])
def test_formula_vs_brute(n, loops):
    A = rand_sym(n, 7 * n + loops)
    ref = oracle.brute(A, loops).value
    for prec, tol in (("d", 1e-11), ("ld", 1e-14), ("dd", 1e-14), ("q", 1e-14)):
        assert rel(oracle.formula(A, loops, prec=prec).value, ref) < tol, prec


@pytest.mark.parametrize("n", [3, 5, 7, 9])
def test_odd_sizes(n):
    A = rand_sym(n, n)
    assert oracle.formula(A).value == 0
    assert rel(oracle.formula(A, True).value, oracle.brute(A, True).value) < 1e-14


def test_integer_exactness_small():
    rng = np.random.default_rng(5)
    for n in (6, 10, 14, 18):
        for loops in (False, True):
            A = rng.integers(-3, 4, (n, n))
            A = np.triu(A) + np.triu(A, 1).T
            exact = oracle.brute_int(A, loops)
            assert oracle.exact_int(A, loops)[0] == exact
            assert round(oracle.formula(A, loops, prec="q").value.real) == exact


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [2, 8, 16, 24, 32])
def test_complete_graph(n):
    """haf(K_n) = (n-1)!!, lhaf(K_n with unit loops) = T(n) (Sec. 4, graph family 1)."""
    J = gi.complete_graph(n)
    assert oracle.exact_int(J)[0] == cf.haf_complete(n)
    assert oracle.exact_int(gi.complete_graph(n, loops=True), True)[0] == cf.telephone(n)
    f = oracle.formula(J.astype(complex), prec="dd").value
    assert rel(f, cf.haf_complete(n)) < 1e-20 * 1e10


@pytest.mark.parametrize("n", [4, 12, 20, 28])
def test_complete_bipartite(n):
    """haf([[0,J],[J,0]]) = per(J) = (n/2)! (Sec. 4, graph family 2)."""
    A = gi.complete_bipartite(n)
    assert oracle.exact_int(A)[0] == cf.haf_complete_bipartite(n)
    assert rel(oracle.ryser(np.ones((n // 2, n // 2)), prec="dd").value, math.factorial(n // 2)) < 1e-25 * 1e10


@pytest.mark.parametrize("ab", [(2, 3), (4, 4), (4, 6), (6, 6)])
def test_grid_graph(ab):
    a, b = ab
    A = gi.grid_graph(a, b)
    want = cf.grid_perfect_matchings(a, b)
    assert abs(cf.grid_kasteleyn(a, b) - want) < 1e-6 * want
    assert oracle.exact_int(A)[0] == want
    if a * b <= 16:
        assert oracle.brute_int(A) == want


@pytest.mark.parametrize("n", [6, 11, 20])
def test_path_with_unit_loops(n):
    """With unit diagonal, lhaf counts all matchings (end of Sec. 2): F(n+1) on a path."""
    A = gi.path_graph(n) + np.eye(n, dtype=np.int64)
    assert oracle.exact_int(A, True)[0] == cf.path_matchings(n)


@pytest.mark.parametrize("n", [6, 12, 20])
def test_rank_one(n):
    """haf(v v^T) = (n-1)!! prod v_i; lhaf(off-diag v_i v_j, diag v_i) = T(n) prod v_i."""
    rng = np.random.default_rng(n)
    v = rng.normal(size=n) + 1j * rng.normal(size=n)
    V = np.outer(v, v)
    assert rel(oracle.formula(V, prec="dd").value, cf.haf_complete(n) * np.prod(v)) < 1e-13
    W = V.copy()
    np.fill_diagonal(W, v)
    assert rel(oracle.formula(W, True, prec="dd").value, cf.telephone(n) * np.prod(v)) < 1e-13


def _series_coeff(factors, N):
    """[x^N] of prod (1 - a x)^(-e) for (a, e) with rational a, e (binomial series)."""
    poly = [Fraction(1)] + [Fraction(0)] * N
    for a, e in factors:
        ser = [Fraction(1)]
        for k in range(1, N + 1):
            ser.append(ser[-1] * (e + k - 1) / k * a)
        poly = [sum(poly[i] * ser[k - i] for i in range(k + 1)) for k in range(N + 1)]
    return poly[N]


@pytest.mark.parametrize("n", [8, 14, 20])
def test_single_term_complete_graph(n):
    """For A = J - I, B = J - X on a subset of m pairs has spectrum 2m-1, -1 (m-1 times),
    +1 (m times), so f(Z) = [l^N] (1-(2m-1)l)^(-1/2) (1+l)^(-(m-1)/2) (1-l)^(-m/2)."""
    N = n // 2
    J = gi.complete_graph(n).astype(complex)
    for mask in (1, 3, (1 << N) - 1, 0b1011 & ((1 << N) - 1), 1 << (N - 1)):
        m = bin(mask).count("1")
        want = _series_coeff([(2 * m - 1, Fraction(1, 2)), (-1, Fraction(m - 1, 2)), (1, Fraction(m, 2))], N)
        got = oracle.term(J, mask, prec="q").value
        assert abs(got - float(want)) <= 1e-25 * max(1.0, abs(float(want))) * 1e10


@pytest.mark.parametrize("n", [8, 12, 16])
def test_kappa_complete_graph_closed_form(n):
    """kappa = sum_Z |f(Z)| / |haf| for A = J - I from the closed-form single terms above:
    f(Z) depends only on m = |Z|, so sum_Z |f(Z)| = sum_m C(N, m) |f_m| and haf = (n-1)!!.
    Every parity tolerance scales with the oracle's kappa, so an over-estimate would
    loosen every GPU test; this pins it."""
    N = n // 2
    J = gi.complete_graph(n).astype(complex)
    total = Fraction(0)
    for m in range(1, N + 1):
        fm = _series_coeff([(2 * m - 1, Fraction(1, 2)), (-1, Fraction(m - 1, 2)), (1, Fraction(m, 2))], N)
        total += math.comb(N, m) * abs(fm)
    want = float(total / cf.haf_complete(n))
    for prec in ("d", "ld", "dd", "q"):
        r, kappa = oracle.formula(J, prec=prec, want_kappa=True)
        assert abs(kappa - want) <= 1e-12 * want, (prec, kappa, want)


@pytest.mark.parametrize("n", [6, 10, 14])
def test_formula_masks_against_closed_forms_and_brute_force(n):
    """formula_masks: one mask of J - I gives (-1)^(N-m) f_m (the closed-form term with
    the sign of Eq. Pset); all nonzero masks of a random matrix give the brute-force haf."""
    N = n // 2
    J = gi.complete_graph(n).astype(complex)
    for mask in (1, (1 << N) - 1, 0b101 & ((1 << N) - 1) or 1):
        m = bin(mask).count("1")
        fm = _series_coeff([(2 * m - 1, Fraction(1, 2)), (-1, Fraction(m - 1, 2)), (1, Fraction(m, 2))], N)
        want = float(fm) * (-1) ** (N - m)
        got = oracle.formula_masks(J, np.array([mask], dtype=np.uint32), prec="q").value
        assert abs(got - want) <= 1e-25 * max(1.0, abs(want)) * 1e10
    A = rand_sym(n, 500 + n)
    masks = np.arange(1, 1 << N, dtype=np.uint32)
    for loops in (False, True):
        got = oracle.formula_masks(A, masks, loops=loops, prec="dd").value
        assert rel(got, oracle.brute(A, loops).value) < 1e-13


@pytest.mark.parametrize("n", [8, 14])
def test_single_term_complete_graph_loops(n):
    """A = J (unit loops): l_k = s (2m-1)^(k-1), so the loop factor is exp(sum_{k<=N} m (2m-1)^(k-1) l^k)."""
    N = n // 2
    J = gi.complete_graph(n, loops=True).astype(complex)
    for mask in (1, 5 & ((1 << N) - 1), (1 << N) - 1):
        m = bin(mask).count("1")
        det_part = [Fraction(0)] * (N + 1)
        for k in range(N + 1):
            det_part[k] = _series_coeff([(2 * m - 1, Fraction(1, 2)), (-1, Fraction(m - 1, 2)),
                                         (1, Fraction(m, 2))], k)
        c = [Fraction(0)] + [Fraction(m) * (2 * m - 1) ** (k - 1) for k in range(1, N + 1)]
        e = [Fraction(1)] + [Fraction(0)] * N      # exp of sum c_k l^k
        for j in range(1, N + 1):
            e[j] = sum(k * c[k] * e[j - k] for k in range(1, j + 1)) / j
        want = sum(det_part[i] * e[N - i] for i in range(N + 1))
        got = oracle.term(J, mask, True, prec="q").value
        assert abs(got - float(want)) <= 1e-15 * max(1.0, abs(float(want)))


# ---------------------------------------------------------------- invariances
def test_scaling_laws():
    """haf(mu A) = mu^(n/2) haf(A);  lhaf(sqrt(mu) A_diag + mu A_off) = mu^(n/2) lhaf(A)  (Eq. scaling)."""
    n = 12
    A = rand_sym(n, 9)
    mu = 1.7
    assert rel(oracle.formula(mu * A, prec="dd").value, mu ** (n // 2) * oracle.formula(A, prec="dd").value) < 1e-13
    D = np.diag(np.diag(A))
    Off = A - D
    lhs = oracle.formula(np.sqrt(mu) * D + mu * Off, True, prec="dd").value
    assert rel(lhs, mu ** (n // 2) * oracle.formula(A, True, prec="dd").value) < 1e-13


def test_lhaf_zero_diagonal_is_haf():
    A = rand_sym(14, 11)
    np.fill_diagonal(A, 0)
    assert rel(oracle.formula(A, True, prec="dd").value, oracle.formula(A, prec="dd").value) < 1e-14


def test_haf_ignores_diagonal():
    A = rand_sym(12, 12)
    B = A.copy()
    np.fill_diagonal(B, 3.0 + 1j)
    assert rel(oracle.formula(A, prec="dd").value, oracle.formula(B, prec="dd").value) < 1e-14


@pytest.mark.parametrize("loops", [False, True])
def test_permutation_invariance(loops):
    """Any pairing of the vertices will do (Fig. graph caption): haf(P A P^T) = haf(A)."""
    A = rand_sym(16, 13)
    p = gi.random_permutation(16, 3)
    B = A[np.ix_(p, p)]
    assert rel(oracle.formula(B, loops, prec="dd").value, oracle.formula(A, loops, prec="dd").value) < 1e-14


def test_block_diagonal_factorisation():
    A1, A2 = rand_sym(6, 1), rand_sym(8, 2)
    A = np.zeros((14, 14), complex)
    A[:6, :6] = A1
    A[6:, 6:] = A2
    for loops in (False, True):
        want = oracle.formula(A1, loops, prec="dd").value * oracle.formula(A2, loops, prec="dd").value
        assert rel(oracle.formula(A, loops, prec="dd").value, want) < 1e-14


def test_bipartite_identity_and_ryser():
    """haf([[0,W],[W^T,0]]) = per(W) (Eq. bipartite); Ryser against a permutation sum."""
    import itertools
    W = gi.gaussian_square(6, 17)
    perm = sum(np.prod([W[i, s[i]] for i in range(6)]) for s in itertools.permutations(range(6)))
    assert rel(oracle.ryser(W, prec="dd").value, perm) < 1e-14
    A = gi.bipartite_embed(W)
    assert rel(oracle.formula(A, prec="dd").value, perm) < 1e-13
    assert rel(oracle.brute(A).value, perm) < 1e-13


# ---------------------------------------------------------------- exact mod-p route
def test_modp_term_vs_exact_term():
    """Per-term f(Z) of an integer matrix: Hessenberg/charpoly over F_p against the
    binary128 explicit-power term rounded to an integer (two unrelated routes)."""
    A = gi.random_graph(16, 0.5, 21)
    N = 8
    for mask in (1, 7, 0b10110101, (1 << N) - 1, 0b01010010):
        exact = round(oracle.term(A.astype(complex), mask, prec="q").value.real)
        for p in oracle.PRIMES[:2]:
            assert oracle.modp_term(A, mask, p) == exact % p


def test_modp_negative_and_loops():
    rng = np.random.default_rng(8)
    A = rng.integers(-5, 6, (12, 12))
    A = np.triu(A) + np.triu(A, 1).T
    for loops in (False, True):
        assert oracle.exact_int(A, loops)[0] == oracle.brute_int(A, loops)


def test_precision_ladder():
    """Lower precisions agree with binary128 within a small multiple of eps * kappa."""
    A = gi.gaussian_symmetric(20, 31)
    ref, kappa = oracle.formula(A, prec="q", want_kappa=True)
    for prec in ("d", "ld", "dd"):
        err = ref.relerr_hp(oracle.formula(A, prec=prec))
        assert err <= 16 * oracle.EPS[prec] * kappa + 1e-30, (prec, err, kappa)
