"""GPU tests of the low-rank hafnian (haf_lowrank_c128, App. C) through the C ABI.

The result is the hafnian of G G^T (above the diagonal), so the oracle is the
plain definition: brute-force matching enumeration at small n, the formula
route in double-double at mid n; closed forms for rank 1 (haf(v v^T) =
(n-1)!! prod v_i) and for G with orthonormal-like columns.  The tolerance is
the cancellation of the final even-monomial sum (cond) times a few eps per
factor."""
import math

import numpy as np
import pytest

import oracle
from oracle import closed_forms as cf

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -53


@pytest.fixture(scope="module")
def hg():
    import paper_1805_12498_amd as hg
    hg.load()
    return hg


def factor(n, r, seed, scale=0.8):
    rng = np.random.default_rng(seed)
    return scale * (rng.normal(0, 1, (n, r)) + 1j * rng.normal(0, 1, (n, r))) / math.sqrt(2)


def hp(x):
    return oracle.HighPrec(x)


@pytest.mark.parametrize("n", [0, 1, 2, 4, 7, 10, 14, 18])
@pytest.mark.parametrize("r", [1, 2, 3, 5, 8])
def test_vs_brute_force(hg, n, r):
    G = factor(n, r, 10 * n + r)
    got, cond = hg.haf_lowrank(G)
    if n % 2:
        assert got == (0.0, 0.0, 0.0, 0.0)
        return
    A = G @ G.T
    ref = oracle.brute(A, False)
    err = ref.relerr_hp(hp(got))
    assert err <= max(1e-13, 8 * n * EPS * cond), (n, r, err, cond)


@pytest.mark.parametrize("n,r", [(28, 2), (32, 3), (36, 4)])
def test_vs_oracle_formula(hg, n, r):
    G = factor(n, r, 500 + n)
    got, cond = hg.haf_lowrank(G)
    A = G @ G.T
    ref, kappa = oracle.formula(A, False, prec="dd", want_kappa=True)
    err = ref.relerr_hp(hp(got))
    print("n=%d r=%d relerr %.3g cond %.3g (subset-sum kappa %.3g)" % (n, r, err, cond, kappa), flush=True)
    assert err <= 8 * n * EPS * cond + 64 * 2.0 ** -104 * kappa, (err, cond)


@pytest.mark.parametrize("n", [2, 20, 40, 64])
def test_rank_one_closed_form(hg, n):
    v = (np.arange(n) % 5 + 1).astype(float) * 0.5
    got, cond = hg.haf_lowrank(v.reshape(n, 1))
    want = cf.double_factorial(n - 1) * math.prod(float(x) for x in v)
    assert abs((got[0] + got[1]) - want) <= 4 * n * EPS * abs(want) and got[2] == 0.0


def test_matches_hafnian_path_at_n44(hg):
    """rank 3 at n = 44: the App. C expansion (C(46, 2) = 1035 monomials) against the
    2^22-term subset sum of the same matrix with double-double terms."""
    n, r = 44, 3
    G = factor(n, r, 4444, scale=0.6)
    got, cond = hg.haf_lowrank(G)
    A = np.ascontiguousarray(G @ G.T)
    dd = hg.haf_host_dd(A, 0)
    err = hp(dd).relerr_hp(hp(got))
    print("n=44 r=3: lowrank vs subset sum (double-double terms) %.3g, cond %.3g" % (err, cond), flush=True)
    assert err <= 8 * n * EPS * cond + 1e-12


def test_errors(hg):
    from paper_1805_12498_amd._native import HafError
    with pytest.raises(HafError, match="TOO_LARGE"):
        hg.haf_lowrank(factor(10, 9, 1))
    with pytest.raises(HafError, match="TOO_LARGE"):
        hg.haf_lowrank(factor(66, 2, 1))
    with pytest.raises(HafError, match="TOO_LARGE"):
        hg.haf_lowrank(factor(64, 8, 1))               # C(71, 7) monomials > 2^28
    G = factor(6, 2, 2)
    G[3, 1] = np.nan
    with pytest.raises(HafError, match="NONFINITE"):
        hg.haf_lowrank(G)
