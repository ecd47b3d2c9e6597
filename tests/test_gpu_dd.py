"""GPU tests of the per-term double-double mode (haf_dd_c128x2_*) through the C ABI.

Every step of each term runs in complex double-double, so the error of the
alternating sum is bounded by ~eps_dd * kappa (eps_dd = 2^-104) instead of
~eps64 * kappa.  Checks: the 16x16 and 40x40 configuration matrices against the
oracle's stored binary128 / double-double values, with the target of at most
1e-10 relative error at n <= 40 asserted next to the kappa bound; brute force at
small n (limited by the long-double oracle); closed forms far beyond double
precision's reach; odd n, n = 0, the host and device entries bitwise equal,
bitwise reproducibility.
"""
import json
import os
import time

import numpy as np
import pytest

import oracle
from gen import inputs as gi
from oracle import closed_forms as cf

pytestmark = pytest.mark.gpu

EPS_DD = 2.0 ** -104
C_TOL = 128.0
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")))


@pytest.fixture(scope="module")
def hg():
    import paper_1805_12498_amd as hg
    hg.load()
    return hg


def gold(name):
    g = GOLD[name]
    v = g["value"]
    return oracle.HighPrec((v["re"][0], v["re"][1], v["im"][0], v["im"][1])), g["kappa"]


def hp(x):
    return oracle.HighPrec(x)


@pytest.mark.parametrize("name,n,kind", [("n16_haf", 16, 0), ("n16_lhaf", 16, 1), ("n40_haf", 40, 0),
                                         ("n40_lhaf", 40, 1)])
def test_configs_vs_oracle(hg, name, n, kind):
    A = gi.gaussian_symmetric(n, gi.SEED_N16 if n == 16 else gi.SEED_N40)
    ref, kappa = gold(name)
    t0 = time.time()
    got = hp(hg.haf_host_dd(A, kind))
    dt = time.time() - t0
    err = ref.relerr_hp(got)
    # the oracle's own double-double error (n = 40) is of the same order as the bound
    print("%s: dd relerr %.3g (kappa %.3g, bound %.3g), %.2f s" % (name, err, kappa, C_TOL * EPS_DD * kappa, dt),
          flush=True)
    assert err <= 1e-10
    assert err <= max(C_TOL * EPS_DD * kappa, 1e-30), (err, kappa)


@pytest.mark.parametrize("n", [2, 5, 8, 11, 14])
@pytest.mark.parametrize("kind", [0, 1])
def test_small_vs_brute_force(hg, n, kind):
    rng = np.random.default_rng(40 * n + kind)
    G = rng.normal(0, 0.7, (n, n)) + 1j * rng.normal(0, 0.7, (n, n))
    A = (G + G.T) / 2
    ref = oracle.brute(A, bool(kind))
    got = hp(hg.haf_host_dd(A, kind))
    if n % 2 and kind == 0:
        assert got.value == 0
        return
    assert ref.relerr_hp(got) < 1e-17, (n, kind)


@pytest.mark.parametrize("n", [20, 30, 40])
def test_closed_forms(hg, n):
    """haf(J - I) = (n-1)!!, lhaf(J) = T(n): integers beyond 2^53, alternating sums with
    heavy cancellation."""
    J = np.ones((n, n))
    for kind, M, exact in ((0, J - np.eye(n), cf.haf_complete(n)), (1, J, cf.telephone(n))):
        got = hp(hg.haf_host_dd(M, kind))
        re, im = got.exact_parts()
        err = abs(float(re - exact)) / exact
        print("n=%d kind=%d relerr %.3g" % (n, kind, err), flush=True)
        assert err < 1e-20 and abs(float(im)) < 1e-20 * exact, (n, kind, err)


def test_edges_and_entries(hg):
    import torch
    A = gi.gaussian_symmetric(13, 77)
    assert hg.haf_host_dd(A, 0) == (0.0, 0.0, 0.0, 0.0)
    assert hg.haf_host_dd(np.zeros((0, 0)), 1) == (1.0, 0.0, 0.0, 0.0)
    B = np.zeros((14, 14), complex)
    B[:13, :13] = A
    B[13, 13] = 1.0
    assert hg.haf_host_dd(A, 1) == hg.haf_host_dd(B, 1)          # odd n: lhaf(A (+) [1])
    C = gi.gaussian_symmetric(24, 78)
    d = torch.from_numpy(C).cuda()
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    hg.haf_dev_dd(d.data_ptr(), 24, 24, out.data_ptr(), torch.cuda.current_stream().cuda_stream, kind=1)
    torch.cuda.synchronize()
    assert tuple(out.cpu().numpy()) == hg.haf_host_dd(C, 1) == hg.haf_host_dd(C, 1)


def test_dd_and_double_agree_within_double_bound(hg):
    """The double path's error measured against the double-double mode (n = 28)."""
    A = gi.gaussian_symmetric(28, 2801)
    ref, kappa = oracle.formula(A, False, prec="ld", want_kappa=True)
    dd = hp(hg.haf_host_dd(A, 0))
    d = hg.haf_host(A, 0)
    e_dd, e_d = ref.relerr_hp(dd), dd.relerr(d)
    print("n=28: double vs dd %.3g, dd vs long-double oracle %.3g, kappa %.3g" % (e_d, e_dd, kappa), flush=True)
    assert e_d <= 64 * 2.0 ** -53 * kappa
    assert e_dd <= 64 * 2.0 ** -64 * kappa
