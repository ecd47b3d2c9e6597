"""GPU tests of the continuous-batching request server through the C ABI.

Every result must be bitwise the single-matrix path's result for the same
matrix (alone versus in the mix, whatever the tick budget), match the oracle,
carry ordered timestamps, and the server must finish every request whatever its
arena and slot limits; small requests submitted behind a large one finish
before it.
"""
import math

import numpy as np
import pytest

import oracle
from gen import inputs as gi

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -53
C_TOL = 64.0


@pytest.fixture(scope="module")
def hg():
    import paper_1805_12498_amd as hg
    hg.load()
    print("device:", hg.device_info(), flush=True)
    return hg


def serve(hg, trace, **cfg):
    srv = hg.Server(**cfg)
    try:
        tickets = {}
        for _, kind, A in trace:
            tickets[srv.submit(A, kind)] = (kind, A)
        srv.drain()
        res = srv.poll(len(trace) + 10)
    finally:
        srv.close()
    assert len(res) == len(trace)
    return tickets, res


def test_results_alone_vs_mix_and_oracle(hg):
    trace = gi.serving_trace(120, qps=1e4, seed=gi.SEED_SERVE, nmax=24)
    tickets, res = serve(hg, trace)
    for k, r in enumerate(res):
        kind, A = tickets[r.ticket]
        assert r.status == 0 and r.n == A.shape[0] and r.kind == kind
        assert r.t_submit <= r.t_admit <= r.t_done
        v = complex(r.value.re, r.value.im)
        assert v == hg.haf_host(A, kind), (r.ticket, A.shape[0], kind)       # alone vs in the mix
        if k % 10 == 0:
            ref, kappa = oracle.formula(A, bool(kind), prec="dd", want_kappa=True)
            assert ref.relerr(v) <= max(1e-12, C_TOL * EPS * kappa)


def test_plain_and_continuous_agree(hg):
    trace = gi.serving_trace(60, qps=1e4, seed=11, nmax=28)
    t1, r1 = serve(hg, trace, continuous=1)
    t0, r0 = serve(hg, trace, continuous=0)
    v1 = {t1[r.ticket][1].tobytes(): complex(r.value.re, r.value.im) for r in r1}
    v0 = {t0[r.ticket][1].tobytes(): complex(r.value.re, r.value.im) for r in r0}
    assert v1 == v0
    # the plain server admits in arrival order, one at a time
    adm = sorted((r.t_admit, r.ticket) for r in r0)
    assert [t for _, t in adm] == sorted(t for _, t in adm)
    done = sorted((r.t_done, r.t_admit) for r in r0)
    for (d_prev, _), (_, a_next) in zip(done, done[1:]):
        assert a_next >= d_prev - 1e-3


def request_bytes(n, kind):
    """Device state of an admitted request: matrix, padded copy (odd-n lhaf), exponent,
    partial slots (32 bytes per 256-subset series block of each size class)."""
    al = lambda x: (x + 255) // 256 * 256  # noqa: E731
    ne = n + 1 if (n % 2 and kind == 1) else n
    N = ne // 2
    slots = sum(-(-math.comb(N, m) // 256) for m in range(1, N + 1))
    return al(n * n * 16) + (al(ne * ne * 16) if ne != n else 0) + 256 + al(slots * 32)


def test_small_arena_and_slots(hg):
    """An arena that holds two of the largest requests at a time and three slots:
    everything still finishes."""
    trace = gi.serving_trace(30, qps=1e4, seed=12, nmax=30)
    arena = 2 * max(request_bytes(A.shape[0], k) for _, k, A in trace)
    tickets, res = serve(hg, trace, arena_bytes=arena, max_active=3)
    for r in res:
        kind, A = tickets[r.ticket]
        assert r.status == 0
        assert complex(r.value.re, r.value.im) == hg.haf_host(A, kind)


def test_edge_sizes(hg):
    mats = [(0, np.zeros((0, 0), complex)), (1, gi.gaussian_symmetric(7, 3)), (0, gi.gaussian_symmetric(7, 3)),
            (1, gi.gaussian_symmetric(2, 4)), (0, gi.gaussian_symmetric(50, 5))]
    trace = [(0.0, k, A) for k, A in mats]
    tickets, res = serve(hg, trace)
    for r in res:
        kind, A = tickets[r.ticket]
        assert complex(r.value.re, r.value.im) == hg.haf_host(A, kind)


def test_submit_errors(hg):
    from paper_1805_12498_amd._native import HafError
    srv = hg.Server()
    try:
        A = gi.gaussian_symmetric(6, 1)
        B = A.copy()
        B[0, 1] += 1e-3
        with pytest.raises(HafError, match="NOT_SYMMETRIC"):
            srv.submit(B, 0)
        with pytest.raises(HafError, match="TOO_LARGE"):
            srv.submit(np.zeros((66, 66)), 0)
        C = A.copy()
        C[1, 1] = np.inf
        with pytest.raises(HafError, match="NONFINITE"):
            srv.submit(C, 1)
        t = srv.submit(A, 1)
        srv.drain()
        (r,) = srv.poll(4)
        assert r.ticket == t and r.status == 0
    finally:
        srv.close()
    with pytest.raises(HafError, match="NOMEM"):
        small = hg.Server(arena_bytes=4096)
        try:
            small.submit(gi.gaussian_symmetric(40, 2), 0)
        finally:
            small.close()


def test_tiny_ticks_bitwise(hg):
    """A tick budget far below one request's work: every request spreads over many ticks
    (pieces of 256 subsets) and its result is still bitwise the single-matrix result."""
    trace = gi.serving_trace(16, qps=1e4, seed=14, nmax=36)
    tickets, res = serve(hg, trace, tick_flops=1e6, tick_coef_bytes=1 << 20)
    for r in res:
        kind, A = tickets[r.ticket]
        assert r.status == 0
        assert complex(r.value.re, r.value.im) == hg.haf_host(A, kind), (A.shape[0], kind)


def test_small_requests_pass_a_large_one(hg):
    """A 44x44 loop hafnian (2^22 subsets) submitted first, then 20 small requests: the
    small ones share the ticks with it and finish before it; every result bitwise."""
    B = gi.serving_trace(1, qps=1e4, seed=15, nmin=44, nmax=44)
    small = gi.serving_trace(20, qps=1e4, seed=16, nmin=12, nmax=16)
    trace = [(0.0, 1, B[0][2])] + small
    srv = hg.Server()
    try:
        tickets = {}
        for _, kind, A in trace:
            tickets[srv.submit(A, kind)] = (kind, A)
        srv.drain()
        res = srv.poll(64)
    finally:
        srv.close()
    big = [r for r in res if tickets[r.ticket][1].shape[0] == 44]
    rest = [r for r in res if tickets[r.ticket][1].shape[0] != 44]
    assert len(big) == 1 and len(rest) == 20
    assert max(r.t_done for r in rest) < big[0].t_done
    for r in res:
        kind, A = tickets[r.ticket]
        assert complex(r.value.re, r.value.im) == hg.haf_host(A, kind), (A.shape[0], kind)


def test_destroy_with_pending_requests(hg):
    """Closing a server that still has queued work returns (queued requests are dropped)."""
    srv = hg.Server(max_active=1)
    for _, kind, A in gi.serving_trace(40, qps=1e4, seed=13, nmax=30):
        srv.submit(A, kind)
    srv.close()


@pytest.mark.parametrize("continuous", [1, 0])
def test_failed_launch_recovery(hg, continuous):
    """A tick whose launch fails (forced from the host by the test hook after the launch
    really succeeded, so the device never faults) fails the admitted requests with
    HAF_E_DEVICE; the server replaces its stream and the next requests complete, bitwise
    equal to the single-matrix path."""
    srv = hg.Server(continuous=continuous)
    try:
        srv.debug_fail_ticks(1)
        first = gi.serving_trace(8, qps=1e4, seed=17, nmax=20)
        tickets = {}
        for _, kind, A in first:
            tickets[srv.submit(A, kind)] = (kind, A)
        srv.drain()
        res1 = srv.poll(64)
        assert len(res1) == len(first)
        failed = [r for r in res1 if r.status == 5]
        assert failed, "the forced failure must fail at least the requests of its tick"
        for r in res1:
            assert r.status in (0, 5)
            if r.status == 0:
                kind, A = tickets[r.ticket]
                assert complex(r.value.re, r.value.im) == hg.haf_host(A, kind)
        second = gi.serving_trace(12, qps=1e4, seed=18, nmax=24)
        for _, kind, A in second:
            tickets[srv.submit(A, kind)] = (kind, A)
        srv.drain()
        res2 = srv.poll(64)
        assert len(res2) == len(second)
        for r in res2:
            kind, A = tickets[r.ticket]
            assert r.status == 0
            assert complex(r.value.re, r.value.im) == hg.haf_host(A, kind)
    finally:
        srv.close()


def test_debug_hook_rejects_bad_arguments(hg):
    from paper_1805_12498_amd._native import HafError
    srv = hg.Server()
    try:
        with pytest.raises(HafError, match="INVALID_ARG"):
            srv.debug_fail_ticks(-1)
    finally:
        srv.close()
