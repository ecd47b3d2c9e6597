"""GPU tests of the continuous-batching request server through the C ABI.

Every result must be bitwise the single-matrix path's result for the same
matrix (alone versus in the mix), match the oracle, carry ordered timestamps,
and the server must finish every request whatever its arena and slot limits.
"""
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
    t1, r1 = serve(hg, trace, continuous=1, streams=8)
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


def test_small_arena_and_slots(hg):
    """An arena that holds two requests at a time and three slots: everything still finishes."""
    trace = gi.serving_trace(30, qps=1e4, seed=12, nmax=30)
    nmax = max(A.shape[0] for _, _, A in trace)
    arena = 2 * (((nmax * nmax * 16 + 255) // 256) * 256 + 256)
    tickets, res = serve(hg, trace, arena_bytes=arena, max_active=3, streams=2)
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


def test_destroy_with_pending_requests(hg):
    """Closing a server that still has queued work returns (queued requests are dropped)."""
    srv = hg.Server(max_active=1, streams=1)
    for _, kind, A in gi.serving_trace(40, qps=1e4, seed=13, nmax=30):
        srv.submit(A, kind)
    srv.close()
