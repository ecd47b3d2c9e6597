"""GPU tests of the permanent entry points (perm_c128, perm_c128_dev) through the C ABI.

perm(W) = haf([[0, W], [W^T, 0]]) (the bipartite identity): checked against the
oracle's Ryser permanent, against n! for the all-ones matrix, host against device
bitwise, against the hafnian entry point on the embedding bitwise, and on errors.
"""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

EPS = 2.0 ** -53


@pytest.fixture(scope="module")
def hg():
    import paper_1805_12498_amd as hg
    hg.load()
    return hg


def embed(W):
    n = W.shape[0]
    B = np.zeros((2 * n, 2 * n), complex)
    B[:n, n:] = W
    B[n:, :n] = W.T
    return B


def tolerance(W):
    """The hafnian path's bound on the embedding: 64 eps kappa, kappa of its subset sum."""
    if W.shape[0] == 0:
        return 0.0
    _, kappa = oracle.formula(embed(W), False, prec="dd", want_kappa=True)
    return 64 * EPS * kappa


def rand_c(n, seed, scale=0.7):
    rng = np.random.default_rng(seed)
    return rng.normal(0, scale, (n, n)) + 1j * rng.normal(0, scale, (n, n))


@pytest.mark.parametrize("n", [1, 2, 3, 5, 8, 11, 14])
def test_perm_vs_ryser(hg, n):
    W = rand_c(n, 8100 + n)
    got = hg.perm_host(W)
    ref = oracle.ryser(W, prec="dd")
    assert ref.relerr(got) <= tolerance(W), (n, got, ref.value)


@pytest.mark.parametrize("n", [0, 1, 4, 7, 10])
def test_perm_all_ones_is_factorial(hg, n):
    W = np.ones((n, n))
    got = hg.perm_host(W)
    assert abs(got - math.factorial(n)) <= tolerance(W) * math.factorial(n), (n, got)


def test_perm_host_device_and_embedding_bitwise(hg):
    import torch
    for n in (3, 9, 16):
        W = rand_c(n, 8200 + n)
        host = hg.perm_host(W)
        dW = torch.from_numpy(np.ascontiguousarray(W)).cuda()
        out = torch.zeros(1, dtype=torch.complex128, device="cuda")
        hg.perm_dev(dW.data_ptr(), n, n, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
        torch.cuda.synchronize()
        dev = complex(out.cpu().numpy()[0])
        assert host == dev == hg.haf_host(embed(W), hg.KIND_HAF), (n, host, dev)


def test_perm_strided_device_matrix(hg):
    import torch
    n, ldw = 6, 9
    big = rand_c(ldw, 8300)
    dW = torch.from_numpy(np.ascontiguousarray(big)).cuda()
    out = torch.zeros(1, dtype=torch.complex128, device="cuda")
    hg.perm_dev(dW.data_ptr(), n, ldw, out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    assert complex(out.cpu().numpy()[0]) == hg.perm_host(big[:n, :n])


def test_perm_errors(hg):
    from paper_1805_12498_amd._native import HafError
    with pytest.raises(HafError, match="TOO_LARGE"):
        hg.perm_host(np.zeros((33, 33)))
    W = rand_c(4, 1)
    W[2, 1] = np.nan
    with pytest.raises(HafError, match="NONFINITE"):
        hg.perm_host(W)
