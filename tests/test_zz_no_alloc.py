"""GPU test of the allocation-free entry point haf_c128x2_dev_noalloc, called
through the C ABI: on consecutive calls (each later call smaller than the one
before it, so stale scratch contents from a larger call are present) its
double-double result equals haf_c128x2_dev's bitwise, for both kinds, odd n,
the multi-class path (n <= 32) and the chunked path (n > 32); sizes beyond its
stated limit are rejected with HAF_E_TOO_LARGE."""
import ctypes

import numpy as np
import pytest

from gen import inputs as gi

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hg():
    import paper_1805_12498_amd as hg
    hg.load()
    return hg


def dev_pair(hg, A, kind):
    """(no-alloc result, ordinary result) as 4 doubles each, through the C ABI."""
    import torch
    lib = hg.load()
    n = A.shape[0]
    dA = torch.from_numpy(np.ascontiguousarray(A) if n else np.zeros(1, complex)).cuda()
    out_a = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    out_b = torch.full((4,), float("nan"), dtype=torch.float64, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = lib.haf_c128x2_dev_noalloc(ctypes.c_void_p(dA.data_ptr()), n, max(n, 1), kind,
                                    ctypes.c_void_p(out_a.data_ptr()), st)
    assert rc == 0, lib.haf_last_error()
    rc = lib.haf_c128x2_dev(ctypes.c_void_p(dA.data_ptr()), n, max(n, 1), kind, ctypes.c_void_p(out_b.data_ptr()), st)
    assert rc == 0, lib.haf_last_error()
    torch.cuda.synchronize()
    return out_a.cpu().numpy(), out_b.cpu().numpy()


@pytest.mark.parametrize("kind", [0, 1])
def test_noalloc_matches_ordinary_two_calls(hg, kind):
    for n in (44, 30):                         # second call smaller than the first
        A = gi.gaussian_symmetric(n, 7000 + n)
        a, b = dev_pair(hg, A, kind)
        print("n=%d kind=%d noalloc=%r ordinary=%r" % (n, kind, a, b), flush=True)
        assert np.array_equal(a, b), (n, kind, a, b)


def test_noalloc_sizes_and_edges(hg):
    for n, kind in ((56, 0), (21, 1), (16, 0), (7, 0), (2, 1), (0, 0)):
        A = gi.gaussian_symmetric(n, 7100 + n) if n else np.zeros((0, 0), complex)
        a, b = dev_pair(hg, A, kind)
        assert np.array_equal(a, b), (n, kind, a, b)


def test_noalloc_rejects_beyond_limit(hg):
    import torch
    lib = hg.load()
    A = torch.zeros((60, 60), dtype=torch.complex128, device="cuda")
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for n in (58, 60):
        rc = lib.haf_c128x2_dev_noalloc(ctypes.c_void_p(A.data_ptr()), n, 60, 0, ctypes.c_void_p(out.data_ptr()), st)
        assert rc == 2, (n, rc)                  # HAF_E_TOO_LARGE
        assert b"partial slots" in lib.haf_last_error()
    rc = lib.haf_c128x2_dev_noalloc(ctypes.c_void_p(A.data_ptr()), 4, 60, 0, None, st)
    assert rc == 1                               # HAF_E_INVALID_ARG
