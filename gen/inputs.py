"""Seeded synthetic inputs for the hafnian workloads.

This module is shared by the tests, the oracle checks and the benchmark, so it
holds no arithmetic of the hafnian method itself: only how inputs are drawn.

Workloads (the paper benchmarks complete graphs, complete bipartite graphs and
random complex symmetric matrices, Sec. 4 and Sec. 4.2; GBS-style submatrices
motivate the batched and serving workloads, Sec. 1):

* ``gaussian_symmetric(n, seed)``  A = (G + G^T)/2, Re G and Im G iid N(0, 1/2);
* ``random_graph(n, p, seed)``     0/1 adjacency of G(n, p), zero diagonal;
* ``complete_graph(n)`` / ``complete_bipartite(n)`` / ``grid_graph(a, b)``;
* ``gbs_batch(count, seed)``       submatrices of B = U diag(tanh r) U^T picked with
                                   repetition, diagonal replaced by a displacement;
* ``serving_trace(...)``           a Poisson stream of mixed-size requests.
"""
from __future__ import annotations

import numpy as np

# Seeds of the named workloads.
SEED_N16 = 1601
SEED_N40 = 4001
SEED_N56 = 5601
SEED_N56_GRAPH = 5602
SEED_N56_BIPARTITE = 5603
SEED_BATCH = 4096
SEED_SERVE = 2027


def gaussian_symmetric(n: int, seed: int) -> np.ndarray:
    """Complex symmetric A = (G + G^T)/2 with Re, Im of G iid N(0, 1/2)."""
    rng = np.random.default_rng(seed)
    re = rng.normal(0.0, np.sqrt(0.5), (n, n))
    im = rng.normal(0.0, np.sqrt(0.5), (n, n))
    G = re + 1j * im
    return np.ascontiguousarray((G + G.T) / 2)


def uniform_symmetric(n: int, seed: int) -> np.ndarray:
    """The paper's random family (Sec. 4.2): uniform real and imaginary parts, symmetrised."""
    rng = np.random.default_rng(seed)
    G = rng.uniform(-1, 1, (n, n)) + 1j * rng.uniform(-1, 1, (n, n))
    return np.ascontiguousarray((G + G.T) / 2)


def random_graph(n: int, p: float, seed: int) -> np.ndarray:
    """0/1 symmetric adjacency matrix of G(n, p) with zero diagonal (int64)."""
    rng = np.random.default_rng(seed)
    U = rng.random((n, n)) < p
    M = np.triu(U, 1)
    return (M | M.T).astype(np.int64)


def complete_graph(n: int, loops: bool = False) -> np.ndarray:
    A = np.ones((n, n), dtype=np.int64)
    if not loops:
        np.fill_diagonal(A, 0)
    return A


def complete_bipartite(n: int) -> np.ndarray:
    """[[0, J], [J, 0]] with n/2 vertices per side (Sec. 4, graph family 2)."""
    h = n // 2
    A = np.zeros((n, n), dtype=np.int64)
    A[:h, h:] = 1
    A[h:, :h] = 1
    return A


def bipartite_embed(W: np.ndarray) -> np.ndarray:
    """[[0, W], [W^T, 0]] (Sec. 1.1, Eq. bipartite)."""
    k = W.shape[0]
    A = np.zeros((2 * k, 2 * k), dtype=np.result_type(W.dtype, np.complex128))
    A[:k, k:] = W
    A[k:, :k] = W.T
    return A


def gaussian_square(k: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, np.sqrt(0.5), (k, k)) + 1j * rng.normal(0.0, np.sqrt(0.5), (k, k))


def grid_graph(a: int, b: int) -> np.ndarray:
    """Adjacency of the a x b grid graph P_a x P_b (vertex (i, j) -> i*b + j)."""
    n = a * b
    A = np.zeros((n, n), dtype=np.int64)
    for i in range(a):
        for j in range(b):
            v = i * b + j
            if j + 1 < b:
                A[v, v + 1] = A[v + 1, v] = 1
            if i + 1 < a:
                A[v, v + b] = A[v + b, v] = 1
    return A


def path_graph(n: int) -> np.ndarray:
    A = np.zeros((n, n), dtype=np.int64)
    for i in range(n - 1):
        A[i, i + 1] = A[i + 1, i] = 1
    return A


def haar_unitary(m: int, rng: np.random.Generator) -> np.ndarray:
    """Haar-random unitary: QR of a complex Gaussian matrix with the phases of R fixed."""
    Z = rng.normal(0.0, np.sqrt(0.5), (m, m)) + 1j * rng.normal(0.0, np.sqrt(0.5), (m, m))
    Q, R = np.linalg.qr(Z)
    d = np.diag(R)
    return Q * (d / np.abs(d))


def gbs_parent(seed: int, modes: int = 64, r: float = 0.8):
    """B = U diag(tanh r) U^T for a Haar U, and a complex Gaussian displacement vector."""
    rng = np.random.default_rng(seed)
    U = haar_unitary(modes, rng)
    B = (U * np.tanh(r)) @ U.T
    B = (B + B.T) / 2                 # symmetric to the last bit (the product is only up to rounding)
    gamma = rng.normal(0.0, np.sqrt(0.5), modes) + 1j * rng.normal(0.0, np.sqrt(0.5), modes)
    return B, gamma, rng


def gbs_submatrix(B: np.ndarray, gamma: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Rows/columns idx (with repetition) of B, diagonal replaced by gamma[idx]."""
    A = B[np.ix_(idx, idx)].copy()
    A[np.diag_indices(len(idx))] = gamma[idx]
    return np.ascontiguousarray(A)


def gbs_batch(count: int = 4096, seed: int = SEED_BATCH, nmin: int = 8, nmax: int = 32):
    """``count`` GBS-style loop-hafnian inputs of uneven even sizes in [nmin, nmax]."""
    B, gamma, rng = gbs_parent(seed)
    mats = []
    for _ in range(count):
        n = 2 * int(rng.integers(nmin // 2, nmax // 2 + 1))
        idx = np.sort(rng.integers(0, B.shape[0], n))
        mats.append(gbs_submatrix(B, gamma, idx))
    return mats


def pack(mats):
    """Pack square matrices contiguously: (flat complex128 array, element offsets, sizes)."""
    sizes = np.array([m.shape[0] for m in mats], dtype=np.int32)
    offs = np.zeros(len(mats), dtype=np.int64)
    tot = 0
    for i, m in enumerate(mats):
        offs[i] = tot
        tot += m.shape[0] * m.shape[0]
    flat = np.zeros(max(tot, 1), dtype=np.complex128)
    for i, m in enumerate(mats):
        flat[offs[i]: offs[i] + m.size] = m.ravel()
    return flat, offs, sizes


def serving_trace(num: int, qps: float, seed: int = SEED_SERVE, nmin: int = 12, nmax: int = 44,
                  skew: float = 0.7):
    """Poisson arrivals at ``qps``; n = nmin + 2j with P(j) ~ skew^j; kind 50/50 haf/lhaf.

    Returns a list of (t_arrival_seconds, kind, matrix).
    """
    B, gamma, rng = gbs_parent(seed)
    js = np.arange((nmax - nmin) // 2 + 1)
    pj = skew ** js
    pj = pj / pj.sum()
    t = 0.0
    out = []
    for _ in range(num):
        t += float(rng.exponential(1.0 / qps))
        n = nmin + 2 * int(rng.choice(js, p=pj))
        kind = int(rng.integers(0, 2))
        idx = np.sort(rng.integers(0, B.shape[0], n))
        A = gbs_submatrix(B, gamma, idx)
        if kind == 0:
            A[np.diag_indices(n)] = 0
        out.append((t, kind, A))
    return out


def random_permutation(n: int, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).permutation(n)
