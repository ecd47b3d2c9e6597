"""GPU tests of the batched path (haf_batched_c128) through the C ABI.

Matrices up to 32 rows share launches (one coefficient and one series launch
per register layout and kind, one reduction); larger ones run the
single-matrix path on a pool of streams.  Checks: results against the CPU
oracle (brute force at small n, the formula in double-double at mid n), bitwise
equality with the single-matrix path and independence of a result from the
rest of the batch and from every configuration knob (layout table, subsets
per lane group, coefficient budget, stream count), bitwise reproducibility,
the constant and padded edge cases, the double-double output, errors and the
autotuner.
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
    hg.set_batched_config()
    print("device:", hg.device_info(), flush=True)
    yield hg
    hg.set_batched_config()


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def rand_sym(n, seed, scale=0.7):
    rng = np.random.default_rng(seed)
    G = rng.normal(0, scale, (n, n)) + 1j * rng.normal(0, scale, (n, n))
    return (G + G.T) / 2


def run_batch(hg, mats, kinds):
    import torch
    flat, offs, sizes = gi.pack(mats)
    dA = torch.from_numpy(flat).cuda()
    out = torch.full((max(len(mats), 1),), complex(np.nan, np.nan), dtype=torch.complex128, device="cuda")
    hg.batched_dev(dA.data_ptr(), offs, sizes, np.asarray(kinds, dtype=np.uint8), out.data_ptr(),
                   torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    return out.cpu().numpy()[:len(mats)]


def run_plain(hg, A, kind):
    import torch
    n = A.shape[0]
    dA = torch.from_numpy(np.ascontiguousarray(A) if n else np.zeros(1, complex)).cuda()
    out = torch.zeros(1, dtype=torch.complex128, device="cuda")
    hg.haf_dev(dA.data_ptr(), n, max(n, 1), out.data_ptr(), torch.cuda.current_stream().cuda_stream, kind=kind)
    torch.cuda.synchronize()
    return complex(out.cpu().numpy()[0])


def test_small_mixed_vs_brute_force(hg):
    """n = 0..14, both kinds, odd n included (haf 0, lhaf padded)."""
    mats, kinds = [], []
    for n in range(0, 15):
        for kind in (0, 1):
            mats.append(rand_sym(n, 300 + 2 * n + kind))
            kinds.append(kind)
    got = run_batch(hg, mats, kinds)
    for A, kind, g in zip(mats, kinds, got):
        ref = oracle.brute(A, bool(kind)).value
        if ref == 0:
            assert g == 0, (A.shape[0], kind, g)
        else:
            assert rel(g, ref) < 1e-12, (A.shape[0], kind, g, ref)


@pytest.mark.parametrize("table,span", [(0, 1), (0, 4), (1, 16)])
def test_gbs_batch_vs_oracle_and_plain(hg, table, span):
    """GBS-style loop hafnians n in [8, 32] (the batched workload's construction):
    bitwise the single-matrix path on all, the oracle (double-double formula) on a sample."""
    hg.set_batched_config(table=table, span=span)
    mats = gi.gbs_batch(48, seed=gi.SEED_BATCH + 1)
    kinds = [1] * len(mats)
    got = run_batch(hg, mats, kinds)
    for t, A in enumerate(mats):
        assert got[t] == run_plain(hg, A, 1), (table, span, t, A.shape[0])
    for t in range(0, len(mats), 8):
        ref, kappa = oracle.formula(mats[t], True, prec="dd", want_kappa=True)
        assert ref.relerr(got[t]) <= max(1e-12, C_TOL * EPS * kappa), (table, span, t, mats[t].shape[0])
    hg.set_batched_config()


def test_alone_equals_in_mix_bitwise(hg):
    """A result depends only on its own matrix: alone, in a batch of small items, and in a
    batch that also holds large items it is bitwise equal."""
    mats = gi.gbs_batch(24, seed=7)
    kinds = [t % 2 for t in range(len(mats))]
    mix = run_batch(hg, mats, kinds)
    big = [rand_sym(40, 1), rand_sym(46, 2)]
    mix2 = run_batch(hg, big + mats, [0, 1] + kinds)[2:]
    for t in (0, 5, 11, 23):
        alone = run_batch(hg, [mats[t]], [kinds[t]])[0]
        assert alone == mix[t] == mix2[t], (t, alone, mix[t], mix2[t])
    assert np.array_equal(mix, mix2)


def test_reproducible(hg):
    mats = gi.gbs_batch(32, seed=9)
    kinds = [1] * len(mats)
    assert np.array_equal(run_batch(hg, mats, kinds), run_batch(hg, mats, kinds))


@pytest.mark.parametrize("n", [34, 40, 50])
def test_large_items(hg, n):
    A = gi.gaussian_symmetric(n, 900 + n)
    small = rand_sym(10, 79)
    for kind in (0, 1):
        got = run_batch(hg, [small, A], [kind, kind])
        assert got[1] == run_plain(hg, A, kind), (n, kind)
        assert rel(got[0], oracle.brute(small, bool(kind)).value) < 1e-12
    if n <= 34:
        ref, kappa = oracle.formula(A, False, prec="dd", want_kappa=True)
        assert ref.relerr(run_batch(hg, [A], [0])[0]) <= C_TOL * EPS * kappa


def test_exact_counts(hg):
    """0/1 graphs: perfect-matching counts are exact integers (small enough to be exact in double)."""
    mats = [gi.random_graph(n, 0.5, 40 + n).astype(complex) for n in (8, 12, 16, 20, 24)]
    got = run_batch(hg, mats, [0] * len(mats))
    for A, g in zip(mats, got):
        assert round(g.real) == oracle.brute_int(A.real.astype(np.int64)) and g.imag == 0


def test_errors(hg):
    import torch
    from paper_1805_12498_amd._native import HafError
    dA = torch.zeros(16, dtype=torch.complex128, device="cuda")
    out = torch.zeros(2, dtype=torch.complex128, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    with pytest.raises(HafError, match="INVALID_ARG"):
        hg.batched_dev(dA.data_ptr(), [0], [4], [2], out.data_ptr(), st)
    with pytest.raises(HafError, match="INVALID_ARG"):
        hg.batched_dev(dA.data_ptr(), [0], [-2], [0], out.data_ptr(), st)
    with pytest.raises(HafError, match="TOO_LARGE"):
        hg.batched_dev(dA.data_ptr(), [0], [66], [0], out.data_ptr(), st)
    hg.batched_dev(dA.data_ptr(), [], [], [], out.data_ptr(), st)      # empty batch: nothing to do


def test_grouped_vs_ungrouped_bitwise(hg):
    """Shared launches (grouped, the default) against every matrix on its own launches:
    bitwise equal, over constants, odd n, padded odd-n loop hafnians, sizes past the
    shared range (n > 32), and a stage of n = 32 loop hafnians large enough to be cut into
    several launch pairs by a small coefficient budget; under both layout tables, several
    subsets-per-lane-group settings and 1 or 4 streams."""
    mats, kinds = [], []
    for n in list(range(0, 34)) + [36, 40]:
        for kind in (0, 1):
            mats.append(rand_sym(n, 5000 + 2 * n + kind))
            kinds.append(kind)
    for t in range(9):
        mats.append(rand_sym(32, 6000 + t))
        kinds.append(1)
    mats.append(rand_sym(31, 6100))
    kinds.append(1)
    runs = {}
    try:
        hg.set_batched_config(streams=4, grouped=0)
        u = run_batch(hg, mats, kinds)
        for table, span, streams, budget in ((0, 4, 4, 8192), (1, 1, 1, 64), (0, 16, 2, 64), (1, 64, 4, 8192)):
            hg.set_batched_config(table=table, span=span, streams=streams, coef_budget_mb=budget)
            runs[(table, span, streams, budget)] = run_batch(hg, mats, kinds)
    finally:
        hg.set_batched_config()
    for key, g in runs.items():
        for t in range(len(mats)):
            assert g[t] == u[t], (key, t, mats[t].shape[0], kinds[t], g[t], u[t])
    for t in (0, 5, 17, 40, 60, 71):
        assert u[t] == run_plain(hg, mats[t], kinds[t]), (t, mats[t].shape[0])


def test_double_double_output(hg):
    """haf_batched_c128x2: the (hi, lo) pairs of each result; hi + lo rounds to the
    complex128 result bitwise, and the pair equals the single-matrix x2 result."""
    import torch
    mats = gi.gbs_batch(40, seed=12) + [rand_sym(0, 1), rand_sym(5, 2), rand_sym(36, 3)]
    kinds = [t % 2 for t in range(len(mats))]
    flat, offs, sizes = gi.pack(mats)
    dA = torch.from_numpy(flat).cuda()
    out2 = torch.zeros((len(mats), 4), dtype=torch.float64, device="cuda")
    st = torch.cuda.current_stream().cuda_stream
    hg.batched_dev(dA.data_ptr(), offs, sizes, np.asarray(kinds, np.uint8), out2.data_ptr(), st, x2=True)
    torch.cuda.synchronize()
    got2 = out2.cpu().numpy()
    got = run_batch(hg, mats, kinds)
    one = torch.zeros(4, dtype=torch.float64, device="cuda")
    for t, A in enumerate(mats):
        assert complex(got2[t, 0] + got2[t, 1], got2[t, 2] + got2[t, 3]) == got[t], t
        if t % 7 == 0 or t >= len(mats) - 3:
            n = A.shape[0]
            dM = torch.from_numpy(np.ascontiguousarray(A) if n else np.zeros(1, complex)).cuda()
            hg.haf_dev(dM.data_ptr(), n, max(n, 1), one.data_ptr(), st, kind=kinds[t], x2=True)
            torch.cuda.synchronize()
            assert np.array_equal(one.cpu().numpy(), got2[t]), t


def test_autotuner(hg):
    import torch
    mats = gi.gbs_batch(64, seed=10)
    flat, offs, sizes = gi.pack(mats)
    kinds = np.ones(len(mats), dtype=np.uint8)
    dA = torch.from_numpy(flat).cuda()
    out = torch.zeros(len(mats), dtype=torch.complex128, device="cuda")
    cfg, ms = hg.batched_tune(dA.data_ptr(), offs, sizes, kinds, out.data_ptr(),
                              torch.cuda.current_stream().cuda_stream)
    print("tuned:", cfg, "%.3f ms" % ms, flush=True)
    assert hg.batched_config() == cfg and ms > 0 and cfg["streams"] in (1, 2, 4)
    assert cfg["grouped"] in (0, 1) and cfg["table"] in (0, 1) and 1 <= cfg["span"] <= 16
    tuned = out.cpu().numpy()
    again = run_batch(hg, mats, kinds)
    assert np.array_equal(tuned, again)
    hg.set_batched_config()


def test_autotune_cache(hg, tmp_path, monkeypatch):
    """HAF_AUTOTUNE_CACHE: the autotuner stores its choice as this device's line of the
    file (replacing an older one), and haf_batched_load_cache makes it current again."""
    import torch
    from paper_1805_12498_amd._native import HafError
    path = tmp_path / "tune.txt"
    monkeypatch.delenv("HAF_AUTOTUNE_CACHE", raising=False)
    with pytest.raises(HafError, match="STATE"):
        hg.batched_load_cache()
    monkeypatch.setenv("HAF_AUTOTUNE_CACHE", str(path))
    with pytest.raises(HafError, match="STATE"):        # no file yet: no entry for this device
        hg.batched_load_cache()
    mats = gi.gbs_batch(64, seed=33)
    flat, offs, sizes = gi.pack(mats)
    kinds = np.ones(len(mats), dtype=np.uint8)
    dA = torch.from_numpy(flat).cuda()
    out = torch.zeros(len(mats), dtype=torch.complex128, device="cuda")
    keep = hg.batched_config()
    try:
        path.write_text("# tuned batched configurations\nother:1 1 2 1 0 64\n")
        cfg, _ = hg.batched_tune(dA.data_ptr(), offs, sizes, kinds, out.data_ptr(), 0)
        hg.batched_tune(dA.data_ptr(), offs, sizes, kinds, out.data_ptr(), 0)   # replaces its own line
        lines = path.read_text().splitlines()
        assert lines[:2] == ["# tuned batched configurations", "other:1 1 2 1 0 64"]
        mine = [ln for ln in lines[2:]]
        assert len(mine) == 1 and mine[0].split()[0].startswith("gfx")
        hg.set_batched_config(table=1 - cfg["table"], span=3, streams=1, grouped=1, coef_budget_mb=128)
        got = hg.batched_load_cache()
        key, *vals = mine[0].split()
        assert [got[f] for f in ("table", "span", "streams", "grouped", "coef_budget_mb")] == [int(v) for v in vals]
        path.write_text("%s 0 0 1 1 64\n" % key)           # span 0 is out of range
        with pytest.raises(HafError, match="INVALID_ARG"):
            hg.batched_load_cache()
        path.write_text("%s 0 x\n" % key)
        with pytest.raises(HafError, match="INVALID_ARG"):
            hg.batched_load_cache()
    finally:
        hg.set_batched_config(**keep)
