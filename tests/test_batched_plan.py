"""Host-side plan of the shared batched launches (no GPU): every subset size
class of every matrix up to 32 rows is covered by exactly one coefficient chunk
and one series chunk with the same coefficient area, partial slots are those of
the single-matrix plan and distinct across matrices, workgroup numbering is
contiguous per launch, every chunk sits in a launch whose layout serves its
subset size, coefficient areas of a launch are disjoint and within budget."""
import math

import numpy as np
import pytest

from gen import inputs as gi

SERIES_BLOCK = 256
# (largest s, matrices per wave, family (P, Q, polynomial split)) of the register
# layouts, in table order
LAYOUT_SM = [8, 12, 16, 20, 24, 28, 32, 40, 48]
LAYOUT_W = [4, 4, 4, 4, 2, 2, 2, 1, 1]
LAYOUT_FAMILY = [(4, 4, 0), (4, 4, 0), (4, 4, 0), (4, 4, 3), (8, 4, 0), (8, 4, 1), (8, 4, 1), (8, 8, 2), (8, 8, 2)]


def fine_layout(s):
    return next(i for i, x in enumerate(LAYOUT_SM) if s <= x)


def coarse_layout(s):
    """The first layout of the fine one's family with a multiple of 8 rows, else the fine one."""
    f = fine_layout(s)
    return next((i for i in range(f, len(LAYOUT_SM))
                 if LAYOUT_FAMILY[i] == LAYOUT_FAMILY[f] and LAYOUT_SM[i] % 8 == 0), f)


@pytest.fixture(scope="module")
def hg():
    import paper_1805_12498_amd as hg
    hg.load()
    yield hg
    hg.set_batched_config()


def single_plan_slots(n_eff):
    """Slots of the single-matrix plan: size classes m = 1..N in order, one slot per
    series block of 256 subsets (one chunk per class for N <= 16)."""
    N = n_eff // 2
    slot0, s = {}, 0
    for m in range(1, N + 1):
        slot0[m] = s
        s += -(-math.comb(N, m) // SERIES_BLOCK)
    return slot0, s


def check_plan(hg, sizes, kinds, table, span, budget_mb):
    hg.set_batched_config(table=table, span=span, coef_budget_mb=budget_mb)
    launches, chunks = hg.batched_plan(sizes, kinds)
    expect = {}
    base = {}
    nxt = 0
    for t, (n, k) in enumerate(zip(sizes, kinds)):
        if n == 0 or (n % 2 and k == 0):
            continue                                   # constants: prologue only
        ne = n + (n % 2)
        assert ne <= 32
        slot0, total = single_plan_slots(ne)
        base[t] = nxt
        nxt += total
        for m in range(1, ne // 2 + 1):
            expect[(t, m)] = slot0[m]
    seen = {0: {}, 1: {}}
    budget = budget_mb * (1 << 20) // 16
    assert len(launches) % 2 == 0
    for li, (what, lay, loops, blocks, first, nch, celems, sm) in enumerate(launches):
        assert what == li % 2                          # coefficient launch, then its series launch
        assert sm == LAYOUT_SM[lay]
        rows = chunks[first:first + nch]
        g = 0
        areas = []
        for item, m, count, gstart, coff, slot, N, rank0 in rows:
            assert gstart == g                         # contiguous workgroups
            if what == 0:
                assert sm - 8 < 2 * m <= sm            # the layout serves this subset size
                assert lay == (coarse_layout(2 * m) if table == 1 else fine_layout(2 * m))
                w = LAYOUT_W[lay] * span
                g += -(-count // w)
            else:
                g += -(-count // SERIES_BLOCK)
            assert kinds[item] == loops
            ne = sizes[item] + (sizes[item] % 2)
            assert N == ne // 2 and rank0 == 0 and count == math.comb(N, m)
            assert slot == base[item] + expect[(item, m)]
            key = (item, m)
            assert key not in seen[what], key
            seen[what][key] = (li // 2, coff)
            ncoef = 2 * N if loops else N
            areas.append((coff, coff + count * ncoef))
        assert g == blocks
        areas.sort()
        for (a0, a1), (b0, b1) in zip(areas, areas[1:]):
            assert a1 <= b0                            # disjoint coefficient areas
        assert areas[-1][1] == celems
        assert celems <= budget or nch == 1
    # both launches of a pair see the same chunks at the same coefficient offsets
    assert seen[0] == seen[1]
    assert set(seen[0]) == set(expect)
    return launches


def test_gbs_batch_plan(hg):
    mats = gi.gbs_batch(512, seed=gi.SEED_BATCH)
    sizes = [m.shape[0] for m in mats]
    kinds = [1] * len(mats)
    for table, span in ((0, 1), (0, 4), (1, 8)):
        launches = check_plan(hg, sizes, kinds, table, span, 8192)
        # one launch pair per layout that the batch uses: 9 or 5 stages at most
        assert len(launches) // 2 <= (9 if table == 0 else 5)


def test_mixed_plan_small_budget(hg):
    sizes, kinds = [], []
    for n in range(0, 33):
        for k in (0, 1):
            sizes.append(n)
            kinds.append(k)
    sizes += [32] * 6 + [31, 33, 40]
    kinds += [1] * 6 + [1, 0, 1]
    # 33 (haf, odd: constant) stays in the shared launches; 40 does not
    big = [t for t, n in enumerate(sizes) if n + (n % 2) * kinds[t] > 32 and not (n % 2 and kinds[t] == 0)]
    keep = [t for t in range(len(sizes)) if t not in big]
    launches = check_plan(hg, [sizes[t] for t in keep], [kinds[t] for t in keep], 0, 2, 64)
    assert len(launches) > 2 * 9                       # the 64 MiB budget cuts some stages
    check_plan(hg, [sizes[t] for t in keep], [kinds[t] for t in keep], 1, 64, 64)


def test_plan_lists_only_shared_matrices(hg):
    hg.set_batched_config()
    launches, chunks = hg.batched_plan([34, 40, 12, 0, 7], [0, 1, 0, 1, 0])
    items = set(int(i) for i in chunks[:, 0])
    assert items == {2}


def test_plan_rejects_bad_items(hg):
    from paper_1805_12498_amd._native import HafError
    with pytest.raises(HafError, match="INVALID_ARG"):
        hg.batched_plan([4, 66], [0, 0])
    with pytest.raises(HafError, match="INVALID_ARG"):
        hg.batched_plan([4], [3])
    with pytest.raises(HafError, match="INVALID_ARG"):
        hg.set_batched_config(span=0)
    with pytest.raises(HafError, match="INVALID_ARG"):
        hg.set_batched_config(streams=8)
    hg.set_batched_config()
    assert hg.batched_config() == {"table": 0, "span": 4, "streams": 4, "grouped": 1, "coef_budget_mb": 8192}
    launches, chunks = hg.batched_plan([], [])
    assert len(launches) == 0 and len(chunks) == 0
