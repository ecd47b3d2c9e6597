"""Host-side plan of the batched path (no GPU): every subset of every matrix is
covered exactly once, partial slots are distinct per matrix, chunk numbering is
contiguous per launch, and the largest chunks come first."""
import math

import pytest

from gen import inputs as gi


@pytest.fixture(scope="module")
def hg():
    import paper_1805_12498_amd as hg
    hg.load()
    return hg


def check_plan(hg, sizes, kinds):
    cls, nchunks, variant = hg.batched_plan(sizes, kinds)
    covered = {}
    slots = {}
    launch_chunks = [0, 0]
    launch = 0
    prev_cost = math.inf
    for item, m, cap, total, j0, base, slot_base, nslots in cls:
        if 2 * m <= 32 and launch == 0:
            launch, prev_cost = 1, math.inf
        assert base == launch_chunks[launch]                  # contiguous numbering
        # default layout table: 4 matrices per wave up to 16 rows, 2 up to 32, then 1
        W = 4 if 2 * m <= 16 else (2 if 2 * m <= 32 else 1)
        cost = -(-cap // W) * (2 * m) ** 3
        assert cost <= prev_cost                               # largest chunks first
        prev_cost = cost
        n_here = (total + cap - 1) // cap - j0
        launch_chunks[launch] += n_here
        assert 1 <= cap <= 64 and j0 == 0
        N = sizes[item] // 2 + (sizes[item] % 2)
        assert total == math.comb(N, m)
        covered[(item, m)] = covered.get((item, m), 0) + total
        for j in range(n_here):
            s = slot_base + j
            assert 0 <= s < nslots
            assert (item, s) not in slots
            slots[(item, s)] = True
    assert sum(launch_chunks) == nchunks
    for t, n in enumerate(sizes):
        if n == 0 or (n % 2 == 1 and kinds[t] == 0) or n + (n % 2) > 48:
            assert not any(k[0] == t for k in covered)
            continue
        N = (n + (n % 2)) // 2
        assert sum(v for (i, m), v in covered.items() if i == t) == 2 ** N - 1
        # every slot of the item is used
        item_slots = [s for (i, s) in slots if i == t]
        assert sorted(item_slots) == list(range(len(item_slots)))
    return cls, nchunks, variant


def test_plan_small_mixed(hg):
    sizes = list(range(0, 15)) * 2
    kinds = [0] * 15 + [1] * 15
    check_plan(hg, sizes, kinds)


def test_plan_gbs_batch(hg):
    mats = gi.gbs_batch(256, seed=gi.SEED_BATCH)
    sizes = [m.shape[0] for m in mats]
    cls, nchunks, variant = check_plan(hg, sizes, [1] * len(sizes))
    assert variant in (0, 1, 3)                # all items up to 32 rows: series bound 16
    assert all(2 * c[1] <= 32 for c in cls)


def test_plan_with_large_items(hg):
    sizes = [8, 40, 46, 50, 33]
    kinds = [1, 0, 1, 0, 1]
    cls, nchunks, variant = check_plan(hg, sizes, kinds)
    assert variant in (4, 5, 6)                # items above 32 rows: series bound 24
    big = [c for c in cls if 2 * c[1] > 32]
    assert big and all(2 * c[1] > 32 for c in cls[:len(big)])    # the large-subset launch comes first
    assert not any(c[0] == 3 for c in cls)      # n = 50 goes to the single-matrix path


def test_plan_chunk_sizes(hg):
    """Subsets per chunk shrink as (16/s)^3 (group_work 16 per matrix slot at 16 rows),
    between one per matrix slot and 64 per wave."""
    cls, _, _ = check_plan(hg, [32], [1])
    cap = {2 * c[1]: c[2] for c in cls}
    assert cap[16] == 64 and cap[8] == 64 and cap[2] == 64
    assert cap[24] == 2 * (16 * 4096 // 24 ** 3) and cap[32] == 2 * 2
