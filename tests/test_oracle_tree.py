"""Pins of the oracle's two-means tree (paper Sec. 3.1: bisection by two-means
clustering down to clusters no bigger than the threshold) against hand-traced
splits, closed forms and invariants."""
import itertools

import numpy as np
import pytest

from paper_1701_08475_amd import datagen
from tests.golden import load_splits

SPLITS = load_splits()


def test_splitmix64_published_vectors(orc):
    # SplitMix64 seeded with 0: first three outputs (Steele, Lea, Flood 2014;
    # the same stream as java.util.SplittableRandom with seed 0).
    g = 0x9E3779B97F4A7C15
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    got = [orc.mix64((g * i) & 0xFFFFFFFFFFFFFFFF) for i in (1, 2, 3)]
    assert got == want


@pytest.mark.parametrize("case", SPLITS, ids=[c["case"] for c in SPLITS])
def test_split_hand_traced(orc, case):
    X = np.array(case["points"], np.float32)[:, None]
    mem = np.arange(len(X), dtype=np.int32)
    a, b = case["init"]
    lab, n0, c, rep, passes = orc.split_init(X, mem, case["min_leaf"][0], case["max_iter"][0], a, b)
    assert sorted(mem[lab == 0].tolist()) == case["left"]
    assert sorted(mem[lab == 1].tolist()) == case["right"]
    assert n0 == len(case["left"])
    assert passes == case["passes"][0]
    assert rep == bool(case["repaired"][0])
    np.testing.assert_allclose(c[:, 0], case["centres"], rtol=1e-15)


def test_two_clusters_every_ordered_init(orc):
    """{0, 1, 10, 11}: every ordered starting pair ends at {0,1} | {10,11}."""
    X = np.array([[0], [1], [10], [11]], np.float32)
    mem = np.arange(4, dtype=np.int32)
    for a, b in itertools.permutations(range(4), 2):
        lab, n0, _, rep, _ = orc.split_init(X, mem, 1, 10, a, b)
        sides = {tuple(mem[lab == 0]), tuple(mem[lab == 1])}
        assert sides == {(0, 1), (2, 3)}, (a, b)
        assert not rep
    # and the tree with threshold 2 has exactly these two leaves for any seed
    for seed in range(20):
        t = orc.tree(X, 2, 1, 10, seed, 0)
        leaves = [tuple(sorted(t["perm"][s:e])) for s, e in zip(t["leaf_off"][:-1], t["leaf_off"][1:])]
        assert sorted(leaves) == [(0, 1), (2, 3)]


def test_init_pair_distinct_in_range_and_keyed(orc):
    seen = set()
    for seed in range(400):
        a, b = orc.init_pair(seed, 0, 0, 4)
        assert 0 <= a < 4 and 0 <= b < 4 and a != b
        seen.add((a, b))
    assert len(seen) == 12  # every ordered pair occurs
    for m in (2, 3, 101, 1_000_000):
        for seed in range(30):
            a, b = orc.init_pair(seed, 3, 17, m)
            assert 0 <= a < m and 0 <= b < m and a != b
    # the key depends on tree, smallest id and size
    base = orc.key_hash(7, 0, 5, 100, 0)
    assert len({base, orc.key_hash(7, 1, 5, 100, 0), orc.key_hash(7, 0, 6, 100, 0),
                orc.key_hash(7, 0, 5, 101, 0), orc.key_hash(7, 0, 5, 100, 1)}) == 5


def _leaves(t):
    lo = t["leaf_off"]
    return [t["perm"][s:e] for s, e in zip(lo[:-1], lo[1:])]


@pytest.mark.parametrize("n,D,L,ml,seed", [(3000, 32, 50, 11, 1), (2500, 8, 40, 5, 2), (777, 3, 20, 1, 3)])
def test_tree_invariants(orc, n, D, L, ml, seed):
    X = datagen.gmm_uniform(n, D, 20, -10, 10, 1.0, seed)
    t = orc.tree(X, L, ml, 10, seed, 0, with_nodes=True)
    perm = t["perm"]
    assert sorted(perm.tolist()) == list(range(n))
    lo = t["leaf_off"]
    assert lo[0] == 0 and lo[-1] == n and np.all(np.diff(lo) > 0)
    for leaf in _leaves(t):
        assert ml <= len(leaf) <= L
        assert np.all(np.diff(leaf) > 0)  # stable partition keeps ids ascending
    for s, m, n0, _ in t["nodes"]:
        assert m > L and ml <= n0 <= m - ml
    assert t["stats"]["internal_nodes"] == len(lo) - 2  # binary tree


def test_tree_single_leaf_when_small(orc):
    X = datagen.random_points(50, 4, 0)
    t = orc.tree(X, 50, 11, 10, 3, 0)
    assert t["leaf_off"].tolist() == [0, 50]
    assert t["perm"].tolist() == list(range(50))


def test_tree_identical_points_closed_form(orc):
    """All points equal: every split is a tie, every margin 0, so each node
    of m points splits into the floor(m/2) smallest ids | the rest.
    300 -> 150|150 -> 75|75 -> 37|38, leaves of threshold 50."""
    X = np.full((300, 6), 3.5, np.float32)
    t = orc.tree(X, 50, 11, 10, 9, 0)
    assert t["leaf_off"].tolist() == [0, 37, 75, 112, 150, 187, 225, 262, 300]
    assert t["perm"].tolist() == list(range(300))


def test_tree_1d_leaves_are_intervals(orc):
    rng = np.random.default_rng(4)
    x = rng.standard_normal(2000).astype(np.float32)
    X = x[:, None]
    t = orc.tree(X, 30, 4, 10, 5, 0)
    rank = np.empty(2000, np.int64)
    rank[np.argsort(x, kind="stable")] = np.arange(2000)
    for leaf in _leaves(t):
        r = np.sort(rank[leaf])
        assert r[-1] - r[0] == len(r) - 1


def test_tree_power_of_two_scaling_invariant(orc):
    X = datagen.gmm_uniform(2000, 16, 10, -5, 5, 1.0, 8)
    t1 = orc.tree(X, 40, 6, 10, 11, 2)
    for p in (-3, 5):
        t2 = orc.tree(X * np.float32(2.0 ** p), 40, 6, 10, 11, 2)
        assert np.array_equal(t1["perm"], t2["perm"])
        assert np.array_equal(t1["leaf_off"], t2["leaf_off"])


def test_split_converged_is_lloyd_fixed_point(orc):
    """A split that stopped because no label changed has centres equal to the
    means of its sides and every point on the side of its nearer centre."""
    X = datagen.gmm_uniform(600, 5, 6, -4, 4, 1.0, 12)
    mem = np.arange(600, dtype=np.int32)
    checked = 0
    for seed in range(25):
        lab, n0, c, rep, passes = orc.split_init(X, mem, 1, 50, *orc.init_pair(seed, 0, 0, 600))
        if rep or passes >= 50 or n0 in (0, 600):
            continue
        x = X.astype(np.float64)
        np.testing.assert_allclose(c[0], x[lab == 0].mean(0), rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(c[1], x[lab == 1].mean(0), rtol=1e-12, atol=1e-12)
        d0 = ((x - c[0]) ** 2).sum(1)
        d1 = ((x - c[1]) ** 2).sum(1)
        assert np.array_equal(lab.astype(bool), d1 < d0)
        checked += 1
    assert checked >= 10


def test_tree_deterministic_and_keyed_by_tree_index(orc):
    X = datagen.gmm_uniform(1500, 8, 10, -5, 5, 1.0, 13)
    a = orc.tree(X, 40, 6, 10, 21, 0)
    b = orc.tree(X, 40, 6, 10, 21, 0)
    c = orc.tree(X, 40, 6, 10, 21, 1)
    assert np.array_equal(a["perm"], b["perm"])
    assert not np.array_equal(a["perm"], c["perm"])
