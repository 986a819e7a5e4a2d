"""Pins of the oracle's graph (paper Alg. 1: exhaustive comparison inside each
cluster, update of G[i] and G[j], repeated over rounds) against brute force,
special cases and invariants."""
import numpy as np
import pytest

from paper_1701_08475_amd import datagen


def _brute_graph_from_leaves(X, k, perms, leaf_offs):
    """Row i: the k smallest (d, j) over the distinct co-leaf members of i in
    any tree, exact integer arithmetic (X holds small integers)."""
    Xi = X.astype(np.int64)
    n = len(X)
    cands = [set() for _ in range(n)]
    for perm, lo in zip(perms, leaf_offs):
        for s, e in zip(lo[:-1], lo[1:]):
            leaf = perm[s:e].tolist()
            for i in leaf:
                cands[i].update(j for j in leaf if j != i)
    ids = np.full((n, k), -1, np.int64)
    ds = np.full((n, k), np.inf)
    for i in range(n):
        c = sorted((int(((Xi[i] - Xi[j]) ** 2).sum()), j) for j in cands[i])[:k]
        for p, (d, j) in enumerate(c):
            ids[i, p] = j
            ds[i, p] = d
    return ids, ds


def test_graph_from_leaves_vs_brute_force(orc):
    X = datagen.random_points(300, 6, 21, "small_int")  # many exact ties
    k, L, ml = 7, 30, 8
    perms, offs = [], []
    for t in range(3):
        tr = orc.tree(X, L, ml, 10, 5, t)
        perms.append(tr["perm"])
        offs.append(tr["leaf_off"])
    ids, ds = orc.graph_from_leaves(X, k, np.stack(perms), offs)
    e_ids, e_ds = _brute_graph_from_leaves(X, k, perms, offs)
    assert np.array_equal(ids, e_ids)
    assert np.array_equal(ds, e_ds)


def _check_rows(X, ids, ds, k):
    n = len(X)
    x = X.astype(np.float64)
    for i in range(n):
        r = ids[i]
        assert len(set(r.tolist())) == k and i not in r and (r >= 0).all()
        d = ((x[r] - x[i]) ** 2).sum(1)
        np.testing.assert_allclose(ds[i], d, rtol=1e-13)
        key = list(zip(ds[i].tolist(), r.tolist()))
        assert key == sorted(key)


def test_graph_row_invariants(orc):
    X = datagen.make("c1", n=3000)
    ids, ds, st = orc.graph(X, 10, 3, 50, 1)
    _check_rows(X, ids, ds, 10)
    # symmetry of the distance in the output
    for i in range(0, 3000, 97):
        for p in range(10):
            j = ids[i, p]
            assert orc.d64(X, i, j) == orc.d64(X, j, i) == ds[i, p]


def test_graph_single_leaf_is_exact_knn(orc):
    X = datagen.make("c1", n=400)
    ids, ds, _ = orc.graph(X, 10, 2, 400, 3)
    e_ids, e_ds = orc.exact_knn(X, 10)
    assert np.array_equal(ids, e_ids) and np.array_equal(ds, e_ds)


def test_graph_merge_order_independent(orc):
    X = datagen.make("c1", n=2000)
    perms, offs = [], []
    for t in range(4):
        tr = orc.tree(X, 50, 11, 10, 7, t)
        perms.append(tr["perm"])
        offs.append(tr["leaf_off"])
    a = orc.graph_from_leaves(X, 10, np.stack(perms), offs)
    order = [2, 0, 3, 1]
    b = orc.graph_from_leaves(X, 10, np.stack([perms[o] for o in order]), [offs[o] for o in order])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    # and graph() builds the same trees (tree index keys the random pairs)
    g_ids, g_ds, _ = orc.graph(X, 10, 4, 50, 7)
    assert np.array_equal(a[0], g_ids) and np.array_equal(a[1], g_ds)


def test_graph_kth_distance_non_increasing_in_rounds(orc):
    X = datagen.make("c1", n=2500)
    prev = None
    for T in (1, 2, 3, 5):
        _, ds, _ = orc.graph(X, 10, T, 50, 4)
        if prev is not None:
            assert np.all(ds[:, -1] <= prev[:, -1])
            assert np.all(ds <= prev)  # every rank, since candidate sets only grow
        prev = ds


def test_recall_pins(orc):
    X = datagen.make("c1", n=1500)
    rows = datagen.sample_rows(1500, 200)
    E, Ed = orc.exact_knn(X, 10, rows)
    assert orc.recall(X, rows, E, E, Ed) == 1.0
    # a graph of the 10 farthest points has recall 0
    far = np.empty_like(E)
    x = X.astype(np.float64)
    for q, i in enumerate(rows):
        d = ((x - x[i]) ** 2).sum(1)
        far[q] = np.argsort(d)[-10:]
    assert orc.recall(X, rows, far, E, Ed) == 0.0
    # recall of the graph grows with the number of rounds (C1-shaped data)
    r = [orc.recall(X, rows, orc.graph(X, 10, T, 50, 1)[0][rows], E, Ed) for T in (1, 4)]
    assert 0.2 < r[0] < r[1] <= 1.0


def test_rows_from_leaves_matches_full_graph(orc):
    X = datagen.make("c1", n=2000)
    perms, offs = [], []
    for t in range(3):
        tr = orc.tree(X, 50, 11, 10, 2, t)
        perms.append(tr["perm"])
        offs.append(tr["leaf_off"])
    ids, ds = orc.graph_from_leaves(X, 10, np.stack(perms), offs)
    rows = datagen.sample_rows(2000, 300, seed=3)
    r_ids, r_ds = orc.rows_from_leaves(X, 10, np.stack(perms), offs, rows)
    assert np.array_equal(r_ids, ids[rows]) and np.array_equal(r_ds, ds[rows])
