"""Pins of the oracle's distance and exact-kNN functions against things other
than itself: exact rational arithmetic, a closed form, and scipy."""
from fractions import Fraction

import numpy as np
import pytest

from paper_1701_08475_amd import datagen


def _brute_exact(X, k):
    """Exact kNN with rational arithmetic on the float32 inputs."""
    Xf = [[Fraction(float(v)) for v in row] for row in X]
    n = len(Xf)
    out_ids, out_d = [], []
    for i in range(n):
        c = []
        for j in range(n):
            if j != i:
                c.append((sum((a - b) * (a - b) for a, b in zip(Xf[i], Xf[j])), j))
        c.sort()
        out_ids.append([j for _, j in c[:k]])
        out_d.append([d for d, _ in c[:k]])
    return out_ids, out_d


@pytest.mark.parametrize("n,D,k,kind,seed", [
    (2, 1, 1, "normal", 0), (5, 3, 4, "normal", 1), (9, 2, 3, "small_int", 2),
    (9, 4, 8, "small_int", 3), (30, 5, 6, "normal", 4), (40, 3, 7, "small_int", 5)])
def test_exact_knn_vs_rational_enumeration(orc, n, D, k, kind, seed):
    X = datagen.random_points(n, D, seed, kind)
    ids, ds = orc.exact_knn(X, k)
    e_ids, e_d = _brute_exact(X, k)
    # small_int data has many exact ties: the (d, id) order must match exactly
    assert ids.tolist() == e_ids
    for i in range(n):
        for p in range(k):
            assert ds[i, p] == pytest.approx(float(e_d[i][p]), rel=1e-15, abs=0)


@pytest.mark.parametrize("n,k,h,axis_dim", [(37, 6, 0.5, 3), (64, 10, 2.0, 1), (12, 11, 0.25, 5)])
def test_exact_knn_1d_lattice_closed_form(orc, n, k, h, axis_dim):
    """x_i = i*h on one axis: the neighbours of i are i-1, i+1, i-2, i+2, ...
    (ties at equal offset go to the smaller id), continuing on the open side
    at the boundary; the o-th offset is at squared distance (o*h)^2."""
    X = np.zeros((n, axis_dim), np.float32)
    X[:, axis_dim // 2] = np.arange(n, dtype=np.float32) * np.float32(h)
    ids, ds = orc.exact_knn(X, k)
    for i in range(n):
        exp = []
        o = 1
        while len(exp) < k:
            if i - o >= 0:
                exp.append(i - o)
            if i + o < n and len(exp) < k:
                exp.append(i + o)
            o += 1
        assert ids[i].tolist() == exp
        assert ds[i].tolist() == [float((abs(j - i) * h) ** 2) for j in exp]


def test_exact_knn_vs_scipy(orc):
    from scipy.spatial import cKDTree
    X = datagen.random_points(3000, 8, 11, "normal")
    rows = datagen.sample_rows(3000, 300, seed=5)
    k = 10
    ids, ds = orc.exact_knn(X, k, rows)
    tr = cKDTree(X.astype(np.float64))
    sd, si = tr.query(X[rows].astype(np.float64), k=k + 1)
    for q, i in enumerate(rows):
        keep = si[q] != i
        s_ids, s_d = si[q][keep][:k], sd[q][keep][:k] ** 2
        np.testing.assert_allclose(ds[q], s_d, rtol=1e-12)
        # ids agree wherever the neighbouring distances are not near-ties
        for p in range(k):
            lo = ds[q, p - 1] if p > 0 else -np.inf
            hi = ds[q, p + 1] if p + 1 < k else np.inf
            if ds[q, p] - lo > 1e-9 * ds[q, p] and hi - ds[q, p] > 1e-9 * ds[q, p]:
                assert ids[q, p] == s_ids[p]


def test_d64_symmetric_and_exact_on_integers(orc):
    X = datagen.random_points(50, 128, 3, "int")
    for i, j in [(0, 1), (5, 49), (17, 30)]:
        a, b = orc.d64(X, i, j), orc.d64(X, j, i)
        assert a == b
        exact = int(((X[i].astype(np.int64) - X[j].astype(np.int64)) ** 2).sum())
        assert a == float(exact)
    assert orc.d64(X, 7, 7) == 0.0


def test_exact_knn_pads_when_k_exceeds_n_minus_1(orc):
    X = datagen.random_points(4, 2, 0, "normal")
    ids, ds = orc.exact_knn(X, 6)
    assert (ids[:, 3:] == -1).all() and np.isinf(ds[:, 3:]).all()
    assert (ids[:, :3] >= 0).all()
