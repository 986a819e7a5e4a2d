"""The benchmark's recall ground truth (its own FP64 brute force) against the
oracle's exact kNN and recall on small inputs."""
import numpy as np

import bench
from paper_1701_08475_amd import datagen


def test_exact_knn_matches_oracle_rows(orc):
    X = datagen.make("c1", n=3000)
    rows = datagen.sample_rows(3000, 60, seed=3)
    E, Ed = bench.exact_knn_fp64(X, X[rows], 10, self_ids=rows, block=1000)
    oE, oEd = orc.exact_knn(X, 10, rows)
    assert np.array_equal(E, oE)
    np.testing.assert_allclose(Ed, oEd, rtol=1e-12)


def test_exact_knn_integer_ties_and_external_queries(orc):
    X = datagen.random_points(2000, 16, 4, "small_int")  # many equal distances
    Q = datagen.random_points(40, 16, 5, "small_int")
    E, Ed = bench.exact_knn_fp64(X, Q, 12, block=700)
    oE, oEd = orc.exact_knn_points(X, Q, 12)
    assert np.array_equal(E, oE) and np.array_equal(Ed, oEd)


def test_recalls_match_oracle(orc):
    X = datagen.make("c1", n=3000)
    G, _, _ = orc.graph(X, 10, 1, 50, 1)
    rows = datagen.sample_rows(3000, 80, seed=7)
    E, Ed = bench.exact_knn_fp64(X, X[rows], 10, self_ids=rows)
    assert bench.graph_recall(X, rows, G[rows], E, Ed) == orc.recall(X, rows, G[rows], E, Ed)
    assert bench.search_recall(G[rows], E) == orc.search_recall(G[rows], E)
