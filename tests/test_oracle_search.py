"""The oracle's E-GNNS search (Alg. 2, readings R10-R13) against values fixed
independently of it: brute force where the search provably reaches every
node, hand-traced walks on a chain graph, exact integer distances."""
import numpy as np
import pytest

from paper_1701_08475_amd import datagen


def _brute_topk(X, q, cand, k):
    """k smallest (d64, id) over the candidate ids, padded with (-1, inf)."""
    cand = sorted(set(int(c) for c in cand if 0 <= c < len(X)))
    d = [float(np.sum((X[c].astype(np.float64) - q.astype(np.float64)) ** 2)) for c in cand]
    order = sorted(range(len(cand)), key=lambda i: (d[i], cand[i]))[:k]
    ids = [cand[i] for i in order] + [-1] * (k - len(order))
    ds = [d[i] for i in order] + [np.inf] * (k - len(order))
    return np.array(ids, np.int32), np.array(ds)


def test_d32_exact_on_integers(orc):
    """Integer data: every term and partial sum of d32 is an exact FP32
    integer, so d32 is the exact squared distance."""
    a = np.arange(32, dtype=np.float32)
    assert orc.d32(a, np.zeros(32, np.float32)) == sum(i * i for i in range(32))  # 10416
    rng = np.random.default_rng(3)
    x = rng.integers(0, 256, size=(40, 128)).astype(np.float32)
    for i in range(0, 40, 2):
        exact = int(np.sum((x[i].astype(np.int64) - x[i + 1].astype(np.int64)) ** 2))
        assert orc.d32(x[i], x[i + 1]) == exact


def test_d32_blocks_of_32_hand_worked(orc):
    """Non-integer d32 at D = 33, worked by hand (u = 2^-24, FP32 round to
    nearest even; the ulp is 2u on [1, 2) and 4u on [2, 4)).

    b: dims 0, 1, 32 differ by 1, 1.5 * 2^-12, 1 + 2^-12.
       block 0..31: fma(1,1,0) = 1; 1 + 2.25u rounds to 1 + 2u.
       block 32:    (1 + 2^-12)^2 = 1 + 2^-11 + u, a tie, to even 1 + 2^-11.
       total:       2 + 2^-11 + 2u, a tie, to even 2 + 2^-11.
       One sequential chain over all 33 dims instead ends with
       1 + 2u + (1 + 2^-11 + u) = 2 + 2^-11 + 3u, rounded up to 2 + 2^-11 + 4u.
    c: dims 0, 16, 17, 32 differ by 1, 2^-12, 2^-12, 2^-12.
       block 0..31: 1 + u twice, each a tie, to even 1; block 32: u;
       total 1 + u, a tie, to even: 1.  Blocks of 16 would give
       1 + (u + u) = 1 + 2u, then + u = 1 + 3u, a tie, to even 1 + 4u."""
    a = np.zeros(33, np.float32)
    b = a.copy()
    b[0], b[1], b[32] = 1.0, 1.5 * 2.0 ** -12, 1.0 + 2.0 ** -12
    c = a.copy()
    c[0], c[16], c[17], c[32] = 1.0, 2.0 ** -12, 2.0 ** -12, 2.0 ** -12
    assert orc.d32(a, b) == 2.0 + 2.0 ** -11
    assert orc.d32(b, a) == 2.0 + 2.0 ** -11
    assert orc.d32(a, c) == 1.0
    assert orc.d32(c, a) == 1.0
    # the FP64 distances differ from both (D = 33, dims in order)
    X = np.stack([a, b, c])
    assert orc.d64(X, 0, 1) == 1.0 + 2.25 * 2.0 ** -24 + (1.0 + 2.0 ** -12) ** 2
    assert orc.d64(X, 0, 2) == 1.0 + 3 * 2.0 ** -24


def test_d32_d40_last_block_partial(orc):
    """D = 40: the second block holds 8 dimensions.  Dims 0 and 39 differ by
    1 and 2^-12: block 0 = 1, block 1 = u, total 1 + u, a tie, to even 1
    (a block of 40 would also give 1; dims 0, 38, 39 by 1, 2^-12, 2^-12
    give 1 + 2u within block 1 first: 1 + 2u exactly)."""
    a = np.zeros(40, np.float32)
    b = a.copy()
    b[0], b[39] = 1.0, 2.0 ** -12
    c = a.copy()
    c[0], c[38], c[39] = 1.0, 2.0 ** -12, 2.0 ** -12
    assert orc.d32(a, b) == 1.0
    assert orc.d32(a, c) == 1.0 + 2.0 ** -23


def test_zero_rounds_is_topk_of_the_seeds(orc):
    X = datagen.random_points(300, 12, 5, "normal")
    Q = datagen.random_points(20, 12, 6, "normal")
    G = np.full((300, 4), -1, np.int32)
    rng = np.random.default_rng(7)
    S = rng.integers(0, 300, size=(20, 9)).astype(np.int32)
    ids, ds = orc.egnns(X, G, Q, S, 5, 0, dist_mode=0)
    for q in range(20):
        bi, bd = _brute_topk(X, Q[q], S[q], 5)
        assert np.array_equal(ids[q], bi)
        np.testing.assert_allclose(ds[q], bd, rtol=1e-12)


def test_complete_graph_gives_exact_knn(orc):
    """Every node is a neighbour of every other: one round from any seed
    visits all n points, so R is the exact k nearest (O2)."""
    n, D, k = 60, 7, 6
    X = datagen.random_points(n, D, 11, "normal")
    Q = datagen.random_points(10, D, 12, "normal")
    G = np.array([[j for j in range(n) if j != i] for i in range(n)], np.int32)
    S = (np.arange(10, dtype=np.int32) * 5).reshape(10, 1)
    ids, ds = orc.egnns(X, G, Q, S, k, 1, dist_mode=0)
    for q in range(10):
        bi, bd = _brute_topk(X, Q[q], range(n), k)
        assert np.array_equal(ids[q], bi)
        np.testing.assert_allclose(ds[q], bd, rtol=1e-12)


def _chain():
    X = np.arange(10, dtype=np.float32).reshape(10, 1)  # points 0..9 on a line
    G = np.array([[i - 1 if i > 0 else -1, i + 1 if i < 9 else -1] for i in range(10)], np.int32)
    return X, G


def test_chain_walk_hand_traced(orc):
    """Points 0..9 on a line, each linked to its two neighbours, query 7.3,
    seed {0}.  k = 1: each round moves the best one step right, so after r
    rounds R = {min(r, 7)}; at 7 the only new neighbour (8, d 0.49) loses and
    the next round has nothing to expand.  k = 2: after r rounds R = {r, r-1}
    up to r = 7 (round 7 adds 7 next to 6), then round 8 expands 7 and swaps
    6 (d 1.69) for 8 (d 0.49): {7, 8} from then on."""
    X, G = _chain()
    Q = np.array([[7.3]], np.float32)
    S = np.array([[0]], np.int32)
    for r in range(12):
        ids, ds = orc.egnns(X, G, Q, S, 1, r, dist_mode=0)
        assert ids[0, 0] == min(r, 7)
        ids2, _ = orc.egnns(X, G, Q, S, 2, r, dist_mode=0)
        want = [0, -1] if r == 0 else ([r, r - 1] if r <= 7 else [7, 8])
        assert ids2[0].tolist() == want, (r, ids2[0].tolist())
    _, ds = orc.egnns(X, G, Q, S, 2, 20, dist_mode=0)
    q = float(np.float32(7.3))  # the query as stored
    np.testing.assert_allclose(ds[0], [(q - 7) ** 2, (8 - q) ** 2], rtol=1e-12)


def test_seed_duplicates_and_invalid_ids(orc):
    X, G = _chain()
    Q = np.array([[4.6], [0.2]], np.float32)
    a = orc.egnns(X, G, Q, np.array([[2, 2, 2, -1], [9, 9, 12, 9]], np.int32), 3, 4, dist_mode=0)
    b = orc.egnns(X, G, Q, np.array([[2], [9]], np.int32), 3, 4, dist_mode=0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_unreachable_nodes_pad(orc):
    """Two disconnected pairs: from a seed in the first only two nodes are
    ever visited, so a k = 4 list holds two entries and two paddings."""
    X = np.array([[0.0], [1.0], [10.0], [11.0]], np.float32)
    G = np.array([[1], [0], [3], [2]], np.int32)
    ids, ds = orc.egnns(X, G, np.array([[10.5]], np.float32), np.array([[0]], np.int32), 4, 5,
                        dist_mode=0)
    assert ids[0].tolist() == [1, 0, -1, -1]
    assert np.isinf(ds[0, 2]) and np.isinf(ds[0, 3])


def test_more_rounds_never_worse(orc):
    """The k-th distance of R never grows, so every rank of the output is
    non-increasing in the number of rounds."""
    X = datagen.make("c1", n=3000)
    ids_g, _, _ = orc.graph(X, 10, 1, 50, 1)
    Q = datagen.random_points(30, X.shape[1], 21, "normal") * 4.0
    S = np.random.default_rng(22).integers(0, len(X), size=(30, 4)).astype(np.int32)
    prev = None
    for r in range(0, 8):
        _, ds = orc.egnns(X, ids_g, Q, S, 10, r, dist_mode=1)
        if prev is not None:
            assert np.all(ds <= prev)
        prev = ds


def test_d32_order_equals_d64_on_integer_data(orc):
    """Integer data in [0, 255]: d32 = d64 exactly, so both rank orders
    give the same search."""
    X = datagen.random_points(2000, 32, 31, "int")
    ids_g, _, _ = orc.graph(X, 8, 2, 40, 3)
    Q = datagen.random_points(25, 32, 32, "int")
    S = np.random.default_rng(33).integers(0, 2000, size=(25, 6)).astype(np.int32)
    a = orc.egnns(X, ids_g, Q, S, 8, 6, dist_mode=0)
    b = orc.egnns(X, ids_g, Q, S, 8, 6, dist_mode=1)
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1], b[1])


def test_exact_knn_points_brute_force(orc):
    """Tiny inputs: against a sort of all distances (numpy, FP64)."""
    X = datagen.random_points(150, 5, 41, "normal")
    Q = datagen.random_points(12, 5, 42, "normal")
    ids, ds = orc.exact_knn_points(X, Q, 7)
    for q in range(12):
        d = np.sum((X.astype(np.float64) - Q[q].astype(np.float64)) ** 2, axis=1)
        order = np.lexsort((np.arange(150), d))[:7]
        assert np.array_equal(ids[q], order)
        np.testing.assert_allclose(ds[q], d[order], rtol=1e-12)


def test_query_generator_shares_the_mixture():
    """Queries come from the same centres as the config's data: every
    query of the small C1 mixture lies near some data point's centre."""
    X = datagen.make("c1", n=20000)
    Q = datagen.queries("c1", 50)
    d = ((Q[:, None, :].astype(np.float64) - X[None, :2000, :]) ** 2).sum(-1).min(1)
    # same mixture: nearest of 2000 data points is within the noise scale
    # (sigma = 1, D = 32: squared distances ~ 2 * 32); an unrelated draw of
    # centres in [-10, 10]^32 would be hundreds away
    assert np.median(d) < 150


def test_work_counts_hand_traced(orc):
    """Chain 0..9, query 7.3, seed 0, k = 1: round t (t <= 8) expands the
    current best and takes one new distance (its unvisited right neighbour);
    round 8 expands 7, whose new neighbour 8 does not enter R, and round 9
    has nothing to expand.  So r rounds take 1 + min(r, 8) distances and
    expand min(r, 8) nodes.  A complete graph of n nodes: one round from one
    seed takes n distances and expands one node."""
    X, G = _chain()
    Q = np.array([[7.3]], np.float32)
    S = np.array([[0]], np.int32)
    for r in range(12):
        _, _, (nd, ne) = orc.egnns(X, G, Q, S, 1, r, dist_mode=0, with_work=True)
        assert (nd, ne) == (1 + min(r, 8), min(r, 8)), r
    n = 40
    Xc = datagen.random_points(n, 3, 50, "normal")
    Gc = np.array([[j for j in range(n) if j != i] for i in range(n)], np.int32)
    Qc = datagen.random_points(4, 3, 51, "normal")
    Sc = np.arange(4, dtype=np.int32).reshape(4, 1)
    _, _, (nd, ne) = orc.egnns(Xc, Gc, Qc, Sc, 5, 1, dist_mode=0, with_work=True)
    assert (nd, ne) == (4 * n, 4)
