"""The oracle's RVQ inverted index and cascaded seeds (Sec. 4.1-4.2, Eqns
1-3, readings R14-R19) against values fixed independently of it: cluster
means known in closed form, the k-means fixed point and monotone objective,
hand-made vocabularies whose codes are known, the direct form of Eqn 2, and
brute-force key rankings on tiny inputs."""
import numpy as np
import pytest

from paper_1701_08475_amd import datagen


def _sqd(P, W):
    """All squared distances, direct form in FP64 (numpy)."""
    return ((P[:, None, :].astype(np.float64) - W[None, :, :].astype(np.float64)) ** 2).sum(-1)


def test_kmeans_recovers_separated_cluster_means(orc):
    """Four clusters, each a centre plus the offsets +-e_d / 2: the mean of
    every cluster is its centre exactly, and Lloyd started from one member of
    each cluster must reach it and stop."""
    D = 6
    centres = np.array([[0] * D, [40] * D, [-40] + [0] * (D - 1), [0, 0, 0, 0, 0, 80]], np.float64)
    rows, lab = [], []
    for c in range(4):
        for d in range(D):
            for s in (0.5, -0.5):
                v = centres[c].copy()
                v[d] += s
                rows.append(v)
                lab.append(c)
    P = np.array(rows)
    init = np.array([0, 2 * D + 3, 4 * D + 1, 6 * D + 7], np.int32)  # one member of each
    W, codes, rounds = orc.kmeans(P, init, 20)
    assert np.array_equal(W, centres)
    assert np.array_equal(codes, np.array(lab))
    # the starting words already give every row its cluster's code, so the
    # first round (update to the means, assign) changes no code and ends
    assert rounds == 1


def test_kmeans_zero_rounds_is_nearest_start_word(orc):
    P = datagen.random_points(300, 9, 1, "normal").astype(np.float64)
    init = np.array([5, 17, 100, 250], np.int32)
    W, codes, rounds = orc.kmeans(P, init, 0)
    assert rounds == 0 and np.array_equal(W, P[init])
    assert np.array_equal(codes, np.argmin(_sqd(P, W), axis=1))


def test_kmeans_fixed_point(orc):
    """Converged Lloyd: every code is the nearest word (brute force) and every
    word is the mean of its members (numpy)."""
    P = datagen.random_points(2000, 12, 2, "normal").astype(np.float64)
    init = np.random.default_rng(3).choice(2000, 16, replace=False).astype(np.int32)
    W, codes, rounds = orc.kmeans(P, init, 200)
    assert rounds < 200
    d = _sqd(P, W)
    best = d.min(1)
    assert np.all(d[np.arange(2000), codes] <= best * (1 + 1e-12) + 1e-12)
    for j in range(16):
        mem = P[codes == j]
        assert len(mem) > 0
        np.testing.assert_allclose(W[j], mem.mean(0), rtol=1e-12, atol=1e-13)


def test_kmeans_objective_never_grows(orc):
    """Lloyd's sum of squares is non-increasing in the number of rounds."""
    P = datagen.random_points(1500, 8, 4, "normal").astype(np.float64) * 3.0
    init = np.arange(0, 1500, 150, dtype=np.int32)
    prev = np.inf
    for r in range(8):
        W, codes, _ = orc.kmeans(P, init, r)
        sse = float(((P - W[codes]) ** 2).sum())
        assert sse <= prev * (1 + 1e-12)
        prev = sse


def test_kmeans_word_without_members_keeps_its_value(orc):
    """Two starting words on identical rows: ties go to the lower index, so
    the higher one has no member after the first assignment; the first update
    keeps its value and moves the others to their members' means."""
    P = datagen.random_points(200, 5, 6, "normal").astype(np.float64)
    P[7] = P[3]
    init = np.array([3, 7, 50, 120], np.int32)
    _, codes0, _ = orc.kmeans(P, init, 0)
    assert not np.any(codes0 == 1)
    W, _, _ = orc.kmeans(P, init, 1)
    assert np.array_equal(W[1], P[7])
    for j in (0, 2, 3):
        np.testing.assert_allclose(W[j], P[codes0 == j].mean(0), rtol=1e-13, atol=1e-14)


def _handmade(K1=5, K2=4, D=8):
    rng = np.random.default_rng(8)
    V1 = rng.integers(-3, 4, size=(K1, D)).astype(np.float64) * 100.0
    V1[:, 0] = np.arange(K1) * 100.0  # distinct words
    V2 = np.zeros((K2, D))
    for l in range(K2):
        V2[l, l % D] = 4.0 * (1 + l // D)
    return V1, V2


def test_encode_recovers_handmade_codes(orc):
    """x = V1[a] + V2[b] + noise, with the V1 words 100 apart and the V2
    words 4 apart: the codes are (a, b) (R17)."""
    V1, V2 = _handmade()
    rng = np.random.default_rng(9)
    a = rng.integers(0, len(V1), 400)
    b = rng.integers(0, len(V2), 400)
    X = (V1[a] + V2[b] + rng.normal(0, 0.05, size=(400, V1.shape[1]))).astype(np.float32)
    key = orc.rvq_encode(X, V1, V2)
    assert np.array_equal(key, a * len(V2) + b)


def test_rvq_train_stages(orc):
    """Stage 1 is k-means of the sample rows; stage 2 is k-means of their
    residues x - w1[c1] (R14); the sample's codes are the encoding's."""
    X = datagen.random_points(3000, 10, 10, "normal")
    train, init1, init2 = datagen.rvq_sample(3000, 1200, 8, 6)
    W1, W2, c1, c2, rounds = orc.rvq_train(X, train, init1, init2, 15)
    P = X[train].astype(np.float64)
    W1b, c1b, r1 = orc.kmeans(P, init1, 15)
    assert np.array_equal(W1, W1b) and np.array_equal(c1, c1b) and rounds[0] == r1
    R = P - W1[c1]
    W2b, c2b, r2 = orc.kmeans(R, init2, 15)
    assert np.array_equal(W2, W2b) and np.array_equal(c2, c2b) and rounds[1] == r2
    assert np.array_equal(orc.rvq_encode(X[train], W1, W2), c1 * 6 + c2)


def test_ivf_lists_brute_force(orc):
    key = np.random.default_rng(11).integers(0, 37, 5000).astype(np.int32)
    key[key == 5] = 6  # an empty list
    offsets, ids = orc.ivf_lists(key, 40)
    assert offsets[0] == 0 and offsets[-1] == 5000
    for I in range(40):
        want = np.nonzero(key == I)[0]
        assert np.array_equal(ids[offsets[I]:offsets[I + 1]], want)


def test_key_distance_is_eqn2(orc):
    """term1 = |q - w1|^2 and d(q, I) = |q - w1 - w2|^2 (direct form, numpy):
    the reading of Eqn 3's garbled signs (R18).  A dropped factor 2 or a flipped
    sign moves the value by the size of a dot product, far above rounding."""
    rng = np.random.default_rng(12)
    D = 24
    W1 = rng.normal(0, 5, size=(7, D))
    W2 = rng.normal(0, 1, size=(5, D))
    for t in range(5):
        q = rng.normal(0, 5, size=D).astype(np.float32)
        t1, dist = orc.ivf_key_dist(q, W1, W2)
        qd = q.astype(np.float64)
        want1 = ((qd - W1) ** 2).sum(1)
        want = ((qd[None, None, :] - W1[:, None, :] - W2[None, :, :]) ** 2).sum(-1)
        scale = (qd @ qd) + (W1 ** 2).sum(1).max() + (W2 ** 2).sum(1).max()
        np.testing.assert_allclose(t1, want1, rtol=0, atol=1e-12 * scale)
        np.testing.assert_allclose(dist, want, rtol=0, atol=1e-12 * scale)


def _brute_seeds(q, W1, W2, offsets, ids, n1, ns):
    qd = q.astype(np.float64)
    t1 = ((qd - W1) ** 2).sum(1)
    first = sorted(range(len(W1)), key=lambda j: (t1[j], j))[:n1]
    keys = []
    for j in first:
        for l in range(len(W2)):
            keys.append((float(((qd - W1[j] - W2[l]) ** 2).sum()), j * len(W2) + l))
    keys.sort()
    out = []
    for _, I in keys:
        out.extend(ids[offsets[I]:offsets[I + 1]].tolist())
    out = out[:ns]
    return out + [-1] * (ns - len(out))


@pytest.mark.parametrize("n1,ns", [(4, 60), (2, 60), (1, 10), (4, 1000)])
def test_seeds_brute_force(orc, n1, ns):
    """Tiny index (K1 = K2 = 4): the cascade's seeds equal a brute-force walk
    of the lists under the n1 nearest first-stage words, in the order of the
    direct key distance (R19); more seeds than ids pads with -1."""
    X = datagen.random_points(300, 6, 13, "normal") * 3.0
    train, init1, init2 = datagen.rvq_sample(300, 300, 4, 4, seed=14)
    W1, W2, _, _, _ = orc.rvq_train(X, train, init1, init2, 10)
    key = orc.rvq_encode(X, W1, W2)
    offsets, ids = orc.ivf_lists(key, 16)
    Q = datagen.random_points(25, 6, 15, "normal") * 3.0
    S = orc.ivf_seeds(Q, W1, W2, offsets, ids, n1, ns)
    for qi in range(25):
        assert S[qi].tolist() == _brute_seeds(Q[qi], W1, W2, offsets, ids, n1, ns)
    if ns > 300 and n1 == 4:
        assert np.array_equal(np.sort(S[:, :300], axis=1), np.tile(np.arange(300), (25, 1)))
        assert np.all(S[:, 300:] == -1)
