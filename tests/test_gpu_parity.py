"""Parity of the HIP path with the CPU oracle (through the C ABI).

The GPU computes the two-means margins and centroid sums in FP64 like the
oracle, so trees are compared exactly (index work, bit-exact); graphs are
compared with the G1 rule (tests/gpu_helpers.py): FP32 distances within
1e-5 relative of FP64, ids equal except inside near-tie classes, and bit-exact
on integer data whose FP32 arithmetic is exact."""
import numpy as np
import pytest

from paper_1701_08475_amd import datagen
from tests.gpu_helpers import TAU, graph_parity, log, rows_sorted, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1701_08475_amd import knng
    knng.lib()
    return knng


def _np(t):
    return t.detach().cpu().numpy()


def _gpu_tree(K, Xd, L, ml, seed, t, max_iter=0):
    r = K.partition(Xd, L, ml, seed, t, max_iter=max_iter, with_nodes=True)
    return _np(r["perm"]), _np(r["leaf_off"]), _np(r["nodes"])


def _nodes_key(nodes):
    return sorted(map(tuple, np.asarray(nodes).tolist()))


# ------------------------------------------------------------------ trees
@pytest.mark.parametrize("name,n,L,ml,seed,trees", [
    ("c1", 10_000, 50, 11, 1, (0, 1, 2)),
    ("c2", 30_000, 100, 21, 2, (0, 5)),
])
def test_partition_identical_to_oracle(K, orc, name, n, L, ml, seed, trees):
    X = datagen.make(name, n=n)
    Xd = to_dev(X)
    for t in trees:
        log("partition %s n=%d tree=%d" % (name, n, t))
        perm, loff, nodes = _gpu_tree(K, Xd, L, ml, seed, t)
        o = orc.tree(X, L, ml, 10, seed, t, with_nodes=True)
        assert np.array_equal(loff, o["leaf_off"])
        assert np.array_equal(perm, o["perm"])
        assert _nodes_key(nodes) == _nodes_key(o["nodes"])


@pytest.mark.parametrize("n,D,kind,L,ml,max_iter", [
    (3001, 3, "normal", 20, 4, 10),       # D % 4 != 0, scalar loads
    (2000, 1, "normal", 16, 3, 10),       # 1-D
    (2500, 960, "normal", 64, 8, 10),     # wide rows (64 lanes per row)
    (2100, 130, "normal", 40, 7, 10),     # 130: scalar loads, 64 lanes
    (4096, 96, "normal", 30, 5, 1),       # one-pass budget
    (5000, 16, "small_int", 25, 13, 10),  # many exact ties and duplicates
    (1500, 8, "normal", 40, 1, 10),       # min_leaf 1
])
def test_partition_variants(K, orc, n, D, kind, L, ml, max_iter):
    X = datagen.random_points(n, D, n + D, kind)
    log("partition variant n=%d D=%d kind=%s" % (n, D, kind))
    perm, loff, nodes = _gpu_tree(K, to_dev(X), L, ml, 9, 3, max_iter=max_iter)
    o = orc.tree(X, L, ml, max_iter, 9, 3, with_nodes=True)
    assert np.array_equal(loff, o["leaf_off"])
    assert np.array_equal(perm, o["perm"])
    assert _nodes_key(nodes) == _nodes_key(o["nodes"])


# Integer data in [0, 255] (uint8 copy): nodes of at most 1024 rows (512 for
# D > 128) are split to leaves by the subtree kernel, one workgroup per node.
@pytest.mark.parametrize("n,D,kind,L,ml,max_iter", [
    (20000, 128, "c2", 100, 21, 10),      # level loop hands over at ~1000 rows
    (900, 128, "c2", 50, 11, 10),         # the root itself is a subtree
    (5000, 64, "int", 60, 30, 10),        # min_leaf = L/2: repairs on most splits
    (6000, 32, "small_int", 40, 5, 3),    # exact ties, three-pass budget
    (4000, 112, "int", 100, 21, 10),      # 7 chunks per row: no LDS swizzle
    (3000, 48, "small_int", 30, 1, 10),   # D = 48: part of a lane group idle
])
def test_subtree_kernel_matches_oracle(K, orc, n, D, kind, L, ml, max_iter, monkeypatch):
    X = datagen.make("c2", n=n) if kind == "c2" else datagen.random_points(n, D, n + D, kind)
    log("subtree n=%d D=%d kind=%s L=%d" % (n, D, kind, L))
    o = orc.tree(X, L, ml, max_iter, 4, 2, with_nodes=True)
    for sub, overlap in (("1", "1"), ("2", "0"), ("3", "1"), ("3", "0"), ("0", "1")):
        # overlap: subtree kernels on a second stream while the levels go on
        monkeypatch.setenv("KNNG_SUBTREE", sub)
        monkeypatch.setenv("KNNG_SUBTREE_OVERLAP", overlap)
        perm, loff, nodes = _gpu_tree(K, to_dev(X), L, ml, 4, 2, max_iter=max_iter)
        assert np.array_equal(loff, o["leaf_off"])
        assert np.array_equal(perm, o["perm"])
        assert _nodes_key(nodes) == _nodes_key(o["nodes"])
        # documented order of the node log: by depth, then start
        keys = [(int(d), int(st)) for st, _, _, d in nodes.tolist()]
        assert keys == sorted(keys)


# Integer data in [0, 255] through the level passes alone (no subtree kernel):
# the matrix-core assignment kernel with one and with four wavefronts per
# chunk, and the FP64 VALU kernel, each give the oracle's tree.
@pytest.mark.parametrize("n,D,kind,L,ml,max_iter", [
    (30000, 128, "c2", 100, 21, 10),
    (9000, 64, "int", 60, 30, 10),        # repairs on most splits
    (7000, 48, "small_int", 30, 1, 10),   # ties; D = 48: one lane of four idle
    (6000, 112, "int", 80, 5, 4),
    (5000, 16, "small_int", 25, 3, 10),   # one 16-byte slice per row
])
def test_level_assignment_kernels_match_oracle(K, orc, n, D, kind, L, ml, max_iter, monkeypatch):
    X = datagen.make("c2", n=n) if kind == "c2" else datagen.random_points(n, D, n + D, kind)
    o = orc.tree(X, L, ml, max_iter, 7, 1, with_nodes=True)
    monkeypatch.setenv("KNNG_SUBTREE", "0")
    for mfma, wide, order in (("1", "0", "0"), ("1", "1000000", "1"), ("0", "0", "3"),
                              ("1", "1000000", "2")):
        log("level kernels n=%d D=%d kind=%s mfma=%s wide_max=%s order=%s" % (
            n, D, kind, mfma, wide, order))
        monkeypatch.setenv("KNNG_ASSIGN_MFMA", mfma)
        monkeypatch.setenv("KNNG_ASSIGN_WIDE_MAX", wide)
        monkeypatch.setenv("KNNG_CHUNK_ORDER", order)
        monkeypatch.setenv("KNNG_CHUNK_ORDER_MIN", "0")  # small cases: order every level
        perm, loff, nodes = _gpu_tree(K, to_dev(X), L, ml, 7, 1, max_iter=max_iter)
        assert np.array_equal(loff, o["leaf_off"])
        assert np.array_equal(perm, o["perm"])
        assert _nodes_key(nodes) == _nodes_key(o["nodes"])


def test_partition_identical_points_closed_form(K):
    X = np.full((300, 6), 3.5, np.float32)
    perm, loff, _ = _gpu_tree(K, to_dev(X), 50, 11, 9, 0)
    assert loff.tolist() == [0, 37, 75, 112, 150, 187, 225, 262, 300]
    assert perm.tolist() == list(range(300))


def test_partition_single_leaf(K):
    X = datagen.random_points(64, 5, 1)
    perm, loff, nodes = _gpu_tree(K, to_dev(X), 64, 11, 9, 0)
    assert loff.tolist() == [0, 64] and perm.tolist() == list(range(64)) and len(nodes) == 0


# ------------------------------------------------------------------ graphs
def test_build_c1_matches_oracle(K, orc):
    c = datagen.CONFIGS["c1"]
    X = datagen.make("c1")
    log("build c1")
    ids, ds = K.build(to_dev(X), c["k"], c["n_trees"], c["leaf_max"], seed=c["seed"])
    o_ids, o_d, _ = orc.graph(X, c["k"], c["n_trees"], c["leaf_max"], c["seed"])
    rows = np.arange(len(X))
    frac = graph_parity(orc, X, rows, _np(ids), _np(ds), o_ids, o_d)
    log("c1 identical id fraction %.6f" % frac)
    assert frac > 0.999
    assert rows_sorted(_np(ids), _np(ds))


@pytest.mark.parametrize("n,D,k,T,L,seed", [(6000, 24, 8, 4, 40, 5), (4000, 7, 5, 3, 30, 6)])
def test_build_multi_tree_matches_oracle(K, orc, n, D, k, T, L, seed):
    X = datagen.gmm_uniform(n, D, 30, -8, 8, 1.0, seed)
    log("build multi n=%d D=%d T=%d" % (n, D, T))
    ids, ds = K.build(to_dev(X), k, T, L, seed=seed)
    o_ids, o_d, _ = orc.graph(X, k, T, L, seed)
    frac = graph_parity(orc, X, np.arange(n), _np(ids), _np(ds), o_ids, o_d)
    assert frac > 0.999


def test_build_integer_data_bit_exact(K, orc):
    """Integers 0..255, D=128: every FP32 partial sum is an exact integer
    below 2^24, so d32 == d64 and the whole graph matches bit for bit."""
    X = datagen.make("c2", n=20_000)
    log("build integer n=20000")
    ids, ds = K.build(to_dev(X), 20, 3, 100, seed=2)
    o_ids, o_d, _ = orc.graph(X, 20, 3, 100, 2)
    graph_parity(orc, X, np.arange(len(X)), _np(ids), _np(ds), o_ids, o_d, strict=True)


@pytest.mark.parametrize("k,L,rerank", [(100, 256, 2), (20, 100, 8), (70, 512, 2)])
def test_integer_data_fp32_request_any_rerank(K, orc, k, L, rerank):
    """FP32 requests on integer data take the exact BF16 leaf pass, which keeps
    the k best whatever rerank_factor is; where its kernels cannot serve
    (k, leaf_max) (k = 70 with leaves above 256 points) the FP32 direct kernel
    does.  Either way the graph equals the oracle's bit for bit."""
    X = datagen.make("c2", n=5000)
    log("integer data fp32 request k=%d L=%d rerank=%d" % (k, L, rerank))
    ids, ds, st = K.build(to_dev(X), k, 2, L, seed=5, rerank_factor=rerank, stats=True)
    assert st["exact_first_pass"] == (0 if k > 64 and L > 256 else 1)
    o_ids, o_d, _ = orc.graph(X, k, 2, L, 5)
    graph_parity(orc, X, np.arange(len(X)), _np(ids), _np(ds), o_ids, o_d, strict=True)


def test_leaf_search_on_oracle_leaves(K, orc):
    import torch
    X = datagen.make("c1", n=8000)
    perms, offs = [], []
    for t in range(3):
        tr = orc.tree(X, 50, 11, 10, 4, t)
        perms.append(tr["perm"])
        offs.append(tr["leaf_off"])
    log("leaf search on oracle leaves")
    ids, ds = K.leaf_search(to_dev(X), 10, torch.from_numpy(np.stack(perms)).cuda(),
                            [torch.from_numpy(o).cuda() for o in offs])
    o_ids, o_d = orc.graph_from_leaves(X, 10, np.stack(perms), offs)
    frac = graph_parity(orc, X, np.arange(len(X)), _np(ids), _np(ds), o_ids, o_d)
    assert frac > 0.999


def test_single_leaf_is_exact_knn(K, orc):
    X = datagen.make("c1", n=500)
    ids, ds = K.build(to_dev(X), 10, 2, 512, seed=3)
    e_ids, e_d = orc.exact_knn(X, 10)
    graph_parity(orc, X, np.arange(500), _np(ids), _np(ds), e_ids, e_d)


def test_k_is_n_minus_1(K, orc):
    X = datagen.random_points(12, 5, 2)
    ids, ds = K.build(to_dev(X), 11, 1, 23, seed=1)
    e_ids, e_d = orc.exact_knn(X, 11)
    graph_parity(orc, X, np.arange(12), _np(ids), _np(ds), e_ids, e_d)


def test_duplicate_rows(K, orc):
    base = datagen.random_points(400, 10, 3, "small_int")
    X = np.concatenate([base, base, base[:200]])  # every row duplicated
    ids, ds = K.build(to_dev(X), 6, 2, 30, seed=8)
    o_ids, o_d, _ = orc.graph(X, 6, 2, 30, 8)
    graph_parity(orc, X, np.arange(len(X)), _np(ids), _np(ds), o_ids, o_d, strict=True)


def test_small_min_leaf_pads_rows(K, orc):
    """min_leaf 2 < k+1: leaves of 2..L points; rows with fewer than k
    distinct candidates are padded with (-1, +inf) like the oracle."""
    X = datagen.random_points(500, 4, 5)
    ids, ds = K.build(to_dev(X), 8, 1, 6, seed=3, min_leaf=2)
    o_ids, o_d, _ = orc.graph(X, 8, 1, 6, 3, min_leaf=2)
    graph_parity(orc, X, np.arange(500), _np(ids), _np(ds), o_ids, o_d)
    assert (_np(ids) == -1).any()
    assert np.isinf(_np(ds)[_np(ids) == -1]).all()


def test_plain_schedule_equals_batched(K):
    X = to_dev(datagen.make("c1", n=6000))
    a = K.build(X, 10, 3, 50, seed=11)
    b = K.build(X, 10, 3, 50, seed=11, plain=True)
    assert np.array_equal(_np(a[0]), _np(b[0])) and np.array_equal(_np(a[1]), _np(b[1]))


def test_deterministic(K):
    X = to_dev(datagen.make("c1"))
    a = K.build(X, 10, 2, 50, seed=1)
    b = K.build(X, 10, 2, 50, seed=1)
    assert np.array_equal(_np(a[0]), _np(b[0]))
    assert np.array_equal(_np(a[1]).view(np.int32), _np(b[1]).view(np.int32))


def test_power_of_two_scaling(K):
    X = datagen.make("c1", n=5000)
    a = K.build(to_dev(X), 10, 2, 50, seed=3)
    b = K.build(to_dev(X * np.float32(8.0)), 10, 2, 50, seed=3)
    assert np.array_equal(_np(a[0]), _np(b[0]))
    assert np.array_equal(_np(a[1]) * np.float32(64.0), _np(b[1]))


def test_nonfinite_rejected_outputs_untouched(K):
    import torch
    X = datagen.random_points(300, 8, 1)
    X[17, 3] = np.nan
    Xd = to_dev(X)
    ids = torch.full((300, 5), 7, dtype=torch.int32, device="cuda")
    ds = torch.full((300, 5), 3.0, dtype=torch.float32, device="cuda")
    with pytest.raises(K.KnngError) as e:
        K.build(Xd, 5, 1, 20, out=(ids, ds))
    assert e.value.status == K.KNNG_ERR_NONFINITE
    assert bool((ids == 7).all()) and bool((ds == 3.0).all())


def test_runs_on_a_side_stream(K):
    import torch
    X = to_dev(datagen.make("c1", n=3000))
    ref = K.build(X, 10, 2, 50, seed=4)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        got = K.build(X, 10, 2, 50, seed=4)
    torch.cuda.synchronize()
    assert np.array_equal(_np(ref[0]), _np(got[0]))


def test_stats(K):
    X = to_dev(datagen.make("c1"))
    ids, ds, st = K.build(X, 10, 2, 50, seed=1, stats=True)
    assert st["leaves"] > 2 * 10_000 // 50 - 10
    assert st["ordered_pairs"] > 0 and st["assign_rows"] >= 2 * 10_000
    assert st["ms_total"] > 0


def test_compact_storage_is_lossless(K, orc):
    """Integer data in [0, 255]: the uint8 copy the partition streams holds the
    same values, so the graph is bit-identical to the FP32-storage build."""
    X = datagen.make("c2", n=30_000)
    Xd = to_dev(X)
    a_ids, a_d, a_st = K.build(Xd, 20, 3, 100, seed=7, stats=True)
    b_ids, b_d, b_st = K.build(Xd, 20, 3, 100, seed=7, stats=True, compact=False)
    assert a_st["compact_used"] == 1 and b_st["compact_used"] == 0
    assert np.array_equal(_np(a_ids), _np(b_ids))
    assert np.array_equal(_np(a_d).view(np.int32), _np(b_d).view(np.int32))
    # and a value outside [0, 255] (or a fraction) disables it
    Y = X.copy()
    Y[5, 5] = 255.5
    _, _, c_st = K.build(to_dev(Y), 20, 1, 100, seed=7, stats=True)
    assert c_st["compact_used"] == 0
