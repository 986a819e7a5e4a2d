"""Reduced-precision leaf search on MFMA (BF16 / FP16 / FP8-e4m3 first pass,
FP32 re-rank) against the oracle's emulation (reading R9) and the FP32 path.

Exact cases are compared bit for bit: integer data is exact in BF16 (so the
first pass is exact), and a candidate budget covering the whole leaf makes
the first pass irrelevant.  Otherwise the first pass rounds differently on
the GPU (FP32 accumulation in the matrix cores) than in the FP64 emulation,
so the comparison is: every GPU row is valid (distinct co-leaf ids, d32
within 1e-5 of d64, sorted) and agrees with the emulation on nearly all
positions."""
import numpy as np
import pytest

from paper_1701_08475_amd import datagen
from tests.gpu_helpers import TAU, graph_parity, log, reduced_parity, rows_sorted, to_dev

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


def _oracle_leaves(orc, X, T, L, ml, seed):
    perms, offs = [], []
    for t in range(T):
        tr = orc.tree(X, L, ml, 10, seed, t)
        perms.append(tr["perm"])
        offs.append(tr["leaf_off"])
    return np.stack(perms), offs


def _gpu_leaf_search(K, X, k, perms, offs, precision, rerank=2):
    import torch
    return K.leaf_search(to_dev(X), k, torch.from_numpy(perms).cuda(),
                         [torch.from_numpy(o).cuda() for o in offs], precision=precision,
                         rerank_factor=rerank)


def _co_leaf_sets(perms, offs, n):
    sets = [set() for _ in range(n)]
    for perm, lo in zip(perms, offs):
        for s, e in zip(lo[:-1], lo[1:]):
            leaf = perm[s:e].tolist()
            for i in leaf:
                sets[i].update(leaf)
    return sets


def _valid_rows(orc, X, ids, ds, co, k):
    n = len(X)
    d64 = orc.pair_d64(X, np.arange(n), np.where(ids >= 0, ids, 0))
    for i in range(n):
        r = ids[i][ids[i] >= 0]
        assert len(set(r.tolist())) == len(r) and i not in r
        assert set(r.tolist()) <= co[i]
        dv = ds[i][: len(r)].astype(np.float64)
        assert np.all(np.abs(dv - d64[i][: len(r)]) <= TAU * d64[i][: len(r)])
    assert rows_sorted(ids, ds)


def test_bf16_integer_data_bit_identical_to_fp32(K, orc):
    """Integers 0..255, D=128: the BF16 first pass is exact, so the exact
    matrix-core path (taken for FP32 and BF16 requests) gives the FP32 direct
    path's graph bit for bit."""
    X = datagen.make("c2", n=20_000)
    Xd = to_dev(X)
    log("bf16 build on integer data")
    a = K.build(Xd, 20, 3, 100, seed=2, compact=False, stats=True)   # FP32 rows, FP32 leaves
    b = K.build(Xd, 20, 3, 100, seed=2, precision="bf16", stats=True)
    f = K.build(Xd, 20, 3, 100, seed=2, stats=True)                  # FP32 request
    assert a[2]["exact_first_pass"] == 0 and b[2]["exact_first_pass"] == 1
    assert f[2]["exact_first_pass"] == 1
    for r in (b, f):
        assert np.array_equal(_np(a[0]), _np(r[0]))
        assert np.array_equal(_np(a[1]).view(np.int32), _np(r[1]).view(np.int32))
    o_ids, o_d, _ = orc.graph(X, 20, 3, 100, 2)
    graph_parity(orc, X, np.arange(len(X)), _np(b[0]), _np(b[1]), o_ids, o_d, strict=True)


@pytest.mark.parametrize("precision,L,rerank", [
    ("bf16", 50, 5), ("fp16", 50, 5), ("fp8", 50, 5),       # wave-per-row kernel (c = 50)
    ("bf16", 30, 3), ("fp16", 30, 3), ("fp8", 30, 3),       # thread-per-row kernel (c = 30)
])
def test_full_candidate_budget_equals_fp32(K, orc, precision, L, rerank):
    """rerank * k >= leaf size - 1: every co-leaf member is re-ranked with
    d32, so the result is the FP32 path's, bit for bit."""
    X = datagen.make("c1", n=5000)
    perms, offs = _oracle_leaves(orc, X, 2, L, 11, 4)
    a = _gpu_leaf_search(K, X, 10, perms, offs, "fp32")
    b = _gpu_leaf_search(K, X, 10, perms, offs, precision, rerank=rerank)
    assert np.array_equal(_np(a[0]), _np(b[0]))
    assert np.array_equal(_np(a[1]).view(np.int32), _np(b[1]).view(np.int32))


@pytest.mark.parametrize("precision,n,D,k,T,L,kind", [
    ("bf16", 6000, 32, 10, 2, 50, "c1"),      # thread-per-row kernel (c = 20)
    ("fp16", 6000, 128, 16, 2, 100, "unit960"),  # thread-per-row, 112-point tiles (c = 32)
    ("fp8", 5000, 64, 12, 2, 128, "c1"),      # thread-per-row, 128-point tiles (c = 24)
    ("fp16", 3000, 960, 20, 2, 200, "unit960"),
    ("fp8", 6000, 96, 32, 2, 500, "unit96"),
    ("fp8", 4000, 32, 10, 2, 100, "c1"),
    ("fp16", 2000, 40, 6, 1, 30, "c1"),      # D not a multiple of 32
])
def test_reduced_matches_emulation(K, orc, precision, n, D, k, T, L, kind):
    if kind == "c1":
        X = datagen.gmm_uniform(n, D, 20, -10, 10, 1.0, 11)
    elif kind == "unit960" and D != 960:
        X = datagen.gmm_unit(n, D, 16, 0.35, 13)
    else:
        X = datagen.gmm_unit(n, D, 16, 0.35, 12)
    perms, offs = _oracle_leaves(orc, X, T, L, k + 1, 5)
    log("reduced %s n=%d D=%d L=%d" % (precision, n, D, L))
    ids, ds = _gpu_leaf_search(K, X, k, perms, offs, precision)
    ids, ds = _np(ids), _np(ds)
    _valid_rows(orc, X, ids, ds, _co_leaf_sets(perms, offs, n), k)
    rows = np.arange(n)
    same = reduced_parity(orc, X, precision, k, 2 * k, perms, offs, rows, ids, ds)
    log("  rows identical to the emulation %.5f" % same)


@pytest.mark.parametrize("precision", ["fp8", "fp16", "bf16"])
def test_reduced_build_end_to_end(K, orc, precision):
    """The whole build (C1 data, 2 trees) with a reduced first pass: every
    row satisfies the widened G1 rule against the emulation on the GPU's own
    leaves (the trees equal the oracle's), and recall@10 on all rows, paired
    with the plain FP32 build on the same rows, is within 0.1 percentage
    point of it."""
    import torch
    X = datagen.make("c1")
    Xd = to_dev(X)
    ids, ds, st = K.build(Xd, 10, 2, 50, seed=1, precision=precision, stats=True)
    p_ids, _ = K.build(Xd, 10, 2, 50, seed=1, plain=True)
    assert st["leaves"] > 0
    # the build equals the leaf search on the GPU's own partitions
    parts = [K.partition(Xd, 50, 11, 1, t) for t in range(2)]
    l_ids, l_ds = K.leaf_search(Xd, 10, torch.stack([r["perm"] for r in parts]),
                                [r["leaf_off"] for r in parts], precision=precision)
    assert torch.equal(ids, l_ids) and torch.equal(ds.view(torch.int32), l_ds.view(torch.int32))
    perms = np.stack([_np(r["perm"]) for r in parts])
    offs = [_np(r["leaf_off"]) for r in parts]
    rows = np.arange(len(X))
    same = reduced_parity(orc, X, precision, 10, 20, perms, offs, rows, _np(ids), _np(ds))
    E, Ed = orc.exact_knn(X, 10, rows)
    r_red = orc.recall(X, rows, _np(ids), E, Ed)
    r_plain = orc.recall(X, rows, _np(p_ids), E, Ed)
    log("%s: rows identical to the emulation %.4f; recall %.5f vs plain FP32 %.5f"
        % (precision, same, r_red, r_plain))
    assert abs(r_red - r_plain) <= 0.001


@pytest.mark.parametrize("precision,L", [
    ("fp32", 50), ("fp32", 200),                  # FP32 direct kernel
    ("bf16", 50), ("fp16", 50), ("fp8", 50),      # thread-per-row kernel (c = 20)
    ("bf16", 200), ("fp8", 200),                  # wave-per-row kernel
])
def test_ties_fall_to_smaller_id_on_shuffled_leaves(K, orc, precision, L):
    """Integers 0..3 (many equal distances; exact in every first-pass format,
    so d~ = d32 = d64) with each leaf's ids shuffled: the c = 2k pre-selection
    and the final list must break distance ties by id, not by position, so the
    result equals the oracle's (d, id)-ordered graph bit for bit."""
    X = datagen.random_points(3000, 16, 21, "small_int")
    perms, offs = _oracle_leaves(orc, X, 2, L, 11, 6)
    rng = np.random.default_rng(5)
    sh = perms.copy()
    for t in range(len(offs)):
        for s, e in zip(offs[t][:-1], offs[t][1:]):
            sh[t, s:e] = rng.permutation(sh[t, s:e])
    log("shuffled leaves %s L=%d" % (precision, L))
    ids, ds = _gpu_leaf_search(K, X, 10, sh, offs, precision)
    o_ids, o_d = orc.graph_from_leaves(X, 10, perms, offs)
    assert np.array_equal(_np(ids), o_ids)
    assert np.array_equal(_np(ds).astype(np.float64), o_d)


@pytest.mark.parametrize("precision,n,D,k,L,kind,ml", [
    ("fp8", 8000, 96, 32, 500, "unit96", 33),      # leaves from 33 to 500 points: four buckets
    ("fp16", 4000, 960, 20, 200, "unit960", 21),   # up to 256 points
    ("bf16", 6000, 128, 20, 300, "int", 21),       # exact first pass (integer data)
    ("fp8", 5000, 64, 16, 260, "unit96", 2),       # tiny leaves next to large ones
])
def test_leaf_size_buckets_identical(K, orc, precision, n, D, k, L, kind, ml, monkeypatch):
    """Leaves grouped by size (at most 64, 128, 256, 512 points), each group
    run by the kernel shaped for it, give the same lists bit for bit as one
    launch shaped by the largest leaf."""
    if kind == "int":
        X = datagen.random_points(n, D, 17, "int")
    elif kind == "unit960" and D == 960:
        X = datagen.gmm_unit(n, D, 16, 0.35, 12)
    else:
        X = datagen.gmm_unit(n, D, 16, 0.35, 13)
    perms, offs = _oracle_leaves(orc, X, 2, L, ml, 7)
    sizes = np.concatenate([np.diff(o) for o in offs])
    log("leaf buckets %s n=%d D=%d sizes %d..%d" % (precision, n, D, sizes.min(), sizes.max()))
    assert sizes.max() > 128
    monkeypatch.setenv("KNNG_LEAF_BUCKETS", "0")
    a = _gpu_leaf_search(K, X, k, perms, offs, precision)
    monkeypatch.setenv("KNNG_LEAF_BUCKETS", "1")
    b = _gpu_leaf_search(K, X, k, perms, offs, precision)
    assert np.array_equal(_np(a[0]), _np(b[0]))
    assert np.array_equal(_np(a[1]).view(np.int32), _np(b[1]).view(np.int32))


@pytest.mark.parametrize("precision,n,D,k,L,rerank,kind", [
    ("fp8", 8000, 96, 32, 500, 2, "unit"),      # 512-point tiles, c = 64
    ("fp8", 6000, 36, 10, 300, 5, "unit"),      # D % 8 == 4, c = 50
    ("fp16", 3000, 960, 20, 200, 2, "unit"),    # 256-point tiles, c = 40
    ("bf16", 5000, 40, 16, 260, 4, "c1"),       # c = 64
    ("fp8", 4000, 64, 64, 256, 1, "unit"),      # k = c = 64
    ("fp16", 3000, 32, 8, 400, 8, "unit"),      # c = 64 with k = 8
])
def test_wide_leaf_kernel_equals_panel_kernel(K, orc, precision, n, D, k, L, rerank, kind,
                                              monkeypatch):
    """Leaves above 128 points with at most 64 candidates per row run the
    wide kernel (batches of 64 rows, radix selection over each row's key
    range, lane-per-candidate re-rank); its lists equal those of the panel
    kernel (k_leaf_mfma) bit for bit: same first pass, same selection rule,
    same d32 and order."""
    if kind == "c1":
        X = datagen.gmm_uniform(n, D, 20, -10, 10, 1.0, 23)
    else:
        X = datagen.gmm_unit(n, D, 16, 0.35, 24)
    perms, offs = _oracle_leaves(orc, X, 2, L, k + 1, 9)
    log("wide vs panel %s n=%d D=%d k=%d L=%d c=%d" % (precision, n, D, k, L, rerank * k))
    monkeypatch.setenv("KNNG_LEAF_WIDE", "0")
    a = _gpu_leaf_search(K, X, k, perms, offs, precision, rerank=rerank)
    monkeypatch.setenv("KNNG_LEAF_WIDE", "1")
    b = _gpu_leaf_search(K, X, k, perms, offs, precision, rerank=rerank)
    assert np.array_equal(_np(a[0]), _np(b[0]))
    assert np.array_equal(_np(a[1]).view(np.int32), _np(b[1]).view(np.int32))


@pytest.mark.parametrize("precision,n,D,k,T,L,kind", [
    ("fp8", 120_000, 96, 32, 2, 500, "unit"),    # C5-shaped rows, FP8 copy
    ("fp16", 40_000, 960, 20, 2, 200, "unit"),   # C4-shaped rows, FP16 copy
    ("bf16", 50_000, 64, 16, 2, 150, "c1"),      # BF16 copy of GMM rows
    ("fp8", 30_000, 36, 10, 2, 60, "c1"),        # D % 8 == 4, wide value range
    ("fp8", 60_000, 64, 16, 2, 120, "offset"),   # a large common offset: the per-row bound decides
])
def test_partition_filter_changes_nothing(K, orc, precision, n, D, k, T, L, kind, monkeypatch):
    """FP32 rows with a reduced copy: the partition's later passes label rows
    from the copy where its error bound decides them and read the FP32 row
    only inside the band or for a changed label.  The graph is bit-identical
    with the filter off, the filter decides most rows, and tree 0 equals the
    oracle's tree."""
    if kind == "c1":
        X = datagen.gmm_uniform(n, D, 40, -10, 10, 1.0, 41)
    elif kind == "offset":
        # every row near (4, ..., 4): margins are small against |x||w|, as in
        # the deep levels of unit-norm data
        X = datagen.gmm_uniform(n, D, 40, 3, 5, 0.3, 43)
    else:
        X = datagen.gmm_unit(n, D, 64, 0.35, 42)
    Xd = to_dev(X)
    log("partition filter %s n=%d D=%d %s" % (precision, n, D, kind))
    monkeypatch.setenv("KNNG_PARTITION_FILTER", "1")
    a = K.build(Xd, k, T, L, seed=3, precision=precision, stats=True)
    monkeypatch.setenv("KNNG_PARTITION_FILTER", "0")
    b = K.build(Xd, k, T, L, seed=3, precision=precision, stats=True)
    assert a[2]["filter_rows"] > 0 and b[2]["filter_rows"] == 0
    log("  filtered rows %d, of which read as FP32 %d; level rows %d"
        % (a[2]["filter_rows"], a[2]["filter_exact_rows"], a[2]["assign_rows"]))
    assert a[2]["filter_exact_rows"] < a[2]["filter_rows"]
    assert a[2]["assign_rows"] == b[2]["assign_rows"] and a[2]["levels"] == b[2]["levels"]
    assert np.array_equal(_np(a[0]), _np(b[0]))
    assert np.array_equal(_np(a[1]).view(np.int32), _np(b[1]).view(np.int32))
    # the partition itself against the oracle (knng_partition: the same kernels
    # without a reduced copy)
    g = K.partition(Xd, L, k + 1, 3, 0, with_nodes=True)
    tr = orc.tree(X, L, k + 1, 10, 3, 0)
    assert np.array_equal(_np(g["perm"]), tr["perm"])
    assert np.array_equal(_np(g["leaf_off"]), tr["leaf_off"])
