"""The C2 workload at full size, in the calls the benchmark times: 10^6
SIFT-shaped rows (integers 0..255, D = 128), k = 20, 8 trees, leaf_max =
100, seed 2, FP32 leaves, batched trees and compact uint8 rows.

- Build (Alg. 1, Sec. 3.1): the whole graph against the oracle's graph of
  the same input, every id and every distance bit for bit.  On this integer
  data every FP32 partial sum is an exact integer below 2^24, so d32 == d64.
- The same build with BF16 leaf distances (C3): BF16 holds these integers
  exactly, so the graph is again the oracle's bit for bit.
- GIST-shaped (10^6 x 960, FP16 leaves, 4 trees) and Deep-shaped (10^7 x
  96, FP8 leaves, 8 trees) builds at full size: the build equals the
  composition of its stages (partition, leaf search) bit for bit; 500
  sampled rows satisfy the widened G1 rule against the oracle's emulation of
  the reduced first pass on the same clusters; bisected nodes of tree 0,
  re-split by the oracle from their members, give the same sides.
- Search (Alg. 2): the benchmark's batch of 10,000 queries with 64 random
  seeds and 10 rounds, over the oracle's graph, on float rows and on the
  uint8 copy; a sample of 300 queries is compared with the oracle's E-GNNS
  query by query (each query's walk is independent of the others).

The oracle's graph takes about half a minute on 16 host threads; it is
computed once for the module.  Every input comes from the seeded
generators."""
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


@pytest.fixture(scope="module")
def c2(orc):
    c = datagen.CONFIGS["c2"]
    X = datagen.make("c2")
    assert X.shape == (c["n"], 128)
    log("full size: oracle graph of c2 (n=%d, %d trees)" % (c["n"], c["n_trees"]))
    o_ids, o_d, _ = orc.graph(X, c["k"], c["n_trees"], c["leaf_max"], c["seed"])
    return c, X, o_ids, o_d


def test_c2_build_full_size(K, orc, c2):
    import torch
    c, X, o_ids, o_d = c2
    n, k = c["n"], c["k"]
    xd = to_dev(X)
    ids = torch.empty((n, k), dtype=torch.int32, device="cuda")
    ds = torch.empty((n, k), dtype=torch.float32, device="cuda")
    log("full size: c2 build on the GPU")
    r = K.build(xd, k, c["n_trees"], c["leaf_max"], seed=c["seed"], precision=c["precision"],
                stats=True, out=(ids, ds))
    assert r[2]["compact_used"] == 1
    g_ids = ids.cpu().numpy()
    g_d = ds.cpu().numpy().astype(np.float64)
    bad = np.flatnonzero(np.any(g_ids != o_ids, axis=1))
    assert bad.size == 0, "rows %s differ" % bad[:10].tolist()
    assert np.array_equal(g_d, o_d)
    rows = np.random.default_rng(3).choice(n, 2000, replace=False)
    graph_parity(orc, X, rows, g_ids[rows], g_d[rows], o_ids[rows], o_d[rows], strict=True)


def test_c3_bf16_build_full_size(K, c2):
    c, X, o_ids, o_d = c2
    c3 = datagen.CONFIGS["c3"]
    assert c3["precision"] == "bf16" and c3["n"] == c["n"] and c3["seed"] == c["seed"]
    log("full size: c3 build (bf16 leaves) on the GPU")
    ids, ds = K.build(to_dev(X), c3["k"], c3["n_trees"], c3["leaf_max"], seed=c3["seed"],
                      precision="bf16")
    assert np.array_equal(ids.cpu().numpy(), o_ids)
    assert np.array_equal(ds.cpu().numpy().astype(np.float64), o_d)


@pytest.mark.parametrize("name", ["c4", "c5"])
def test_reduced_build_full_size(K, orc, name):
    """GIST- and Deep-shaped builds at full size with their reduced first pass
    (FP16, FP8), in the call the benchmark times.

    - The build equals, bit for bit, the composition of its stages through
      the C ABI: knng_partition of every tree, then knng_leaf_search on those
      clusters.
    - 500 sampled rows satisfy the widened G1 rule against the oracle's
      emulation of the first pass on the same clusters (tests/gpu_helpers.py:
      reduced_parity).
    - Tree parity by decomposition (T1): bisected nodes of tree 0 from the
      node log, re-split by the oracle from their member sets, give the same
      left side bit for bit."""
    import torch
    c = datagen.CONFIGS[name]
    n, D, k, T, L, seed, fmt = (c["n"], c["D"], c["k"], c["n_trees"], c["leaf_max"], c["seed"],
                                c["precision"])
    log("full size: %s data" % name)
    X = datagen.make(name)
    xd = to_dev(X)
    log("full size: %s partitions of %d trees" % (name, T))
    parts = [K.partition(xd, L, k + 1, seed, t, with_nodes=(t == 0)) for t in range(T)]
    perms_d = torch.stack([r["perm"] for r in parts])
    log("full size: %s leaf search and build (%s first pass)" % (name, fmt))
    l_ids, l_ds = K.leaf_search(xd, k, perms_d, [r["leaf_off"] for r in parts], precision=fmt)
    ids, ds = K.build(xd, k, T, L, seed=seed, precision=fmt)
    assert torch.equal(ids, l_ids)
    assert torch.equal(ds.view(torch.int32), l_ds.view(torch.int32))
    del l_ids, l_ds
    rows = datagen.sample_rows(n, 500)
    rsel = torch.from_numpy(rows).cuda()
    g_ids = ids[rsel].cpu().numpy()
    g_d = ds[rsel].cpu().numpy()
    perms = perms_d.cpu().numpy()
    offs = [r["leaf_off"].cpu().numpy() for r in parts]
    nodes = parts[0]["nodes"].cpu().numpy()
    del xd, ids, ds, perms_d, parts
    torch.cuda.empty_cache()
    log("full size: %s widened G1 on %d rows" % (name, len(rows)))
    same = reduced_parity(orc, X, fmt, k, 2 * k, perms, offs, rows, g_ids, g_d)
    log("  rows identical to the emulation %.4f" % same)
    # T1 by decomposition: up to 24 nodes of at most 10^5 points, spread
    # over the depths, and their left sides
    small = nodes[nodes[:, 1] <= 100_000]
    pick = small[np.linspace(0, len(small) - 1, min(24, len(small))).astype(int)]
    log("full size: %s re-split %d logged nodes (sizes %d..%d)"
        % (name, len(pick), pick[:, 1].min(), pick[:, 1].max()))
    for start, size, left, depth in pick.tolist():
        mem = np.sort(perms[0][start:start + size])
        lab, n0, _, _ = orc.split(X, mem, k + 1, 10, seed, 0)
        assert n0 == left, (start, size, depth, n0, left)
        assert np.array_equal(np.sort(mem[lab == 0]), np.sort(perms[0][start:start + left])), \
            (start, size, depth)


@pytest.mark.parametrize("rows", ["float", "uint8"])
def test_c2_search_full_size(K, orc, c2, rows):
    import torch
    c, X, o_ids, _ = c2
    n, k = c["n"], c["k"]
    Q = datagen.queries("c2", 10_000)
    S = datagen.seeds(n, len(Q), 64)
    xd = to_dev(X)
    G = torch.from_numpy(np.ascontiguousarray(o_ids)).cuda()
    qd, sd = to_dev(Q), torch.from_numpy(S).cuda()
    log("full size: search over %s rows, %d queries" % (rows, len(Q)))
    if rows == "uint8":
        g_ids, g_d = K.search_u8(K.to_u8(xd), G, qd, sd, k, 10)
    else:
        g_ids, g_d = K.search(xd, G, qd, sd, k, 10)
    pick = np.sort(np.random.default_rng(4).choice(len(Q), 300, replace=False))
    e_ids, e_d = orc.egnns(X, o_ids, Q[pick], S[pick], k, 10, dist_mode=1)
    assert np.array_equal(g_ids.cpu().numpy()[pick], e_ids)
    assert np.array_equal(g_d.cpu().numpy()[pick].astype(np.float64), e_d)
