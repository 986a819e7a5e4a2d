"""ctypes front end of the CPU oracle (``knng_oracle.c``).

Test infrastructure only: the tests, the GPU smoke check and the benchmark's
CPU-baseline leg use it.  It follows the paper's Sec. 3.1 / Algorithm 1 with
the readings listed at the top of ``knng_oracle.c``; nothing here imports the
GPU package.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "knng_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

GCC_FLAGS = ["-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
             "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(force=False):
    """Compile the oracle with gcc (plain C11, OpenMP)."""
    if not force and os.path.exists(_LIB_PATH) and \
            os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", *GCC_FLAGS, _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        i64, i32, u64, vp = ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_void_p
        L.orc_mix64.restype = u64
        L.orc_mix64.argtypes = [u64]
        L.orc_key_hash.restype = u64
        L.orc_key_hash.argtypes = [u64, u64, u64, u64, u64]
        L.orc_init_pair.restype = None
        L.orc_init_pair.argtypes = [u64, i32, i32, i64, vp, vp]
        L.orc_d64.restype = ctypes.c_double
        L.orc_d64.argtypes = [vp, i32, i64, i64]
        L.orc_exact_knn.restype = i32
        L.orc_exact_knn.argtypes = [vp, i64, i32, i32, vp, i64, vp, vp]
        L.orc_split.restype = i64
        L.orc_split.argtypes = [vp, i32, vp, i64, i32, i32, u64, i32, vp, vp, vp, vp]
        L.orc_split_init.restype = i64
        L.orc_split_init.argtypes = [vp, i32, vp, i64, i32, i32, i64, i64, vp, vp, vp, vp]
        L.orc_tree.restype = i64
        L.orc_tree.argtypes = [vp, i64, i32, i32, i32, i32, u64, i32, vp, vp, vp, i64, vp]
        L.orc_graph_from_leaves.restype = i32
        L.orc_graph_from_leaves.argtypes = [vp, i64, i32, i32, i32, vp, vp, vp, vp, vp]
        L.orc_rows_from_leaves.restype = i32
        L.orc_rows_from_leaves.argtypes = [vp, i64, i32, i32, i32, vp, vp, vp, vp, i64, vp, vp]
        L.orc_rows_from_leaves_reduced.restype = i32
        L.orc_rows_from_leaves_reduced.argtypes = [vp, i64, i32, i32, i32, vp, vp, vp, i32, i32,
                                                   vp, i64, vp, vp, vp]
        L.orc_dtilde.restype = ctypes.c_double
        L.orc_dtilde_row.restype = i32
        L.orc_dtilde_row.argtypes = [vp, i32, i32, i64, vp, i64, vp]
        L.orc_dtilde.argtypes = [vp, i32, i32, i64, i64]
        L.orc_round_fmt.restype = ctypes.c_double
        L.orc_round_fmt.argtypes = [ctypes.c_double, i32, i32]
        L.orc_quantize.restype = ctypes.c_double
        L.orc_quantize.argtypes = [i32, ctypes.c_double]
        L.orc_row_scale.restype = ctypes.c_double
        L.orc_row_scale.argtypes = [i32, vp, i32]
        L.orc_graph_from_leaves_reduced.restype = i32
        L.orc_graph_from_leaves_reduced.argtypes = [vp, i64, i32, i32, i32, vp, vp, vp, i32, i32,
                                                    vp, vp]
        L.orc_graph.restype = i32
        L.orc_graph.argtypes = [vp, i64, i32, i32, i32, i32, i32, i32, u64, vp, vp, vp]
        L.orc_d32.restype = ctypes.c_double
        L.orc_d32.argtypes = [vp, vp, i32]
        L.orc_egnns.restype = i32
        L.orc_egnns.argtypes = [vp, i64, i32, vp, i32, vp, i64, vp, i32, i32, i32, i32, vp, vp, vp]
        L.orc_exact_knn_points.restype = i32
        L.orc_exact_knn_points.argtypes = [vp, i64, i32, vp, i64, i32, vp, vp]
        L.orc_kmeans.restype = i32
        L.orc_kmeans.argtypes = [vp, i64, i32, i32, vp, i32, vp, vp]
        L.orc_rvq_train.restype = i32
        L.orc_rvq_train.argtypes = [vp, i64, i32, vp, i64, i32, i32, vp, vp, i32, vp, vp, vp, vp,
                                    vp]
        L.orc_rvq_encode.restype = i32
        L.orc_rvq_encode.argtypes = [vp, i64, i32, vp, i32, vp, i32, vp]
        L.orc_ivf_lists.restype = i32
        L.orc_ivf_lists.argtypes = [vp, i64, i32, vp, vp]
        L.orc_ivf_key_dist.restype = i32
        L.orc_ivf_key_dist.argtypes = [vp, i32, vp, i32, vp, i32, vp, vp]
        L.orc_ivf_seeds.restype = i32
        L.orc_ivf_seeds.argtypes = [vp, i64, i32, vp, i32, vp, i32, vp, vp, i32, i32, vp]
        L.orc_num_threads.restype = i32
        L.orc_set_num_threads.restype = None
        L.orc_set_num_threads.argtypes = [i32]
        _lib = L
    return _lib


def _f32(X):
    X = np.ascontiguousarray(X, dtype=np.float32)
    assert X.ndim == 2
    return X


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads():
    return lib().orc_num_threads()


def set_num_threads(t):
    lib().orc_set_num_threads(int(t))


def mix64(z):
    return lib().orc_mix64(ctypes.c_uint64(z & 0xFFFFFFFFFFFFFFFF))


def key_hash(seed, tree, min_id, size, j):
    return lib().orc_key_hash(seed, tree, min_id, size, j)


def init_pair(seed, tree, min_id, m):
    a = np.zeros(1, np.int64)
    b = np.zeros(1, np.int64)
    lib().orc_init_pair(seed, tree, min_id, m, _p(a), _p(b))
    return int(a[0]), int(b[0])


def d64(X, i, j):
    X = _f32(X)
    return lib().orc_d64(_p(X), X.shape[1], int(i), int(j))


def exact_knn(X, k, rows=None):
    """Exact k nearest neighbours (FP64, ties by id) of `rows` (default all)."""
    X = _f32(X)
    n, D = X.shape
    rows = np.arange(n, dtype=np.int64) if rows is None else np.ascontiguousarray(rows, np.int64)
    ids = np.empty((len(rows), k), np.int32)
    ds = np.empty((len(rows), k), np.float64)
    rc = lib().orc_exact_knn(_p(X), n, D, k, _p(rows), len(rows), _p(ids), _p(ds))
    assert rc == 0
    return ids, ds


def split(X, members, min_leaf, max_iter, seed, tree):
    """One bisection of `members` (ascending ids).  Returns (labels, n_left,
    centres[2, D], repaired)."""
    X = _f32(X)
    mem = np.ascontiguousarray(members, np.int32)
    m = len(mem)
    assert m >= 2 * min_leaf and np.all(np.diff(mem) > 0)
    lab = np.empty(m, np.uint8)
    c = np.empty((2, X.shape[1]), np.float64)
    rep = ctypes.c_int(0)
    n0 = lib().orc_split(_p(X), X.shape[1], _p(mem), m, min_leaf, max_iter, seed, tree,
                         _p(lab), _p(c), ctypes.byref(rep), None)
    return lab, int(n0), c, bool(rep.value)


def split_init(X, members, min_leaf, max_iter, a, b):
    """One bisection with the starting centres given as member positions
    a != b.  Returns (labels, n_left, centres[2, D], repaired, passes)."""
    X = _f32(X)
    mem = np.ascontiguousarray(members, np.int32)
    m = len(mem)
    lab = np.empty(m, np.uint8)
    c = np.empty((2, X.shape[1]), np.float64)
    rep = ctypes.c_int(0)
    st = np.zeros(4, np.int64)
    n0 = lib().orc_split_init(_p(X), X.shape[1], _p(mem), m, min_leaf, max_iter, a, b,
                              _p(lab), _p(c), ctypes.byref(rep), _p(st))
    return lab, int(n0), c, bool(rep.value), int(st[1])


def tree(X, leaf_max, min_leaf, max_iter, seed, t, with_nodes=False):
    """One tree.  Returns dict(perm, leaf_off, nodes, stats)."""
    X = _f32(X)
    n, D = X.shape
    perm = np.empty(n, np.int32)
    loff = np.empty(n + 1, np.int32)
    cap = n if with_nodes else 0
    nodes = np.empty((max(cap, 1), 4), np.int32)
    st = np.zeros(6, np.int64)
    nl = lib().orc_tree(_p(X), n, D, leaf_max, min_leaf, max_iter, seed, t, _p(perm),
                        _p(loff), _p(nodes) if with_nodes else None, cap, _p(st))
    out = dict(perm=perm, leaf_off=loff[: nl + 1].copy(),
               stats=dict(assign_rows=int(st[0]), passes=int(st[1]), splits=int(st[2]),
                          repairs=int(st[3]), internal_nodes=int(st[4]), depth=int(st[5])))
    if with_nodes:
        out["nodes"] = nodes[: st[4]].copy()
    return out


def graph_from_leaves(X, k, perms, leaf_offs):
    """G from given leaves: perms [T, n]; leaf_offs list of T boundary arrays."""
    X = _f32(X)
    n, D = X.shape
    perms = np.ascontiguousarray(perms, np.int32).reshape(-1, n)
    T = perms.shape[0]
    assert len(leaf_offs) == T
    cat = np.ascontiguousarray(np.concatenate([np.asarray(o, np.int32) for o in leaf_offs]))
    nl = np.array([len(o) - 1 for o in leaf_offs], np.int64)
    ids = np.empty((n, k), np.int32)
    ds = np.empty((n, k), np.float64)
    rc = lib().orc_graph_from_leaves(_p(X), n, D, k, T, _p(perms), _p(cat), _p(nl),
                                     _p(ids), _p(ds))
    assert rc == 0
    return ids, ds


def rows_from_leaves(X, k, perms, leaf_offs, rows):
    """Rows `rows` of graph_from_leaves(X, k, perms, leaf_offs)."""
    X = _f32(X)
    n, D = X.shape
    perms = np.ascontiguousarray(perms, np.int32).reshape(-1, n)
    T = perms.shape[0]
    cat = np.ascontiguousarray(np.concatenate([np.asarray(o, np.int32) for o in leaf_offs]))
    nl = np.array([len(o) - 1 for o in leaf_offs], np.int64)
    rows = np.ascontiguousarray(rows, np.int64)
    ids = np.empty((len(rows), k), np.int32)
    ds = np.empty((len(rows), k), np.float64)
    rc = lib().orc_rows_from_leaves(_p(X), n, D, k, T, _p(perms), _p(cat), _p(nl), _p(rows),
                                    len(rows), _p(ids), _p(ds))
    assert rc == 0
    return ids, ds


FORMATS = {"bf16": 1, "fp16": 2, "fp8": 3}


def quantize(fmt, x):
    """Round x (float) to the format, ties to even (reading R9)."""
    return lib().orc_quantize(FORMATS[fmt], float(x))


def row_scale(fmt, row):
    row = np.ascontiguousarray(row, np.float32)
    return lib().orc_row_scale(FORMATS[fmt], _p(row), len(row))


def graph_from_leaves_reduced(X, k, perms, leaf_offs, fmt, c):
    """G from given leaves with the reduced-precision first pass (R9)."""
    X = _f32(X)
    n, D = X.shape
    perms = np.ascontiguousarray(perms, np.int32).reshape(-1, n)
    T = perms.shape[0]
    cat = np.ascontiguousarray(np.concatenate([np.asarray(o, np.int32) for o in leaf_offs]))
    nl = np.array([len(o) - 1 for o in leaf_offs], np.int64)
    ids = np.empty((n, k), np.int32)
    ds = np.empty((n, k), np.float64)
    rc = lib().orc_graph_from_leaves_reduced(_p(X), n, D, k, T, _p(perms), _p(cat), _p(nl),
                                             FORMATS[fmt], c, _p(ids), _p(ds))
    assert rc == 0
    return ids, ds


def rows_from_leaves_reduced(X, k, perms, leaf_offs, fmt, c, rows):
    """Rows `rows` of graph_from_leaves_reduced, plus per row and tree the
    first-pass distances of the c-th kept and the first dropped candidate
    (thr [len(rows), T, 2], +inf where the leaf has no such entry)."""
    X = _f32(X)
    n, D = X.shape
    perms = np.ascontiguousarray(perms, np.int32).reshape(-1, n)
    T = perms.shape[0]
    cat = np.ascontiguousarray(np.concatenate([np.asarray(o, np.int32) for o in leaf_offs]))
    nl = np.array([len(o) - 1 for o in leaf_offs], np.int64)
    rows = np.ascontiguousarray(rows, np.int64)
    ids = np.empty((len(rows), k), np.int32)
    ds = np.empty((len(rows), k), np.float64)
    thr = np.empty((len(rows), T, 2), np.float64)
    rc = lib().orc_rows_from_leaves_reduced(_p(X), n, D, k, T, _p(perms), _p(cat), _p(nl),
                                            FORMATS[fmt], c, _p(rows), len(rows), _p(ids),
                                            _p(ds), _p(thr))
    assert rc == 0
    return ids, ds, thr


def dtilde(X, fmt, i, j):
    """First-pass distance of the pair (i, j) under the reduced format (R9)."""
    X = _f32(X)
    return lib().orc_dtilde(_p(X), X.shape[1], FORMATS[fmt], int(i), int(j))


def dtilde_row(X, fmt, i, js):
    """First-pass distances of row i to the rows js under the reduced format
    (R9), FP64 array."""
    X = _f32(X)
    js = np.ascontiguousarray(js, np.int32)
    out = np.empty(len(js), np.float64)
    rc = lib().orc_dtilde_row(_p(X), X.shape[1], FORMATS[fmt], int(i), _p(js), len(js), _p(out))
    assert rc == 0
    return out


def graph(X, k, n_trees, leaf_max, seed, min_leaf=None, max_iter=10):
    """Algorithm 1 end to end.  Returns (ids [n,k] int32, dists [n,k] f64, stats)."""
    X = _f32(X)
    n, D = X.shape
    ml = k + 1 if min_leaf is None else min_leaf
    ids = np.empty((n, k), np.int32)
    ds = np.empty((n, k), np.float64)
    st = np.zeros(6, np.int64)
    rc = lib().orc_graph(_p(X), n, D, k, n_trees, leaf_max, ml, max_iter, seed,
                         _p(ids), _p(ds), _p(st))
    assert rc == 0
    return ids, ds, dict(assign_rows=int(st[0]), passes=int(st[1]), splits=int(st[2]),
                         repairs=int(st[3]), internal_nodes=int(st[4]), depth=int(st[5]))


def pair_d64(X, rows, cols):
    """FP64 squared distances d(rows[q], cols[q, p]) (numpy, direct form)."""
    X = _f32(X)
    rows = np.asarray(rows, np.int64)
    cols = np.asarray(cols, np.int64)
    out = np.full(cols.shape, np.inf)
    for q, i in enumerate(rows):
        c = cols[q]
        ok = c >= 0
        diff = X[c[ok]].astype(np.float64) - X[i].astype(np.float64)
        out[q, ok] = np.einsum("pd,pd->p", diff, diff)
    return out


def recall(X, rows, G_ids, E_ids, E_d):
    """Tie-tolerant recall@k of graph rows G_ids[q] (for point rows[q]) against
    exact lists (E_ids, E_d): an id counts when it is in the exact list or no
    farther than the exact k-th neighbour."""
    G_ids = np.asarray(G_ids)
    k = E_ids.shape[1]
    dG = pair_d64(X, rows, G_ids)
    hits = 0
    for q in range(len(rows)):
        ex = set(E_ids[q].tolist())
        kth = E_d[q, k - 1]
        for p in range(k):
            j = int(G_ids[q, p])
            if j >= 0 and (j in ex or dG[q, p] <= kth):
                hits += 1
    return hits / float(len(rows) * k)


def d32(a, b):
    """Canonical FP32 distance of two vectors (reading R13)."""
    a, b = _f32(np.asarray(a).reshape(1, -1)), _f32(np.asarray(b).reshape(1, -1))
    return lib().orc_d32(_p(a), _p(b), a.shape[1])


def egnns(X, G, Q, seeds, k, rounds, dist_mode=1, with_work=False):
    """Alg. 2 (E-GNNS, readings R10-R13) for every query row of Q.

    G: [n, kg] int32 graph (-1 padding); seeds: [nq, ns] int32.
    Returns (ids int32 [nq, k], dists float64 [nq, k]) and, with with_work,
    (distances taken, nodes expanded) over all queries."""
    X, Q = _f32(X), _f32(Q)
    G = np.ascontiguousarray(G, dtype=np.int32)
    S = np.ascontiguousarray(seeds, dtype=np.int32)
    n, D = X.shape
    nq = Q.shape[0]
    assert Q.shape[1] == D and G.shape[0] == n and S.shape[0] == nq
    ids = np.empty((nq, k), np.int32)
    ds = np.empty((nq, k), np.float64)
    work = np.zeros(2, np.int64)
    rc = lib().orc_egnns(_p(X), n, D, _p(G), G.shape[1], _p(Q), nq, _p(S), S.shape[1], k,
                         rounds, dist_mode, _p(ids), _p(ds), _p(work))
    if rc != 0:
        raise MemoryError("orc_egnns")
    if with_work:
        return ids, ds, (int(work[0]), int(work[1]))
    return ids, ds


def exact_knn_points(X, Q, k):
    """Exact k nearest rows of X for each query row of Q (FP64 brute force)."""
    X, Q = _f32(X), _f32(Q)
    ids = np.empty((Q.shape[0], k), np.int32)
    ds = np.empty((Q.shape[0], k), np.float64)
    rc = lib().orc_exact_knn_points(_p(X), X.shape[0], X.shape[1], _p(Q), Q.shape[0], k,
                                    _p(ids), _p(ds))
    assert rc == 0
    return ids, ds


def search_recall(ids, E_ids):
    """Mean fraction of the exact k nearest ids found per query."""
    k = E_ids.shape[1]
    hit = 0
    for a, b in zip(ids, E_ids):
        hit += len(set(a[a >= 0].tolist()) & set(b[b >= 0].tolist()))
    return hit / float(E_ids.shape[0] * k)


# ---------------------------------------------------------------- RVQ index
# Sec. 4.1-4.2 and Eqns 1-3, readings R14-R19 in knng_oracle.c.

def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def kmeans(P, init, iters):
    """Lloyd k-means (R15, R16) of the FP64 rows P from the rows init.
    Returns (W float64 [K, D], codes int32 [m], update rounds)."""
    P, init = _f64(P), _i32(init)
    m, D = P.shape
    W = np.empty((len(init), D), np.float64)
    codes = np.empty(m, np.int32)
    r = lib().orc_kmeans(_p(P), m, D, len(init), _p(init), iters, _p(W), _p(codes))
    if r < 0:
        raise ValueError("orc_kmeans")
    return W, codes, r


def rvq_train(X, train_ids, init1, init2, iters):
    """Two-stage RVQ vocabularies (R14).  Returns (W1, W2, codes1, codes2,
    rounds [2]); codes are those of the sample rows."""
    X, train_ids, init1, init2 = _f32(X), _i32(train_ids), _i32(init1), _i32(init2)
    m, D = len(train_ids), X.shape[1]
    W1 = np.empty((len(init1), D), np.float64)
    W2 = np.empty((len(init2), D), np.float64)
    c1 = np.empty(m, np.int32)
    c2 = np.empty(m, np.int32)
    rounds = np.zeros(2, np.int32)
    rc = lib().orc_rvq_train(_p(X), X.shape[0], D, _p(train_ids), m, len(init1), len(init2),
                             _p(init1), _p(init2), iters, _p(W1), _p(W2), _p(c1), _p(c2),
                             _p(rounds))
    if rc != 0:
        raise ValueError("orc_rvq_train")
    return W1, W2, c1, c2, rounds


def rvq_encode(X, W1, W2):
    """Index key c1 * K2 + c2 of every row (R17)."""
    X, W1, W2 = _f32(X), _f64(W1), _f64(W2)
    key = np.empty(X.shape[0], np.int32)
    rc = lib().orc_rvq_encode(_p(X), X.shape[0], X.shape[1], _p(W1), W1.shape[0], _p(W2),
                              W2.shape[0], _p(key))
    assert rc == 0
    return key


def ivf_lists(key, nkeys):
    """Inverted lists (R17): (offsets int32 [nkeys + 1], ids int32 [n])."""
    key = _i32(key)
    offsets = np.empty(nkeys + 1, np.int32)
    ids = np.empty(len(key), np.int32)
    rc = lib().orc_ivf_lists(_p(key), len(key), nkeys, _p(offsets), _p(ids))
    if rc != 0:
        raise ValueError("orc_ivf_lists")
    return offsets, ids


def ivf_key_dist(q, W1, W2):
    """term1 [K1] and d(q, I) [K1, K2] of one query (R18)."""
    q = _f32(np.asarray(q).reshape(1, -1))
    W1, W2 = _f64(W1), _f64(W2)
    t1 = np.empty(W1.shape[0], np.float64)
    dist = np.empty((W1.shape[0], W2.shape[0]), np.float64)
    rc = lib().orc_ivf_key_dist(_p(q), q.shape[1], _p(W1), W1.shape[0], _p(W2), W2.shape[0],
                                _p(t1), _p(dist))
    assert rc == 0
    return t1, dist


def ivf_seeds(Q, W1, W2, offsets, ids, n1, ns):
    """Cascaded seeds of each query (R18, R19): int32 [nq, ns], -1 padded."""
    Q, W1, W2 = _f32(Q), _f64(W1), _f64(W2)
    offsets, ids = _i32(offsets), _i32(ids)
    out = np.empty((Q.shape[0], ns), np.int32)
    rc = lib().orc_ivf_seeds(_p(Q), Q.shape[0], Q.shape[1], _p(W1), W1.shape[0], _p(W2),
                             W2.shape[0], _p(offsets), _p(ids), n1, ns, _p(out))
    if rc != 0:
        raise ValueError("orc_ivf_seeds")
    return out
