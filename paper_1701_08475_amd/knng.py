"""Python binding of libknng.so (include/knng.h).  Argument marshalling only:
every step of the build runs in the library's HIP kernels.  PyTorch provides
device memory and the current stream.

    ids, dists = knng.build(x, k=20, n_trees=8, leaf_max=100, seed=0)

raises ``KnngError`` on a non-zero status and ``RuntimeError`` when the
library has not been built (there is no fallback path).
"""
import ctypes
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB_PATH = os.path.join(PKG, "libknng.so")
HEADER = os.path.join(ROOT, "include", "knng.h")

KNNG_OK = 0
KNNG_ERR_INVALID_ARG = -1
KNNG_ERR_UNSUPPORTED = -2
KNNG_ERR_OOM = -3
KNNG_ERR_HIP = -4
KNNG_ERR_NONFINITE = -5
PRECISION = {"fp32": 0, "bf16": 1, "fp16": 2, "fp8": 3, "fp8_e4m3": 3}


class KnngOptions(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("rerank_factor", ctypes.c_int32), ("min_leaf", ctypes.c_int32),
                ("max_iter", ctypes.c_int32), ("plain", ctypes.c_int32),
                ("check_finite", ctypes.c_int32), ("time_kernels", ctypes.c_int32),
                ("compact", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p)]

# knng_autotune's knobs, in the order of its chosen_out array
TUNE_KNOBS = ("assign_unroll", "filter", "assign_m_u", "assign_m_pd", "chunk_order",
              "leaf_wide", "leaf_buckets", "merge_network")


class KnngStats(ctypes.Structure):
    _fields_ = [("assign_rows", ctypes.c_int64), ("ordered_pairs", ctypes.c_int64),
                ("leaves", ctypes.c_int64), ("splits", ctypes.c_int64),
                ("repairs", ctypes.c_int64), ("levels", ctypes.c_int32),
                ("launches", ctypes.c_int32), ("ms_prep", ctypes.c_float),
                ("ms_partition", ctypes.c_float), ("ms_leaf", ctypes.c_float),
                ("ms_merge", ctypes.c_float), ("ms_total", ctypes.c_float),
                ("ms_k_assign", ctypes.c_float), ("n_k_assign", ctypes.c_int32),
                ("ms_k_leaf", ctypes.c_float), ("n_k_leaf", ctypes.c_int32),
                ("ms_k_merge", ctypes.c_float), ("n_k_merge", ctypes.c_int32),
                ("compact_used", ctypes.c_int32), ("exact_first_pass", ctypes.c_int32),
                ("subtree_rows", ctypes.c_int64), ("filter_rows", ctypes.c_int64),
                ("filter_exact_rows", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class KnngError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("knng status %d: %s" % (status, msg))
        self.status = status


_lib = None


def declared_functions():
    """Names of the functions include/knng.h declares."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(knng_\w+)\s*\(", txt)))


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libknng.so is not built (run __graft_entry__.build() or "
                           "python -m paper_1701_08475_amd.build_lib)")
    # torch's HIP runtime is brought up first (where a GPU is present): when
    # the library was loaded before it, its HIP calls found no device (the
    # process then holds two HIP runtimes and the library's saw none)
    try:
        import torch
        torch.cuda.is_available()
    except ImportError:
        pass
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64
    L.knng_build.restype = ctypes.c_int
    L.knng_build.argtypes = [vp, i64, i32, i32, i32, i32, u64, vp, vp, vp]
    L.knng_build_ex.restype = ctypes.c_int
    L.knng_build_ex.argtypes = [vp, i64, i32, i32, i32, i32, u64, vp, vp,
                                ctypes.POINTER(KnngOptions), ctypes.POINTER(KnngStats), vp]
    L.knng_partition.restype = ctypes.c_int
    L.knng_partition.argtypes = [vp, i64, i32, i32, i32, i32, u64, i32, vp, vp,
                                 ctypes.POINTER(i32), vp, ctypes.POINTER(i32), vp]
    L.knng_leaf_search.restype = ctypes.c_int
    L.knng_leaf_search.argtypes = [vp, i64, i32, i32, i32, vp, vp, ctypes.POINTER(i32),
                                   ctypes.POINTER(KnngOptions), vp, vp, vp]
    L.knng_leaf_search_noalloc.restype = ctypes.c_int
    L.knng_leaf_search_noalloc.argtypes = L.knng_leaf_search.argtypes
    L.knng_search.restype = ctypes.c_int
    L.knng_search.argtypes = [vp, i64, i32, vp, i32, vp, i64, vp, i32, i32, i32, vp, vp, vp]
    L.knng_search_ex.argtypes = [vp, i64, i32, vp, i32, vp, i64, vp, i32, i32, i32, vp, vp,
                                 ctypes.POINTER(ctypes.c_uint64), vp]
    L.knng_search_u8.argtypes = [vp, i64, i32, vp, i32, vp, i64, vp, i32, i32, i32, vp, vp,
                                 ctypes.POINTER(ctypes.c_uint64), vp]
    L.knng_to_u8.argtypes = [vp, i64, vp, vp]
    L.knng_release_workspace.restype = None
    L.knng_release_workspace.argtypes = []
    L.knng_rvq_train.argtypes = [vp, i64, i32, vp, i64, i32, i32, vp, vp, i32, vp, vp, vp, vp,
                                 ctypes.POINTER(i32), vp]
    L.knng_ivf_build.argtypes = [vp, i64, i32, vp, i32, vp, i32, vp, vp, vp, vp]
    L.knng_ivf_seeds.argtypes = [vp, i64, i32, vp, i32, vp, i32, vp, vp, i64, i32, i32, vp, vp]
    L.knng_autotune.restype = ctypes.c_int
    L.knng_autotune.argtypes = [vp, i64, i32, i32, i32, i32, u64, ctypes.POINTER(KnngOptions),
                                ctypes.c_char_p, ctypes.POINTER(i32), vp]
    L.knng_default_options.restype = None
    L.knng_default_options.argtypes = [ctypes.POINTER(KnngOptions)]
    L.knng_status_string.restype = ctypes.c_char_p
    L.knng_status_string.argtypes = [ctypes.c_int]
    L.knng_last_error.restype = ctypes.c_char_p
    L.knng_last_error.argtypes = []
    L.knng_version.restype = ctypes.c_int
    L.knng_version.argtypes = []
    _lib = L
    return L


def _check(rc):
    if rc != KNNG_OK:
        raise KnngError(rc, lib().knng_last_error().decode(errors="replace"))


def options(precision="fp32", rerank_factor=2, min_leaf=0, max_iter=0, plain=False,
            check_finite=True, time_kernels=False, compact=True, tune_cache=None):
    o = KnngOptions()
    lib().knng_default_options(ctypes.byref(o))
    o.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    o.rerank_factor = int(rerank_factor)
    o.min_leaf = int(min_leaf)
    o.max_iter = int(max_iter)
    o.plain = 1 if plain else 0
    o.check_finite = 1 if check_finite else 0
    o.time_kernels = 1 if time_kernels else 0
    o.compact = 1 if compact else 0
    # the path must outlive the call: ctypes keeps this bytes object with o
    o.tune_cache = tune_cache.encode() if isinstance(tune_cache, str) else tune_cache
    return o


def _stream(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _dev_f32(x):
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32
            and x.dim() == 2 and x.is_contiguous()):
        raise ValueError("x must be a contiguous 2-D float32 CUDA tensor")
    return x


def build(x, k, n_trees, leaf_max, seed=0, precision="fp32", rerank_factor=2, min_leaf=0,
          max_iter=0, plain=False, stats=False, time_kernels=False, compact=True, out=None,
          stream=None, tune_cache=None):
    """kNN graph of the rows of x.  Returns (ids int32 [n,k], dists f32 [n,k])
    and a stats dict when stats=True."""
    import torch
    x = _dev_f32(x)
    n, D = x.shape
    if out is None:
        ids = torch.empty((n, k), dtype=torch.int32, device=x.device)
        ds = torch.empty((n, k), dtype=torch.float32, device=x.device)
    else:
        ids, ds = out
    o = options(precision, rerank_factor, min_leaf, max_iter, plain,
                time_kernels=time_kernels, compact=compact, tune_cache=tune_cache)
    st = KnngStats() if stats else None
    rc = lib().knng_build_ex(ctypes.c_void_p(x.data_ptr()), n, D, k, n_trees, leaf_max,
                             ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF),
                             ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(ds.data_ptr()),
                             ctypes.byref(o), ctypes.byref(st) if st is not None else None,
                             _stream(stream))
    _check(rc)
    return (ids, ds, st.as_dict()) if stats else (ids, ds)


def autotune(x, k, n_trees, leaf_max, cache_path, seed=0, precision="fp32", rerank_factor=2,
             min_leaf=0, max_iter=0, compact=True, stream=None):
    """knng_autotune: time the build's result-invariant choices on x, check that
    each gives the default build's graph bit for bit, store the fastest in
    cache_path.  Returns {knob: value}."""
    x = _dev_f32(x)
    n, D = x.shape
    o = options(precision, rerank_factor, min_leaf, max_iter, compact=compact)
    chosen = (ctypes.c_int32 * len(TUNE_KNOBS))()
    rc = lib().knng_autotune(ctypes.c_void_p(x.data_ptr()), n, D, k, n_trees, leaf_max,
                             ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), ctypes.byref(o),
                             str(cache_path).encode(), chosen, _stream(stream))
    _check(rc)
    return dict(zip(TUNE_KNOBS, list(chosen)))


def build_plain_call(x, k, n_trees, leaf_max, seed, ids, ds, stream=None):
    """knng_build (the options-free entry point) into given outputs."""
    rc = lib().knng_build(ctypes.c_void_p(x.data_ptr()), x.shape[0], x.shape[1], k, n_trees,
                          leaf_max, ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF),
                          ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(ds.data_ptr()),
                          _stream(stream))
    _check(rc)


def partition(x, leaf_max, min_leaf, seed, tree, max_iter=0, with_nodes=False, stream=None):
    """One tree's clustering.  Returns dict(perm [n] int32, leaf_off [n_leaves+1]
    int32, nodes [n_nodes, 4] int32 if with_nodes), all CUDA tensors."""
    import torch
    x = _dev_f32(x)
    n, D = x.shape
    perm = torch.empty(n, dtype=torch.int32, device=x.device)
    loff = torch.empty(n + 1, dtype=torch.int32, device=x.device)
    nodes = torch.empty((n, 4), dtype=torch.int32, device=x.device) if with_nodes else None
    nl = ctypes.c_int32(0)
    nn = ctypes.c_int32(0)
    rc = lib().knng_partition(ctypes.c_void_p(x.data_ptr()), n, D, leaf_max, min_leaf, max_iter,
                              ctypes.c_uint64(seed & 0xFFFFFFFFFFFFFFFF), tree,
                              ctypes.c_void_p(perm.data_ptr()), ctypes.c_void_p(loff.data_ptr()),
                              ctypes.byref(nl),
                              ctypes.c_void_p(nodes.data_ptr()) if with_nodes else None,
                              ctypes.byref(nn), _stream(stream))
    _check(rc)
    out = dict(perm=perm, leaf_off=loff[: nl.value + 1])
    if with_nodes:
        out["nodes"] = nodes[: nn.value]
    return out


def leaf_search(x, k, perms, leaf_offs, precision="fp32", rerank_factor=2, stream=None,
                noalloc=False):
    """G from given clusters.  perms: int32 CUDA [T, n]; leaf_offs: list of T
    int32 CUDA boundary tensors.  Returns (ids, dists).  noalloc=True calls
    knng_leaf_search_noalloc (scratch from the library's fixed array)."""
    import torch
    x = _dev_f32(x)
    n, D = x.shape
    perms = perms.reshape(-1, n).contiguous()
    T = perms.shape[0]
    cat = torch.cat([o.to(torch.int32) for o in leaf_offs]).contiguous()
    nl = (ctypes.c_int32 * T)(*[int(o.numel()) - 1 for o in leaf_offs])
    ids = torch.empty((n, k), dtype=torch.int32, device=x.device)
    ds = torch.empty((n, k), dtype=torch.float32, device=x.device)
    o = options(precision, rerank_factor)
    fn = lib().knng_leaf_search_noalloc if noalloc else lib().knng_leaf_search
    rc = fn(ctypes.c_void_p(x.data_ptr()), n, D, k, T,
                                ctypes.c_void_p(perms.data_ptr()), ctypes.c_void_p(cat.data_ptr()),
                                nl, ctypes.byref(o), ctypes.c_void_p(ids.data_ptr()),
                                ctypes.c_void_p(ds.data_ptr()), _stream(stream))
    _check(rc)
    return ids, ds


def search(x, graph, queries, seeds, k, rounds, stream=None, work=False):
    """E-GNNS (Alg. 2) for a batch of queries over a kNN graph.

    x: float32 CUDA [n, D]; graph: int32 CUDA [n, kg]; queries: float32 CUDA
    [nq, D]; seeds: int32 CUDA [nq, ns].  Returns (ids int32 [nq, k], dists
    float32 [nq, k]) and, with work=True, (distances taken, nodes expanded)."""
    import torch
    x = _dev_f32(x)
    queries = _dev_f32(queries)
    n, D = x.shape
    if queries.shape[1] != D:
        raise ValueError("queries must have D columns")
    for name, t in (("graph", graph), ("seeds", seeds)):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int32
                and t.dim() == 2 and t.is_contiguous()):
            raise ValueError("%s must be a contiguous 2-D int32 CUDA tensor" % name)
    if graph.shape[0] != n or seeds.shape[0] != queries.shape[0]:
        raise ValueError("graph needs n rows and seeds one row per query")
    nq = queries.shape[0]
    ids = torch.empty((nq, k), dtype=torch.int32, device=x.device)
    ds = torch.empty((nq, k), dtype=torch.float32, device=x.device)
    w = (ctypes.c_uint64 * 2)()
    rc = lib().knng_search_ex(ctypes.c_void_p(x.data_ptr()), n, D,
                              ctypes.c_void_p(graph.data_ptr()), graph.shape[1],
                              ctypes.c_void_p(queries.data_ptr()), nq,
                              ctypes.c_void_p(seeds.data_ptr()), seeds.shape[1], k, rounds,
                              ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(ds.data_ptr()),
                              w if work else None, _stream(stream))
    _check(rc)
    if work:
        return ids, ds, (int(w[0]), int(w[1]))
    return ids, ds


def to_u8(x, stream=None):
    """The lossless uint8 copy of a float32 CUDA tensor whose values are all
    integers in [0, 255] (raises KnngError otherwise)."""
    import torch
    if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32
            and x.is_contiguous()):
        raise ValueError("x must be a contiguous float32 CUDA tensor")
    out = torch.empty(x.shape, dtype=torch.uint8, device=x.device)
    _check(lib().knng_to_u8(ctypes.c_void_p(x.data_ptr()), x.numel(),
                            ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def search_u8(x8, graph, queries, seeds, k, rounds, stream=None, work=False):
    """search() over the uint8 copy of integer data (to_u8): the same results
    from a quarter of the row bytes."""
    import torch
    if not (isinstance(x8, torch.Tensor) and x8.is_cuda and x8.dtype == torch.uint8
            and x8.dim() == 2 and x8.is_contiguous()):
        raise ValueError("x8 must be a contiguous 2-D uint8 CUDA tensor")
    queries = _dev_f32(queries)
    n, D = x8.shape
    if queries.shape[1] != D:
        raise ValueError("queries must have D columns")
    _dev_i32(graph, "graph", 2)
    _dev_i32(seeds, "seeds", 2)
    if graph.shape[0] != n or seeds.shape[0] != queries.shape[0]:
        raise ValueError("graph needs n rows and seeds one row per query")
    nq = queries.shape[0]
    ids = torch.empty((nq, k), dtype=torch.int32, device=x8.device)
    ds = torch.empty((nq, k), dtype=torch.float32, device=x8.device)
    w = (ctypes.c_uint64 * 2)()
    rc = lib().knng_search_u8(ctypes.c_void_p(x8.data_ptr()), n, D,
                              ctypes.c_void_p(graph.data_ptr()), graph.shape[1],
                              ctypes.c_void_p(queries.data_ptr()), nq,
                              ctypes.c_void_p(seeds.data_ptr()), seeds.shape[1], k, rounds,
                              ctypes.c_void_p(ids.data_ptr()), ctypes.c_void_p(ds.data_ptr()),
                              w if work else None, _stream(stream))
    _check(rc)
    if work:
        return ids, ds, (int(w[0]), int(w[1]))
    return ids, ds


def release_workspace():
    """Free the scratch blocks the library keeps cached on the current device."""
    lib().knng_release_workspace()


def _dev_i32(t, name, dim=1):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.int32
            and t.dim() == dim and t.is_contiguous()):
        raise ValueError("%s must be a contiguous %d-D int32 CUDA tensor" % (name, dim))
    return t


def _dev_f64(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
            and t.dim() == 2 and t.is_contiguous()):
        raise ValueError("%s must be a contiguous 2-D float64 CUDA tensor" % name)
    return t


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def rvq_train(x, train_ids, init1, init2, iters, codes=False, stream=None):
    """Two-stage RVQ vocabularies by Lloyd k-means (Sec. 4.1, Eqn 1).

    x: float32 CUDA [n, D]; train_ids: int32 CUDA [m] sample rows; init1,
    init2: int32 CUDA [K1] / [K2] starting positions in the sample.  Returns
    (words1 float64 [K1, D], words2 float64 [K2, D], rounds (r1, r2)) and,
    with codes=True, the sample's codes (int32 [m] each) as well."""
    import torch
    x = _dev_f32(x)
    _dev_i32(train_ids, "train_ids")
    _dev_i32(init1, "init1")
    _dev_i32(init2, "init2")
    n, D = x.shape
    m, K1, K2 = train_ids.shape[0], init1.shape[0], init2.shape[0]
    W1 = torch.empty((K1, D), dtype=torch.float64, device=x.device)
    W2 = torch.empty((K2, D), dtype=torch.float64, device=x.device)
    c1 = torch.empty(m, dtype=torch.int32, device=x.device) if codes else None
    c2 = torch.empty(m, dtype=torch.int32, device=x.device) if codes else None
    rounds = (ctypes.c_int * 2)()
    rc = lib().knng_rvq_train(_ptr(x), n, D, _ptr(train_ids), m, K1, K2, _ptr(init1), _ptr(init2),
                              iters, _ptr(W1), _ptr(W2), _ptr(c1) if codes else None,
                              _ptr(c2) if codes else None, rounds, _stream(stream))
    _check(rc)
    if codes:
        return W1, W2, (rounds[0], rounds[1]), c1, c2
    return W1, W2, (rounds[0], rounds[1])


def ivf_build(x, words1, words2, stream=None):
    """Keys and inverted lists of every point (Sec. 4.2).  Returns (keys int32
    [n], offsets int32 [K1 K2 + 1], ids int32 [n])."""
    import torch
    x = _dev_f32(x)
    _dev_f64(words1, "words1")
    _dev_f64(words2, "words2")
    n, D = x.shape
    if words1.shape[1] != D or words2.shape[1] != D:
        raise ValueError("vocabularies must have D columns")
    K1, K2 = words1.shape[0], words2.shape[0]
    keys = torch.empty(n, dtype=torch.int32, device=x.device)
    offsets = torch.empty(K1 * K2 + 1, dtype=torch.int32, device=x.device)
    ids = torch.empty(n, dtype=torch.int32, device=x.device)
    rc = lib().knng_ivf_build(_ptr(x), n, D, _ptr(words1), K1, _ptr(words2), K2, _ptr(keys),
                              _ptr(offsets), _ptr(ids), _stream(stream))
    _check(rc)
    return keys, offsets, ids


def ivf_seeds(queries, words1, words2, offsets, ids, n1, ns, stream=None):
    """Cascaded seeds (Eqns 2-3): int32 [nq, ns], -1 padded."""
    import torch
    queries = _dev_f32(queries)
    _dev_f64(words1, "words1")
    _dev_f64(words2, "words2")
    _dev_i32(offsets, "offsets")
    _dev_i32(ids, "ids")
    nq, D = queries.shape
    if words1.shape[1] != D or words2.shape[1] != D:
        raise ValueError("vocabularies must have D columns")
    K1, K2 = words1.shape[0], words2.shape[0]
    if offsets.shape[0] != K1 * K2 + 1:
        raise ValueError("offsets must hold K1 * K2 + 1 entries")
    seeds = torch.empty((nq, ns), dtype=torch.int32, device=queries.device)
    rc = lib().knng_ivf_seeds(_ptr(queries), nq, D, _ptr(words1), K1, _ptr(words2), K2,
                              _ptr(offsets), _ptr(ids), ids.shape[0], n1, ns, _ptr(seeds),
                              _stream(stream))
    _check(rc)
    return seeds
