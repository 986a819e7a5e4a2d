"""The C ABI without a GPU: the library loads, exports every function that
include/knng.h declares, and rejects invalid arguments on the host before any
HIP call (so these calls are safe on a machine without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_1701_08475_amd import knng

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(knng.LIB_PATH):
        from paper_1701_08475_amd import build_lib
        build_lib.build()
    return knng.lib()


def test_exports_every_declared_function(L):
    names = knng.declared_functions()
    assert set(names) >= {"knng_build", "knng_build_ex", "knng_partition", "knng_leaf_search",
                          "knng_status_string", "knng_last_error", "knng_default_options",
                          "knng_version"}
    for nm in names:
        assert hasattr(L, nm), nm


def test_status_codes_match_header(L):
    txt = open(os.path.join(ROOT, "include", "knng.h")).read()
    codes = {m.group(1): int(m.group(2)) for m in
             re.finditer(r"#define\s+(KNNG_(?:OK|ERR_\w+))\s+(-?\d+)", txt)}
    for nm, v in codes.items():
        assert getattr(knng, nm) == v
        assert L.knng_status_string(v) not in (None, b"unknown status")
    assert L.knng_status_string(12345) == b"unknown status"


def test_options_struct_layout(L):
    o = knng.KnngOptions()
    L.knng_default_options(ctypes.byref(o))
    # ten int32, then the tune-cache path pointer
    assert o.struct_size == ctypes.sizeof(knng.KnngOptions) == 48
    assert (o.precision, o.rerank_factor, o.min_leaf, o.max_iter, o.plain, o.check_finite,
            o.time_kernels, o.compact) == (0, 2, 0, 10, 0, 1, 0, 1)
    assert o.tune_cache is None
    # 5 int64, 2 int32, 5 float, 3 (float, int32) pairs, 2 int32 = 100 bytes,
    # padded to 104, then three int64
    assert ctypes.sizeof(knng.KnngStats) == 128


FAKE = 0x10000  # aligned, never dereferenced: validation fails first


def _build(L, data=FAKE, n=100, D=8, k=5, T=1, leaf=20, ids=FAKE, ds=FAKE, opt=None):
    return L.knng_build_ex(ctypes.c_void_p(data), n, D, k, T, leaf, 0, ctypes.c_void_p(ids),
                           ctypes.c_void_p(ds), opt, None, None)


@pytest.mark.parametrize("kw,status,msg", [
    (dict(data=0), knng.KNNG_ERR_INVALID_ARG, "null"),
    (dict(ids=0), knng.KNNG_ERR_INVALID_ARG, "null"),
    (dict(data=FAKE + 4), knng.KNNG_ERR_INVALID_ARG, "aligned"),
    (dict(n=1), knng.KNNG_ERR_INVALID_ARG, "n="),
    (dict(n=1 << 31), knng.KNNG_ERR_INVALID_ARG, "n="),
    (dict(D=0), knng.KNNG_ERR_INVALID_ARG, "D="),
    (dict(D=4100), knng.KNNG_ERR_UNSUPPORTED, "D="),
    (dict(D=1027), knng.KNNG_ERR_UNSUPPORTED, "D="),
    (dict(k=0), knng.KNNG_ERR_INVALID_ARG, "k="),
    (dict(k=100), knng.KNNG_ERR_INVALID_ARG, "k="),
    (dict(n=2000, k=600, leaf=1500), knng.KNNG_ERR_UNSUPPORTED, "k="),
    (dict(T=0), knng.KNNG_ERR_INVALID_ARG, "n_trees"),
    (dict(leaf=10), knng.KNNG_ERR_INVALID_ARG, "leaf_max"),   # needs >= 2*(k+1)-1 = 11
    (dict(n=5000, leaf=513), knng.KNNG_ERR_UNSUPPORTED, "leaf_max"),
])
def test_build_rejects_invalid_arguments(L, kw, status, msg):
    assert _build(L, **kw) == status
    assert msg in L.knng_last_error().decode()


def test_build_rejects_bad_options(L):
    o = knng.KnngOptions()
    L.knng_default_options(ctypes.byref(o))
    o.struct_size = 8
    assert _build(L, opt=ctypes.byref(o)) == knng.KNNG_ERR_INVALID_ARG
    L.knng_default_options(ctypes.byref(o))
    o.precision = 9
    assert _build(L, opt=ctypes.byref(o)) == knng.KNNG_ERR_INVALID_ARG
    L.knng_default_options(ctypes.byref(o))
    o.min_leaf = -1
    assert _build(L, opt=ctypes.byref(o)) == knng.KNNG_ERR_INVALID_ARG
    L.knng_default_options(ctypes.byref(o))
    o.min_leaf = 15  # leaf_max 20 < 2*15-1
    assert _build(L, opt=ctypes.byref(o)) == knng.KNNG_ERR_INVALID_ARG


def test_partition_and_leaf_search_reject_invalid_arguments(L):
    nl = ctypes.c_int32(0)
    f = ctypes.c_void_p(FAKE)
    assert L.knng_partition(None, 100, 8, 20, 1, 10, 0, 0, f, f, ctypes.byref(nl), None, None,
                            None) == knng.KNNG_ERR_INVALID_ARG
    assert L.knng_partition(f, 100, 8, 20, 11, 10, 0, 0, f, f, ctypes.byref(nl), None, None,
                            None) == knng.KNNG_ERR_INVALID_ARG  # 20 < 2*11-1
    assert L.knng_partition(f, 100, 8, 20, 1, 10, 0, -1, f, f, ctypes.byref(nl), None, None,
                            None) == knng.KNNG_ERR_INVALID_ARG
    nls = (ctypes.c_int32 * 1)(0)
    assert L.knng_leaf_search(f, 100, 8, 5, 1, f, f, nls, None, f, f, None) == \
        knng.KNNG_ERR_INVALID_ARG  # zero leaves
    nls = (ctypes.c_int32 * 1)(3)
    assert L.knng_leaf_search(f, 100, 8, 5, 1, None, f, nls, None, f, f, None) == \
        knng.KNNG_ERR_INVALID_ARG


def test_version(L):
    assert L.knng_version() >= 100


def test_search_and_index_reject_invalid_arguments(L):
    """Host-side checks of knng_search, knng_rvq_train, knng_ivf_build and
    knng_ivf_seeds: each case returns before any HIP call."""
    f = ctypes.c_void_p(FAKE)
    E, U = knng.KNNG_ERR_INVALID_ARG, knng.KNNG_ERR_UNSUPPORTED

    def search(data=f, n=100, D=8, kg=4, nq=3, ns=2, k=5, rounds=2):
        return L.knng_search(data, n, D, f, kg, f, nq, f, ns, k, rounds, f, f, None)
    assert search(data=None) == E
    assert search(n=0) == E
    assert search(D=0) == E
    assert search(D=5000) == U
    assert search(kg=0) == E
    assert search(ns=0) == E
    assert search(k=0) == E
    assert search(rounds=-1) == E
    assert search(k=2048, kg=1024) == U          # k x graph degree above 2^20

    def train(data=f, n=100, D=8, m=50, K1=4, K2=4, iters=5):
        return L.knng_rvq_train(data, n, D, f, m, K1, K2, f, f, iters, f, f, None, None, None,
                                None)
    assert train(data=None) == E
    assert train(m=0) == E
    assert train(m=101) == E                      # more sample rows than points
    assert train(K1=0) == E
    assert train(K2=300) == U                     # at most 256 words per stage
    assert train(iters=-1) == E
    assert train(D=0) == E

    def build(n=100, D=8, K1=4, K2=4, w1=f):
        return L.knng_ivf_build(f, n, D, w1, K1, f, K2, None, f, f, None)
    assert build(w1=None) == E
    assert build(n=-1) == E
    assert build(K1=257) == U
    assert build(D=4097) == U

    def seeds(nq=3, D=8, K1=32, K2=256, n1=4, ns=8, n_ids=100):
        return L.knng_ivf_seeds(f, nq, D, f, K1, f, K2, f, f, n_ids, n1, ns, f, None)
    assert seeds(n1=0) == E
    assert seeds(n1=33) == E                      # more than K1 first-stage words
    assert seeds(n1=17) == U                      # 17 x 256 keys above 4096
    assert seeds(ns=0) == E
    assert seeds(nq=-1) == E
    assert seeds(n_ids=-5) == E
    assert "n_ids" in L.knng_last_error().decode()


def test_u8_entry_points_reject_invalid_arguments(L):
    f = ctypes.c_void_p(FAKE)
    E = knng.KNNG_ERR_INVALID_ARG
    assert L.knng_to_u8(None, 10, f, None) == E
    assert L.knng_to_u8(f, -1, f, None) == E
    assert L.knng_to_u8(f, 0, f, None) == knng.KNNG_OK      # nothing to convert
    assert L.knng_search_u8(None, 100, 8, f, 4, f, 3, f, 2, 5, 2, f, f, None, None) == E
    assert L.knng_search_u8(ctypes.c_void_p(FAKE + 1), 100, 8, f, 4, f, 3, f, 2, 5, 2, f, f, None,
                            None) == E                         # not 16-byte aligned
    assert L.knng_search_u8(f, 100, 8, f, 0, f, 3, f, 2, 5, 2, f, f, None, None) == E


def test_leaf_search_noalloc_rejects_oversized_requests(L):
    """The no-allocation leaf search computes its scratch need on the host and
    rejects what does not fit its fixed array before any HIP call: here 8 trees
    of 10^6 rows with k = 32 need 8 * 10^6 * 32 * 8 B of candidate lists."""
    n, T, k = 1_000_000, 8, 32
    nl = (ctypes.c_int32 * T)(*([n // 40] * T))
    rc = L.knng_leaf_search_noalloc(ctypes.c_void_p(FAKE), n, 32, k, T, ctypes.c_void_p(FAKE),
                                    ctypes.c_void_p(FAKE), nl, None, ctypes.c_void_p(FAKE),
                                    ctypes.c_void_p(FAKE), None)
    assert rc == knng.KNNG_ERR_UNSUPPORTED
    assert b"scratch" in L.knng_last_error()
    # an absurd tree count saturates instead of wrapping around
    T2 = 1 << 20
    nl2 = (ctypes.c_int32 * T2)(*([1] * T2))
    rc = L.knng_leaf_search_noalloc(ctypes.c_void_p(FAKE), 1 << 30, 4096, 512, T2,
                                    ctypes.c_void_p(FAKE), ctypes.c_void_p(FAKE), nl2, None,
                                    ctypes.c_void_p(FAKE), ctypes.c_void_p(FAKE), None)
    assert rc == knng.KNNG_ERR_UNSUPPORTED


def test_autotune_knob_list_matches_header(L):
    txt = open(os.path.join(ROOT, "include", "knng.h")).read()
    m = re.search(r"#define\s+KNNG_TUNE_KNOBS\s+(\d+)", txt)
    assert m and int(m.group(1)) == len(knng.TUNE_KNOBS)


def test_autotune_rejects_empty_cache_path(L):
    # checked before any HIP call, so it runs without a GPU
    rc = L.knng_autotune(None, 100, 8, 5, 1, 50, 0, None, b"", None, None)
    assert rc == knng.KNNG_ERR_INVALID_ARG
    assert b"cache_path" in L.knng_last_error()
