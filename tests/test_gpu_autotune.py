"""The autotuner (knng_autotune) and its cache: every candidate value of every
knob gives the default build's graph bit for bit (the tuner checks that on
the caller's data and fails otherwise), and a build that reads the cache
equals the default build, also with every knob forced to its other value."""
import numpy as np
import pytest

from paper_1701_08475_amd import datagen
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def K():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1701_08475_amd import knng
    knng.lib()
    return knng


SHAPES = [
    # C5-shaped float rows, FP8 leaves (FP32 assignment, filter, wide leaves)
    ("fp8", 60_000, 96, 16, 2, 300, "unit"),
    # C2-shaped integer rows (uint8 assignment, exact BF16 leaves, merge)
    ("fp32", 40_000, 128, 10, 2, 100, "int"),
    # C4-shaped wide rows, FP16 leaves
    ("fp16", 12_000, 960, 20, 2, 200, "unit"),
]


def _data(kind, n, D):
    if kind == "int":
        return np.clip(np.rint(datagen.gmm_uniform(n, D, 32, 0, 80, 16.0, 61)), 0, 255).astype(np.float32)
    return datagen.gmm_unit(n, D, 32, 0.35, 62)


@pytest.mark.parametrize("precision,n,D,k,T,L,kind", SHAPES)
def test_autotune_choices_change_no_bits(K, tmp_path, precision, n, D, k, T, L, kind):
    import torch
    X = torch.from_numpy(_data(kind, n, D)).cuda()
    path = tmp_path / "tune.txt"
    log("autotune %s n=%d D=%d k=%d T=%d L=%d" % (precision, n, D, k, T, L))
    chosen = K.autotune(X, k, T, L, str(path), seed=5, precision=precision)
    log("  chosen %s" % chosen)
    assert set(chosen) == set(K.TUNE_KNOBS)
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and "|" in lines[0]
    key, rest = lines[0].split("|")
    assert all(("%s=" % nm) in rest for nm in K.TUNE_KNOBS)
    a_ids, a_d, a_st = K.build(X, k, T, L, seed=5, precision=precision, stats=True)
    b_ids, b_d = K.build(X, k, T, L, seed=5, precision=precision, tune_cache=str(path))
    assert torch.equal(a_ids, b_ids)
    assert torch.equal(a_d.view(torch.int32), b_d.view(torch.int32))
    # every knob at its other value, through the cache: the same graph, and
    # the choices are applied (the filter's row counter drops to zero)
    other = {"assign_unroll": 1, "filter": 0, "assign_m_u": 2, "assign_m_pd": 2,
             "chunk_order": 0, "leaf_wide": 0, "leaf_buckets": 0, "merge_network": 1}
    flipped = tmp_path / "flipped.txt"
    flipped.write_text(key + "|" + " ".join("%s=%d" % kv for kv in other.items()) + "\n")
    c_ids, c_d, c_st = K.build(X, k, T, L, seed=5, precision=precision, stats=True,
                               tune_cache=str(flipped))
    assert torch.equal(a_ids, c_ids)
    assert torch.equal(a_d.view(torch.int32), c_d.view(torch.int32))
    assert c_st["filter_rows"] == 0
    if kind != "int":  # float rows: the filter and the leaf buckets show
        assert a_st["filter_rows"] > 0
        assert c_st["launches"] != a_st["launches"]


def test_autotune_cache_keeps_other_shapes(K, tmp_path):
    """A second shape adds a line; tuning the first shape again replaces its
    line only."""
    import torch
    X = torch.from_numpy(_data("unit", 20_000, 32)).cuda()
    path = tmp_path / "tune.txt"
    K.autotune(X, 8, 1, 100, str(path), seed=1, precision="fp32")
    K.autotune(X, 8, 2, 100, str(path), seed=1, precision="fp32")
    K.autotune(X, 8, 1, 100, str(path), seed=1, precision="fp32")
    keys = [ln.split("|")[0] for ln in path.read_text().splitlines()]
    assert len(keys) == 2 and len(set(keys)) == 2
