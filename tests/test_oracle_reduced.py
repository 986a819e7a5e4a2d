"""Pins of the oracle's reduced-precision first pass (reading R9 in
knng_oracle.c): the rounding functions against torch's CPU casts and an
exhaustive round trip, the row scale against its closed form, and the
reduced graph against the exact graph where the two must coincide."""
import numpy as np
import pytest
import torch

from paper_1701_08475_amd import datagen

FMT_TORCH = {"bf16": torch.bfloat16, "fp16": torch.float16, "fp8": torch.float8_e4m3fn}


def _torch_round(fmt, vals):
    t = torch.tensor(vals, dtype=torch.float32).to(FMT_TORCH[fmt]).to(torch.float64)
    return t.numpy()


@pytest.mark.parametrize("fmt", ["bf16", "fp16"])
def test_every_16bit_value_rounds_to_itself(orc, fmt):
    pats = np.arange(1 << 16, dtype=np.uint32)
    if fmt == "bf16":
        vals = (pats << 16).view(np.float32).astype(np.float64)
    else:
        vals = pats.astype(np.uint16).view(np.float16).astype(np.float64)
    vals = vals[np.isfinite(vals)]
    got = np.array([orc.quantize(fmt, v) for v in vals])
    assert np.array_equal(got, vals)


@pytest.mark.parametrize("fmt", ["bf16", "fp16", "fp8"])
def test_rounding_matches_torch_casts(orc, fmt):
    rng = np.random.default_rng(7)
    hi = {"bf16": 1e30, "fp16": 60000.0, "fp8": 440.0}[fmt]
    lo = {"bf16": 1e-30, "fp16": 1e-7, "fp8": 2.0 ** -10}[fmt]
    mags = np.exp(rng.uniform(np.log(lo), np.log(hi), 20000))
    vals = (mags * rng.choice([-1.0, 1.0], 20000)).astype(np.float32).astype(np.float64)
    # plus exact ties: midpoints between neighbouring representable values
    if fmt == "fp8":
        grid = np.array([orc.quantize(fmt, v) for v in np.linspace(0.5, 300, 4000)])
        grid = np.unique(grid)
        ties = (grid[:-1] + grid[1:]) / 2
        vals = np.concatenate([vals, ties, -ties])
    got = np.array([orc.quantize(fmt, v) for v in vals])
    want = _torch_round(fmt, vals.astype(np.float32))
    assert np.array_equal(got, want)


def test_row_scale_closed_form(orc):
    row = np.array([0.3, -0.7, 0.05], np.float32)     # max 0.7 = 1.4 * 2^-1
    assert orc.row_scale("bf16", row) == 1.0
    assert orc.row_scale("fp16", row) == 2.0 ** (15 - (-1) - 1)
    assert orc.row_scale("fp8", row) == 2.0 ** (8 - (-1) - 1)
    row2 = np.array([255.0, 3.0], np.float32)          # floor(log2 255) = 7
    assert orc.row_scale("fp8", row2) == 1.0            # 2^(8-7-1)
    assert orc.row_scale("fp16", np.zeros(4, np.float32)) == 1.0
    # the scaled maximum stays below 2^E
    for fmt, E in (("fp16", 15), ("fp8", 8)):
        for mx in (1e-3, 0.999, 1.0, 17.5, 200.0):
            r = np.array([mx, -mx / 3], np.float32)
            assert abs(float(np.float32(mx)) * orc.row_scale(fmt, r)) < 2.0 ** E


def _trees(orc, X, T, L, ml, seed):
    perms, offs = [], []
    for t in range(T):
        tr = orc.tree(X, L, ml, 10, seed, t)
        perms.append(tr["perm"])
        offs.append(tr["leaf_off"])
    return np.stack(perms), offs


@pytest.mark.parametrize("fmt", ["bf16", "fp16", "fp8"])
def test_reduced_with_all_candidates_equals_exact(orc, fmt):
    """c >= leaf size - 1: every co-leaf member is re-ranked by d64, so the
    first pass's rounding cannot matter."""
    X = datagen.make("c1", n=1500)
    perms, offs = _trees(orc, X, 2, 40, 11, 3)
    a = orc.graph_from_leaves(X, 10, perms, offs)
    b = orc.graph_from_leaves_reduced(X, 10, perms, offs, fmt, 40)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_reduced_bf16_exact_on_small_integers(orc):
    """Integers below 256 are exact in BF16 and every product and sum of the
    first pass is exact in FP64, so d~ = d and the 2k pre-selection keeps the
    exact top k."""
    X = datagen.random_points(1200, 16, 4, "int")
    perms, offs = _trees(orc, X, 2, 60, 9, 5)
    a = orc.graph_from_leaves(X, 8, perms, offs)
    b = orc.graph_from_leaves_reduced(X, 8, perms, offs, "bf16", 16)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_reduced_fp8_loses_little(orc):
    """FP8 first pass with a 2k pre-selection: rows stay valid and nearly all
    of the exact graph's neighbours survive (C1-shaped data)."""
    X = datagen.make("c1", n=3000)
    perms, offs = _trees(orc, X, 2, 50, 11, 6)
    a_ids, a_d = orc.graph_from_leaves(X, 10, perms, offs)
    b_ids, b_d = orc.graph_from_leaves_reduced(X, 10, perms, offs, "fp8", 20)
    same = np.mean([len(set(a_ids[i]) & set(b_ids[i])) / 10.0 for i in range(len(X))])
    assert same > 0.97
    # every kept distance is the exact d64 of its pair
    for i in range(0, 3000, 37):
        for p in range(10):
            assert b_d[i, p] == orc.d64(X, i, b_ids[i, p])
