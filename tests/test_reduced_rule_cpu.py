"""The widened G1 rule of the reduced path (tests/gpu_helpers.py:
reduced_parity) on the CPU: the oracle's own emulated rows pass it, and rows
with a planted mistake (an id that is not a co-leaf member, an id the first
pass cannot keep, a kept candidate missing) fail it."""
import numpy as np
import pytest

from paper_1701_08475_amd import datagen
from tests.gpu_helpers import inverse_perms, leaf_members, reduced_parity


@pytest.fixture(scope="module")
def case(orc):
    X = datagen.gmm_unit(3000, 64, 12, 0.35, 21)
    perms, offs = [], []
    for t in range(2):
        tr = orc.tree(X, 200, 11, 10, 3, t)
        perms.append(tr["perm"])
        offs.append(tr["leaf_off"])
    perms = np.stack(perms)
    rows = datagen.sample_rows(len(X), 60, seed=2)
    ids, ds = orc.rows_from_leaves_reduced(X, 10, perms, offs, "fp8", 20, rows)[:2]
    return X, perms, offs, rows, ids, ds.astype(np.float32)


def test_emulation_passes(orc, case):
    X, perms, offs, rows, ids, ds = case
    # d32 of the emulated ids: the oracle's d64 rounded to FP32 is within tau
    assert reduced_parity(orc, X, "fp8", 10, 20, perms, offs, rows, ids, ds) == 1.0


def test_foreign_id_fails(orc, case):
    X, perms, offs, rows, ids, ds = case
    inv = inverse_perms(perms)
    bad = ids.copy()
    i = rows[0]
    co = set(np.concatenate(leaf_members(perms, offs, inv, i)).tolist())
    j = next(j for j in range(len(X)) if j not in co)
    bad[0, -1] = j
    d = ds.copy()
    d[0, -1] = np.float32(np.sum((X[i].astype(np.float64) - X[j]) ** 2))
    order = np.lexsort((bad[0], d[0]))
    bad[0], d[0] = bad[0][order], d[0][order]
    with pytest.raises(AssertionError):
        reduced_parity(orc, X, "fp8", 10, 20, perms, offs, rows, bad, d)


def test_missing_sure_candidate_fails(orc, case):
    X, perms, offs, rows, ids, ds = case
    # drop row 0's nearest id and append a co-leaf member ranked after the
    # emulation's k-th: the nearest one is a first-pass keep in some tree
    inv = inverse_perms(perms)
    i = rows[0]
    co = np.unique(np.concatenate(leaf_members(perms, offs, inv, i)))
    co = co[(co != i) & ~np.isin(co, ids[0])]
    d64 = np.sum((X[co].astype(np.float64) - X[i]) ** 2, axis=1)
    j = co[np.argmax(d64)]
    bad = np.concatenate([ids[0][1:], [j]])
    d = np.concatenate([ds[0][1:], [np.float32(d64.max())]])
    order = np.lexsort((bad, d))
    bad_ids, bad_d = ids.copy(), ds.copy()
    bad_ids[0], bad_d[0] = bad[order], d[order]
    with pytest.raises(AssertionError):
        reduced_parity(orc, X, "fp8", 10, 20, perms, offs, rows, bad_ids, bad_d)


def test_graph_parity_accepts_the_oracle_graph(orc):
    """The G1 checker of the FP32 path (tests/gpu_helpers.py: graph_parity)
    accepts the oracle's own graph and rejects a row with a wrong id."""
    from tests.gpu_helpers import graph_parity
    X = datagen.make("c1", n=2000)
    ids, ds, _ = orc.graph(X, 10, 2, 50, 1)
    rows = np.arange(len(X))
    assert graph_parity(orc, X, rows, ids, ds.astype(np.float32), ids, ds) == 1.0
    bad = ids.copy()
    bad[5, 0] = bad[5, -1]
    with pytest.raises(AssertionError):
        graph_parity(orc, X, rows, bad, ds.astype(np.float32), ids, ds)
