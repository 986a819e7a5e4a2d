"""Shared checks of GPU results against the oracle (used by the gpu tests)."""
import sys

import numpy as np

# Relative tolerance of FP32 results against FP64 (distance gaps below it are
# near-ties; FP32 distances must be within it of the FP64 value).
TAU = 1e-5


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(X):
    import torch
    return torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()


def graph_parity(orc, X, rows, g_ids, g_d, o_ids, o_d, strict=False):
    """G1: GPU rows vs oracle rows for points `rows`.

    - GPU ids are distinct, non-self, and present wherever the oracle has one;
    - each GPU distance (d32) is within TAU of d64 of the same pair;
    - at every rank p, d64(i, gpu_id[p]) is within TAU of the oracle's p-th
      distance (so ids can differ only inside near-tie classes).
    strict: ids identical and d32 == d64 exactly (data exact in FP32).
    Returns the fraction of positions with identical ids."""
    g_ids = np.asarray(g_ids)
    g_d = np.asarray(g_d, np.float64)
    k = o_ids.shape[1]
    d_true = orc.pair_d64(X, rows, np.where(g_ids >= 0, g_ids, 0))
    same = 0
    for q, i in enumerate(rows):
        gi, oi = g_ids[q], o_ids[q]
        valid = oi >= 0
        assert np.array_equal(gi >= 0, valid), (i, gi, oi)
        gv = gi[valid]
        assert len(set(gv.tolist())) == len(gv) and i not in gv, (i, gi)
        dt = d_true[q][valid]
        assert np.all(np.abs(g_d[q][valid] - dt) <= TAU * dt), (i, g_d[q], dt)
        od = o_d[q][valid]
        assert np.all(np.abs(dt - od) <= TAU * od), (i, gi, oi, dt, od)
        same += int(np.sum(gi == oi))
        if strict:
            assert np.array_equal(gi, oi), (i, gi, oi)
            assert np.array_equal(g_d[q][valid], od), (i, g_d[q], od)
    return same / float(len(rows) * k)


def rows_sorted(ids, d):
    """Every row ascending by (d, id)."""
    for r in range(len(ids)):
        key = list(zip(d[r].tolist(), ids[r].tolist()))
        if key != sorted(key):
            return False
    return True
