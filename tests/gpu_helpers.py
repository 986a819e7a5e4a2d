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


def inverse_perms(perms):
    """inv[t][perm[t][p]] = p."""
    perms = np.asarray(perms)
    inv = np.empty(perms.shape, np.int64)
    for t in range(perms.shape[0]):
        inv[t][perms[t]] = np.arange(perms.shape[1])
    return inv


def leaf_members(perms, offs, inv, i):
    """Per tree, the members of the leaf that holds point i (perms [T, n],
    offs a list of T boundary arrays, inv = inverse_perms(perms))."""
    out = []
    for t, (perm, lo) in enumerate(zip(perms, offs)):
        l = int(np.searchsorted(lo, inv[t][i], "right")) - 1
        out.append(np.asarray(perm[lo[l]:lo[l + 1]]))
    return out


# Bound on |d~_gpu - d~_emulated| for the pair (i, j) (unit roundoff u = 2^-24):
# the GPU's first pass takes the squared norms of the dequantised rows in FP32
# (error <= (D/64 + 7) u n~), the scaled dot product in FP32 inside the matrix
# cores (any order: <= Dp u |x~_i| |x~_j| <= Dp u (n~_i + n~_j) / 2 after the
# exact power-of-two unscaling), and the combination n~_i + n~_j - 2 g with two
# roundings (<= 2 u (n~_i + n~_j)); the emulation is FP64.  Together at most
# (Dp + D/64 + 11) u (n~_i + n~_j); the factor 2 and the +16 leave slack.
# n~ <= (1 + rel)^2 |x|^2 with rel the format's half-ulp (2^-4 FP8, 2^-11 FP16,
# 2^-8 BF16) bounds the dequantised norms from the input rows.
FMT_REL = {"fp8": 2.0 ** -4, "fp16": 2.0 ** -11, "bf16": 2.0 ** -8}


def first_pass_bound(X, fmt, i, js):
    D = X.shape[1]
    Dp = (D + 31) // 32 * 32
    nx = lambda r: (1.0 + FMT_REL[fmt]) ** 2 * np.sum(np.asarray(r, np.float64) ** 2, axis=-1)
    return 2.0 * (Dp + D / 64.0 + 16) * 2.0 ** -24 * (nx(X[i]) + nx(X[js])) + 1e-12


def reduced_parity(orc, X, fmt, k, c, perms, offs, rows, g_ids, g_d):
    """The G1 rule widened to the reduced first pass.  GPU rows g_ids/g_d for
    points `rows`, built from leaves (perms, offs) with a first pass in `fmt`
    keeping c candidates per row and leaf.  The emulation (reading R9) gives,
    per row and tree, the first-pass distances e of the c-th kept (thr0) and
    the first dropped (thr1) candidate; beta bounds the GPU's first-pass error
    against it (first_pass_bound).  Then:
      (a) every GPU id is a co-leaf member that some tree's first pass may
          keep: e(i, j) <= thr0 + 2 beta;
      (b) every co-leaf member that a tree's first pass must keep
          (e(i, j) < thr1 - 2 beta) and that is nearer in d64 than the GPU's
          k-th entry (beyond tau) is in the GPU row;
      (c) ids distinct and non-self, d32 within tau of d64, rows ascending by
          (d32, id).
    Returns the fraction of rows identical to the emulation's."""
    g_ids = np.asarray(g_ids)
    g_d = np.asarray(g_d, np.float64)
    e_ids, e_d, thr = orc.rows_from_leaves_reduced(X, k, perms, offs, fmt, c, rows)
    d_true = orc.pair_d64(X, rows, np.where(g_ids >= 0, g_ids, 0))
    inv = inverse_perms(perms)
    same = 0
    for q, i in enumerate(rows):
        gi = g_ids[q]
        ok = gi >= 0
        assert np.array_equal(ok, e_ids[q] >= 0), (i, gi, e_ids[q])
        gv = gi[ok]
        assert len(set(gv.tolist())) == len(gv) and i not in gv, (i, gi)
        dt = d_true[q][ok]
        assert np.all(np.abs(g_d[q][ok] - dt) <= TAU * dt), (i, g_d[q], dt)
        key = list(zip(g_d[q][ok].tolist(), gv.tolist()))
        assert key == sorted(key), (i, key)
        members = leaf_members(perms, offs, inv, i)
        in_row = set(gv.tolist())
        kth = dt[-1] if len(dt) == k else np.inf
        valid = set()
        for t, mem in enumerate(members):
            js = mem[mem != i]
            e = orc.dtilde_row(X, fmt, i, js)
            beta = first_pass_bound(X, fmt, i, js)
            valid.update(js[e <= thr[q, t, 0] + 2 * beta].tolist())
            sure = js[e < thr[q, t, 1] - 2 * beta]
            if len(sure):
                ds = orc.pair_d64(X, np.array([i]), sure.reshape(1, -1))[0]
                need = sure[ds < kth * (1.0 - TAU)]
                missing = set(need.tolist()) - in_row
                assert not missing, (i, t, sorted(missing), gi)
        assert in_row <= valid, (i, sorted(in_row - valid))
        same += int(np.array_equal(gi, e_ids[q]))
    return same / float(len(rows))
