#!/usr/bin/env python3
"""kNN-graph build throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c5]

One step = one full build (knng_build_ex: partition of every tree, leaf
search, merge) of the resident synthetic input.  The headline workload is the
largest single-GPU configuration, c5 (10^7 x 96 unit-norm rows, k = 32, 8
trees, leaves up to 500 points, FP8 first pass with FP32 re-rank).  Prints one
JSON line with points/s, the roofline position of the dominant kernel (the
two-means assignment pass, HBM-bound), the plain FP32 schedule on the same
data with the paired recall difference, the first-pass and output error
against FP64, and the CPU oracle timed on a bounded sample on the host.  A
second workload (c2, SIFT-shaped) is reported under "extra", together with
the graph's consumers: E-GNNS search (Alg. 2) from random seeds and from the
seeds of an RVQ inverted index (Sec. 4).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "kNN-graph build points/sec at recall@k≥target; leaf MFMA util vs plain FP32"
HBM_PEAK_GBS = 8000.0
FP32_VALU_PEAK_TFLOPS = 157.3
MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp16": 2500.0, "fp8": 5000.0}
PROFILES = os.path.join(ROOT, "profiles")
CSRC = os.path.join(ROOT, "paper_1701_08475_amd", "csrc")
# sources of the assignment kernels: stored HBM counters are void once they change
ASSIGN_SRCS = [os.path.join(CSRC, f) for f in ("partition.hip", "assign_mfma.hip", "assign_f32.hip")]
# rows of the CPU oracle's bounded sample, per workload (about 10-30 s on 16 threads)
CPU_SAMPLE = {"c1": 10_000, "c2": 500_000, "c3": 500_000, "c4": 40_000, "c5": 800_000}
DTYPE = {
    "u8": "bf16 exact first pass (integer data) / u8 rows, int8 MFMA + f64 two-means",
    "fp32": "fp32 leaves / f64 two-means margins and centroid sums",
    "bf16": "bf16 first pass + fp32 re-rank / f64 two-means",
    "fp16": "fp16 first pass + fp32 re-rank / f64 two-means",
    "fp8": "fp8-e4m3 first pass + fp32 re-rank / f64 two-means",
}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def source_sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def stored_traffic(config):
    """HBM bytes per assignment launch from the committed rocprofv3 counter
    summary, or None when it is missing or the kernel source changed since."""
    path = os.path.join(PROFILES, "k_assign_%s_hbm_counters.md" % config)
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"traffic_bytes_per_launch\s*=\s*([0-9.eE+]+)", txt)
    s = re.search(r"assign_sources_sha256_16\s*=\s*([0-9a-f]+)", txt)
    if not m or not s or s.group(1) != source_sha(ASSIGN_SRCS):
        return None
    return float(m.group(1))


# ------------------------------------------------------------ evaluation
# Ground truth for the recall figures: exact nearest rows of X in FP64 by
# brute force.  Candidates come from FP64 matrix products on the GPU
# (|x|^2 - 2 q.x, ranked per query); the best k + 32 of each query are
# re-measured on the host in the direct form sum (x_d - q_d)^2 and ranked by
# (distance, id).

def _d64_direct(X, q, ids):
    diff = X[ids].astype(np.float64) - q.astype(np.float64)[None, :]
    return (diff * diff).sum(1)


def exact_knn_fp64(X, Q, k, self_ids=None, block=1 << 21, xd=None):
    """(ids int64 [nq, k], d float64 [nq, k]); self_ids[q] (optional) is
    excluded.  xd: X on the GPU (float32) for the candidate products, or None
    to take them on the host."""
    import torch
    if xd is None:
        xd = torch.from_numpy(np.ascontiguousarray(X, np.float32))
    nq = len(Q)
    extra = k + 32
    Qd = torch.from_numpy(np.ascontiguousarray(Q, np.float64)).to(xd.device)
    best_d, best_i = None, None
    for b0 in range(0, xd.shape[0], block):
        Xb = xd[b0:b0 + block].to(torch.float64)
        d = (Xb * Xb).sum(1)[None, :] - 2.0 * (Qd @ Xb.T)
        t = min(extra, d.shape[1])
        v, i = torch.topk(d, t, dim=1, largest=False)
        i = i + b0
        if best_d is None:
            best_d, best_i = v, i
        else:
            v2, j = torch.topk(torch.cat([best_d, v], 1), min(extra, best_d.shape[1] + t), dim=1,
                               largest=False)
            best_i = torch.gather(torch.cat([best_i, i], 1), 1, j)
            best_d = v2
        del Xb, d
    cand = best_i.cpu().numpy()
    ids = np.empty((nq, k), np.int64)
    ds = np.empty((nq, k), np.float64)
    for q in range(nq):
        ci = cand[q]
        if self_ids is not None:
            ci = ci[ci != self_ids[q]]
        dd = _d64_direct(X, Q[q], ci)
        order = np.lexsort((ci, dd))[:k]
        ids[q], ds[q] = ci[order], dd[order]
    return ids, ds


def graph_recall(X, rows, G, E, Ed):
    """Tie-tolerant recall@k: a graph id counts when it is an exact neighbour
    or no farther than the exact k-th neighbour."""
    k = E.shape[1]
    hits = 0
    for q, i in enumerate(rows):
        g = G[q][G[q] >= 0]
        dg = _d64_direct(X, X[i], g)
        ex = set(E[q].tolist())
        hits += sum(1 for j, dj in zip(g.tolist(), dg) if j in ex or dj <= Ed[q, k - 1])
    return hits / float(len(rows) * k)


def search_recall(ids, E):
    """Mean fraction of the exact k nearest ids found per query."""
    hit = 0
    for a, b in zip(ids, E):
        hit += len(set(a[a >= 0].tolist()) & set(b.tolist()))
    return hit / float(E.shape[0] * E.shape[1])


FIRST_PASS_FMT = {"bf16": ("bfloat16", None), "fp16": ("float16", 15), "fp8": ("float8_e4m3fn", 8)}


def first_pass_error(X, rows, G, precision):
    """Relative error against FP64 of the reduced first pass on the pairs the
    build kept (each sampled row with its k neighbours): the rows are scaled by
    their power of two sigma = 2^(E - floor(log2 max|x|) - 1) (1 for BF16),
    rounded to the format by torch's CPU cast, and the squared distance of the
    dequantised rows is taken in FP64."""
    import torch
    name, E = FIRST_PASS_FMT[precision]
    dt = getattr(torch, name)

    def dq(V):
        V = V.astype(np.float64)
        if E is None:
            s = np.ones(len(V))
        else:
            mx = np.abs(V).max(1)
            s = np.where(mx > 0, np.ldexp(1.0, E - (np.frexp(mx)[1] - 1) - 1), 1.0)
        q = torch.from_numpy((V * s[:, None]).astype(np.float32)).to(dt).to(torch.float64).numpy()
        return q / s[:, None]

    errs = []
    for q, i in enumerate(rows):
        g = G[q][G[q] >= 0]
        a, b = dq(X[i:i + 1]), dq(X[g])
        dt_ = ((b - a) ** 2).sum(1)
        d64 = _d64_direct(X, X[i], g)
        ok = d64 > 0
        errs.append(np.abs(dt_[ok] - d64[ok]) / d64[ok])
    e = np.concatenate(errs)
    return {"median": float(np.median(e)), "p99": float(np.quantile(e, 0.99)),
            "max": float(e.max()), "pairs": int(len(e)),
            "definition": "|d~ - d64| / d64 of the kept pairs, d~ from the power-of-two scaled "
                          "rows rounded to %s" % precision}


def output_error(X, rows, G, Gd):
    """Largest relative error of the output distances (d32) against FP64."""
    worst = 0.0
    for q, i in enumerate(rows):
        ok = G[q] >= 0
        d64 = _d64_direct(X, X[i], G[q][ok])
        nz = d64 > 0
        if nz.any():
            worst = max(worst, float(np.max(np.abs(Gd[q][ok][nz] - d64[nz]) / d64[nz])))
    return worst


def search_roofline(knng, xd, graph, qd, sd, k, rounds, ms, x8=None):
    """Algorithmic bytes of an E-GNNS batch from its work report (one extra,
    untimed call; the search is deterministic): a row of D elements (4 bytes,
    or 1 for the uint8 copy x8) per distance taken, kg graph entries per node
    expanded, plus each query, its seeds and its k results."""
    if x8 is None:
        _, _, (n_dist, n_exp) = knng.search(xd, graph, qd, sd, k, rounds, work=True)
    else:
        _, _, (n_dist, n_exp) = knng.search_u8(x8, graph, qd, sd, k, rounds, work=True)
    D, kg = xd.shape[1], graph.shape[1]
    nq, ns = sd.shape
    eb = 1 if x8 is not None else 4
    alg = n_dist * D * eb + n_exp * kg * 4 + nq * (D * 4 + ns * 4 + k * 8)
    gbs = alg / (ms * 1e6)
    return {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "distances": n_dist, "expanded": n_exp,
            "bytes": alg, "kernel": "k_egnns (row gathers of visited nodes)"}


# ------------------------------------------------------------ one workload
def run_workload(args, name, steps, warmup, headline):
    import torch
    from paper_1701_08475_amd import datagen, knng

    c = dict(datagen.CONFIGS[name])
    if headline and args.precision:
        c["precision"] = args.precision
    n, D, k, T, L = c["n"], c["D"], c["k"], c["n_trees"], c["leaf_max"]
    seed, prec = c["seed"], c["precision"]
    log("config %s: n=%d D=%d k=%d trees=%d leaf_max=%d precision=%s" % (name, n, D, k, T, L, prec))
    t = time.perf_counter()
    X = datagen.make(name)
    log("data generated in %.1fs" % (time.perf_counter() - t))
    dev = torch.device("cuda:0")
    xd = torch.from_numpy(X).to(dev)
    ids = torch.empty((n, k), dtype=torch.int32, device=dev)
    ds = torch.empty((n, k), dtype=torch.float32, device=dev)
    compact = not args.no_compact

    def step(timed_kernels=False):
        return knng.build(xd, k, T, L, seed=seed, precision=prec, stats=True,
                          time_kernels=timed_kernels, compact=compact, out=(ids, ds))

    for w in range(warmup):
        step()
        log("warmup %d done" % w)
    torch.cuda.synchronize()
    sts, marks = [], []  # each build call returns after its work is done
    t0 = time.perf_counter()
    for s in range(steps):
        # HIP events around every launch of the assignment, leaf and merge
        # kernels (hundreds per build) cost milliseconds per build: they are
        # recorded in the last timed step only
        sts.append(step(timed_kernels=(s == steps - 1))[2])
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms = [(b - a) * 1e3 for a, b in zip([t0] + marks[:-1], marks)]
    ms_per_step = (t1 - t0) * 1e3 / steps
    value = n / (ms_per_step / 1e3)
    log("timed %d steps: %.2f ms/step, %.3e points/s" % (steps, ms_per_step, value))
    st = sts[-1]
    u8 = bool(st["compact_used"])
    leaf_fmt = "bf16" if st["exact_first_pass"] else prec

    # dominant kernel: the two-means assignment pass of the level kernels,
    # bound by HBM.  Its rows are the assigned rows minus those assigned inside
    # the subtree kernels (rows held in LDS); kernel times from the last timed
    # step, the one with per-launch events.
    # Filtered passes (FP32 rows with a reduced leaf copy) read each row's
    # reduced copy (D elements, its 4-byte scale and 4-byte error norm) and the FP32 values of
    # the rows the filter leaves undecided or that changed side.
    elem_bytes = 1.0 if u8 else 4.0  # uint8 copy or FP32 rows
    red_bytes = {"bf16": 2.0, "fp16": 2.0, "fp8": 1.0}.get(prec, 0.0)
    level_rows = st["assign_rows"] - st["subtree_rows"]
    f_rows, fx_rows = st.get("filter_rows", 0), st.get("filter_exact_rows", 0)
    a_bytes = ((level_rows - f_rows) * D * elem_bytes + f_rows * (D * red_bytes + 8.0)
               + fx_rows * D * 4.0)
    a_ms, a_launches = st["ms_k_assign"], st["n_k_assign"]
    achieved = a_bytes / (a_ms / 1e3) / 1e9
    roofline = {
        "bound": "hbm", "kernel": "k_assign (two-means assignment pass, level kernels)",
        "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": stored_traffic(name),
        "bytes_per_launch": a_bytes / a_launches, "avg_launch_ms": a_ms / a_launches,
        "algorithmic_bytes": ("rows streamed by the level kernels x D x %d B" % elem_bytes
                              if not f_rows else
                              "unfiltered rows x D x 4 B + filtered rows x (D x %d B + 8 B: 1/sigma and e) + "
                              "rows read as FP32 by filtered passes x D x 4 B" % red_bytes),
        "row_storage": ("uint8 (lossless: integer data)" if u8 else
                        "fp32, %s filter copy" % prec if f_rows else "fp32"),
        "filter_rows": f_rows, "filter_exact_rows": fx_rows,
        "filter_band_frac": round(fx_rows / f_rows, 4) if f_rows else None,
        "launches_per_step": a_launches,
        "subtree_rows_excluded": st["subtree_rows"],
        "events_in": "last timed step",
    }

    pairs = st["ordered_pairs"]
    leaf_ms, merge_ms = st["ms_k_leaf"], st["ms_k_merge"]
    gram_flops = 2.0 * D * pairs  # one D-long dot product per ordered pair
    c_keep = k if st["exact_first_pass"] or prec == "fp32" else 2 * k
    # re-rank: c candidates per row and tree, D subtractions and D FMAs each
    rerank_flops = 0.0 if (st["exact_first_pass"] or prec == "fp32") else 3.0 * D * c_keep * n * T
    leaf = {"ms": round(leaf_ms, 3), "path": leaf_fmt if leaf_fmt != "fp32" else "fp32 direct",
            "gram_tflops": round(gram_flops / leaf_ms / 1e9, 2)}
    if leaf_fmt in MFMA_PEAK_TFLOPS:
        leaf["mfma_peak_tflops"] = MFMA_PEAK_TFLOPS[leaf_fmt]
        leaf["mfma_frac"] = round(gram_flops / leaf_ms / 1e9 / MFMA_PEAK_TFLOPS[leaf_fmt], 5)
    if rerank_flops:
        leaf["rerank_valu_tflops"] = round(rerank_flops / leaf_ms / 1e9, 2)
        leaf["valu_peak_tflops"] = FP32_VALU_PEAK_TFLOPS
        leaf["rerank_valu_frac"] = round(rerank_flops / leaf_ms / 1e9 / FP32_VALU_PEAK_TFLOPS, 4)
    merge_bytes = (T * n * k * 8.0 + n * k * 8.0) if T > 1 else 0.0
    phases = {
        "ms_prep": round(st["ms_prep"], 3),
        "ms_partition": round(sum(s["ms_partition"] for s in sts) / steps, 3),
        "ms_leaf": round(sum(s["ms_leaf"] for s in sts) / steps, 3),
        "ms_merge": round(sum(s["ms_merge"] for s in sts) / steps, 3),
        "leaf_kernel": leaf,
        "merge_kernel": {"ms": round(merge_ms, 3),
                         "gbs": round(merge_bytes / merge_ms / 1e6, 1) if merge_ms > 0 else None},
        "pairs_per_s": pairs / (ms_per_step / 1e3),
        "assign_passes_per_point_per_tree": st["assign_rows"] / float(n * T),
        "leaves": st["leaves"], "levels": st["levels"], "repairs": st["repairs"],
        "launches": st["launches"],
    }
    G = ids.cpu().numpy()
    Gd = ds.cpu().numpy()

    plain = None
    Gp = None
    if not args.no_plain:
        # the plain FP32 path: trees one after another, FP32 rows (no uint8
        # copy), FP32 direct leaf distances; one untimed call first
        pids = torch.empty_like(ids)
        pds = torch.empty_like(ds)

        def plain_call():
            knng.build(xd, k, T, L, seed=seed, precision="fp32", plain=True, compact=False,
                       out=(pids, pds))
        plain_call()
        torch.cuda.synchronize()
        tp = time.perf_counter()
        reps = 2
        for _ in range(reps):
            plain_call()
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - tp) * 1e3 / reps
        plain = {"ms_per_step": round(plain_ms, 2),
                 "speedup_of_batched": round(plain_ms / ms_per_step, 3),
                 "definition": "same rules; trees one after another; FP32 rows; FP32 direct "
                               "leaf distances; one sync per level"}
        Gp = pids.cpu().numpy()
        del pids, pds
        log("plain schedule: %.2f ms/step" % plain_ms)

    recall = None
    errors = None
    if not args.no_recall:
        rows = datagen.sample_rows(n, args.recall_rows)
        tr = time.perf_counter()
        E, Ed = exact_knn_fp64(X, X[rows], k, self_ids=rows, xd=xd)
        rb = graph_recall(X, rows, G[rows], E, Ed)
        recall = {"recall_at_k": round(rb, 5), "rows": len(rows), "k": k,
                  "ground_truth": "FP64 brute force, tie-tolerant"}
        if Gp is not None:
            rp = graph_recall(X, rows, Gp[rows], E, Ed)
            recall["plain_fp32_recall_at_k"] = round(rp, 5)
            recall["diff_pp_batched_minus_plain"] = round(100.0 * (rb - rp), 4)
            recall["rows_identical_to_plain"] = int(sum(
                np.array_equal(G[i], Gp[i]) for i in rows))
        errors = {"output_d32_max_rel_err_vs_fp64": output_error(X, rows, G[rows], Gd[rows])}
        if leaf_fmt in FIRST_PASS_FMT:
            errors["first_pass_vs_fp64"] = first_pass_error(X, rows[:100], G[rows[:100]], leaf_fmt)
        log("recall@%d = %.4f on %d rows (%.1fs)%s" % (
            k, rb, len(rows), time.perf_counter() - tr,
            "" if Gp is None else ", plain %.4f" % recall["plain_fp32_recall_at_k"]))

    cpu = None
    if headline and not args.no_cpu:
        # the CPU baseline is the oracle itself, timed on a bounded sample
        from oracle import oracle
        oracle.build()
        ns = min(args.cpu_sample or CPU_SAMPLE.get(name, 100_000), n)
        Xs = np.ascontiguousarray(X[:ns])
        threads = oracle.num_threads()
        tc = time.perf_counter()
        oracle.graph(Xs, k, T, L, seed)
        el = time.perf_counter() - tc
        cpu = {"value": round(ns / el, 1), "unit": "points/s", "cores": threads, "kind": "oracle",
               "seconds": round(el, 2),
               "sample": "first %d of the %d rows, all %d trees, k=%d, leaf_max=%d, FP64 "
                         "leaves (per-point cost grows with log n, so the full-size rate is "
                         "somewhat lower)" % (ns, n, T, k, L)}
        log("cpu oracle: %d points in %.1fs on %d threads" % (ns, el, threads))
        if args.cpu_sample_1t > 0:
            # the paper times its construction on one thread (Sec. 5)
            n1 = min(args.cpu_sample_1t, n)
            oracle.set_num_threads(1)
            t1_ = time.perf_counter()
            oracle.graph(np.ascontiguousarray(X[:n1]), k, T, L, seed)
            el1 = time.perf_counter() - t1_
            oracle.set_num_threads(threads)
            cpu["one_thread"] = {"value": round(n1 / el1, 1), "unit": "points/s",
                                 "seconds": round(el1, 2),
                                 "sample": "first %d rows, all %d trees" % (n1, T)}
            log("cpu oracle, one thread: %d points in %.1fs" % (n1, el1))

    res = {
        "value": round(value, 1), "ms_per_step": round(ms_per_step, 3),
        "step_ms": [round(v, 3) for v in step_ms],
        "median_ms_without_kernel_events": (round(float(np.median(step_ms[:-1])), 3)
                                            if len(step_ms) > 1 else None),
        "dtype": DTYPE["u8"] if (u8 and st["exact_first_pass"]) else DTYPE[leaf_fmt],
        "config": {"workload": "%s: n=%d D=%d k=%d trees=%d leaf_max=%d, %s first pass, batched"
                               % (name, n, D, k, T, L, leaf_fmt),
                   "n": n, "D": D, "k": k, "n_trees": T, "leaf_max": L, "seed": seed,
                   "precision": prec},
        "roofline": roofline, "cpu_baseline": cpu, "recall": recall, "errors": errors,
        "plain_schedule": plain, "phases": phases,
    }
    if not headline and not args.no_search:
        res["search"], res["ivf_search"] = run_search(args, name, X, xd, ids, k, st)
    del xd, ids, ds
    torch.cuda.empty_cache()
    return res


def run_search(args, name, X, xd, ids, k, st):
    """E-GNNS (Alg. 2) over the graph just built, from random seeds and from
    the seeds of an RVQ inverted index (Sec. 4); queries from the config's
    mixture, recall against FP64 brute force."""
    import torch
    from paper_1701_08475_amd import datagen, knng
    n = len(X)
    dev = xd.device
    Qn = datagen.queries(name, args.search_queries)
    S = datagen.seeds(n, len(Qn), args.search_seeds)
    qd = torch.from_numpy(Qn).to(dev)
    sd = torch.from_numpy(S).to(dev)
    rounds = args.search_rounds
    knng.search(xd, ids, qd, sd, k, rounds)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    reps = 3
    for _ in range(reps):
        s_ids, s_d = knng.search(xd, ids, qd, sd, k, rounds)
    torch.cuda.synchronize()
    s_ms = (time.perf_counter() - ts) * 1e3 / reps
    search = {"queries": len(Qn), "k": k, "graph_degree": k, "rounds": rounds,
              "seeds": args.search_seeds, "ms": round(s_ms, 3),
              "queries_per_s": round(len(Qn) / (s_ms / 1e3), 1),
              "data": "synthetic queries from the config's mixture",
              "roofline": search_roofline(knng, xd, ids, qd, sd, k, rounds, s_ms)}
    x8 = None
    if st["exact_first_pass"] or (X.min() >= 0 and X.max() <= 255 and np.array_equal(X, np.rint(X))):
        # integer data: the same search over the lossless uint8 copy
        x8 = knng.to_u8(xd)
        knng.search_u8(x8, ids, qd, sd, k, rounds)
        torch.cuda.synchronize()
        tu = time.perf_counter()
        for _ in range(reps):
            u_ids, _ = knng.search_u8(x8, ids, qd, sd, k, rounds)
        torch.cuda.synchronize()
        u_ms = (time.perf_counter() - tu) * 1e3 / reps
        search["uint8_rows"] = {
            "ms": round(u_ms, 3), "queries_per_s": round(len(Qn) / (u_ms / 1e3), 1),
            "same_results": bool(torch.equal(u_ids, s_ids)),
            "roofline": search_roofline(knng, xd, ids, qd, sd, k, rounds, u_ms, x8=x8)}
        log("search over uint8 rows: %.2f ms" % u_ms)
    rq = min(200, len(Qn))
    Eq = None
    if not args.no_recall:
        Eq, _ = exact_knn_fp64(X, Qn[:rq], k, xd=xd)
        search["recall_at_k"] = round(search_recall(s_ids.cpu().numpy()[:rq], Eq), 5)
        search["recall_queries"] = rq
    log("search: %d queries in %.2f ms (%s)" % (len(Qn), s_ms, search.get("recall_at_k")))
    if args.no_ivf:
        return search, None
    K1 = K2 = args.ivf_words
    tr, i1, i2 = datagen.rvq_sample(n, args.ivf_train, K1, K2)
    trd, i1d, i2d = (torch.from_numpy(a).to(dev) for a in (tr, i1, i2))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    W1, W2, rounds_tr = knng.rvq_train(xd, trd, i1d, i2d, args.ivf_iters)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    _, offs, lids = knng.ivf_build(xd, W1, W2)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    ns_ivf = args.search_seeds
    knng.ivf_seeds(qd, W1, W2, offs, lids, args.ivf_n1, ns_ivf)
    torch.cuda.synchronize()
    ta = time.perf_counter()
    for _ in range(reps):
        S_ivf = knng.ivf_seeds(qd, W1, W2, offs, lids, args.ivf_n1, ns_ivf)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for _ in range(reps):
        v_ids, _ = knng.search(xd, ids, qd, S_ivf, k, rounds)
    torch.cuda.synchronize()
    tc2 = time.perf_counter()
    seed_ms = (tb - ta) * 1e3 / reps
    srch_ms = (tc2 - tb) * 1e3 / reps
    srch8_ms = None
    if x8 is not None:
        td = time.perf_counter()
        for _ in range(reps):
            knng.search_u8(x8, ids, qd, S_ivf, k, rounds)
        torch.cuda.synchronize()
        srch8_ms = (time.perf_counter() - td) * 1e3 / reps
    ivf = {"search_roofline": search_roofline(knng, xd, ids, qd, S_ivf, k, rounds, srch_ms),
           "words": [K1, K2], "train_rows": len(tr), "iters": args.ivf_iters,
           "rounds": list(rounds_tr), "train_ms": round((t1 - t0) * 1e3, 2),
           "build_ms": round((t2 - t1) * 1e3, 2), "n1": args.ivf_n1, "seeds": ns_ivf,
           "seeds_ms": round(seed_ms, 3), "search_ms": round(srch_ms, 3),
           "search_uint8_ms": round(srch8_ms, 3) if srch8_ms is not None else None,
           "queries_per_s": round(len(Qn) / ((seed_ms + srch_ms) / 1e3), 1),
           "non_empty_lists": int((offs[1:] > offs[:-1]).sum().item())}
    # encoding work: per point and stage, K words x D dimensions of one FP64
    # subtraction and one FMA (3 flops); the call also sorts the keys, so this
    # rate is a lower bound for the encoding kernel
    enc_flops = 2 * n * K1 * X.shape[1] * 3
    ivf["encode_fp64_tflops_whole_call"] = round(enc_flops / ((t2 - t1) * 1e12), 2)
    ivf["fp64_peak_tflops"] = 78.6
    if Eq is not None:
        ivf["recall_at_k"] = round(search_recall(v_ids.cpu().numpy()[:rq], Eq), 5)
    log("ivf: train %.1f ms, build %.1f ms, seeds %.2f ms + search %.2f ms (%s)"
        % (ivf["train_ms"], ivf["build_ms"], seed_ms, srch_ms, ivf.get("recall_at_k")))
    return search, ivf


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c5", help="headline workload (c1..c5)")
    ap.add_argument("--extra-config", default="c2",
                    help="second workload reported under 'extra' ('none' to skip)")
    ap.add_argument("--extra-steps", type=int, default=5)
    ap.add_argument("--precision", default=None, help="override the headline's leaf precision")
    ap.add_argument("--recall-rows", type=int, default=500)
    ap.add_argument("--cpu-sample", type=int, default=0, help="oracle rows (0: per workload)")
    ap.add_argument("--cpu-sample-1t", type=int, default=50_000,
                    help="rows of the one-thread oracle timing (the paper's setting)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-recall", action="store_true")
    ap.add_argument("--no-plain", action="store_true", help="skip timing the plain schedule")
    ap.add_argument("--no-compact", action="store_true",
                    help="stream FP32 rows in the partition even for integer data")
    ap.add_argument("--no-search", action="store_true",
                    help="skip the E-GNNS search over the extra workload's graph")
    ap.add_argument("--search-queries", type=int, default=10_000)
    ap.add_argument("--search-seeds", type=int, default=64)
    ap.add_argument("--search-rounds", type=int, default=10)
    ap.add_argument("--no-ivf", action="store_true",
                    help="skip the RVQ inverted index (training, lists, seeded search)")
    ap.add_argument("--ivf-train", type=int, default=65536, help="RVQ training rows")
    ap.add_argument("--ivf-words", type=int, default=256, help="words per RVQ stage")
    ap.add_argument("--ivf-iters", type=int, default=10, help="Lloyd rounds per stage")
    ap.add_argument("--ivf-n1", type=int, default=8, help="first-stage words kept per query")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 1 GiB elementwise copy first (HBM counter calibration)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU; multi-GPU sharding by tree is a design "
              "note only (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1701_08475_amd import knng

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    knng.lib()
    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()
        del a, b
        log("copy calibration kernel: 1 GiB read + 1 GiB write")

    head = run_workload(args, args.config, args.steps, args.warmup, headline=True)
    extra = None
    if args.extra_config and args.extra_config != "none" and args.extra_config != args.config:
        extra = run_workload(args, args.extra_config, args.extra_steps, 1, headline=False)

    out = {
        "metric": METRIC, "value": head["value"], "unit": "points/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "step_ms": head["step_ms"],
        "median_ms_without_kernel_events": head["median_ms_without_kernel_events"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": head["dtype"],
        "data": "synthetic (seeded Gaussian mixture shaped like the paper's workloads)",
        "config": head["config"],
        "roofline": head["roofline"],
        "cpu_baseline": head["cpu_baseline"],
        "recall": head["recall"],
        "errors": head["errors"],
        "plain_schedule": head["plain_schedule"],
        "phases": head["phases"],
        "extra": {args.extra_config: extra} if extra else None,
        "gpu": torch.cuda.get_device_name(0),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
