"""Seeded synthetic inputs shaped like the paper's workloads (Sec. 5: SIFT1M,
GIST1M; plus a Deep-shaped large set).  The datasets themselves are not
available; these generators stand in for their shapes and value ranges only.

This module holds no arithmetic of the method: it draws Gaussian-mixture
points and nothing else.  Both the oracle tests and the GPU path take their
inputs from here.

Every generator draws in fixed chunks of rows from one numpy PCG64 stream, so
the output depends only on (config, seed), never on memory limits.
"""
import numpy as np

CHUNK = 1 << 16

# name -> build parameters.  k / n_trees / leaf_max / precision describe the
# run configured on that data; `data` names the generator below.
CONFIGS = {
    # small plain-method case: 50 isotropic clusters, one tree
    "c1": dict(n=10_000, D=32, k=10, n_trees=1, leaf_max=50, precision="fp32",
               data="gmm_uniform", K=50, lo=-10.0, hi=10.0, sigma=1.0, seed=1),
    # SIFT-shaped: integers 0..255 stored as FP32
    "c2": dict(n=1_000_000, D=128, k=20, n_trees=8, leaf_max=100, precision="fp32",
               data="gmm_sift", K=256, lo=0.0, hi=80.0, sigma=16.0, seed=2),
    "c3": dict(n=1_000_000, D=128, k=20, n_trees=8, leaf_max=100, precision="bf16",
               data="gmm_sift", K=256, lo=0.0, hi=80.0, sigma=16.0, seed=2),
    # GIST-shaped: unit-norm rows, D=960
    "c4": dict(n=1_000_000, D=960, k=20, n_trees=4, leaf_max=200, precision="fp16",
               data="gmm_unit", K=512, sigma=0.5, seed=3),
    # Deep-shaped: unit-norm rows, D=96, 10M points
    "c5": dict(n=10_000_000, D=96, k=32, n_trees=8, leaf_max=500, precision="fp8",
               data="gmm_unit", K=4096, sigma=0.35, seed=4),
}


def gmm_uniform(n, D, K, lo, hi, sigma, seed):
    """K centres ~ U[lo, hi]^D; x = centre + sigma * N(0, I), FP32."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.uniform(lo, hi, size=(K, D)).astype(np.float32)
    out = np.empty((n, D), np.float32)
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        lab = rng.integers(0, K, size=e - s)
        z = rng.standard_normal(size=(e - s, D), dtype=np.float32)
        out[s:e] = centres[lab] + np.float32(sigma) * z
    return out


def gmm_sift(n, D, K, lo, hi, sigma, seed):
    """SIFT-like: as gmm_uniform, then clipped to [0, 255] and rounded to
    integers (half to even); stored as FP32 (exact)."""
    x = gmm_uniform(n, D, K, lo, hi, sigma, seed)
    np.clip(x, 0.0, 255.0, out=x)
    np.rint(x, out=x)
    return x


def gmm_unit(n, D, K, sigma, seed):
    """K centres ~ N(0, I_D); x = centre + sigma * N(0, I), each row scaled to
    unit L2 norm (computed in FP64, stored FP32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    centres = rng.standard_normal(size=(K, D))
    out = np.empty((n, D), np.float32)
    for s in range(0, n, CHUNK):
        e = min(n, s + CHUNK)
        lab = rng.integers(0, K, size=e - s)
        z = rng.standard_normal(size=(e - s, D))
        x = centres[lab] + sigma * z
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        out[s:e] = x
    return out


def make(name, n=None):
    """Data of config `name`; `n` overrides the row count (same generator and
    seed, so a smaller n gives a different draw, not a prefix)."""
    c = dict(CONFIGS[name])
    n = c["n"] if n is None else int(n)
    kind = c["data"]
    if kind == "gmm_uniform":
        return gmm_uniform(n, c["D"], c["K"], c["lo"], c["hi"], c["sigma"], c["seed"])
    if kind == "gmm_sift":
        return gmm_sift(n, c["D"], c["K"], c["lo"], c["hi"], c["sigma"], c["seed"])
    if kind == "gmm_unit":
        return gmm_unit(n, c["D"], c["K"], c["sigma"], c["seed"])
    raise ValueError(kind)


def queries(name, nq, seed=77):
    """nq query points from the mixture of config `name`: the same centres
    (the generator's first draw from the config seed), labels and noise from
    their own stream `seed`."""
    c = CONFIGS[name]
    kind, D, K = c["data"], c["D"], c["K"]
    rc = np.random.Generator(np.random.PCG64(c["seed"]))
    rng = np.random.Generator(np.random.PCG64(seed))
    if kind in ("gmm_uniform", "gmm_sift"):
        centres = rc.uniform(c["lo"], c["hi"], size=(K, D)).astype(np.float32)
        lab = rng.integers(0, K, size=nq)
        z = rng.standard_normal(size=(nq, D), dtype=np.float32)
        x = centres[lab] + np.float32(c["sigma"]) * z
        if kind == "gmm_sift":
            np.clip(x, 0.0, 255.0, out=x)
            np.rint(x, out=x)
        return x.astype(np.float32)
    if kind == "gmm_unit":
        centres = rc.standard_normal(size=(K, D))
        lab = rng.integers(0, K, size=nq)
        x = centres[lab] + c["sigma"] * rng.standard_normal(size=(nq, D))
        x /= np.linalg.norm(x, axis=1, keepdims=True)
        return x.astype(np.float32)
    raise ValueError(kind)


def seeds(n, nq, ns, seed=78):
    """Random starting points for the search: nq x ns ids in [0, n)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, n, size=(nq, ns)).astype(np.int32)


def sample_rows(n, q, seed=99):
    """q distinct row indices (ascending) for recall / sampled parity."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q = min(q, n)
    return np.sort(rng.choice(n, size=q, replace=False)).astype(np.int64)


def random_points(n, D, seed, kind="normal"):
    """Small generic test inputs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if kind == "normal":
        return rng.standard_normal(size=(n, D)).astype(np.float32)
    if kind == "int":
        return rng.integers(0, 256, size=(n, D)).astype(np.float32)
    if kind == "small_int":
        return rng.integers(0, 4, size=(n, D)).astype(np.float32)
    raise ValueError(kind)


def rvq_sample(n, m, K1, K2, seed=91):
    """Training sample of the RVQ vocabularies: m distinct row ids of [0, n)
    in increasing order, and the starting words of each stage as K1 and K2
    distinct positions in that sample."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = min(m, n)
    train = np.sort(rng.choice(n, size=m, replace=False)).astype(np.int32)
    init1 = rng.choice(m, size=K1, replace=False).astype(np.int32)
    init2 = rng.choice(m, size=K2, replace=False).astype(np.int32)
    return train, init1, init2
