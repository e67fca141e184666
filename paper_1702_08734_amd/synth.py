"""Seeded synthetic inputs.

This module only draws random numbers; it holds none of the search method's
arithmetic.  Both the GPU path's tests/benchmarks and the CPU oracle consume
the arrays it returns, so the two sides see identical inputs.

Recipe (numpy PCG64, float64 draws cast once to float32 with round to
nearest even):

* ``gaussian(n, d, seed)``: i.i.d. N(0, 1) rows.
* ``Mixture(ncomp, d, seed)``: ``ncomp`` components with uniform weights,
  centres mu_c ~ N(0, 4 I) (standard deviation 2) and per-component scale
  sigma_c ~ U[0.5, 1.5]; a sample is mu_c + sigma_c * N(0, I), optionally
  normalised to unit length in float64 before the cast.  The mixture
  parameters are drawn once per seed and shared by database, query and
  training draws, which use their own seeds.
* ``uniform_rows(nrows, length, seed)``: U[0, 1) float32 rows (k-selection
  benchmark input).
* Large draws are split into chunks of max(1, 2^22 // columns) rows, chunk i
  seeded by ``SeedSequence(seed).spawn`` child i, so any chunk can be
  regenerated alone and chunks are drawn on several threads.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CHUNK_ELEMS = 1 << 22


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def _chunked(n: int, d: int, seed: int, fill) -> np.ndarray:
    out = np.empty((n, d), np.float32)
    rows = max(1, CHUNK_ELEMS // max(d, 1))
    nchunks = (n + rows - 1) // rows
    children = np.random.SeedSequence(seed).spawn(max(nchunks, 1))

    def work(i):
        lo = i * rows
        hi = min(n, lo + rows)
        rng = np.random.Generator(np.random.PCG64(children[i]))
        fill(rng, out[lo:hi])

    if nchunks <= 1:
        for i in range(nchunks):
            work(i)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, range(nchunks)))
    return out


def gaussian(n: int, d: int, seed: int) -> np.ndarray:
    """n x d float32 rows drawn i.i.d. N(0, 1)."""
    def fill(rng, dst):
        dst[...] = rng.standard_normal(dst.shape, dtype=np.float64)
    return _chunked(n, d, seed, fill)


def uniform_rows(nrows: int, length: int, seed: int) -> np.ndarray:
    """nrows x length float32 values drawn U[0, 1)."""
    def fill(rng, dst):
        dst[...] = rng.random(dst.shape, dtype=np.float64)
    return _chunked(nrows, length, seed, fill)


class Mixture:
    """Gaussian mixture with uniform weights, centres N(0, 4I), scales U[0.5, 1.5]
    (or, with log_scales=(lo, hi), scales log-uniform in [lo, hi]: components
    of very different densities)."""

    def __init__(self, ncomp: int, d: int, seed: int, log_scales=None):
        rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
        self.ncomp = ncomp
        self.d = d
        self.mu = 2.0 * rng.standard_normal((ncomp, d))
        if log_scales is None:
            self.sigma = rng.uniform(0.5, 1.5, size=ncomp)
        else:
            lo, hi = log_scales
            self.sigma = np.exp(rng.uniform(np.log(lo), np.log(hi), size=ncomp))

    def sample(self, n: int, seed: int, unit_norm: bool = False) -> np.ndarray:
        mu, sigma, ncomp = self.mu, self.sigma, self.ncomp

        def fill(rng, dst):
            comp = rng.integers(0, ncomp, size=dst.shape[0])
            v = mu[comp] + sigma[comp, None] * rng.standard_normal(dst.shape, dtype=np.float64)
            if unit_norm:
                v /= np.linalg.norm(v, axis=1, keepdims=True)
            dst[...] = v
        return _chunked(n, self.d, seed, fill)


def choose_rows(n: int, count: int, seed: int) -> np.ndarray:
    """The first `count` entries of a seeded permutation of range(n): used for
    Forgy k-means initialisation and for drawing training samples without
    replacement."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence(seed)))
    if count > n:
        raise ValueError("cannot choose more rows than exist")
    return rng.permutation(n)[:count].astype(np.int64)


def pq_init_rows(n: int, M: int, seed) -> np.ndarray:
    """[M, 256] Forgy rows for the M sub-quantizers: sub-quantizer m draws
    with seed + m (integer seed) or entropy (*seed, m) (tuple seed)."""
    if isinstance(seed, tuple):
        return np.stack([choose_rows(n, 256, (*seed, m)) for m in range(M)])
    return np.stack([choose_rows(n, 256, seed + m) for m in range(M)])


# ---------------------------------------------------------------- workloads
# Each workload draws its arrays from SeedSequence entropy (base, offset).
def exact_small():
    """50,000 x 64 N(0, 1) database, 500 queries of the same law, k = 10."""
    return {"xb": gaussian(50_000, 64, (101, 0)), "xq": gaussian(500, 64, (101, 1)), "k": 10}


def exact_large(nb: int = 1_000_000, nq: int = 10_000):
    """1,000-component mixture in d = 128: database and queries."""
    mix = Mixture(1000, 128, (102, 99))
    return {"xb": mix.sample(nb, (102, 0)), "xq": mix.sample(nq, (102, 1)),
            "ks": (1, 32, 256, 1024)}


def kselect_rows(nrows: int = 10_000, length: int = 128_000):
    """Row-wise k-selection input: U[0, 1) float32 rows."""
    return uniform_rows(nrows, length, (106, 0))


def ivfpq_workload(nb: int = 10_000_000, nq: int = 10_000, nt: int = 500_000):
    """IVFADC workload: database and queries from a 1,000-component mixture in
    d = 128, a training sample of nt database rows drawn without replacement,
    Forgy rows for 4,096 coarse centroids and 16 sub-quantizers."""
    mix = Mixture(1000, 128, (103, 99))
    xb = mix.sample(nb, (103, 0))
    xq = mix.sample(nq, (103, 1))
    sample = choose_rows(nb, nt, (103, 2))
    return {"xb": xb, "xq": xq, "sample": sample, "nlist": 4096, "M": 16,
            "coarse_init": choose_rows(nt, 4096, (103, 3)),
            "pq_init": pq_init_rows(nt, 16, (103, 4)), "k": 100,
            "nprobes": (1, 8, 16, 32, 64, 128), "rerank": (256, 1024),
            "learn_rerank": 256, "learn_cap": 32, "learn_fixed_nprobes": tuple(range(1, 13)),
            "learn_train": 200_000, "learn_epochs": 30, "serve_requests": 2000,
            "serve_load": (0.5, 0.8), "base": 103, "mix": (1000, 128, (103, 99)),
            "graph_settings": ((4, 0), (16, 0), (4, 64), (8, 128), (16, 256))}


def ivfpq_large_workload(nb: int = 50_000_000, nq: int = 10_000, nt: int = 500_000):
    """Learned-probe and serving workload: 50,000,000 x 128 rows of a
    1,000-component mixture, 16,384 coarse centroids, PQ 16 x 8 bit."""
    mix = Mixture(1000, 128, (105, 99))
    xb = mix.sample(nb, (105, 0))
    xq = mix.sample(nq, (105, 1))
    sample = choose_rows(nb, nt, (105, 2))
    return {"xb": xb, "xq": xq, "sample": sample, "nlist": 16384, "M": 16,
            "coarse_init": choose_rows(nt, 16384, (105, 3)),
            "pq_init": pq_init_rows(nt, 16, (105, 4)), "k": 10,
            "learn_rerank": 1024, "learn_cap": 64, "learn_fixed_nprobes": tuple(range(1, 25)),
            "learn_train": 200_000, "learn_epochs": 30, "serve_requests": 2000,
            "serve_load": (0.5, 0.8), "base": 105, "mix": (1000, 128, (105, 99))}


def lowp_workload(nb: int = 20_000_000, nq: int = 10_000):
    """Low-precision brute-force workload: unit-norm rows of a 2,000-component
    mixture in d = 96 (database and queries), k = 100, re-rank depth 4k."""
    mix = Mixture(2000, 96, (104, 99))
    return {"xb": mix.sample(nb, (104, 0), unit_norm=True),
            "xq": mix.sample(nq, (104, 1), unit_norm=True), "k": 100, "R": 400,
            "metrics": ("ip", "l2")}


def mlp_init(din: int, hidden: int, seed) -> np.ndarray:
    """He-uniform initial parameters of the probe-count network, flat float32
    in the order W1 [hidden, din], b1, W2 [hidden, hidden], b2, w3, b3:
    weights U(-sqrt(6 / fan_in), +sqrt(6 / fan_in)), biases zero."""
    rng = np.random.default_rng(np.random.SeedSequence(seed if isinstance(seed, tuple) else (seed,)))
    w1 = rng.uniform(-1, 1, (hidden, din)) * np.sqrt(6.0 / din)
    w2 = rng.uniform(-1, 1, (hidden, hidden)) * np.sqrt(6.0 / hidden)
    w3 = rng.uniform(-1, 1, hidden) * np.sqrt(6.0 / hidden)
    z = np.zeros(hidden)
    return np.concatenate([w1.ravel(), z, w2.ravel(), z, w3, [0.0]]).astype(np.float32)


def permutation(n: int, seed) -> np.ndarray:
    """Seeded permutation of 0 .. n-1 (int64), e.g. the row order of a
    training epoch."""
    rng = np.random.default_rng(np.random.SeedSequence(seed if isinstance(seed, tuple) else (seed,)))
    return rng.permutation(n).astype(np.int64)
