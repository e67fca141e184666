"""Lossless training fixture for the IVFADC quantizers (Section 2, "The
quantizers" and "Product quantizer": q1 by k-means, then one 256-centroid
k-means per contiguous sub-vector of the residuals y - q1(y)).

The training set is built so that the right answer is known by
construction:

* two coarse centres c_0 = -100 * 1 and c_1 = +100 * 1 in d = 8;
* per sub-space m (M = 4, sub-vectors of 2 components) a set of 256 distinct
  codewords, the 16 x 16 grid of odd integers {-15, ..., 15}^2 scaled by
  (m + 1) -- symmetric under negation, so the codewords sum to zero, and
  different in every sub-space;
* 512 training rows: row L * 256 + i = c_L + concat_m cw_m[perm_m(i)] for
  fixed permutations perm_m, so each cluster holds every codeword of every
  sub-space exactly once.

Any initial coarse centroids with one row from each cluster give the exact
partition at the first assignment (the clusters are 200 apart per
coordinate, their spread at most 120), and the mean of a cluster is exactly
c_L (the residuals sum to zero; every sum is an integer, exact in FP64 and
FP32).  The residuals to the final centroids are then exactly the codewords,
so a sub-space's k-means started from 256 rows whose residual sub-vectors
are its 256 distinct codewords assigns every residual to the centroid equal
to it and never moves: codebook m, entry j = the residual sub-vector m of
init row j.  pq_init_rows[m] takes the rows of cluster m % 2 in an order
rotated by 37 m, so each sub-space's init rows differ.

Plausible mistakes change the result: residuals taken to the initial coarse
centroids (rows, not c_L) shift every codeword; a sub-vector slice off by a
block takes another sub-space's (differently scaled) codewords; the init rows
of another sub-space give another order.
"""
import numpy as np

D, NLIST, M, DS, NT = 8, 2, 4, 2, 512


def codewords(m):
    g = np.arange(-15, 16, 2, dtype=np.float64)          # 16 odd integers
    a, b = np.meshgrid(g, g, indexing="ij")
    return np.stack([a.ravel(), b.ravel()], axis=1) * (m + 1)   # [256, 2]


def build():
    centres = np.stack([np.full(D, -100.0), np.full(D, 100.0)])
    perms = [np.random.default_rng(1000 + m).permutation(256) for m in range(M)]
    rows = []
    for L in range(NLIST):
        for i in range(256):
            parts = [codewords(m)[perms[m][i]] for m in range(M)]
            rows.append(centres[L] + np.concatenate(parts))
    xt = np.array(rows, np.float32)
    coarse_init = np.array([5, 256 + 77], np.int64)   # one row of each cluster
    pq_init = np.stack([(m % 2) * 256 + (np.arange(256) + 37 * m) % 256 for m in range(M)])
    # expected quantizers, by construction
    exp_coarse = centres.astype(np.float32)
    exp_books = np.empty((M, 256, DS), np.float32)
    for m in range(M):
        for j in range(256):
            r = pq_init[m, j]
            L = r // 256
            exp_books[m, j] = (xt[r].astype(np.float64) - centres[L])[m * DS:(m + 1) * DS]
    return {"xt": xt, "coarse_init": coarse_init, "pq_init": pq_init.astype(np.int64),
            "coarse": exp_coarse, "books": exp_books}
