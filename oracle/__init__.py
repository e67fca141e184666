"""Reference oracle (CPU, float64) for the k-NN / IVFADC hot path.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` are the only users.  The GPU product path
never imports this package, and this package imports nothing from it.

The arithmetic lives in ``oracle.c`` (plain loops, double precision, full
sorts); this module only marshals numpy arrays to it and adds the plain host
logic that strings the steps together (k-means iterations, PQ training on
residuals, building inverted lists in insertion order).  Each function names
the passage of "Billion-scale similarity search with GPUs" it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

METRIC_L2 = 0
METRIC_IP = 1

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc (-O2, OpenMP over queries)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB)
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = None
    lib.oracle_get_threads.argtypes = []
    lib.oracle_get_threads.restype = ctypes.c_int
    lib.oracle_knn.argtypes = [_f32p, _i64, _f32p, _i64, _i32, _i32, _i32, ctypes.c_void_p,
                               _f64p, _i64p]
    lib.oracle_kselect.argtypes = [_f32p, _i64, _i64, _i32, _i32, _f64p, _i64p]
    lib.oracle_kmeans_assign.argtypes = [_f64p, _i64, _i32, _f32p, _i32, _i64p, _f64p]
    lib.oracle_kmeans_update.argtypes = [_f64p, _i64, _i32, _i64p, _i32, _f32p, _i64p]
    lib.oracle_pq_encode.argtypes = [_f64p, _i64, _i32, _i32, _f32p, _u8p]
    lib.oracle_ivfpq_search.argtypes = [_f32p, _i64, _i32, _f32p, _i32, _i32, _f32p, _i64p,
                                        _u8p, _i64p, _i32, _i32, ctypes.c_void_p, ctypes.c_void_p,
                                        _f64p, _i64p]
    for fn in ("oracle_knn", "oracle_kselect", "oracle_kmeans_assign", "oracle_kmeans_update",
               "oracle_pq_encode", "oracle_ivfpq_search"):
        getattr(lib, fn).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with status {rc}")


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# Exact search and k-selection (Section 2, Eq. 1; Section 4 contract)
# --------------------------------------------------------------------------
def _opt_i64(a):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, np.int64)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def knn(xq, xb, k: int, metric: int = METRIC_L2, exclude=None):
    """Exact k-NN by full sort in float64 (Section 2, Eq. 1).

    Returns (D float64 [nq, k], I int64 [nq, k]); squared L2 ascending or
    inner product descending, ties to the lower index, padded (+-inf, -1).
    exclude [nq] (optional): a database row left out of each query's
    candidates (the node itself when building a k-NN graph, Section 6.5).
    """
    xq = _f32(xq)
    xb = _f32(xb)
    nq, d = xq.shape
    nb = xb.shape[0]
    if nb:
        assert xb.shape[1] == d
    D = np.empty((nq, k), np.float64)
    I = np.empty((nq, k), np.int64)
    ex, exp = _opt_i64(exclude)
    assert ex is None or ex.shape == (nq,)
    _check(_load().oracle_knn(xq, nq, xb if nb else np.zeros((1, d), np.float32), nb, d, k,
                              metric, exp, D, I), "knn")
    return D, I


def kselect(a, k: int, largest: bool = False):
    """Row-wise k-selection of a float32 matrix by full sort (Section 2)."""
    a = _f32(a)
    nrows, length = a.shape
    vals = np.empty((nrows, k), np.float64)
    idx = np.empty((nrows, k), np.int64)
    _check(_load().oracle_kselect(a if a.size else np.zeros((1, 1), np.float32), nrows, length,
                                  k, int(bool(largest)), vals, idx), "kselect")
    return vals, idx


def pair_distance(xq, xb, qi, bi, metric: int = METRIC_L2):
    """float64 distance of query qi to database row bi (direct form)."""
    x = np.asarray(xq, np.float64)[qi]
    y = np.asarray(xb, np.float64)[bi]
    if metric == METRIC_L2:
        return ((x - y) ** 2).sum(-1)
    return (x * y).sum(-1)


# --------------------------------------------------------------------------
# k-means (Section 2 "The quantizers"; Section 6.2 k = 1 assignment)
# --------------------------------------------------------------------------
def kmeans_assign(x, c):
    """Nearest centroid per point (float64, ties to lower index)."""
    x = _f64(x)
    c = _f32(c)
    n, d = x.shape
    a = np.empty(n, np.int64)
    dist = np.empty(n, np.float64)
    _check(_load().oracle_kmeans_assign(x, n, d, c, c.shape[0], a, dist), "kmeans_assign")
    return a, dist


def kmeans_update(x, assign, c):
    """One centroid update (float64 sums, float32 result, empty-cluster split)."""
    x = _f64(x)
    c = _f32(c).copy()
    n, d = x.shape
    counts = np.empty(c.shape[0], np.int64)
    _check(_load().oracle_kmeans_update(x, n, d, np.ascontiguousarray(assign, np.int64),
                                        c.shape[0], c, counts), "kmeans_update")
    return c, counts


def kmeans(x, init_rows, niter: int):
    """Lloyd's k-means: Forgy initialisation from the given rows, then `niter`
    rounds of (assign, update).  Returns (centroids float32, objective per
    iteration measured at its assignment step)."""
    x = _f64(x)
    c = np.ascontiguousarray(x[np.asarray(init_rows, np.int64)], np.float32)
    objs = []
    for _ in range(niter):
        a, dist = kmeans_assign(x, c)
        objs.append(float(dist.sum()))
        c, _ = kmeans_update(x, a, c)
    return c, objs


# --------------------------------------------------------------------------
# Product quantizer and IVFADC (Section 2 Eq. 3-6; Section 5.2-5.3)
# --------------------------------------------------------------------------
def pq_encode(r, codebooks):
    """PQ codes of (residual) vectors r, codebooks [M, 256, d/M]."""
    r = _f64(r)
    cb = _f32(codebooks)
    n, d = r.shape
    M = cb.shape[0]
    codes = np.empty((n, M), np.uint8)
    _check(_load().oracle_pq_encode(r, n, d, M, cb, codes), "pq_encode")
    return codes


def pq_decode(codes, codebooks):
    """Reconstruct q2 values (float64) from codes: concatenation of the
    selected sub-quantizer centroids."""
    cb = np.asarray(codebooks, np.float64)
    M = cb.shape[0]
    parts = [cb[m][np.asarray(codes)[:, m]] for m in range(M)]
    return np.concatenate(parts, axis=1)


def rotate_rows(x, rot):
    """Linear pre-processing of the input vectors (an OPQ rotation, Sections
    1 and 6.4): out[i][j] = sum_t rot[j][t] x[i][t], float64."""
    return _f64(x) @ _f64(rot).T


def ivfpq_train(xt, nlist: int, M: int, niter: int, coarse_init_rows, pq_init_rows):
    """Train q1 (k-means, nlist centroids) then q2 (M independent 256-centroid
    k-means on contiguous residual sub-vectors), Section 2 "The quantizers"
    and "Product quantizer".  Residuals are taken to the final coarse
    centroids.  pq_init_rows is [M, 256]."""
    xt = _f64(xt)
    n, d = xt.shape
    ds = d // M
    coarse, _ = kmeans(xt, coarse_init_rows, niter)
    a, _ = kmeans_assign(xt, coarse)
    res = xt - coarse[a].astype(np.float64)
    books = np.empty((M, 256, ds), np.float32)
    for m in range(M):
        sub = np.ascontiguousarray(res[:, m * ds:(m + 1) * ds])
        books[m], _ = kmeans(sub, np.asarray(pq_init_rows)[m], niter)
    return coarse, books


def ivf_encode(xb, coarse, codebooks):
    """Coarse list (q1) and PQ code of the residual (q2) of each vector,
    Section 2 Eq. 3."""
    xb = _f64(xb)
    lists, _ = kmeans_assign(xb, coarse)
    res = xb - np.asarray(coarse, np.float64)[lists]
    return lists, pq_encode(res, codebooks)


def build_lists(list_of, codes, nlist: int, id0: int = 0, prev=None):
    """Inverted lists in CSR form, entries in insertion order within each list
    (ids are sequential from id0).  prev = (offsets, codes, ids) of an
    existing index, whose entries stay in front of the new ones."""
    list_of = np.asarray(list_of, np.int64)
    codes = np.asarray(codes, np.uint8)
    ids = id0 + np.arange(len(list_of), dtype=np.int64)
    if prev is not None:
        po, pc, pi = prev
        prev_list = np.repeat(np.arange(nlist), np.diff(po))
        list_of = np.concatenate([prev_list, list_of])
        codes = np.concatenate([pc, codes])
        ids = np.concatenate([pi, ids])
    order = np.argsort(list_of, kind="stable")
    counts = np.bincount(list_of, minlength=nlist)
    offsets = np.zeros(nlist + 1, np.int64)
    offsets[1:] = np.cumsum(counts)
    return offsets, np.ascontiguousarray(codes[order]), np.ascontiguousarray(ids[order])


def ivfpq_search(xq, coarse, codebooks, offsets, codes, ids, k: int, nprobe: int,
                 nprobe_per_query=None, exclude=None):
    """IVFADC search, Algorithm 4 with Eq. 5, 6 and 10 (float64, full sort).

    exclude [nq] (optional): an id whose entries are skipped for each query.
    """
    xq = _f32(xq)
    coarse = _f32(coarse)
    cb = _f32(codebooks)
    nq, d = xq.shape
    M = cb.shape[0]
    D = np.empty((nq, k), np.float64)
    I = np.empty((nq, k), np.int64)
    npq = None
    if nprobe_per_query is not None:
        npq = np.ascontiguousarray(nprobe_per_query, np.int32)
    codes = np.ascontiguousarray(codes, np.uint8)
    if codes.size == 0:
        codes = np.zeros((1, M), np.uint8)
    ids_a = np.ascontiguousarray(ids, np.int64)
    if ids_a.size == 0:
        ids_a = np.zeros(1, np.int64)
    ex, exp = _opt_i64(exclude)
    assert ex is None or ex.shape == (nq,)
    _check(_load().oracle_ivfpq_search(
        xq, nq, d, coarse, coarse.shape[0], M, cb, np.ascontiguousarray(offsets, np.int64),
        codes, ids_a, k, nprobe,
        npq.ctypes.data_as(ctypes.c_void_p) if npq is not None else None, exp, D, I),
        "ivfpq_search")
    return D, I


def ivfpq_search_rerank(xq, coarse, codebooks, offsets, codes, ids, xb, k: int, nprobe: int,
                        R: int, exclude=None):
    """IVFADC short list re-ranked exactly (an extension of Algorithm 4).

    The R best entries by ADC distance (``ivfpq_search`` with k = R) are
    re-scored by their exact squared L2 distance to the database row of their
    id (float64 direct form) and the first k by (distance, id) are returned,
    padded with (+inf, -1) where fewer than k entries were scanned.
    exclude [nq] (optional): an id left out of each query's short list.
    """
    xq = _f32(xq)
    xb = _f32(xb)
    _, Ia = ivfpq_search(xq, coarse, codebooks, offsets, codes, ids, R, nprobe,
                         exclude=exclude)
    nq = xq.shape[0]
    D = np.full((nq, k), np.inf)
    I = np.full((nq, k), -1, np.int64)
    for j in range(nq):
        cand = Ia[j][Ia[j] >= 0]
        diff = xb[cand].astype(np.float64) - xq[j].astype(np.float64)
        dist = (diff * diff).sum(1)
        order = np.lexsort((cand, dist))[:k]
        D[j, :len(order)] = dist[order]
        I[j, :len(order)] = cand[order]
    return D, I
