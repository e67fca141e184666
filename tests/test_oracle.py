"""Pins of the CPU oracle against facts other than itself.

Each test checks the oracle against hand-worked values from the paper's
definitions (tests/golden), against independent library routines on small
inputs (scipy's cdist and numpy's stable sorts), against closed forms and
special cases, or against invariants the definitions imply.
"""
import json
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle

L2, IP = oracle.METRIC_L2, oracle.METRIC_IP


def _load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


def _num(v):
    return float("inf") if v == "inf" else float(v)


def _ref_topk(dist, k, largest):
    """Independent top-k: numpy lexsort on (index, value) per row."""
    nq, nb = dist.shape
    D = np.full((nq, k), -np.inf if largest else np.inf)
    I = np.full((nq, k), -1, np.int64)
    for j in range(nq):
        keyv = -dist[j] if largest else dist[j]
        order = np.lexsort((np.arange(nb), keyv))[:k]
        D[j, :len(order)] = dist[j, order]
        I[j, :len(order)] = order
    return D, I


# ---------------------------------------------------------------- exact k-NN
def test_knn_handworked(golden_dir):
    g = _load(golden_dir, "knn_handworked.json")
    xb = np.array(g["xb"], np.float32)
    for c in g["cases"]:
        D, I = oracle.knn(np.array([c["x"]], np.float32), xb, c["k"],
                          L2 if c["metric"] == "l2" else IP)
        assert I[0].tolist() == c["I"]
        assert D[0].tolist() == [_num(v) for v in c["D"]]


@pytest.mark.parametrize("d", [1, 3, 8, 17])
@pytest.mark.parametrize("nb", [0, 1, 5, 37, 200])
@pytest.mark.parametrize("k", [1, 4, 64])
@pytest.mark.parametrize("metric", [L2, IP])
def test_knn_vs_library_small_integers(d, nb, k, metric):
    # small integers: every distance is exact in float64 and ties are common,
    # so the index tie-break is exercised.
    rng = np.random.default_rng(1000 * d + 10 * nb + k + metric)
    xq = rng.integers(-3, 4, size=(7, d)).astype(np.float32)
    xb = rng.integers(-3, 4, size=(nb, d)).astype(np.float32)
    D, I = oracle.knn(xq, xb, k, metric)
    if nb:
        dist = cdist(xq.astype(np.float64), xb.astype(np.float64), "sqeuclidean") \
            if metric == L2 else xq.astype(np.float64) @ xb.astype(np.float64).T
    else:
        dist = np.zeros((7, 0))
    Dr, Ir = _ref_topk(dist, k, metric == IP)
    np.testing.assert_array_equal(I, Ir)
    np.testing.assert_array_equal(D, Dr)


def test_knn_invariants_continuous():
    rng = np.random.default_rng(7)
    xq = rng.standard_normal((20, 24)).astype(np.float32)
    xb = rng.standard_normal((500, 24)).astype(np.float32)
    for metric in (L2, IP):
        D, I = oracle.knn(xq, xb, 50, metric)
        for j in range(20):
            assert len(set(I[j].tolist())) == 50
            diffs = np.diff(D[j])
            assert np.all(diffs >= 0) if metric == L2 else np.all(diffs <= 0)
            again = oracle.pair_distance(xq, xb, j, I[j], metric)
            np.testing.assert_allclose(D[j], again, rtol=1e-13, atol=1e-12)
            # nothing left out beats the k-th value
            full = oracle.pair_distance(xq, xb, j, np.arange(500), metric)
            rest = np.setdiff1d(np.arange(500), I[j])
            if metric == L2:
                assert full[rest].min() >= D[j, -1]
            else:
                assert full[rest].max() <= D[j, -1]


def test_knn_special_cases():
    rng = np.random.default_rng(3)
    xq = rng.standard_normal((5, 6)).astype(np.float32)
    xb = rng.standard_normal((40, 6)).astype(np.float32)
    # k = nb is a full sort
    D, I = oracle.knn(xq, xb, 40)
    dist = cdist(xq.astype(np.float64), xb.astype(np.float64), "sqeuclidean")
    np.testing.assert_array_equal(I, np.argsort(dist, axis=1, kind="stable"))
    # k = 1 is the argmin
    D1, I1 = oracle.knn(xq, xb, 1)
    np.testing.assert_array_equal(I1[:, 0], dist.argmin(1))
    # empty query batch
    D0, I0 = oracle.knn(np.zeros((0, 6), np.float32), xb, 3)
    assert D0.shape == (0, 3) and I0.shape == (0, 3)


def test_knn_uses_direct_form():
    # Far from the origin the norm decomposition of Eq. 2 loses every digit
    # in double; the direct form keeps them.
    xb = np.array([[1e8, 0.0], [1e8, 1.0]], np.float32)
    xq = np.array([[1e8, 0.25]], np.float32)
    D, I = oracle.knn(xq, xb, 2)
    assert I[0].tolist() == [0, 1]
    assert D[0].tolist() == [0.0625, 0.5625]


# ---------------------------------------------------------------- k-selection
@pytest.mark.parametrize("length", [0, 1, 63, 64, 65, 500])
@pytest.mark.parametrize("k", [1, 10, 64, 100])
@pytest.mark.parametrize("largest", [False, True])
def test_kselect_vs_stable_argsort(length, k, largest):
    rng = np.random.default_rng(length * 7 + k)
    a = rng.integers(0, 20, size=(6, length)).astype(np.float32)  # many ties
    vals, idx = oracle.kselect(a, k, largest)
    for r in range(6):
        order = np.argsort(-a[r] if largest else a[r], kind="stable")[:k]
        n = len(order)
        assert idx[r, :n].tolist() == order.tolist()
        assert vals[r, :n].tolist() == a[r, order].astype(np.float64).tolist()
        assert np.all(idx[r, n:] == -1)
        assert np.all(np.isinf(vals[r, n:]))


def test_kselect_handworked():
    a = np.array([[5.0, 1.0, 3.0, 1.0, -2.0]], np.float32)
    v, i = oracle.kselect(a, 3)
    assert v[0].tolist() == [-2.0, 1.0, 1.0] and i[0].tolist() == [4, 1, 3]
    v, i = oracle.kselect(a, 2, largest=True)
    assert v[0].tolist() == [5.0, 3.0] and i[0].tolist() == [0, 2]


# ---------------------------------------------------------------- k-means
def test_kmeans_1d_handworked(golden_dir):
    g = _load(golden_dir, "kmeans_1d.json")
    x = np.array(g["points"], np.float64)
    c = np.array(g["init"], np.float32)
    for it in g["iterations"]:
        a, dist = oracle.kmeans_assign(x, c)
        assert a.tolist() == it["assign"]
        assert dist.sum() == pytest.approx(it["objective"], rel=1e-6)
        c, _ = oracle.kmeans_update(x, a, c)
        np.testing.assert_allclose(c, np.array(it["centroids"]), rtol=1e-7)


def test_kmeans_empty_cluster_split(golden_dir):
    g = _load(golden_dir, "kmeans_empty_split.json")
    c, counts = oracle.kmeans_update(np.array(g["points"]), np.array(g["assign"]),
                                     np.array(g["init"], np.float32))
    assert c.tolist() == g["centroids"]
    assert counts.tolist() == g["counts"]


def test_kmeans_assign_vs_library():
    rng = np.random.default_rng(11)
    x = rng.integers(-4, 5, size=(300, 5)).astype(np.float64)  # exact ties
    c = rng.integers(-4, 5, size=(17, 5)).astype(np.float32)
    a, dist = oracle.kmeans_assign(x, c)
    ref = cdist(x, c.astype(np.float64), "sqeuclidean")
    np.testing.assert_array_equal(a, ref.argmin(1))  # argmin: first = lower index
    np.testing.assert_array_equal(dist, ref.min(1))


def test_kmeans_update_is_mean():
    rng = np.random.default_rng(12)
    x = rng.standard_normal((400, 6))
    a = rng.integers(0, 9, size=400)
    a[:9] = np.arange(9)  # no empty cluster
    c, counts = oracle.kmeans_update(x, a, np.zeros((9, 6), np.float32))
    for j in range(9):
        np.testing.assert_array_equal(c[j], x[a == j].mean(0).astype(np.float32))
    np.testing.assert_array_equal(counts, np.bincount(a, minlength=9))


def test_kmeans_objective_monotone_and_k_eq_n():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((600, 4))
    _, objs = oracle.kmeans(x, np.arange(0, 600, 40), 12)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(objs, objs[1:]))
    # K = n with distinct points: every point is its own centroid -> zero loss
    pts = rng.standard_normal((30, 3))
    c, objs = oracle.kmeans(pts, np.arange(30), 2)
    assert objs[-1] < 1e-10


# ---------------------------------------------------------------- PQ
def test_pq_encode_vs_library_and_roundtrip():
    rng = np.random.default_rng(21)
    M, ds = 4, 3
    books = rng.standard_normal((M, 256, ds)).astype(np.float32)
    r = rng.standard_normal((200, M * ds))
    codes = oracle.pq_encode(r, books)
    for m in range(M):
        ref = cdist(r[:, m * ds:(m + 1) * ds], books[m].astype(np.float64), "sqeuclidean")
        np.testing.assert_array_equal(codes[:, m], ref.argmin(1))
    # encode(decode(c)) = c for distinct codewords
    c0 = rng.integers(0, 256, size=(100, M)).astype(np.uint8)
    np.testing.assert_array_equal(oracle.pq_encode(oracle.pq_decode(c0, books), books), c0)


# ---------------------------------------------------------------- IVFADC
def _handworked_index(g):
    d, M = g["d"], g["M"]
    ds = d // M
    books = np.tile(np.array(g["codebook_defaults"], np.float32), (M, 256, 1)).reshape(M, 256, ds)
    for m, entries in g["codebook_set"].items():
        for j, v in entries.items():
            books[int(m), int(j)] = v
    coarse = np.array(g["coarse"], np.float32)
    return coarse, books


def test_ivfpq_handworked(golden_dir):
    g = _load(golden_dir, "ivfpq_handworked.json")
    coarse, books = _handworked_index(g)
    xb = np.array(g["xb"], np.float32)
    lists, codes = oracle.ivf_encode(xb, coarse, books)
    assert lists.tolist() == g["lists"]
    assert codes.tolist() == g["codes"]
    offs, lc, lid = oracle.build_lists(lists, codes, len(coarse))
    q = np.array([g["query"]], np.float32)
    for c in g["cases"]:
        D, I = oracle.ivfpq_search(q, coarse, books, offs, lc, lid, c["k"], c["nprobe"])
        assert I[0].tolist() == c["I"]
        np.testing.assert_allclose(D[0], [_num(v) for v in c["D"]], rtol=1e-6)
    # Eq. 11 on y0: term1 + term2 - 2 term3
    e = g["eq11_y0"]
    q1 = coarse[0].astype(np.float64)
    q2 = oracle.pq_decode(np.array([g["codes"][0]]), books)[0]
    x = np.array(g["query"], np.float64)
    assert q2 @ q2 + 2 * q1 @ q2 == e["term1"]
    assert (x - q1) @ (x - q1) == e["term2"]
    assert x @ q2 == e["term3"]


def test_ivfpq_rerank_handworked(golden_dir):
    g = _load(golden_dir, "ivfpq_rerank_handworked.json")
    coarse, books = _handworked_index(g)
    xb = np.array(g["xb"], np.float32)
    lists, codes = oracle.ivf_encode(xb, coarse, books)
    assert lists.tolist() == g["lists"]
    assert codes.tolist() == g["codes"]
    offs, lc, lid = oracle.build_lists(lists, codes, len(coarse))
    q = np.array([g["query"]], np.float32)
    for c in g["cases"]:
        D, I = oracle.ivfpq_search_rerank(q, coarse, books, offs, lc, lid, xb, c["k"],
                                          c["nprobe"], c["R"])
        assert I[0].tolist() == c["I"]
        np.testing.assert_allclose(D[0], [_num(v) for v in c["D"]], rtol=1e-6)


def _random_index(seed, nlist=6, M=4, ds=2, nb=300):
    rng = np.random.default_rng(seed)
    d = M * ds
    coarse = (3 * rng.standard_normal((nlist, d))).astype(np.float32)
    books = rng.standard_normal((M, 256, ds)).astype(np.float32)
    xb = (coarse[rng.integers(0, nlist, nb)] + rng.standard_normal((nb, d))).astype(np.float32)
    lists, codes = oracle.ivf_encode(xb, coarse, books)
    offs, lc, lid = oracle.build_lists(lists, codes, nlist)
    xq = (coarse[rng.integers(0, nlist, 9)] + rng.standard_normal((9, d))).astype(np.float32)
    return xq, xb, coarse, books, lists, codes, offs, lc, lid


def test_ivfpq_full_probe_is_exhaustive_adc():
    # tau = |C1| gives ADC (Section 2): distance to every decoded vector.
    xq, xb, coarse, books, lists, codes, offs, lc, lid = _random_index(31)
    k = 25
    D, I = oracle.ivfpq_search(xq, coarse, books, offs, lc, lid, k, len(coarse))
    dec = coarse[lists].astype(np.float64) + oracle.pq_decode(codes, books)
    dist = cdist(xq.astype(np.float64), dec, "sqeuclidean")
    Dr, Ir = _ref_topk(dist, k, False)
    np.testing.assert_allclose(D, Dr, rtol=1e-12)
    np.testing.assert_array_equal(I, Ir)


def test_ivfpq_table_sum_and_three_terms():
    # Eq. 10: per-sub-space tables summed = decoded distance;
    # Eq. 11: term1 + term2 - 2 term3 = the same value.
    xq, xb, coarse, books, lists, codes, offs, lc, lid = _random_index(32)
    M, ds = books.shape[0], books.shape[2]
    D, I = oracle.ivfpq_search(xq, coarse, books, offs, lc, lid, 20, 3)
    b64 = books.astype(np.float64)
    for j in range(len(xq)):
        x = xq[j].astype(np.float64)
        for r in range(20):
            i = I[j, r]
            L = lists[i]
            c = coarse[L].astype(np.float64)
            tables = [((x - c)[m * ds:(m + 1) * ds][None, :] - b64[m]) ** 2 for m in range(M)]
            tsum = sum(tables[m].sum(1)[codes[i, m]] for m in range(M))
            assert D[j, r] == pytest.approx(tsum, rel=1e-12)
            q2 = oracle.pq_decode(codes[i:i + 1], books)[0]
            t1 = q2 @ q2 + 2 * c @ q2
            t2 = (x - c) @ (x - c)
            t3 = x @ q2
            assert D[j, r] == pytest.approx(t1 + t2 - 2 * t3, rel=1e-9, abs=1e-9)


def test_ivfpq_probe_set_and_padding():
    xq, xb, coarse, books, lists, codes, offs, lc, lid = _random_index(33)
    D, I = oracle.ivfpq_search(xq, coarse, books, offs, lc, lid, 400, 1)
    cd = cdist(xq.astype(np.float64), coarse.astype(np.float64), "sqeuclidean")
    for j in range(len(xq)):
        L = int(np.lexsort((np.arange(len(coarse)), cd[j]))[0])
        members = set(np.nonzero(lists == L)[0].tolist())
        got = [v for v in I[j].tolist() if v >= 0]
        assert set(got) == members
        assert np.all(np.isinf(D[j, len(got):])) and np.all(I[j, len(got):] == -1)
    # per-query nprobe overrides the scalar
    D2, I2 = oracle.ivfpq_search(xq, coarse, books, offs, lc, lid, 400, 99,
                                 nprobe_per_query=np.ones(len(xq), np.int32))
    np.testing.assert_array_equal(I2, I)


def test_ivfpq_lossless_equals_exact():
    # database built exactly from codewords: ADC distance = true distance
    rng = np.random.default_rng(41)
    M, ds, nlist = 2, 2, 3
    d = M * ds
    coarse = rng.integers(-20, 20, size=(nlist, d)).astype(np.float32) * 4
    books = rng.integers(-1, 2, size=(M, 256, ds)).astype(np.float32)
    books[:, :9] = np.array([[a, b] for a in (-1, 0, 1) for b in (-1, 0, 1)], np.float32)
    books[:, 9:] = 50.0
    L = rng.integers(0, nlist, 80)
    cw = rng.integers(0, 9, size=(80, M))
    xb = (coarse[L] + np.concatenate([books[m][cw[:, m]] for m in range(M)], 1)).astype(np.float32)
    lists, codes = oracle.ivf_encode(xb, coarse, books)
    np.testing.assert_array_equal(lists, L)
    offs, lc, lid = oracle.build_lists(lists, codes, nlist)
    xq = rng.integers(-80, 80, size=(6, d)).astype(np.float32)
    D, I = oracle.ivfpq_search(xq, coarse, books, offs, lc, lid, 30, nlist)
    De, Ie = oracle.knn(xq, xb, 30)
    np.testing.assert_array_equal(I, Ie)
    np.testing.assert_array_equal(D, De)


def test_ivfpq_rerank_full_list_is_exact_search():
    # every entry probed and short-listed: the re-rank is exact search
    xq, xb, coarse, books, lists, codes, offs, lc, lid = _random_index(34)
    for k in (1, 7, 50):
        D, I = oracle.ivfpq_search_rerank(xq, coarse, books, offs, lc, lid, xb, k,
                                          len(coarse), len(xb))
        De, Ie = oracle.knn(xq, xb, k)
        np.testing.assert_array_equal(I, Ie)
        np.testing.assert_allclose(D, De, rtol=1e-12)


def test_ivfpq_rerank_short_list():
    # results are the exact-distance order of the ADC short list of length R
    xq, xb, coarse, books, lists, codes, offs, lc, lid = _random_index(35)
    k, R, nprobe = 5, 12, 2
    Da, Ia = oracle.ivfpq_search(xq, coarse, books, offs, lc, lid, R, nprobe)
    D, I = oracle.ivfpq_search_rerank(xq, coarse, books, offs, lc, lid, xb, k, nprobe, R)
    exact = cdist(xq.astype(np.float64), xb.astype(np.float64), "sqeuclidean")
    for j in range(len(xq)):
        cand = Ia[j][Ia[j] >= 0]
        assert set(I[j].tolist()) <= set(cand.tolist())
        ref = sorted((exact[j, i], i) for i in cand)[:k]
        assert I[j].tolist() == [i for _, i in ref]
        np.testing.assert_allclose(D[j], [v for v, _ in ref], rtol=1e-12)


def test_build_lists_insertion_order_and_append():
    lists = np.array([2, 0, 2, 1, 0, 2])
    codes = np.arange(12, dtype=np.uint8).reshape(6, 2)
    offs, lc, lid = oracle.build_lists(lists, codes, 4)
    assert offs.tolist() == [0, 2, 3, 6, 6]
    assert lid.tolist() == [1, 4, 3, 0, 2, 5]
    assert lc[:, 0].tolist() == [2, 8, 6, 0, 4, 10]
    offs2, lc2, lid2 = oracle.build_lists(np.array([0, 3]), np.zeros((2, 2), np.uint8), 4,
                                          id0=6, prev=(offs, lc, lid))
    assert offs2.tolist() == [0, 3, 4, 7, 8]
    assert lid2.tolist() == [1, 4, 6, 3, 0, 2, 5, 7]


def test_ivfpq_train_shapes_and_objective():
    rng = np.random.default_rng(51)
    xt = rng.standard_normal((2000, 8)).astype(np.float32)
    coarse, books = oracle.ivfpq_train(xt, 8, 2, 5, np.arange(8) * 7,
                                       np.stack([np.arange(256) * 3, np.arange(256) * 5]))
    assert coarse.shape == (8, 8) and books.shape == (2, 256, 4)
    assert coarse.dtype == np.float32 and books.dtype == np.float32


# ------------------------------------------------------------ training pins
def test_ivfpq_train_lossless_fixture():
    # quantizers known by construction (tests/train_fixture.py): training must
    # return the two coarse centres and, per sub-space, the codewords of its
    # init rows' residuals, bit for bit
    from train_fixture import NLIST, M, build
    f = build()
    coarse, books = oracle.ivfpq_train(f["xt"], NLIST, M, 4, f["coarse_init"], f["pq_init"])
    np.testing.assert_array_equal(coarse, f["coarse"])
    np.testing.assert_array_equal(books, f["books"])


def test_ivfpq_train_lossless_fixture_catches_planted_mistakes():
    # each plausible mistake, planted in a copy of the oracle's training steps,
    # fails the fixture: residuals to the initial coarse rows, a sub-vector
    # slice off by one block, another sub-space's init rows
    from train_fixture import DS, NLIST, M, build
    f = build()
    xt = f["xt"].astype(np.float64)

    def train(residual_to_init=False, shift=0, same_init=False):
        coarse, _ = oracle.kmeans(xt, f["coarse_init"], 4)
        init = np.ascontiguousarray(xt[f["coarse_init"]], np.float32)
        ref = init if residual_to_init else coarse
        a, _ = oracle.kmeans_assign(xt, ref)
        res = xt - ref[a].astype(np.float64)
        books = np.empty((M, 256, DS), np.float32)
        for m in range(M):
            mm = (m + shift) % M
            sub = np.ascontiguousarray(res[:, mm * DS:(mm + 1) * DS])
            rows = f["pq_init"][0 if same_init else m]
            books[m], _ = oracle.kmeans(sub, rows, 4)
        return books

    np.testing.assert_array_equal(train(), f["books"])  # the copy is faithful
    for bad in ({"residual_to_init": True}, {"shift": 1}, {"same_init": True}):
        assert not np.array_equal(train(**bad), f["books"]), bad


def test_ivfpq_train_residuals_to_final_centroids_handworked(golden_dir):
    with open(os.path.join(golden_dir, "ivfpq_train_handworked.json")) as fh:
        g = json.load(fh)
    i = np.arange(256, dtype=np.float64)
    xt = np.stack([i, 2 * i, -i, 3 * i], axis=1).astype(np.float32)
    pq_init = np.array([[(5 * j + 3 * m) % 256 for j in range(256)] for m in range(4)], np.int64)
    coarse, books = oracle.ivfpq_train(xt, g["nlist"], g["M"], g["niter"], g["coarse_init"],
                                       pq_init)
    assert coarse.tolist() == g["coarse"]
    for e in g["books_sample"]:
        assert books[e["m"], e["j"], 0] == e["value"], e


def test_kmeans_loop_1d_handworked(golden_dir):
    # the Lloyd loop itself (Forgy rows 0 and 1) reproduces the hand-worked
    # iterations: objective measured at each assignment, final centroids
    g = _load(golden_dir, "kmeans_1d.json")
    x = np.array(g["points"], np.float64)
    n = len(g["iterations"])
    c, objs = oracle.kmeans(x, [0, 1], n)
    assert g["init"] == [x[0].tolist(), x[1].tolist()]
    # objectives are measured against FP32-rounded centroids (7.3333335)
    np.testing.assert_allclose(objs, [it["objective"] for it in g["iterations"]], rtol=1e-6)
    np.testing.assert_allclose(c, np.array(g["iterations"][-1]["centroids"]), rtol=1e-7)


# ------------------------------------------------------------ k-NN graph
def test_knn_graph_exact_bruteforce_with_ties():
    # Section 6.5: every node queried against the whole set, the node itself
    # left out.  Pure-Python double loop on small-integer points with many
    # equal distances and duplicate points (a duplicate is a neighbour at 0).
    rng = np.random.default_rng(61)
    x = rng.integers(-2, 3, size=(40, 3)).astype(np.float32)
    x[7] = x[3]
    k = 6
    D, I = oracle.knn(x, x, k, exclude=np.arange(len(x)))
    for i in range(len(x)):
        cand = []
        for j in range(len(x)):
            if j == i:
                continue
            cand.append((sum((float(x[i, t]) - float(x[j, t])) ** 2 for t in range(3)), j))
        cand.sort()
        assert I[i].tolist() == [j for _, j in cand[:k]]
        assert D[i].tolist() == [v for v, _ in cand[:k]]
        assert i not in I[i]
    assert I[3, 0] == 7 and D[3, 0] == 0.0 and I[7, 0] == 3
    # nb - 1 candidates only: the last slot is padding
    D, I = oracle.knn(x[:5], x[:5], 5, exclude=np.arange(5))
    assert np.all(I[:, 4] == -1) and np.all(np.isinf(D[:, 4]))


def test_knn_graph_exclude_is_per_query():
    # excluding another row than the query's own removes exactly that row
    rng = np.random.default_rng(62)
    xb = rng.standard_normal((50, 4)).astype(np.float32)
    xq = rng.standard_normal((5, 4)).astype(np.float32)
    D0, I0 = oracle.knn(xq, xb, 10)
    ex = I0[:, 0].copy()
    D1, I1 = oracle.knn(xq, xb, 9, exclude=ex)
    np.testing.assert_array_equal(I1, I0[:, 1:])
    np.testing.assert_array_equal(D1, D0[:, 1:])
    # an id outside the database excludes nothing
    D2, I2 = oracle.knn(xq, xb, 10, exclude=np.full(5, -1))
    np.testing.assert_array_equal(I2, I0)


def test_ivfpq_graph_lossless_equals_exact_graph():
    # a database made exactly of coarse centroid + codewords, every list
    # probed: the IVFADC graph equals the exact graph (self left out on both)
    rng = np.random.default_rng(63)
    M, ds, nlist = 2, 2, 3
    d = M * ds
    coarse = rng.integers(-20, 20, size=(nlist, d)).astype(np.float32) * 4
    books = rng.integers(-1, 2, size=(M, 256, ds)).astype(np.float32)
    books[:, :9] = np.array([[a, b] for a in (-1, 0, 1) for b in (-1, 0, 1)], np.float32)
    books[:, 9:] = 50.0
    L = rng.integers(0, nlist, 80)
    cw = rng.integers(0, 9, size=(80, M))
    xb = (coarse[L] + np.concatenate([books[m][cw[:, m]] for m in range(M)], 1)).astype(np.float32)
    lists, codes = oracle.ivf_encode(xb, coarse, books)
    offs, lc, lid = oracle.build_lists(lists, codes, nlist)
    self_ids = np.arange(len(xb))
    D, I = oracle.ivfpq_search(xb, coarse, books, offs, lc, lid, 10, nlist, exclude=self_ids)
    De, Ie = oracle.knn(xb, xb, 10, exclude=self_ids)
    np.testing.assert_array_equal(I, Ie)
    np.testing.assert_array_equal(D, De)
    assert not np.any(I == self_ids[:, None])


def test_ivfpq_graph_drops_only_the_node():
    # with the node excluded, the result is the unexcluded search of k + 1
    # with the node's entry removed (wherever it ranked), else its first k
    xq, xb, coarse, books, lists, codes, offs, lc, lid = _random_index(64)
    nodes = np.array([0, 5, 17, 120, 299])
    k = 8
    Da, Ia = oracle.ivfpq_search(xb[nodes], coarse, books, offs, lc, lid, k + 1, 2)
    D, I = oracle.ivfpq_search(xb[nodes], coarse, books, offs, lc, lid, k, 2, exclude=nodes)
    for j, n in enumerate(nodes):
        keep = Ia[j] != n
        np.testing.assert_array_equal(I[j], Ia[j][keep][:k])
        np.testing.assert_array_equal(D[j], Da[j][keep][:k])


def test_rotate_rows_permutation_and_orthogonal():
    # a permutation matrix moves columns exactly; an orthogonal matrix keeps
    # every row's norm and is undone by its transpose; a transposed operand
    # or a wrong index fails one of these
    rng = np.random.default_rng(5)
    x = rng.standard_normal((37, 12))
    perm = rng.permutation(12)
    P = np.eye(12)[perm]                      # row j selects column perm[j]
    assert np.array_equal(oracle.rotate_rows(x, P), x[:, perm])
    Q, _ = np.linalg.qr(rng.standard_normal((12, 12)))
    y = oracle.rotate_rows(x, Q)
    assert np.allclose(np.linalg.norm(y, axis=1), np.linalg.norm(x, axis=1), rtol=1e-12)
    assert np.allclose(oracle.rotate_rows(y, Q.T), x, atol=1e-12)
    # a rectangular projection (dout < d) keeps the first dout coordinates
    assert np.array_equal(oracle.rotate_rows(x, np.eye(12)[:5]), x[:, :5])
