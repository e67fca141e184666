"""GPU parity of k-means steps, PQ encoding and IVFADC search against the
float64 oracle (through the C ABI).  Trained quantizers are exported from the
GPU index and handed to the oracle as data, so both sides search the same
index."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
from paper_1702_08734_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
RTOL = 1e-5


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_08734_amd import api as a
    a.lib()
    return a


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def gap_ok(dist_row, chosen, tol=RTOL):
    """True when `chosen` is the unique argmin of dist_row beyond tolerance,
    i.e. the choice must be bit-exact; False when ties within tol allow
    another answer."""
    srt = np.sort(dist_row)
    return len(srt) < 2 or (srt[1] - srt[0]) > tol * max(abs(srt[0]), 1e-30)


# ------------------------------------------------------------ k-means steps
def test_kmeans_assign_matches_oracle(api):
    say("kmeans assign")
    mix = synth.Mixture(50, 32, (9, 1))
    x = mix.sample(20000, (9, 2))
    c = x[:300].copy()
    a, dist = api.kmeans_assign(dev(x), dev(c))
    torch.cuda.synchronize()
    ao, do = oracle.kmeans_assign(x, c)
    a = a.cpu().numpy()
    diff = np.nonzero(a != ao)[0]
    for i in diff:  # only band-ambiguous points may differ
        di = ((x[i].astype(np.float64) - c.astype(np.float64)) ** 2).sum(1)
        assert abs(di[a[i]] - di[ao[i]]) <= RTOL * di[ao[i]], (i, a[i], ao[i])
    np.testing.assert_allclose(dist.cpu().numpy(), do, rtol=RTOL)


def test_kmeans_update_matches_oracle(api):
    say("kmeans update")
    mix = synth.Mixture(40, 16, (9, 3))
    x = mix.sample(30000, (9, 4))
    K = 64
    a = np.random.default_rng(0).integers(0, K, size=30000)
    a[a == 5] = 6       # cluster 5 empty -> split rule
    a[a == 60] = 6      # cluster 60 empty too
    c0 = x[:K].copy()
    c, counts = api.kmeans_update(dev(x), dev(a.astype(np.int64)), dev(c0))
    torch.cuda.synchronize()
    co, counts_o = oracle.kmeans_update(x, a, c0)
    np.testing.assert_array_equal(counts.cpu().numpy(), counts_o)
    np.testing.assert_allclose(c.cpu().numpy(), co, rtol=1e-6, atol=1e-7)


def test_kmeans_split_rule_handworked(api, golden_dir):
    with open(os.path.join(golden_dir, "kmeans_empty_split.json")) as f:
        g = json.load(f)
    c, counts = api.kmeans_update(dev(np.array(g["points"], np.float32)),
                                  dev(np.array(g["assign"], np.int64)),
                                  dev(np.array(g["init"], np.float32)))
    torch.cuda.synchronize()
    assert c.cpu().numpy().tolist() == g["centroids"]
    assert counts.cpu().numpy().tolist() == g["counts"]


def test_kmeans_1d_handworked(api, golden_dir):
    with open(os.path.join(golden_dir, "kmeans_1d.json")) as f:
        g = json.load(f)
    x = dev(np.array(g["points"], np.float32))
    c = dev(np.array(g["init"], np.float32))
    for it in g["iterations"]:
        a, dist = api.kmeans_assign(x, c)
        assert a.cpu().numpy().tolist() == it["assign"]
        assert float(dist.double().sum()) == pytest.approx(it["objective"], rel=1e-6)
        c, _ = api.kmeans_update(x, a, c)
        np.testing.assert_allclose(c.cpu().numpy(), np.array(it["centroids"]), rtol=1e-7)


# ------------------------------------------------------------ PQ training
def test_train_lossless_fixture_matches_oracle_exactly(api):
    # quantizers known by construction (tests/train_fixture.py): the GPU's
    # coarse k-means, residuals and per-sub-space k-means return them bit for
    # bit, as does the oracle
    from train_fixture import D, M, NLIST, build
    say("train lossless fixture")
    f = build()
    ix = api.IVFPQ(D, NLIST, M)
    ix.train(dev(f["xt"]), 4, f["coarse_init"], f["pq_init"])
    coarse, books = ix.get_quantizers()
    np.testing.assert_array_equal(coarse, f["coarse"])
    np.testing.assert_array_equal(books, f["books"])
    co, bo = oracle.ivfpq_train(f["xt"], NLIST, M, 4, f["coarse_init"], f["pq_init"])
    np.testing.assert_array_equal(coarse, co)
    np.testing.assert_array_equal(books, bo)


def test_train_residuals_to_final_centroids_handworked(api, golden_dir):
    with open(os.path.join(golden_dir, "ivfpq_train_handworked.json")) as f:
        g = json.load(f)
    i = np.arange(256, dtype=np.float64)
    xt = np.stack([i, 2 * i, -i, 3 * i], axis=1).astype(np.float32)
    pq_init = np.array([[(5 * j + 3 * m) % 256 for j in range(256)] for m in range(4)], np.int64)
    ix = api.IVFPQ(g["d"], g["nlist"], g["M"])
    ix.train(dev(xt), g["niter"], np.array(g["coarse_init"], np.int64), pq_init)
    coarse, books = ix.get_quantizers()
    assert coarse.tolist() == g["coarse"]
    for e in g["books_sample"]:
        assert books[e["m"], e["j"], 0] == e["value"], e


def _pq_objectives(xt, coarse, books):
    """Per sub-space mean squared quantisation error of the training
    residuals to their nearest coarse centroid (float64, oracle steps)."""
    a, _ = oracle.kmeans_assign(xt, coarse)
    res = xt.astype(np.float64) - coarse[a].astype(np.float64)
    M, _, ds = books.shape
    out = []
    for m in range(M):
        _, dist = oracle.kmeans_assign(np.ascontiguousarray(res[:, m * ds:(m + 1) * ds]), books[m])
        out.append(dist.mean())
    return np.array(out)


def test_train_mixture_objectives_match_oracle(api):
    # same data and Forgy rows on both sides; trajectories may split after a
    # band-ambiguous assignment, so the coarse and per-sub-space objectives
    # are compared (within 1%), not the centroids
    say("train mixture vs oracle")
    mix = synth.Mixture(60, 32, (12, 0))
    xt = mix.sample(20000, (12, 1))
    nlist, M, niter = 64, 8, 8
    ci, pi = synth.choose_rows(len(xt), nlist, 13), synth.pq_init_rows(len(xt), M, 14)
    ix = api.IVFPQ(32, nlist, M)
    ix.train(dev(xt), niter, ci, pi)
    coarse, books = ix.get_quantizers()
    co, bo = oracle.ivfpq_train(xt, nlist, M, niter, ci, pi)
    _, dg = oracle.kmeans_assign(xt, coarse)
    _, do = oracle.kmeans_assign(xt, co)
    assert abs(dg.mean() / do.mean() - 1) <= 0.01
    og, oo = _pq_objectives(xt, coarse, books), _pq_objectives(xt, co, bo)
    say(f"per-sub-space objective ratio gpu/oracle: {np.round(og / oo, 4).tolist()}")
    assert np.all(np.abs(og / oo - 1) <= 0.01), (og, oo)


@pytest.mark.parametrize("M,ds", [(4, 2), (8, 8), (16, 8), (8, 16), (16, 3)])
def test_pq_encode_matches_oracle(api, M, ds):
    say(f"pq encode M={M} ds={ds}")
    rng = np.random.default_rng(M * 10 + ds)
    books = rng.standard_normal((M, 256, ds)).astype(np.float32)
    r = rng.standard_normal((5000, M * ds)).astype(np.float32)
    codes = api.pq_encode(dev(r), dev(books)).cpu().numpy()
    co = oracle.pq_encode(r, books)
    bad = np.argwhere(codes != co)
    for i, m in bad:
        sub = r[i, m * ds:(m + 1) * ds].astype(np.float64)
        dd = ((sub - books[m].astype(np.float64)) ** 2).sum(1)
        assert not gap_ok(dd, co[i, m]), (i, m)


# ------------------------------------------------------------ IVFADC
def _adc_dist(x, ids, id_pos, lists_of_pos, codes, coarse, books):
    pos = id_pos[ids]
    dec = coarse[lists_of_pos[pos]].astype(np.float64) + oracle.pq_decode(codes[pos], books)
    return ((dec - x.astype(np.float64)) ** 2).sum(1)


def check_ivf(D, I, xq, rows, coarse, books, offs, codes, ids, k, nprobe):
    """Band rule for IVFADC results against the oracle on the same index."""
    nlist = len(coarse)
    Do, Io = oracle.ivfpq_search(xq[rows], coarse, books, offs, codes, ids, k + 64, nprobe)
    lists_of_pos = np.repeat(np.arange(nlist), np.diff(offs))
    id_pos = np.empty(ids.max() + 1 if len(ids) else 0, np.int64)
    id_pos[ids] = np.arange(len(ids))
    fails, ambiguous = [], 0
    for j, q in enumerate(rows):
        x = xq[q]
        cd = ((coarse.astype(np.float64) - x.astype(np.float64)) ** 2).sum(1)
        srt = np.sort(cd)
        if nprobe < nlist and srt[nprobe] - srt[nprobe - 1] <= RTOL * srt[nprobe]:
            ambiguous += 1  # probe set itself is band-ambiguous
            continue
        gi = I[j][I[j] >= 0]
        gd = D[j][: len(gi)].astype(np.float64)
        nexp = min(k, int((Io[j] >= 0).sum()))
        if len(gi) != nexp:
            fails.append(f"q{q}: {len(gi)} results, expected {nexp}")
            continue
        if len(gi) == 0:
            continue
        if np.any(np.diff(gd) < 0):
            fails.append(f"q{q}: not ascending")
        if len(set(gi.tolist())) != len(gi):
            fails.append(f"q{q}: duplicates")
        delta = _adc_dist(x, gi, id_pos, lists_of_pos, codes, coarse, books)
        if np.any(np.abs(gd - delta) > RTOL * np.maximum(delta, 1e-3 * (x.astype(np.float64) ** 2).sum())):
            r = int(np.argmax(np.abs(gd - delta)))
            fails.append(f"q{q}: rank {r} D={gd[r]} oracle={delta[r]}")
        od, oi = Do[j], Io[j]
        nv = int((oi >= 0).sum())
        dk = od[nexp - 1]
        tol = RTOL * max(dk, 1e-30)
        inband = (np.abs(od[:nv] - dk) <= tol) & (oi[:nv] >= 0)
        band = set(oi[:nv][inband].tolist())
        oset = set(oi[:nexp].tolist())
        gset = set(gi.tolist())
        if not (oset - band) <= gset or not gset <= (oset | band):
            fails.append(f"q{q}: sets differ beyond the band")
        for r in range(nexp):
            lo = r == 0 or od[r] - od[r - 1] > RTOL * od[r]
            hi = r + 1 >= nv or od[r + 1] - od[r] > RTOL * od[r]
            if lo and hi and gi[r] != oi[r]:
                fails.append(f"q{q}: rank {r} id {gi[r]} != oracle {oi[r]}")
                break
        same = gd[1:] == gd[:-1]
        if np.any(same & (gi[1:] < gi[:-1])):
            fails.append(f"q{q}: equal distances out of id order")
    return fails, ambiguous


@pytest.fixture(scope="module")
def small_index(api):
    say("build small IVFPQ index")
    mix = synth.Mixture(100, 32, (11, 0))
    xt = mix.sample(20000, (11, 1))
    xb = mix.sample(60000, (11, 2))
    xq = mix.sample(300, (11, 3))
    nlist, M = 64, 8
    ix = api.IVFPQ(32, nlist, M)
    ix.train(dev(xt), 8, synth.choose_rows(len(xt), nlist, 5), synth.pq_init_rows(len(xt), M, 6))
    ix.add(dev(xb[:25000]))
    ix.add(dev(xb[25000:]))   # a second batch appends behind the first
    return {"ix": ix, "xt": xt, "xb": xb, "xq": xq}


def test_ivfpq_train_quality(api, small_index):
    # k-means trajectories may split after one band-ambiguous assignment, so
    # training is compared by the final objective, not bitwise.
    ix, xt = small_index["ix"], small_index["xt"]
    coarse, books = ix.get_quantizers()
    co, _ = oracle.kmeans(xt, synth.choose_rows(len(xt), 64, 5), 8)
    _, dg = oracle.kmeans_assign(xt, coarse)
    _, do = oracle.kmeans_assign(xt, co)
    assert dg.mean() <= do.mean() * 1.01


def test_ivfpq_lists_match_oracle_encoding(api, small_index):
    ix, xb = small_index["ix"], small_index["xb"]
    coarse, books = ix.get_quantizers()
    offs, codes, ids = ix.get_lists()
    assert ix.ntotal == len(xb)
    lo, co = oracle.ivf_encode(xb, coarse, books)
    offs_o, codes_o, ids_o = oracle.build_lists(lo, co, len(coarse))
    if np.array_equal(ids, ids_o):
        np.testing.assert_array_equal(offs, offs_o)
        bad = np.argwhere(codes != codes_o)
    else:
        # a band-ambiguous coarse assignment moved an entry: check each one
        lists_g = np.repeat(np.arange(len(coarse)), np.diff(offs))
        pos = np.empty(len(ids), np.int64)
        pos[ids] = np.arange(len(ids))
        lg = lists_g[pos]
        for i in np.nonzero(lg != lo)[0]:
            dd = ((xb[i].astype(np.float64) - coarse.astype(np.float64)) ** 2).sum(1)
            assert not gap_ok(dd, lo[i]), i
        bad = []
    # ids sequential, insertion order inside each list
    for L in range(len(coarse)):
        seg = ids[offs[L]:offs[L + 1]]
        assert np.all(np.diff(seg) > 0)
    assert sorted(ids.tolist()) == list(range(len(xb)))
    res = xb.astype(np.float64) - coarse[lo].astype(np.float64)
    pos_o = np.empty(len(ids_o), np.int64)
    pos_o[ids_o] = np.arange(len(ids_o))
    for p, m in bad:
        i = ids_o[p]
        ds = books.shape[2]
        dd = ((res[i, m * ds:(m + 1) * ds] - books[m].astype(np.float64)) ** 2).sum(1)
        assert not gap_ok(dd, codes_o[p, m]), (i, m)


@pytest.mark.parametrize("k,nprobe", [(1, 1), (10, 4), (100, 16), (5, 64), (300, 8), (1024, 32)])
def test_ivfpq_search_matches_oracle(api, small_index, k, nprobe):
    say(f"ivfpq search k={k} nprobe={nprobe}")
    ix, xq = small_index["ix"], small_index["xq"]
    D, I = ix.search(dev(xq), k, nprobe)
    torch.cuda.synchronize()
    coarse, books = ix.get_quantizers()
    offs, codes, ids = ix.get_lists()
    rows = np.arange(0, 300, 7)
    fails, amb = check_ivf(D.cpu().numpy()[rows], I.cpu().numpy()[rows], xq, rows, coarse, books,
                           offs, codes, ids, k, nprobe)
    assert not fails, fails[:10]
    assert amb <= 2


def test_ivfpq_handworked(api, golden_dir):
    with open(os.path.join(golden_dir, "ivfpq_handworked.json")) as f:
        g = json.load(f)
    d, M = g["d"], g["M"]
    # the library needs M >= 4: embed the 2-sub-space example in d = 8, M = 4
    # with two extra all-zero sub-spaces whose codebook entry 0 is zero.
    D8, M4 = 8, 4
    ds = d // M
    books = np.full((M4, 256, ds), 100.0, np.float32)
    for m, entries in g["codebook_set"].items():
        for j, v in entries.items():
            books[int(m), int(j)] = v
    books[2:, 0] = 0.0
    coarse = np.zeros((2, D8), np.float32)
    coarse[:, :d] = np.array(g["coarse"], np.float32)
    xb = np.zeros((3, D8), np.float32)
    xb[:, :d] = np.array(g["xb"], np.float32)
    xq = np.zeros((1, D8), np.float32)
    xq[0, :d] = g["query"]
    ix = api.IVFPQ(D8, 2, M4)
    ix.set_quantizers(coarse, books)
    ix.add(dev(xb))
    offs, codes, ids = ix.get_lists()
    assert codes[:, :2].tolist() == [g["codes"][0], g["codes"][2], g["codes"][1]]
    for c in g["cases"]:
        D, I = ix.search(dev(xq), c["k"], c["nprobe"])
        assert I.cpu().numpy()[0].tolist() == c["I"]
        exp = [float("inf") if v == "inf" else v for v in c["D"]]
        np.testing.assert_allclose(D.cpu().numpy()[0], exp, rtol=1e-6)


def test_ivfpq_rerank_handworked(api, golden_dir):
    with open(os.path.join(golden_dir, "ivfpq_rerank_handworked.json")) as f:
        g = json.load(f)
    d, M = g["d"], g["M"]
    # embedded in d = 8, M = 4 as in the plain hand-worked case
    D8, M4 = 8, 4
    ds = d // M
    books = np.full((M4, 256, ds), 100.0, np.float32)
    for m, entries in g["codebook_set"].items():
        for j, v in entries.items():
            books[int(m), int(j)] = v
    books[2:, 0] = 0.0
    coarse = np.zeros((2, D8), np.float32)
    coarse[:, :d] = np.array(g["coarse"], np.float32)
    xb = np.zeros((len(g["xb"]), D8), np.float32)
    xb[:, :d] = np.array(g["xb"], np.float32)
    xq = np.zeros((1, D8), np.float32)
    xq[0, :d] = g["query"]
    ix = api.IVFPQ(D8, 2, M4)
    ix.set_quantizers(coarse, books)
    b = dev(xb)
    ix.add(b)
    for c in g["cases"]:
        say(f"rerank handworked {c}")
        D, I = ix.search_rerank(dev(xq), c["k"], c["nprobe"], c["R"], b)
        assert I.cpu().numpy()[0].tolist() == c["I"]
        exp = [float("inf") if v == "inf" else v for v in c["D"]]
        np.testing.assert_allclose(D.cpu().numpy()[0], exp, rtol=1e-6)


@pytest.mark.parametrize("k,nprobe,R", [(1, 4, 16), (10, 8, 100), (100, 16, 400), (10, 64, 1024)])
def test_ivfpq_rerank_matches_oracle(api, small_index, k, nprobe, R):
    say(f"ivfpq rerank k={k} nprobe={nprobe} R={R}")
    ix, xq, xb = small_index["ix"], small_index["xq"], small_index["xb"]
    D, I = ix.search_rerank(dev(xq), k, nprobe, R, dev(xb))
    torch.cuda.synchronize()
    coarse, books = ix.get_quantizers()
    offs, codes, ids = ix.get_lists()
    rows = np.arange(0, 300, 5)
    fails, skipped = check_rerank(D.cpu().numpy()[rows], I.cpu().numpy()[rows], xq, xb, rows,
                                  coarse, books, offs, codes, ids, k, nprobe, R)
    assert not fails, fails[:10]
    assert skipped <= 3


@pytest.mark.parametrize("k,R", [(10, 100), (10, 1024)])
def test_ivfpq_rerank_independent_of_batch(api, small_index, k, R):
    # a query's re-ranked result does not depend on the batch it is searched
    # in (coarse plan, scan grouping and merge all change with the batch
    # size; the scan's keys are (distance, id), a total order): bit for bit
    say(f"ivfpq rerank small vs large batch k={k} R={R}")
    ix, xb = small_index["ix"], small_index["xb"]
    xq = synth.Mixture(100, 32, (11, 0)).sample(5000, (11, 9))
    Dl, Il = ix.search_rerank(dev(xq), k, 8, R, dev(xb))
    Ds, Is = ix.search_rerank(dev(xq[:300]), k, 8, R, dev(xb))
    torch.cuda.synchronize()
    assert np.array_equal(Is.cpu().numpy(), Il.cpu().numpy()[:300])
    assert np.array_equal(Ds.cpu().numpy(), Dl.cpu().numpy()[:300])


def check_rerank(Dg, Ig, xq, xb, rows, coarse, books, offs, codes, ids, k, nprobe, R):
    """Band rule for re-ranked IVFADC results against the oracle; returns
    (failures, rows skipped as band-ambiguous)."""
    # short lists whose R-th ADC value is band-ambiguous may legitimately
    # differ; the oracle's R + 1 values tell which rows those are
    Da, Ia = oracle.ivfpq_search(xq[rows], coarse, books, offs, codes, ids, R + 1, nprobe)
    Do, Io = oracle.ivfpq_search_rerank(xq[rows], coarse, books, offs, codes, ids, xb, k,
                                        nprobe, R)
    skipped, fails = 0, []
    for j, q in enumerate(rows):
        x = xq[q].astype(np.float64)
        cd = np.sort(((coarse.astype(np.float64) - x) ** 2).sum(1))
        probe_amb = nprobe < len(coarse) and cd[nprobe] - cd[nprobe - 1] <= RTOL * cd[nprobe]
        a = Da[j]
        list_amb = Ia[j, R] >= 0 and a[R] - a[R - 1] <= RTOL * a[R]
        if probe_amb or list_amb:
            skipped += 1
            continue
        gi = Ig[j][Ig[j] >= 0]
        nexp = int((Io[j] >= 0).sum())
        if len(gi) != nexp:
            fails.append(f"q{q}: {len(gi)} results, expected {nexp}")
            continue
        # exact FP32 distances of the returned rows
        delta = ((xb[gi].astype(np.float64) - x) ** 2).sum(1)
        gd = Dg[j][:nexp].astype(np.float64)
        floor = 1e-3 * ((x ** 2).sum() + (xb[gi].astype(np.float64) ** 2).sum(1))
        if np.any(np.abs(gd - delta) > RTOL * np.maximum(delta, floor)):
            fails.append(f"q{q}: distance off")
        od, oi = Do[j][:nexp], Io[j][:nexp]
        dk = od[-1]
        band_ids = set(oi[np.abs(od - dk) <= RTOL * dk].tolist())
        if not (set(oi.tolist()) - band_ids) <= set(gi.tolist()):
            fails.append(f"q{q}: sets differ beyond the band")
        for r in range(nexp):
            lo = r == 0 or od[r] - od[r - 1] > RTOL * od[r]
            hi = r + 1 >= nexp or od[r + 1] - od[r] > RTOL * od[r]
            if lo and hi and gi[r] != oi[r]:
                fails.append(f"q{q}: rank {r} id {gi[r]} != oracle {oi[r]}")
                break
    return fails, skipped


def test_ivfpq_rerank_errors(api, small_index):
    ix, xq, xb = small_index["ix"], small_index["xq"], small_index["xb"]
    with pytest.raises(api.MKError):
        ix.search_rerank(dev(xq[:2]), 10, 4, 5, dev(xb))          # R < k
    with pytest.raises(api.MKError):
        ix.search_rerank(dev(xq[:2]), 10, 4, 20, dev(xb[:100]))   # too few rows


def test_ivfpq_state_errors(api):
    ix = api.IVFPQ(16, 8, 4)
    with pytest.raises(api.MKError) as e:
        ix.search(dev(np.zeros((1, 16), np.float32)), 5, 1)
    assert e.value.status == -5
    with pytest.raises(api.MKError):
        api.IVFPQ(16, 8, 3)
