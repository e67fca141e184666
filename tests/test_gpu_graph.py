"""GPU parity of k-NN graph construction (Section 6.5: every database vector
searched against the whole database or index, a node never its own
neighbour) against the float64 oracle with one excluded id per query,
through the C ABI (mk_knn_graph, mk_ivfpq_knn_graph)."""
import sys

import numpy as np
import pytest

import oracle
from band import check_rows
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


# ------------------------------------------------------------ exact graph
@pytest.mark.parametrize("metric", ["l2", "ip"])
@pytest.mark.parametrize("k", [1, 10, 100])
def test_exact_graph_integer_ties_equals_oracle(api, k, metric):
    # small-integer points with duplicate rows: distances exact in FP32, many
    # exact ties (a node's duplicates tie with distance 0); the graph must
    # equal the oracle's exactly, lower index first
    say(f"exact graph integer ties k={k} {metric}")
    rng = np.random.default_rng(40 + k)
    xb = rng.integers(-2, 3, size=(6000, 12)).astype(np.float32)
    xb[3000:3050] = xb[:50]
    D, I = api.knn_graph(dev(xb), k, metric)
    torch.cuda.synchronize()
    m = oracle.METRIC_L2 if metric == "l2" else oracle.METRIC_IP
    Do, Io = oracle.knn(xb, xb, k, m, exclude=np.arange(6000))
    np.testing.assert_array_equal(I.cpu().numpy(), Io)
    np.testing.assert_array_equal(D.cpu().numpy().astype(np.float64), Do)


def test_exact_graph_node_range_and_padding(api):
    # a sub-range of nodes; and a database of k rows (each node has k - 1
    # neighbours, so the last column is padding)
    say("exact graph node range + padding")
    rng = np.random.default_rng(8)
    xb = rng.integers(-3, 4, size=(2000, 8)).astype(np.float32)
    D, I = api.knn_graph(dev(xb), 20, "l2", node0=700, nnodes=333)
    torch.cuda.synchronize()
    Do, Io = oracle.knn(xb[700:1033], xb, 20, oracle.METRIC_L2, exclude=np.arange(700, 1033))
    np.testing.assert_array_equal(I.cpu().numpy(), Io)
    np.testing.assert_array_equal(D.cpu().numpy().astype(np.float64), Do)
    small = xb[:7]
    D, I = api.knn_graph(dev(small), 7, "l2")
    torch.cuda.synchronize()
    Do, Io = oracle.knn(small, small, 7, oracle.METRIC_L2, exclude=np.arange(7))
    np.testing.assert_array_equal(I.cpu().numpy(), Io)
    assert np.all(I.cpu().numpy()[:, 6] == -1) and np.all(np.isinf(D.cpu().numpy()[:, 6]))


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_exact_graph_mixture_band_rule(api, metric):
    # continuous mixture data, 40,000 x 64, k = 10: every node's row equals
    # an exact search of the node against the database minus itself (band
    # rule against the oracle on sampled nodes)
    say(f"exact graph mixture {metric}")
    mix = synth.Mixture(200, 64, (12, 0))
    xb = mix.sample(40_000, (12, 1))
    D, I = api.knn_graph(dev(xb), 10, metric)
    torch.cuda.synchronize()
    D, I = D.cpu().numpy(), I.cpu().numpy()
    assert not np.any(I == np.arange(40_000)[:, None]), "a node is its own neighbour"
    rows = np.arange(0, 40_000, 401)
    # the database minus node q is xb with row q removed; map indices back
    fails = []
    for q in rows:
        keep = np.ones(40_000, bool)
        keep[q] = False
        sub = xb[keep]
        idx = np.nonzero(keep)[0]
        pos = np.searchsorted(idx, I[q])
        fails += check_rows(D[q:q + 1], pos[None, :], xb, sub, np.array([q]), 10, metric,
                            extra=32)
    assert not fails, fails[:10]


def test_exact_graph_errors(api):
    x = torch.zeros((10, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(api.MKError):
        api.knn_graph(x, 1024)  # one selector entry goes to the node
    with pytest.raises(api.MKError):
        api.knn_graph(x, 5, node0=8, nnodes=5)  # past the database


# ------------------------------------------------------------ IVFADC graph
def _adc(x, gi, id_pos, list_of_pos, codes, coarse, books):
    M, _, ds = books.shape
    out = np.empty(len(gi))
    for j, i in enumerate(gi):
        p = id_pos[i]
        r = x.astype(np.float64) - coarse[list_of_pos[p]].astype(np.float64)
        dec = np.concatenate([books[m, codes[p, m]].astype(np.float64) for m in range(M)])
        out[j] = ((r - dec) ** 2).sum()
    return out


def check_graph_ivf(D, I, xb, rows, coarse, books, offs, codes, ids, k, nprobe):
    """Band rule for IVFADC graph rows D[j], I[j] of nodes rows[j] against the
    oracle's search of the node with its own id excluded."""
    nlist = len(coarse)
    Do, Io = oracle.ivfpq_search(xb[rows], coarse, books, offs, codes, ids, k + 64, nprobe,
                                 exclude=rows)
    list_of_pos = np.repeat(np.arange(nlist), np.diff(offs))
    id_pos = np.empty(ids.max() + 1, np.int64)
    id_pos[ids] = np.arange(len(ids))
    fails, ambiguous = [], 0
    for j, q in enumerate(rows):
        x = xb[q]
        cd = ((coarse.astype(np.float64) - x.astype(np.float64)) ** 2).sum(1)
        srt = np.sort(cd)
        if nprobe < nlist and srt[nprobe] - srt[nprobe - 1] <= RTOL * srt[nprobe]:
            ambiguous += 1  # the probe set itself is band-ambiguous
            continue
        gi = I[j][I[j] >= 0]
        gd = D[j][: len(gi)].astype(np.float64)
        if q in set(gi.tolist()):
            fails.append(f"node {q} is its own neighbour")
        nexp = min(k, int((Io[j] >= 0).sum()))
        if len(gi) != nexp:
            fails.append(f"node {q}: {len(gi)} results, expected {nexp}")
            continue
        if nexp == 0:
            continue
        if np.any(np.diff(gd) < 0) or len(set(gi.tolist())) != len(gi):
            fails.append(f"node {q}: not ascending or duplicates")
        delta = _adc(x, gi, id_pos, list_of_pos, codes, coarse, books)
        if np.any(np.abs(gd - delta) > RTOL * np.maximum(delta, 1e-3 * (x.astype(np.float64) ** 2).sum())):
            fails.append(f"node {q}: distances")
        od, oi = Do[j], Io[j]
        nv = int((oi >= 0).sum())
        dk = od[nexp - 1]
        inband = np.abs(od[:nv] - dk) <= RTOL * max(dk, 1e-30)
        band = set(oi[:nv][inband].tolist())
        oset, gset = set(oi[:nexp].tolist()), set(gi.tolist())
        if not (oset - band) <= gset or not gset <= (oset | band):
            fails.append(f"node {q}: sets differ beyond the band")
        for r in range(nexp):
            lo = r == 0 or od[r] - od[r - 1] > RTOL * od[r]
            hi = r + 1 >= nv or od[r + 1] - od[r] > RTOL * od[r]
            if lo and hi and gi[r] != oi[r]:
                fails.append(f"node {q}: rank {r} id {gi[r]} != oracle {oi[r]}")
                break
        same = gd[1:] == gd[:-1]
        if np.any(same & (gi[1:] < gi[:-1])):
            fails.append(f"node {q}: equal distances out of id order")
    return fails, ambiguous


@pytest.fixture(scope="module")
def graph_index(api):
    say("build IVFPQ index for the graph tests")
    mix = synth.Mixture(80, 32, (13, 0))
    xt = mix.sample(20_000, (13, 1))
    xb = mix.sample(50_000, (13, 2))
    xb[40_000:40_200] = xb[:200]  # duplicate nodes: identical codes, exact ADC ties
    nlist, M = 64, 8
    ix = api.IVFPQ(32, nlist, M)
    ix.train(dev(xt), 8, synth.choose_rows(len(xt), nlist, (13, 3)),
             synth.pq_init_rows(len(xt), M, (13, 4)))
    ix.add(dev(xb))
    torch.cuda.synchronize()
    coarse, books = ix.get_quantizers()
    offs, codes, ids = ix.get_lists()
    return ix, xb, coarse, books, offs, codes, ids


@pytest.mark.parametrize("k,nprobe", [(10, 1), (10, 4), (50, 16), (300, 64)])
def test_ivfpq_graph_matches_oracle(api, graph_index, k, nprobe):
    ix, xb, coarse, books, offs, codes, ids = graph_index
    say(f"ivfpq graph k={k} nprobe={nprobe}")
    D, I = ix.knn_graph(dev(xb), k, nprobe)
    torch.cuda.synchronize()
    D, I = D.cpu().numpy(), I.cpu().numpy()
    assert not np.any(I == np.arange(len(xb))[:, None]), "a node is its own neighbour"
    rows = np.concatenate([np.arange(0, 50_000, 997), np.arange(40_000, 40_010), [49_999]])
    fails, amb = check_graph_ivf(D[rows], I[rows], xb, rows, coarse, books, offs, codes, ids,
                                 k, nprobe)
    assert not fails, fails[:10]
    assert amb <= len(rows) // 10


def test_ivfpq_graph_duplicate_nodes(api, graph_index):
    # nodes 40,000 .. 40,199 are copies of nodes 0 .. 199: identical codes in
    # the same list, so each copy ties with its original at the smallest ADC
    # distance the list offers (its own quantisation error); a node range
    # through the batched call, checked against the oracle, ties by lower id
    ix, xb, coarse, books, offs, codes, ids = graph_index
    say("ivfpq graph duplicate nodes")
    D, I = ix.knn_graph(dev(xb), 5, 8, node0=40_000, nnodes=200)
    torch.cuda.synchronize()
    D, I = D.cpu().numpy(), I.cpu().numpy()
    rows = np.arange(40_000, 40_200)
    fails, amb = check_graph_ivf(D, I, xb, rows, coarse, books, offs, codes, ids, 5, 8)
    assert not fails, fails[:10]
    assert amb <= 20
    # the original is the copy's first neighbour unless the probe order is ambiguous
    assert np.mean(I[:, 0] == np.arange(200)) > 0.9


@pytest.mark.parametrize("k,nprobe,R", [(10, 4, 64), (20, 16, 256)])
def test_ivfpq_graph_rerank_matches_oracle(api, graph_index, k, nprobe, R):
    # ADC short list of R entries (the node excluded), re-ranked exactly
    ix, xb, coarse, books, offs, codes, ids = graph_index
    say(f"ivfpq graph re-rank k={k} nprobe={nprobe} R={R}")
    D, I = ix.knn_graph(dev(xb), k, nprobe, R=R)
    torch.cuda.synchronize()
    D, I = D.cpu().numpy(), I.cpu().numpy()
    assert not np.any(I == np.arange(len(xb))[:, None]), "a node is its own neighbour"
    rows = np.concatenate([np.arange(0, 50_000, 1013), np.arange(40_000, 40_010)])
    Da, Ia = oracle.ivfpq_search(xb[rows], coarse, books, offs, codes, ids, R + 1, nprobe,
                                 exclude=rows)
    Do, Io = oracle.ivfpq_search_rerank(xb[rows], coarse, books, offs, codes, ids, xb, k, nprobe,
                                        R, exclude=rows)
    skipped, fails = 0, []
    for j, q in enumerate(rows):
        x = xb[q].astype(np.float64)
        cd = np.sort(((coarse.astype(np.float64) - x) ** 2).sum(1))
        probe_amb = nprobe < len(coarse) and cd[nprobe] - cd[nprobe - 1] <= RTOL * cd[nprobe]
        a = Da[j]
        list_amb = Ia[j, R] >= 0 and a[R] - a[R - 1] <= RTOL * a[R]
        if probe_amb or list_amb:
            skipped += 1
            continue
        gi, gd = I[q][I[q] >= 0], D[q][I[q] >= 0].astype(np.float64)
        nexp = int((Io[j] >= 0).sum())
        if len(gi) != nexp:
            fails.append(f"node {q}: {len(gi)} results, expected {nexp}")
            continue
        delta = ((xb[gi].astype(np.float64) - x) ** 2).sum(1)
        floor = 1e-3 * ((x ** 2).sum() + (xb[gi].astype(np.float64) ** 2).sum(1))
        if np.any(np.abs(gd - delta) > RTOL * np.maximum(delta, floor)):
            fails.append(f"node {q}: distance off")
        od, oi = Do[j][:nexp], Io[j][:nexp]
        band = set(oi[np.abs(od - od[-1]) <= RTOL * max(od[-1], 1e-30)].tolist())
        if not (set(oi.tolist()) - band) <= set(gi.tolist()):
            fails.append(f"node {q}: sets differ beyond the band")
        for r in range(nexp):
            lo = r == 0 or od[r] - od[r - 1] > RTOL * od[r]
            hi = r + 1 >= nexp or od[r + 1] - od[r] > RTOL * od[r]
            if lo and hi and gi[r] != oi[r]:
                fails.append(f"node {q}: rank {r} id {gi[r]} != oracle {oi[r]}")
                break
    assert not fails, fails[:10]
    assert skipped <= len(rows) // 10


def test_ivfpq_graph_errors(api, graph_index):
    ix, xb, *_ = graph_index
    with pytest.raises(api.MKError):
        ix.knn_graph(dev(xb), 10, 4, node0=49_990, nnodes=20)
    with pytest.raises(api.MKError):
        ix.knn_graph(dev(xb), 10, 4, R=5)  # R < k
