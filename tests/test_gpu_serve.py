"""Serving loop (continuous batching) through the C ABI: a request's results
equal a search of that request alone, bit for bit, whatever batch it shares;
the row limit and the workspace budget bound the batches; errors surface at
submit and wait."""
import sys
import threading

import numpy as np
import pytest

import oracle
from paper_1702_08734_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


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


@pytest.fixture(scope="module")
def index(api):
    say("build IVFPQ index for the serving tests")
    mix = synth.Mixture(100, 64, (51, 0))
    xt = mix.sample(20000, (51, 1))
    xb = mix.sample(60000, (51, 2))
    xq = mix.sample(3000, (51, 3))
    ix = api.IVFPQ(64, 64, 8)
    ix.train(dev(xt), 6, synth.choose_rows(len(xt), 64, 5), synth.pq_init_rows(len(xt), 8, 6))
    ix.add(dev(xb))
    return {"ix": ix, "xb": xb, "xq": xq, "xb_dev": dev(xb)}


def _sizes(n, seed):
    # request sizes log-uniform in [1, 64]
    u = np.random.default_rng(seed).random(n)
    return np.clip(np.floor(np.exp(u * np.log(65))), 1, 64).astype(int)


@pytest.mark.parametrize("mode", ["adc", "rerank"])
def test_requests_equal_alone(api, index, mode):
    ix, xq = index["ix"], index["xq"]
    k, nprobe, R = 10, 8, 64
    kw = {"R": R, "xb": index["xb_dev"]} if mode == "rerank" else {}
    srv = api.Server(ix, k, nprobe=nprobe, max_batch=256, nstreams=3, **kw)
    sizes = _sizes(120, 7)
    starts = np.concatenate([[0], np.cumsum(sizes)])[:-1] % (len(xq) - 64)
    tickets = []
    for s0, n in zip(starts, sizes):
        tickets.append(srv.submit(xq[s0:s0 + n]))
    res = [srv.wait(t) for t in tickets]
    batches, rows = srv.stats()
    srv.close()
    say(f"{mode}: {len(tickets)} requests in {batches} batches, {rows} rows")
    assert rows == sizes.sum()
    assert batches < len(tickets)  # requests were batched together
    for (s0, n), (D, I, lat) in zip(zip(starts, sizes), res):
        q = dev(xq[s0:s0 + n])
        if mode == "rerank":
            Da, Ia = ix.search_rerank(q, k, nprobe, R, index["xb_dev"])
        else:
            Da, Ia = ix.search(q, k, nprobe)
        np.testing.assert_array_equal(I, Ia.cpu().numpy())
        np.testing.assert_array_equal(D, Da.cpu().numpy())
        assert lat > 0


def test_concurrent_submitters(api, index):
    ix, xq = index["ix"], index["xq"]
    srv = api.Server(ix, 5, nprobe=4, max_batch=128, nstreams=2)
    out = {}

    def client(c):
        got = []
        for j in range(20):
            s0 = (c * 97 + j * 13) % (len(xq) - 8)
            t = srv.submit(xq[s0:s0 + 8])
            got.append((s0, t))
        out[c] = [(s0, srv.wait(t)) for s0, t in got]

    th = [threading.Thread(target=client, args=(c,)) for c in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    srv.close()
    for c in range(4):
        for s0, (D, I, _) in out[c]:
            Da, Ia = ix.search(dev(xq[s0:s0 + 8]), 5, 4)
            np.testing.assert_array_equal(I, Ia.cpu().numpy())


def test_budget_and_row_limit(api, index):
    ix, xq = index["ix"], index["xq"]
    # a 1-byte budget admits only the first request of each batch
    srv = api.Server(ix, 10, nprobe=4, max_batch=512, nstreams=1, workspace_budget=1)
    tickets = [srv.submit(xq[i * 3:i * 3 + 3]) for i in range(30)]
    for t in tickets:
        srv.wait(t)
    batches, rows = srv.stats()
    srv.close()
    assert batches == 30 and rows == 90
    # row limit 16 with requests of 10 rows: one request per batch
    srv = api.Server(ix, 10, nprobe=4, max_batch=16, nstreams=2)
    tickets = [srv.submit(xq[i * 10:i * 10 + 10]) for i in range(12)]
    for t in tickets:
        srv.wait(t)
    batches, _ = srv.stats()
    srv.close()
    assert batches == 12
    assert ix.workspace_bytes(100, 10, 4) > ix.workspace_bytes(10, 10, 4) > 0


def test_errors(api, index):
    ix, xq = index["ix"], index["xq"]
    srv = api.Server(ix, 10, nprobe=4, max_batch=16)
    with pytest.raises(api.MKError):
        srv.submit(xq[:17])          # larger than max_batch
    with pytest.raises(api.MKError):
        srv.wait(12345)              # unknown ticket
    srv.close()
    with pytest.raises(api.MKError):
        api.Server(ix, 10, nprobe=4, R=5)   # re-rank without xb / R < k


# ------------------------------------------------------------ exact ties, large batches
@pytest.fixture(scope="module")
def tie_index(api):
    """Index of small-integer data: coarse centroids and codewords are small
    integers and every database vector is a centroid plus one codeword per
    sub-space, so every ADC distance (Eq. 10-11) is an integer computed
    exactly in FP32; distinct entries, within a list and across lists, share
    distances all the time, and each vector is also added twice more."""
    say("build small-integer IVFPQ index with exact ties")
    rng = np.random.default_rng(77)
    d, nlist, M = 16, 64, 4
    ds = d // M
    coarse = rng.integers(-4, 5, size=(nlist, d)).astype(np.float32)
    books = rng.integers(-1, 2, size=(M, 256, ds)).astype(np.float32)
    ix = api.IVFPQ(d, nlist, M)
    ix.set_quantizers(coarse, books)
    n = 6000
    base = coarse[rng.integers(0, nlist, n)]
    parts = [books[m][rng.integers(0, 256, n)] for m in range(M)]
    xb = (base + np.concatenate(parts, axis=1)).astype(np.float32)
    xb = np.concatenate([xb, xb[:2000], xb[:2000]])    # duplicate codes, later ids
    ix.add(dev(xb))
    xq = rng.integers(-4, 5, size=(3000, d)).astype(np.float32)
    offs, codes, ids = ix.get_lists()
    return {"ix": ix, "xq": xq, "coarse": coarse, "books": books, "offs": offs,
            "codes": codes, "ids": ids, "nlist": nlist}


def _big_sizes(n, seed):
    # requests of 300-700 rows: batches of up to 1,024 rows group 4 lists per
    # workgroup at nprobe 8 (the grouping depends on the batch size)
    return np.random.default_rng(seed).integers(300, 700, n)


@pytest.mark.parametrize("mode", ["fixed", "learned"])
def test_large_batches_exact_ties_equal_alone_and_oracle(api, tie_index, mode):
    ix, xq = tie_index["ix"], tie_index["xq"]
    k, nprobe, cap = 20, 8, 32
    kw = {"nprobe": nprobe}
    net = None
    if mode == "learned":
        net = api.MLP(16 + 32, 64, "fp32")
        net.set_params(synth.mlp_init(16 + 32, 64, 5))
        net.fit_standardization(ix.probe_features(dev(xq)))
        kw = {"net": net, "delta": 2.0, "cap": cap}
    srv = api.Server(ix, k, max_batch=1024, nstreams=2, **kw)
    sizes = _big_sizes(10, 3)
    starts = np.random.default_rng(4).integers(0, len(xq) - 700, len(sizes))
    tickets = [srv.submit(xq[s0:s0 + n]) for s0, n in zip(starts, sizes)]
    res = [srv.wait(t) for t in tickets]
    batches, rows = srv.stats()
    srv.close()
    say(f"{mode}: {len(sizes)} requests in {batches} batches")
    assert batches < len(sizes)
    for (s0, n), (D, I, _) in zip(zip(starts, sizes), res):
        q = dev(xq[s0:s0 + n])
        if mode == "learned":
            Da, Ia, tau = ix.search_learned(net, 2.0, q, k, cap)
            tau = tau.cpu().numpy()
            assert tau.min() >= 1 and tau.max() <= cap
        else:
            Da, Ia = ix.search(q, k, nprobe)
            tau = None
        np.testing.assert_array_equal(I, Ia.cpu().numpy())
        np.testing.assert_array_equal(D, Da.cpu().numpy())
    # the request searched alone equals the oracle exactly (integer distances,
    # ties to the lower id), on the first request
    s0, n = starts[0], sizes[0]
    q = xq[s0:s0 + n]
    if mode == "learned":
        _, _, tau = ix.search_learned(net, 2.0, dev(q), k, cap)
        Do, Io = oracle.ivfpq_search(q, tie_index["coarse"], tie_index["books"],
                                     tie_index["offs"], tie_index["codes"], tie_index["ids"], k,
                                     cap, nprobe_per_query=tau.cpu().numpy())
    else:
        Do, Io = oracle.ivfpq_search(q, tie_index["coarse"], tie_index["books"],
                                     tie_index["offs"], tie_index["codes"], tie_index["ids"], k,
                                     nprobe)
    D0, I0, _ = res[0]
    np.testing.assert_array_equal(I0, Io)
    np.testing.assert_array_equal(D0.astype(np.float64), Do)
