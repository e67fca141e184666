"""GPU parity of exact k-NN and row-wise k-selection against the float64
oracle (through the C ABI).  Run on an MI355X: pytest -m gpu."""
import sys

import numpy as np
import pytest

import oracle
from band import check_rows
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


# ------------------------------------------------------------ k-selection
@pytest.mark.parametrize("largest", [False, True])
@pytest.mark.parametrize("length,k", [(0, 5), (1, 1), (7, 10), (63, 64), (64, 64), (65, 64),
                                      (1000, 1), (1000, 100), (1000, 1000), (4099, 128),
                                      (5000, 256), (5000, 513), (20000, 1024), (3, 1024)])
def test_kselect_ties_vs_oracle(api, length, k, largest):
    say(f"kselect len={length} k={k} largest={largest}")
    rng = np.random.default_rng(length * 31 + k)
    a = rng.integers(0, 50, size=(9, length)).astype(np.float32)  # many exact ties
    v, i = api.kselect(dev(a), k, largest)
    torch.cuda.synchronize()
    vo, io = oracle.kselect(a, k, largest)
    np.testing.assert_array_equal(i.cpu().numpy(), io)
    np.testing.assert_array_equal(v.cpu().numpy().astype(np.float64), vo)


@pytest.mark.parametrize("k", [100, 1000])
def test_kselect_segmented_rows(api, k):
    # few long rows -> several segments per row and the merge pass
    say(f"kselect segmented k={k}")
    a = synth.uniform_rows(3, 400_000, (7, k))
    v, i = api.kselect(dev(a), k)
    torch.cuda.synchronize()
    vo, io = oracle.kselect(a, k)
    np.testing.assert_array_equal(i.cpu().numpy(), io)
    np.testing.assert_array_equal(v.cpu().numpy().astype(np.float64), vo)


@pytest.mark.parametrize("k", [77, 300, 1000])
def test_kselect_unaligned_rows(api, k):
    # rows of 10,001 values: every row but the first starts off the 16-byte
    # grid, so the element-wise path runs (k >= 129: candidate pools)
    say(f"kselect unaligned k={k}")
    a = synth.uniform_rows(50, 10_001, (8, 0))
    v, i = api.kselect(dev(a), k)
    torch.cuda.synchronize()
    vo, io = oracle.kselect(a, k)
    np.testing.assert_array_equal(i.cpu().numpy(), io)
    np.testing.assert_array_equal(v.cpu().numpy().astype(np.float64), vo)


@pytest.mark.parametrize("k", [100, 1000])
def test_kselect_benchmark_shape_sampled(api, k):
    # the k-selection benchmark shape (rows of 128,000 U[0,1) values), 2,000 rows
    say(f"kselect 2000x128000 k={k}")
    a = synth.kselect_rows(2000, 128_000)
    v, i = api.kselect(dev(a), k)
    torch.cuda.synchronize()
    rows = np.arange(0, 2000, 97)
    vo, io = oracle.kselect(a[rows], k)
    np.testing.assert_array_equal(i.cpu().numpy()[rows], io)
    np.testing.assert_array_equal(v.cpu().numpy()[rows].astype(np.float64), vo)


@pytest.mark.parametrize("largest", [False, True])
@pytest.mark.parametrize("k", [300, 1000])
def test_kselect_threshold_guess_rows(api, k, largest):
    # 8,200 rows of 33,000 values: one segment per row, long enough for the
    # sampled threshold guess.  Rows 0-63 ascending (the guess, taken from
    # the row's start, is far too low: the plain second pass must run), rows
    # 64-127 descending (far too high), rows 128-191 small-integer ties,
    # the rest U[0,1).
    say(f"kselect guess rows k={k} largest={largest}")
    rng = np.random.default_rng(1000 + k + int(largest))
    a = rng.random((8200, 33_000), dtype=np.float32)
    a[0:64] = np.sort(a[0:64], axis=1)
    a[64:128] = np.sort(a[64:128], axis=1)[:, ::-1]
    a[128:192] = rng.integers(0, 40, size=(64, 33_000)).astype(np.float32)
    v, i = api.kselect(dev(a), k, largest)
    torch.cuda.synchronize()
    rows = np.concatenate([np.arange(0, 8), np.arange(60, 70), np.arange(124, 134),
                           np.arange(186, 196), np.arange(200, 8200, 397)])
    vo, io = oracle.kselect(np.ascontiguousarray(a[rows]), k, largest)
    np.testing.assert_array_equal(i.cpu().numpy()[rows], io)
    np.testing.assert_array_equal(v.cpu().numpy()[rows].astype(np.float64), vo)


# ------------------------------------------------------------ exact k-NN
def test_knn_exact_small_full(api):
    # 50,000 x 64 N(0,1), 500 queries, k = 10: every query against the oracle
    say("knn exact_small full")
    w = synth.exact_small()
    D, I = api.knn_search(dev(w["xq"]), dev(w["xb"]), w["k"])
    torch.cuda.synchronize()
    fails = check_rows(D.cpu().numpy(), I.cpu().numpy(), w["xq"], w["xb"],
                       np.arange(500), w["k"])
    assert not fails, fails[:10]


@pytest.mark.parametrize("metric", ["l2", "ip"])
@pytest.mark.parametrize("d", [1, 3, 8, 63, 64, 96, 128, 200])
@pytest.mark.parametrize("nb,k", [(0, 4), (5, 10), (300, 1), (1000, 64), (5000, 100),
                                  (3000, 300), (2500, 1024)])
def test_knn_shapes(api, d, nb, k, metric):
    say(f"knn d={d} nb={nb} k={k} {metric}")
    rng = np.random.default_rng(d * 1009 + nb + k)
    xb = rng.standard_normal((nb, d)).astype(np.float32)
    xq = rng.standard_normal((37, d)).astype(np.float32)
    if nb > 10:
        xb[nb // 2] = xb[3]  # an exact duplicate
        xq[5] = xb[7]        # a query equal to a database row
    D, I = api.knn_search(dev(xq), dev(xb), k, metric)
    torch.cuda.synchronize()
    fails = check_rows(D.cpu().numpy(), I.cpu().numpy(), xq, xb, np.arange(37), k, metric)
    assert not fails, fails[:10]


def test_knn_integer_ties(api):
    # small-integer data: distances exact in FP32, many exact ties -> lower index wins
    say("knn integer ties")
    rng = np.random.default_rng(5)
    xb = rng.integers(-2, 3, size=(4000, 16)).astype(np.float32)
    xq = rng.integers(-2, 3, size=(50, 16)).astype(np.float32)
    for metric in ("l2", "ip"):
        D, I = api.knn_search(dev(xq), dev(xb), 50, metric)
        torch.cuda.synchronize()
        Do, Io = oracle.knn(xq, xb, 50, oracle.METRIC_L2 if metric == "l2" else oracle.METRIC_IP)
        np.testing.assert_array_equal(I.cpu().numpy(), Io)
        np.testing.assert_array_equal(D.cpu().numpy().astype(np.float64), Do)


@pytest.mark.parametrize("metric", ["l2", "ip"])
@pytest.mark.parametrize("k", [1, 10, 50, 100, 200, 300, 1024])
def test_knn_many_chunks_integer_ties(api, k, metric):
    # 150,000 small-integer rows: many database chunks share score bounds
    # while exact ties abound (distances are exact in FP32); the result must
    # equal the oracle's exactly, lower index first among equal distances.
    # k <= 100 runs the register queues, larger k the candidate pools.
    say(f"knn many chunks, integer ties, k={k} {metric}")
    rng = np.random.default_rng(11 + k)
    xb = rng.integers(-2, 3, size=(150_000, 16)).astype(np.float32)
    xq = rng.integers(-2, 3, size=(100, 16)).astype(np.float32)
    D, I = api.knn_search(dev(xq), dev(xb), k, metric)
    torch.cuda.synchronize()
    Do, Io = oracle.knn(xq, xb, k, oracle.METRIC_L2 if metric == "l2" else oracle.METRIC_IP)
    np.testing.assert_array_equal(I.cpu().numpy(), Io)
    np.testing.assert_array_equal(D.cpu().numpy().astype(np.float64), Do)


@pytest.mark.parametrize("k", [100, 256, 1024])
def test_knn_best_rows_in_last_chunk(api, k):
    # rows ordered from far to near for query 0, so its whole answer sits in
    # the last chunk and every earlier chunk publishes loose points
    say(f"knn best rows last, k={k}")
    rng = np.random.default_rng(29 + k)
    xb = rng.standard_normal((200_000, 32)).astype(np.float32)
    xq = rng.standard_normal((64, 32)).astype(np.float32)
    d0 = ((xb.astype(np.float64) - xq[0]) ** 2).sum(1)
    xb = np.ascontiguousarray(xb[np.argsort(-d0, kind="stable")])
    D, I = api.knn_search(dev(xq), dev(xb), k)
    torch.cuda.synchronize()
    rows = np.array([0, 1, 31, 63])
    fails = check_rows(D.cpu().numpy()[rows], I.cpu().numpy()[rows], xq, xb, rows, k)
    assert not fails, fails[:10]
    assert I[0].min().item() >= 200_000 - 4 * k


def test_knn_empty_query_batch(api):
    xb = dev(np.ones((10, 8), np.float32))
    D, I = api.knn_search(dev(np.zeros((0, 8), np.float32)), xb, 3)
    assert D.shape == (0, 3)


def test_knn_errors(api):
    xb = dev(np.ones((10, 8), np.float32))
    with pytest.raises(api.MKError) as e:
        api.knn_search(xb, xb, 1025)
    assert e.value.status == -2


@pytest.fixture(scope="module")
def large():
    say("generating exact_large (1,000,000 x 128, 10,000 queries)")
    return synth.exact_large()


LARGE_ROWS = np.linspace(0, 9999, 256).astype(np.int64)


@pytest.fixture(scope="module")
def large_oracle(large):
    # the oracle's 1,088 best rows of 256 sampled queries, for every k
    say("oracle on 256 exact_large queries")
    return {m: oracle.knn(large["xq"][LARGE_ROWS], large["xb"], 1024 + 64,
                          oracle.METRIC_L2 if m == "l2" else oracle.METRIC_IP)
            for m in ("l2", "ip")}


@pytest.mark.parametrize("metric,k", [("l2", 1), ("l2", 32), ("l2", 256), ("l2", 1024),
                                      ("ip", 10), ("ip", 1024)])
def test_knn_exact_large_sampled(api, large, large_oracle, k, metric):
    # the full 10,000-query batch in one call (the benchmark's launch shape),
    # 256 queries checked against the oracle
    say(f"knn exact_large k={k} {metric}")
    xq, xb = dev(large["xq"]), dev(large["xb"])
    D, I = api.knn_search(xq, xb, k, metric)
    torch.cuda.synchronize()
    rows = LARGE_ROWS
    fails = check_rows(D.cpu().numpy()[rows], I.cpu().numpy()[rows], large["xq"], large["xb"],
                       rows, k, metric, oracle_result=large_oracle[metric])
    assert not fails, fails[:10]
    # properties that hold for every row: sorted, valid, no duplicates
    Dn, In = D.cpu().numpy(), I.cpu().numpy()
    assert np.all(np.diff(Dn, axis=1) >= 0) if metric == "l2" else np.all(np.diff(Dn, axis=1) <= 0)
    assert In.min() >= 0 and In.max() < xb.shape[0]
    if k > 1:
        s = np.sort(In, axis=1)
        assert np.all(s[:, 1:] != s[:, :-1])


def test_knn_batch_independent(api, large):
    # a query's result does not depend on the rest of its batch
    say("knn batch independence")
    xb = dev(large["xb"][:200_000])
    xq_all = dev(large["xq"][:3000])
    for k in (10, 300):
        D, I = api.knn_search(xq_all, xb, k)
        sub = [0, 1, 17, 2999]
        D1, I1 = api.knn_search(xq_all[sub].contiguous(), xb, k)
        torch.cuda.synchronize()
        assert torch.equal(I[sub], I1) and torch.equal(D[sub], D1)


def test_knn_prenorm_matches(api, large):
    say("knn prenorm")
    xb = dev(large["xb"][:100_000])
    xq = dev(large["xq"][:500])
    yn = api.norms(xb)
    D, I = api.knn_search(xq, xb, 20)
    D2, I2 = api.knn_search(xq, xb, 20, yn=yn)
    torch.cuda.synchronize()
    assert torch.equal(I, I2) and torch.equal(D, D2)
    ref = (xb.double() ** 2).sum(1)
    assert torch.allclose(yn.double(), ref, rtol=1e-5)


def test_candidate_pools_never_dropped_a_key(api):
    # queues of 256+ entries keep unsorted pools that are cut before they can
    # fill; the library counts any key a full pool would have had to drop.
    # This runs after every pool search above (same process) plus one more.
    rng = np.random.default_rng(3)
    xb = dev(rng.standard_normal((300_000, 48)).astype(np.float32))
    xq = dev(rng.standard_normal((700, 48)).astype(np.float32))
    for k in (256, 600, 1024):
        api.knn_search(xq, xb, k)
    torch.cuda.synchronize()
    assert api.debug_pool_drops() == 0
