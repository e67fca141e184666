"""GPU test of the allocation-free exact search (mk_knn_search_noalloc): its
results equal mk_knn_search's on the same inputs, bit for bit, on two calls
in a row (the second smaller, so it reuses the fixed scratch array holding
the first call's contents), and a call too large for the array is refused
before any work is enqueued.  Both entry points are called through the C ABI;
the first call is also checked against the float64 oracle."""
import sys

import numpy as np
import pytest

import oracle
from band import check_rows

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


def _pair(api, xq, xb, k, metric):
    D0, I0 = api.knn_search(xq, xb, k, metric)
    D1, I1 = api.knn_search_noalloc(xq, xb, k, metric)
    torch.cuda.synchronize()
    return D0.cpu().numpy(), I0.cpu().numpy(), D1.cpu().numpy(), I1.cpu().numpy()


@pytest.mark.parametrize("metric", ["l2", "ip"])
@pytest.mark.parametrize("k", [10, 100, 300])
def test_noalloc_equals_allocating_search(api, k, metric):
    rng = np.random.default_rng(1234 + k)
    # first call: 300 queries x 60,000 rows (several chunks, ragged tail)
    xb = rng.standard_normal((60_003, 64)).astype(np.float32)
    xq = rng.standard_normal((300, 64)).astype(np.float32)
    xb[777] = xb[12]  # an exact duplicate row
    say(f"noalloc call 1: nq=300 nb=60003 d=64 k={k} {metric}")
    D0, I0, D1, I1 = _pair(api, dev(xq), dev(xb), k, metric)
    np.testing.assert_array_equal(I1, I0)
    np.testing.assert_array_equal(D1, D0)
    rows = np.arange(0, 300, 7)
    fails = check_rows(D1[rows], I1[rows], xq, xb, rows, k, metric)
    assert not fails, fails[:10]
    # second call, smaller: fewer queries, a shorter database, another d
    xb2 = rng.standard_normal((9_001, 32)).astype(np.float32)
    xq2 = rng.standard_normal((41, 32)).astype(np.float32)
    say(f"noalloc call 2: nq=41 nb=9001 d=32 k={k} {metric}")
    D0, I0, D1, I1 = _pair(api, dev(xq2), dev(xb2), k, metric)
    np.testing.assert_array_equal(I1, I0)
    np.testing.assert_array_equal(D1, D0)


def test_noalloc_integer_ties_vs_oracle(api):
    # exact FP32 distances with many ties: both entry points equal the oracle
    rng = np.random.default_rng(77)
    for nb, nq in ((50_000, 120), (3_000, 17)):
        xb = rng.integers(-2, 3, size=(nb, 16)).astype(np.float32)
        xq = rng.integers(-2, 3, size=(nq, 16)).astype(np.float32)
        say(f"noalloc integer ties nq={nq} nb={nb}")
        D0, I0, D1, I1 = _pair(api, dev(xq), dev(xb), 50, "l2")
        Do, Io = oracle.knn(xq, xb, 50, oracle.METRIC_L2)
        np.testing.assert_array_equal(I1, Io)
        np.testing.assert_array_equal(D1.astype(np.float64), Do)
        np.testing.assert_array_equal(I0, I1)


def test_noalloc_rejects_oversize_and_empty(api):
    # 20,000 queries at k = 1024 need far more than the fixed array; the call
    # is refused on the host, before any kernel is enqueued
    say("noalloc oversize refusal")
    xb = torch.zeros((200_000, 8), dtype=torch.float32, device="cuda")
    xq = torch.zeros((20_000, 8), dtype=torch.float32, device="cuda")
    with pytest.raises(api.MKError) as e:
        api.knn_search_noalloc(xq, xb, 1024)
    assert e.value.status == -2 and "scratch" in str(e.value)
    # nq = 0 is a no-op
    D, I = api.knn_search_noalloc(xq[:0], xb, 5)
    assert D.shape == (0, 5)
    # the array still works after the refusal
    rng = np.random.default_rng(3)
    xb2 = rng.standard_normal((5_000, 24)).astype(np.float32)
    xq2 = rng.standard_normal((13, 24)).astype(np.float32)
    D0, I0, D1, I1 = _pair(api, dev(xq2), dev(xb2), 7, "l2")
    np.testing.assert_array_equal(I1, I0)
    np.testing.assert_array_equal(D1, D0)
