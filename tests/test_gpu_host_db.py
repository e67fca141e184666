"""Exact k-NN against a host-resident database streamed in chunks
(mk_knn_search_host, Section 5.1's inputs from the CPU) through the C ABI,
against the float64 oracle."""
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


def pinned(x):
    t = torch.empty(x.shape, dtype=torch.float32, pin_memory=True)
    t.copy_(torch.from_numpy(np.ascontiguousarray(x)))
    return t


@pytest.mark.parametrize("metric", ["l2", "ip"])
@pytest.mark.parametrize("k,chunk", [(1, 7_000), (10, 10_000), (100, 3_001), (300, 25_000),
                                     (1024, 9_000), (50, 100_000)])
def test_host_db_integer_ties_equal_oracle(api, k, chunk, metric):
    # distances exact in FP32, many ties spanning chunk boundaries: the merged
    # result equals the oracle's exactly, lower row first among equal values
    say(f"host db integer ties k={k} chunk={chunk} {metric}")
    rng = np.random.default_rng(70 + k)
    xb = rng.integers(-2, 3, size=(50_000, 16)).astype(np.float32)
    xb[40_000:40_100] = xb[:100]  # equal rows in different chunks
    xq = rng.integers(-2, 3, size=(64, 16)).astype(np.float32)
    D, I = api.knn_search_host(torch.from_numpy(xq).cuda(), pinned(xb), k, metric, chunk)
    m = oracle.METRIC_L2 if metric == "l2" else oracle.METRIC_IP
    Do, Io = oracle.knn(xq, xb, k, m)
    np.testing.assert_array_equal(I.cpu().numpy(), Io)
    np.testing.assert_array_equal(D.cpu().numpy().astype(np.float64), Do)


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_host_db_mixture_band_rule(api, metric):
    say(f"host db mixture {metric}")
    mix = synth.Mixture(300, 96, (71, 0))
    xb = mix.sample(200_003, (71, 1))
    xq = mix.sample(200, (71, 2))
    D, I = api.knn_search_host(torch.from_numpy(xq).cuda(), pinned(xb), 32, metric, 65_536)
    rows = np.arange(0, 200, 3)
    fails = check_rows(D.cpu().numpy()[rows], I.cpu().numpy()[rows], xq, xb, rows, 32, metric)
    assert not fails, fails[:10]


def test_host_db_small_and_pageable(api):
    # one chunk, and a pageable (not pinned) host array: still correct
    rng = np.random.default_rng(72)
    xb = rng.integers(-3, 4, size=(5_000, 8)).astype(np.float32)
    xq = rng.integers(-3, 4, size=(9, 8)).astype(np.float32)
    Do, Io = oracle.knn(xq, xb, 20)
    for chunk in (10_000, 1_234):
        D, I = api.knn_search_host(torch.from_numpy(xq).cuda(), torch.from_numpy(xb), 20, "l2",
                                   chunk)
        np.testing.assert_array_equal(I.cpu().numpy(), Io)
    with pytest.raises(api.MKError):
        api.knn_search_host(torch.from_numpy(xq).cuda(), torch.from_numpy(xb), 20, "l2", 0)
