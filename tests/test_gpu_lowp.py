"""BF16 / FP8 brute force with exact FP32 re-rank (through the C ABI).

Pins: the quantizers against torch's own BF16 and float8_e4m3fn conversions
(round to nearest even) on the CPU; inputs exactly representable in both
formats must give exactly the FP32 exact-search result; on mixture data the
re-ranked distances are exact FP32 (within 1e-5 of the float64 oracle) and
recall@k is measured against the oracle."""
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


@pytest.mark.parametrize("d", [5, 64, 96, 130])
def test_quantize_bf16_matches_torch(api, d):
    say(f"quantize bf16 d={d}")
    rng = np.random.default_rng(d)
    x = (rng.standard_normal((300, d)) * np.exp(rng.uniform(-8, 8, (300, 1)))).astype(np.float32)
    out, inv = api.quantize_rows(dev(x), "bf16")
    ld = api.lib().mk_lowp_stride(d)
    got = out.cpu().numpy().view(np.uint16).reshape(300, ld)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(got[:, :d], ref)
    assert np.all(got[:, d:] == 0)
    assert np.all(inv.cpu().numpy() == 1.0)


@pytest.mark.parametrize("d", [7, 64, 96])
def test_quantize_fp8_matches_torch(api, d):
    say(f"quantize fp8 d={d}")
    rng = np.random.default_rng(100 + d)
    x = (rng.standard_normal((300, d)) * np.exp(rng.uniform(-6, 6, (300, 1)))).astype(np.float32)
    x[7] = 0.0
    out, inv = api.quantize_rows(dev(x), "fp8")
    ld = api.lib().mk_lowp_stride(d)
    got = out.cpu().numpy().reshape(300, ld)
    m = np.abs(x).max(1).astype(np.float64)
    # largest power of two s with m * s <= 448 (s = 1 for a zero row)
    with np.errstate(divide="ignore"):
        e = np.where(m > 0, np.floor(np.log2(448.0 / np.where(m > 0, m, 1.0))), 0.0)
    s = np.ldexp(1.0, e.astype(np.int64))
    assert np.all(m * s <= 448.0) and np.all((m * s > 224.0) | (m == 0))
    np.testing.assert_array_equal(inv.cpu().numpy(), (1.0 / s).astype(np.float32))
    scaled = (x.astype(np.float64) * s[:, None]).astype(np.float32)
    ref = torch.from_numpy(scaled).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(got[:, :d], ref)
    assert np.all(got[:, d:] == 0)


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("metric", ["l2", "ip"])
@pytest.mark.parametrize("nb,k,R", [(6000, 20, 80), (150_000, 100, 400)])
def test_lowp_exact_on_representable_inputs(api, prec, metric, nb, k, R):
    # small integers are exact in BF16 and E4M3 (and the FP8 scale is a power
    # of two): every product and partial sum is exact in FP32, so the
    # low-precision search equals the FP32 search exactly -- also with many
    # database chunks, memory-resident candidate pools and exact ties
    say(f"lowp representable {prec} {metric} nb={nb} k={k} R={R}")
    rng = np.random.default_rng(3)
    xb = rng.integers(-3, 4, size=(nb, 64)).astype(np.float32)
    xq = rng.integers(-3, 4, size=(70, 64)).astype(np.float32)
    xb[:, 0] = 3.0  # every row has max |x| = 3: one common FP8 scale
    xq[:, 0] = 3.0
    b = dev(xb)
    lp, inv = api.quantize_rows(b, prec)
    D, I = api.knn_search_lowp(dev(xq), b, lp, inv, k, R, prec, metric)
    De, Ie = api.knn_search(dev(xq), b, k, metric)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(I.cpu().numpy(), Ie.cpu().numpy())
    np.testing.assert_array_equal(D.cpu().numpy(), De.cpu().numpy())


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_lowp_mixture_recall_and_exact_distances(api, prec, metric):
    say(f"lowp mixture {prec} {metric}")
    mix = synth.Mixture(200, 96, (104, 99))
    xb = mix.sample(200_000, (104, 0), unit_norm=True)
    xq = mix.sample(64, (104, 1), unit_norm=True)
    b = dev(xb)
    lp, inv = api.quantize_rows(b, prec)
    k, R = 100, 400
    D, I = api.knn_search_lowp(dev(xq), b, lp, inv, k, R, prec, metric)
    torch.cuda.synchronize()
    Dn, In = D.cpu().numpy(), I.cpu().numpy()
    m = oracle.METRIC_L2 if metric == "l2" else oracle.METRIC_IP
    Do, Io = oracle.knn(xq, xb, k, m)
    recall = np.mean([len(set(In[j]) & set(Io[j])) / k for j in range(len(xq))])
    say(f"recall@{k} {prec} {metric}: {recall:.4f}")
    assert recall >= (0.99 if prec == "bf16" else 0.97)
    # reported distances are the exact FP32 direct form of the returned rows
    for j in range(len(xq)):
        delta = oracle.pair_distance(xq, xb, j, In[j], m)
        scale = np.abs(xb[In[j]].astype(np.float64) * xq[j]).sum(1)
        floor = 1e-3 * (1.0 + (xb[In[j]].astype(np.float64) ** 2).sum(1)) if m == 0 else scale
        assert np.all(np.abs(Dn[j] - delta) <= 1e-5 * np.maximum(np.abs(delta), floor))
        order = np.diff(Dn[j])
        assert np.all(order >= 0) if m == 0 else np.all(order <= 0)


def test_lowp_errors(api):
    b = dev(np.ones((10, 8), np.float32))
    lp, inv = api.quantize_rows(b, "bf16")
    with pytest.raises(api.MKError):
        api.knn_search_lowp(b, b, lp, inv, 10, 5, "bf16")  # rerank < k
