"""List-scan options of the IVFADC index through the C ABI
(mk_ivfpq_set_scan_options): the per-query fused scan and any fixed number
of lists per workgroup return exactly the default results; 16-bit lookup
tables (Section 5.3) agree with the float64 oracle within the bound that one
FP16 rounding per table entry implies, also for M = 96 sub-quantizers, which
FP32 tables cannot hold in LDS."""
import sys

import numpy as np
import pytest

import oracle
from paper_1702_08734_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
U16 = 2.0 ** -11  # unit roundoff of FP16 (round to nearest)


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


def _index(api, d, nlist, M, seed, nb=40_000):
    mix = synth.Mixture(70, d, (seed, 0))
    xt = mix.sample(15_000, (seed, 1))
    xb = mix.sample(nb, (seed, 2))
    xq = mix.sample(120, (seed, 3))
    xb[nb - 100:] = xb[:100]  # duplicates: exact ADC ties across ids
    ix = api.IVFPQ(d, nlist, M)
    ix.train(dev(xt), 6, synth.choose_rows(len(xt), nlist, (seed, 4)),
             synth.pq_init_rows(len(xt), M, (seed, 5)))
    ix.add(dev(xb))
    torch.cuda.synchronize()
    return ix, xb, xq


@pytest.fixture(scope="module")
def idx(api):
    say("build index d=64 nlist=40 M=16")
    return _index(api, 64, 40, 16, 51)


def _np(t):
    return [x.cpu().numpy() for x in t]


@pytest.mark.parametrize("group", [-1, 1, 3, 16, 40])
def test_lists_per_group_do_not_change_results(api, idx, group):
    ix, xb, xq = idx
    q, b = dev(xq), dev(xb)
    say(f"lists per group {group}")
    ix.set_scan_options("fp32", 0)
    ref = [_np(ix.search(q, 50, p)) for p in (1, 7, 40)]
    rr = _np(ix.search_rerank(q, 10, 9, 100, b))
    gr = _np(ix.knn_graph(b, 10, 5, 0, 300))
    ix.set_scan_options("fp32", group)
    try:
        for p, r in zip((1, 7, 40), ref):
            for x, y in zip(_np(ix.search(q, 50, p)), r):
                np.testing.assert_array_equal(x, y)
        for x, y in zip(_np(ix.search_rerank(q, 10, 9, 100, b)), rr):
            np.testing.assert_array_equal(x, y)
        for x, y in zip(_np(ix.knn_graph(b, 10, 5, 0, 300)), gr):
            np.testing.assert_array_equal(x, y)
    finally:
        ix.set_scan_options("fp32", 0)


def check_fp16(D, I, xq, ix, k, nprobe):
    """FP16-table results against the oracle: each returned distance within
    tol_q + 1e-5 |delta| of the float64 ADC distance of that id, where
    tol_q = 2^-11 sum_m max_j |2 term3_q[m][j]| bounds the rounding of the
    M looked-up table entries; sets equal outside a band of 2 tol_q at rank k."""
    coarse, books = ix.get_quantizers()
    offs, codes, ids = ix.get_lists()
    M, _, ds = books.shape
    Do, Io = oracle.ivfpq_search(xq, coarse, books, offs, codes, ids, k + 64, nprobe)
    pos = np.empty(ids.max() + 1, np.int64)
    pos[ids] = np.arange(len(ids))
    lists = np.repeat(np.arange(len(coarse)), np.diff(offs))
    b64 = books.astype(np.float64)
    fails = []
    for j in range(len(xq)):
        x = xq[j].astype(np.float64)
        t3 = np.einsum("mjt,mt->mj", b64, x.reshape(M, ds))
        tol = U16 * np.abs(2 * t3).max(1).sum()
        gi = I[j][I[j] >= 0]
        gd = D[j][: len(gi)].astype(np.float64)
        nexp = min(k, int((Io[j] >= 0).sum()))
        if len(gi) != nexp:
            fails.append(f"q{j}: {len(gi)} results, expected {nexp}")
            continue
        for r, i in enumerate(gi):
            p = pos[i]
            res = x - coarse[lists[p]].astype(np.float64)
            dec = np.concatenate([b64[m, codes[p, m]] for m in range(M)])
            delta = ((res - dec) ** 2).sum()
            if abs(gd[r] - delta) > tol + 1e-5 * abs(delta):
                fails.append(f"q{j} rank {r}: D {gd[r]} vs {delta} (tol {tol})")
                break
        dk = Do[j][nexp - 1]
        sure = set(Io[j][: nexp][Do[j][: nexp] < dk - 2 * tol].tolist())
        allowed = set(Io[j][Do[j] <= dk + 2 * tol].tolist())
        g = set(gi.tolist())
        if not sure <= g or not g <= allowed:
            fails.append(f"q{j}: sets differ beyond the FP16 band")
        if np.any(np.diff(gd) < 0):
            fails.append(f"q{j}: not ascending")
    return fails


@pytest.mark.parametrize("k,nprobe", [(10, 1), (50, 8), (200, 40)])
def test_fp16_tables_vs_oracle(api, idx, k, nprobe):
    ix, xb, xq = idx
    say(f"fp16 tables k={k} nprobe={nprobe}")
    ix.set_scan_options("fp16", 0)
    try:
        D, I = _np(ix.search(dev(xq), k, nprobe))
    finally:
        ix.set_scan_options("fp32", 0)
    fails = check_fp16(D, I, xq, ix, k, nprobe)
    assert not fails, fails[:10]


def test_fp16_tables_m96(api):
    # M = 96 sub-quantizers of one component each (d = 96): FP32 tables need
    # 96 KiB of LDS and are refused; FP16 tables (48 KiB) search
    say("fp16 tables with M = 96")
    ix, xb, xq = _index(api, 96, 32, 96, 52, nb=25_000)
    with pytest.raises(api.MKError) as e:
        ix.search(dev(xq), 10, 4)
    assert e.value.status == -2
    ix.set_scan_options("fp16", -1)
    D, I = _np(ix.search(dev(xq), 20, 4))
    fails = check_fp16(D, I, xq, ix, 20, 4)
    assert not fails, fails[:10]


def test_scan_option_errors(api, idx):
    ix, _, _ = idx
    with pytest.raises(api.MKError):
        ix.set_scan_options("fp32", -2)
    with pytest.raises(KeyError):
        ix.set_scan_options("bf16", 0)
