"""Index and network files (mk_ivfpq_save/load, mk_mlp_save/load) through the
C ABI: a loaded index searches exactly as the saved one (fixed probe count,
re-rank, k-NN graph, learned probe count), a loaded network predicts and
keeps training exactly as the saved one, and damaged files are refused."""
import os
import sys

import numpy as np
import pytest

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
def built(api):
    say("build IVFPQ index for save/load")
    mix = synth.Mixture(60, 64, (41, 0))
    xt = mix.sample(12_000, (41, 1))
    xb = mix.sample(30_000, (41, 2))
    xq = mix.sample(150, (41, 3))
    nlist, M = 48, 8
    ix = api.IVFPQ(64, nlist, M)
    ix.train(dev(xt), 5, synth.choose_rows(len(xt), nlist, (41, 4)),
             synth.pq_init_rows(len(xt), M, (41, 5)))
    ix.add(dev(xb[:20_000]))
    ix.add(dev(xb[20_000:]))  # two batches: lists built by appending
    torch.cuda.synchronize()
    return ix, xb, xq


def _same(a, b):
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x.cpu().numpy(), y.cpu().numpy())


def test_index_round_trip_bitwise(api, built, tmp_path):
    ix, xb, xq = built
    p = str(tmp_path / "index.bin")
    ix.save(p)
    say(f"index file {os.path.getsize(p)} bytes")
    ix2 = api.IVFPQ.load(p)
    assert (ix2.d, ix2.nlist, ix2.M, ix2.ntotal) == (ix.d, ix.nlist, ix.M, ix.ntotal)
    for a, b in zip(ix.get_quantizers(), ix2.get_quantizers()):
        np.testing.assert_array_equal(a, b)
    for a, b in zip(ix.get_lists(), ix2.get_lists()):
        np.testing.assert_array_equal(a, b)
    q, b = dev(xq), dev(xb)
    for k, nprobe in ((10, 1), (100, 8), (300, 48)):
        _same(ix.search(q, k, nprobe), ix2.search(q, k, nprobe))
    _same(ix.search_rerank(q, 10, 4, 64, b), ix2.search_rerank(q, 10, 4, 64, b))
    _same(ix.knn_graph(b, 10, 4, 100, 500), ix2.knn_graph(b, 10, 4, 100, 500))
    # the loaded index keeps growing like the original
    extra = synth.Mixture(60, 64, (41, 0)).sample(3_000, (41, 6))
    ix2.add(dev(extra))
    assert ix2.ntotal == ix.ntotal + 3_000


def test_network_round_trip_bitwise(api, built, tmp_path):
    ix, xb, xq = built
    say("network save/load")
    net = api.MLP(64 + 32, 128, "bf16")
    net.set_params(synth.mlp_init(96, 128, (41, 7)))
    rng = np.random.default_rng(41)
    F = dev(rng.standard_normal((2000, 96)).astype(np.float32) * 2 + 1)
    y = dev(rng.uniform(0, 5, 2000).astype(np.float32))
    net.fit_standardization(F)
    net.train_epoch(F, y, dev(synth.permutation(2000, (41, 8))), 256, 1e-3)
    p = str(tmp_path / "net.bin")
    net.save(p)
    net2 = api.MLP.load(p)
    assert (net2.din, net2.hidden, net2.n_params) == (96, 128, net.n_params)
    np.testing.assert_array_equal(net.get_params()[0], net2.get_params()[0])
    _same([net.forward(F)], [net2.forward(F)])
    # Adam state travels with the file: one more epoch on both is identical
    perm = dev(synth.permutation(2000, (41, 9)))
    l1 = net.train_epoch(F, y, perm, 256, 1e-3)
    l2 = net2.train_epoch(F, y, perm, 256, 1e-3)
    _same([l1], [l2])
    np.testing.assert_array_equal(net.get_params()[0], net2.get_params()[0])
    # a learned-probe search with loaded index and network equals the original
    net3 = api.MLP(64 + 32, 128, "bf16")
    net3.set_params(synth.mlp_init(96, 128, (41, 10)))
    net3.fit_standardization(ix.probe_features(dev(xq)))
    p3 = str(tmp_path / "net3.bin")
    net3.save(p3)
    pi = str(tmp_path / "index.bin")
    ix.save(pi)
    ixl, netl = api.IVFPQ.load(pi), api.MLP.load(p3)
    q, b = dev(xq), dev(xb)
    _same(ix.search_learned(net3, 0.5, q, 10, 32, 32, b),
          ixl.search_learned(netl, 0.5, q, 10, 32, 32, b))


def test_damaged_files_refused(api, built, tmp_path):
    ix, _, _ = built
    p = str(tmp_path / "index.bin")
    ix.save(p)
    raw = open(p, "rb").read()
    cases = {"truncated": raw[:-17], "trailing": raw + b"\0",
             "magic": b"X" + raw[1:], "empty": b""}
    for name, data in cases.items():
        q = str(tmp_path / f"bad_{name}.bin")
        with open(q, "wb") as f:
            f.write(data)
        with pytest.raises(api.MKError) as e:
            api.IVFPQ.load(q)
        assert e.value.status == -1, name
    # offsets that do not span the entries: corrupt the last offset
    hdr = 8 + 4 + 4 * 3 + 8
    body = hdr + 4 * ix.nlist * ix.d + 4 * ix.M * 256 * (ix.d // ix.M)
    last = body + 8 * ix.nlist
    bad = bytearray(raw)
    bad[last:last + 8] = (ix.ntotal + 5).to_bytes(8, "little")
    q = str(tmp_path / "bad_offsets.bin")
    with open(q, "wb") as f:
        f.write(bytes(bad))
    with pytest.raises(api.MKError):
        api.IVFPQ.load(q)
    with pytest.raises(api.MKError):
        api.IVFPQ.load(str(tmp_path / "missing.bin"))
    # an untrained index cannot be saved
    with pytest.raises(api.MKError) as e:
        api.IVFPQ(64, 48, 8).save(str(tmp_path / "untrained.bin"))
    assert e.value.status == -5
