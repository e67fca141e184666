"""IVFADC parity at the benchmark's own shape: 10,000,000 x 128 rows of a
1,000-component mixture, 4,096 lists, PQ 16 x 8 bit, trained and searched
as the bench does (all 10,000 queries in one launch, so the list scan runs
in the grouping and grid it is timed in), sampled queries compared with the
oracle on the exported index (Algorithm 4; the band rule of
test_gpu_ivfpq)."""
import sys

import numpy as np
import pytest

from paper_1702_08734_amd import synth
from test_gpu_ivfpq import check_ivf, check_rerank

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def c3():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_08734_amd import api
    say("c3: generating 10,000,000 x 128, training, adding")
    w = synth.ivfpq_workload()
    xb = torch.from_numpy(w["xb"]).cuda()
    xt = xb[torch.from_numpy(w["sample"]).cuda()].contiguous()
    ix = api.IVFPQ(128, w["nlist"], w["M"])
    ix.train(xt, 20, w["coarse_init"], w["pq_init"])
    ix.add(xb)
    torch.cuda.synchronize()
    del xt
    coarse, books = ix.get_quantizers()
    offs, codes, ids = ix.get_lists()
    rows = np.linspace(0, w["xq"].shape[0] - 1, 64).astype(np.int64)
    return {"ix": ix, "w": w, "xb": xb, "xq": torch.from_numpy(w["xq"]).cuda(), "rows": rows,
            "q": (coarse, books, offs, codes, ids)}


@pytest.mark.parametrize("nprobe", [8, 128])
def test_c3_adc_sampled(c3, nprobe):
    say(f"c3 ADC k=100 nprobe={nprobe}")
    D, I = c3["ix"].search(c3["xq"], 100, nprobe)
    torch.cuda.synchronize()
    rows = c3["rows"]
    coarse, books, offs, codes, ids = c3["q"]
    fails, amb = check_ivf(D.cpu().numpy()[rows], I.cpu().numpy()[rows], c3["w"]["xq"], rows,
                           coarse, books, offs, codes, ids, 100, nprobe)
    assert not fails, fails[:10]
    assert amb <= 4


def test_c3_rerank_sampled(c3):
    say("c3 re-rank k=10 nprobe=8 R=256")
    D, I = c3["ix"].search_rerank(c3["xq"], 10, 8, 256, c3["xb"])
    torch.cuda.synchronize()
    rows = c3["rows"]
    coarse, books, offs, codes, ids = c3["q"]
    fails, skipped = check_rerank(D.cpu().numpy()[rows], I.cpu().numpy()[rows], c3["w"]["xq"],
                                  c3["w"]["xb"], rows, coarse, books, offs, codes, ids, 10, 8, 256)
    assert not fails, fails[:10]
    assert skipped <= 4
