"""Linear pre-processing of rows (mk_rotate_rows: an OPQ rotation or a
projection, Sections 1 and 6.4) against the oracle's float64 product."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1702_08734_amd import api as a
    a.lib()
    return a


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda()


def within_dot_bound(got, x, rot):
    # FP32 sum of d products in any order: |error| <= gamma_d sum_t |r_jt x_it|,
    # gamma_d = d u / (1 - d u), u = 2^-24 (twice that, for the inputs'
    # own rounding to FP32 being taken exactly here)
    x64, r64 = x.astype(np.float64), rot.astype(np.float64)
    ref = oracle.rotate_rows(x64, r64)
    d = x.shape[1]
    u = 2.0 ** -24
    gam = d * u / (1 - d * u)
    scale = np.abs(x64) @ np.abs(r64).T
    err = np.abs(got.astype(np.float64) - ref)
    return err <= 2 * gam * scale + 1e-30


def test_rotate_permutation_is_exact(api):
    print("rotate: permutation, 5000 x 96", flush=True)
    rng = np.random.default_rng(31)
    x = rng.standard_normal((5000, 96)).astype(np.float32)
    perm = rng.permutation(96)
    P = np.eye(96, dtype=np.float32)[perm]
    out = api.rotate_rows(dev(x), dev(P)).cpu().numpy()
    assert np.array_equal(out, x[:, perm])


@pytest.mark.parametrize("n,d,dout", [(70000, 128, 128), (1001, 100, 40), (63, 7, 9), (1, 32, 32)])
def test_rotate_matches_oracle(api, n, d, dout):
    print(f"rotate: n={n} d={d} dout={dout}", flush=True)
    rng = np.random.default_rng(n + d)
    x = rng.standard_normal((n, d)).astype(np.float32)
    if dout == d:
        q, _ = np.linalg.qr(rng.standard_normal((d, d)))
        rot = q.astype(np.float32)
    else:
        rot = rng.standard_normal((dout, d)).astype(np.float32)
    out = api.rotate_rows(dev(x), dev(rot)).cpu().numpy()
    ok = within_dot_bound(out, x, rot)
    assert ok.all(), np.argwhere(~ok)[:5]


def test_rotate_across_launch_blocks(api):
    # one launch covers at most 65535 * 64 rows: rows around that boundary
    n, d = 65535 * 64 + 100, 16
    print(f"rotate: n={n} across the launch boundary", flush=True)
    rng = np.random.default_rng(7)
    x = rng.standard_normal((n, d)).astype(np.float32)
    q, _ = np.linalg.qr(rng.standard_normal((d, d)))
    rot = q.astype(np.float32)
    out = api.rotate_rows(dev(x), dev(rot))
    rows = np.r_[0:50, 65535 * 64 - 50:n]
    got = out[torch.from_numpy(rows).cuda()].cpu().numpy()
    assert within_dot_bound(got, x[rows], rot).all()


def test_rotate_errors(api):
    x = torch.zeros((10, 8), dtype=torch.float32, device="cuda")
    rot = torch.eye(8, dtype=torch.float32, device="cuda")
    assert api.rotate_rows(x[:0], rot).shape == (0, 8)
    lib = api.lib()
    # out overlapping x is refused
    rc = lib.mk_rotate_rows(x.data_ptr(), 10, 8, rot.data_ptr(), 8, x.data_ptr(), None)
    assert rc != 0
    with pytest.raises(ValueError):
        api.rotate_rows(x, torch.eye(6, dtype=torch.float32, device="cuda"))
