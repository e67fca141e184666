"""Comparison of GPU k-NN results with the float64 oracle ("band rule").

Indices must match the oracle exactly except where the oracle's distance
gap to the rank-k value is within the FP32 tolerance (1e-5 relative):

 1. D is sorted in metric order and I holds no duplicates besides -1 padding;
 2. every returned distance is within RTOL * max(|delta_i|, phi_i) of the
    oracle's float64 distance of that same index, phi_i being
    1e-3 * (||x||^2 + ||y_i||^2) for L2 (a floor that only matters for
    near-zero distances) and sum_t |x_t y_t| for inner products (the scale
    of the FP32 rounding error of a dot product, which a near-zero inner
    product of large vectors cannot beat);
 3. with d_k the oracle's k-th value and B the band of indices whose oracle
    distance is within tolerance of d_k:
    oracle_set \\ B  <=  gpu_set  <=  oracle_set | B;
 4. at every rank whose oracle value is separated from both neighbours by
    more than the tolerance the index is the oracle's;
 5. equal GPU distances come out in increasing index order.
"""
from __future__ import annotations

import numpy as np

import oracle

RTOL = 1e-5


def _tol(v, phi):
    return RTOL * np.maximum(np.abs(v), phi)


def check_rows(D, I, xq, xb, qrows, k, metric="l2", extra=64):
    """Check GPU rows D[j], I[j] for the queries xq[qrows[j]] (band rule).

    D, I: numpy [len(qrows), k]; xq, xb: float32 numpy arrays.
    Returns a list of failure strings (empty when everything holds).
    """
    m = oracle.METRIC_L2 if metric == "l2" else oracle.METRIC_IP
    nb = xb.shape[0]
    k2 = min(k + extra, nb) if nb else k
    Do, Io = oracle.knn(xq[qrows], xb, max(k2, 1), m)
    fails = []
    for j, q in enumerate(qrows):
        x = xq[q].astype(np.float64)
        g_I = I[j]
        g_D = D[j].astype(np.float64)
        valid = g_I >= 0
        nvalid = int(valid.sum())
        exp_valid = min(k, nb)
        if nvalid != exp_valid or not np.all(valid[:nvalid]):
            fails.append(f"q{q}: {nvalid} valid results, expected {exp_valid}")
            continue
        pad_ok = np.all(np.isinf(g_D[nvalid:])) and (
            np.all(g_D[nvalid:] > 0) if m == oracle.METRIC_L2 else np.all(g_D[nvalid:] < 0))
        if not pad_ok:
            fails.append(f"q{q}: bad padding")
        gi = g_I[:nvalid]
        gd = g_D[:nvalid]
        if len(set(gi.tolist())) != nvalid:
            fails.append(f"q{q}: duplicate indices")
        if nvalid == 0:
            continue
        if m == oracle.METRIC_L2:
            if np.any(np.diff(gd) < 0):
                fails.append(f"q{q}: D not ascending")
        else:
            if np.any(np.diff(gd) > 0):
                fails.append(f"q{q}: D not descending")
        # 2. distances of the returned indices
        y = xb[gi].astype(np.float64)
        if m == oracle.METRIC_L2:
            delta = ((y - x) ** 2).sum(1)
            phi = 1e-3 * ((x * x).sum() + (y * y).sum(1))
        else:
            delta = y @ x
            phi = np.abs(y * x).sum(1)
        bad = np.abs(gd - delta) > _tol(delta, phi)
        if np.any(bad):
            r = int(np.nonzero(bad)[0][0])
            fails.append(f"q{q}: rank {r} id {gi[r]} D={gd[r]!r} oracle={delta[r]!r}")
        # 3. sets up to the band at rank k
        od = Do[j]
        oi = Io[j]
        kk = exp_valid
        dk = od[kk - 1]
        yk = xb[oi[kk - 1]].astype(np.float64)
        phik = 1e-3 * ((x * x).sum() + (yk * yk).sum()) if m == oracle.METRIC_L2 else \
            np.abs(yk * x).sum()
        tolk = _tol(dk, phik)
        nor = min(k2, nb)
        inband = np.abs(od[:nor] - dk) <= tolk
        if nor > kk and inband[nor - 1] and nor < nb:
            fails.append(f"q{q}: band wider than the oracle's extra candidates")
        band = set(oi[:nor][inband].tolist())
        oset = set(oi[:kk].tolist())
        gset = set(gi.tolist())
        if not (oset - band) <= gset:
            fails.append(f"q{q}: missing {sorted((oset - band) - gset)[:5]}")
        if not gset <= (oset | band):
            fails.append(f"q{q}: extra {sorted(gset - (oset | band))[:5]}")
        # 4. isolated ranks
        yo = xb[oi[:nor]].astype(np.float64)
        phio = 1e-3 * ((x * x).sum() + (yo * yo).sum(1)) if m == oracle.METRIC_L2 else \
            np.abs(yo * x).sum(1)
        for r in range(kk):
            tr = _tol(od[r], phio[r])
            lo_ok = r == 0 or abs(od[r] - od[r - 1]) > tr
            hi_ok = r + 1 >= nor or abs(od[r + 1] - od[r]) > tr
            if lo_ok and hi_ok and gi[r] != oi[r]:
                fails.append(f"q{q}: rank {r} id {gi[r]} != oracle {oi[r]}")
                break
        # 5. exact ties in index order
        same = gd[1:] == gd[:-1]
        if np.any(same & (gi[1:] < gi[:-1])):
            fails.append(f"q{q}: equal distances out of index order")
    return fails
