"""Comparison of GPU k-NN results with the float64 oracle ("band rule").

Indices must match the oracle exactly except where the oracle's distance
gap to the rank-k value is within the FP32 tolerance (1e-5 relative):

 1. D is sorted in metric order and I holds no duplicates besides -1 padding;
 2. every returned distance is within tol_i of the oracle's float64
    distance of that same index: for L2, tol_i = RTOL * max(|delta_i|,
    1e-3 * (||x||^2 + ||y_i||^2)) (the floor only matters for near-zero
    distances); for inner products tol_i = max(RTOL * |delta_i|,
    gamma_d * sum_t |x_t y_it|), gamma_d = d u / (1 - d u), u = 2^-24: an
    FP32 dot product of d terms, summed in any order with each partial sum
    rounded once, is off by at most gamma_d * sum |x_t y_t| (the standard
    bound for floating-point summation), which a near-zero inner product of
    large vectors cannot beat, so no tolerance below it is attainable;
 3. with d_k the oracle's k-th value and B the band of indices i whose
    oracle distance is within the pair tolerance of d_k, max(RTOL * |d_k|,
    floor_i + floor_k) (floor: the absolute part of tol above; two FP32
    values each carry their own error, so their difference can be off by
    the sum):  oracle_set \\ B  <=  gpu_set  <=  oracle_set | B;
 4. at every rank whose oracle value is separated from both neighbours by
    more than the pair tolerance the index is the oracle's (values closer
    than the FP32 error bound can be ordered either way by any FP32
    computation);
 5. equal GPU distances come out in increasing index order.
"""
from __future__ import annotations

import numpy as np

import oracle

RTOL = 1e-5


U32 = 2.0 ** -24


def gamma(n):
    """Bound factor of an n-term FP32 sum of exact products: n u / (1 - n u)."""
    return n * U32 / (1.0 - n * U32)


def _tol(v, floor):
    """max(RTOL * |v|, floor): floor is absolute."""
    return np.maximum(RTOL * np.abs(v), floor)


def floor_abs(x, y, metric_l2):
    """Absolute tolerance floor for query x (float64 [d]) against rows y
    (float64 [n, d]): RTOL * 1e-3 (||x||^2 + ||y||^2) for L2, gamma_d *
    sum_t |x_t y_t| for inner products."""
    if metric_l2:
        return RTOL * 1e-3 * ((x * x).sum() + (y * y).sum(-1))
    return gamma(x.shape[-1]) * np.abs(y * x).sum(-1)


def check_rows(D, I, xq, xb, qrows, k, metric="l2", extra=64, oracle_result=None):
    """Check GPU rows D[j], I[j] for the queries xq[qrows[j]] (band rule).

    D, I: numpy [len(qrows), k]; xq, xb: float32 numpy arrays.
    oracle_result: optional (Do, Io) of oracle.knn for these rows with at
    least k + extra columns (reused across k).
    Returns a list of failure strings (empty when everything holds).
    """
    m = oracle.METRIC_L2 if metric == "l2" else oracle.METRIC_IP
    nb = xb.shape[0]
    k2 = min(k + extra, nb) if nb else k
    if oracle_result is not None:
        Do, Io = oracle_result[0][:, :max(k2, 1)], oracle_result[1][:, :max(k2, 1)]
    else:
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
        l2 = m == oracle.METRIC_L2
        delta = ((y - x) ** 2).sum(1) if l2 else y @ x
        bad = np.abs(gd - delta) > _tol(delta, floor_abs(x, y, l2))
        if np.any(bad):
            r = int(np.nonzero(bad)[0][0])
            fails.append(f"q{q}: rank {r} id {gi[r]} D={gd[r]!r} oracle={delta[r]!r}")
        # 3. sets up to the band at rank k
        od = Do[j]
        oi = Io[j]
        kk = exp_valid
        dk = od[kk - 1]
        nor = min(k2, nb)
        yo = xb[oi[:nor]].astype(np.float64)
        flo = floor_abs(x, yo, l2)
        inband = np.abs(od[:nor] - dk) <= _tol(dk, flo + flo[kk - 1])
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
        for r in range(kk):
            lo_ok = r == 0 or abs(od[r] - od[r - 1]) > _tol(od[r], flo[r] + flo[r - 1])
            hi_ok = r + 1 >= nor or abs(od[r + 1] - od[r]) > _tol(od[r], flo[r] + flo[r + 1])
            if lo_ok and hi_ok and gi[r] != oi[r]:
                fails.append(f"q{q}: rank {r} id {gi[r]} != oracle {oi[r]}")
                break
        # 5. exact ties in index order
        same = gd[1:] == gd[:-1]
        if np.any(same & (gi[1:] < gi[:-1])):
            fails.append(f"q{q}: equal distances out of index order")
    return fails
