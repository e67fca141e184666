#!/usr/bin/env python3
"""Benchmark of the exact brute-force k-NN hot path on one MI355X.

Workload (synthetic, seeded): a 1,000,000 x 128 float32 database drawn from a
1,000-component Gaussian mixture and 10,000 queries of the same law; one step
is one L2 search of all queries for each k in {1, 32, 256, 1024} (database
norms, fused MFMA distance tiles + register k-selection, chunk merge and
direct-form re-rank).  The metric is TFLOP/s at 2 flop per multiply-add of
the q.y term, 2 * nq * nb * d per search.

Prints ONE JSON line.  Inputs are resident in device memory before timing
starts.  `roofline` reports the dominant kernel (knn_fused) timed with
HIP events inside the library over the timed steps; `cpu_baseline` times the
float64 oracle on a bounded sample of the same queries on the host cores.

Two further measurements ride along in `extra` (not part of `value`):
* `ivfpq`: a 10,000,000 x 128 mixture database, 4,096-list coarse quantizer
  and 16 x 8-bit PQ trained on a 500,000-row sample (20 iterations), 10,000
  queries, k = 100: QPS and recall@10 per nprobe in {1, 8, 32, 128}, with
  ground truth from the exact GPU search (itself parity-checked against the
  oracle), and the list-scan kernel's algorithmic code bytes per second.
* `kselect`: row-wise k-selection of 10,000 x 128,000 U[0,1) floats (5.12 GB
  resident) at k = 100 and 1,000, as GB/s of input against 8 TB/s.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
FP32_MFMA_PEAK_TFLOPS = 157.3
BF16_MFMA_PEAK_TFLOPS = 2500.0
FP8_MFMA_PEAK_TFLOPS = 5000.0
KS = (1, 32, 256, 1024)
PMC_FILE = os.path.join(ROOT, "profiles", "knn_fused_exact_large_pmc.json")
# sources of the fused kernel and its launch configuration
KERNEL_SOURCES = ["fused.hpp", "wave_select.hpp", "kselect.hpp", "knn_impl.hpp", "common.hpp"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1702_08734_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_counters(launch_flops_per_byte=None):
    """HBM bytes per launch of the dominant kernel from committed rocprofv3
    FETCH_SIZE / WRITE_SIZE counters, if they were taken on this source."""
    try:
        with open(PMC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(xq, xb, target_s: float):
    """The float64 oracle (direct-form distances, full sort per query) on a
    bounded sample of the queries against the full database: all host cores
    (OpenMP over queries) and one thread."""
    import oracle
    d = xq.shape[1]
    nb = xb.shape[0]
    cores = oracle.get_threads()

    def rate(q0, n):
        t0 = time.perf_counter()
        oracle.knn(xq[q0:q0 + n], xb, 32)
        dt = time.perf_counter() - t0
        return 2.0 * n * nb * d / dt / 1e12, dt

    _, dt = rate(0, 16)
    n_all = int(max(16, min(2000, 16 * 0.75 * target_s / max(dt, 1e-3))))
    all_rate, dt_all = rate(16, n_all)
    oracle.set_threads(1)
    try:
        _, dt = rate(16 + n_all, 1)
        n_one = int(max(1, min(200, 0.25 * target_s / max(dt, 1e-3))))
        one_rate, dt_one = rate(17 + n_all, n_one)
    finally:
        oracle.set_threads(cores)
    return {
        "value": all_rate,
        "unit": "TFLOP/s",
        "cores": cores,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "single_thread_value": one_rate,
        "sample": f"{n_all} of {xq.shape[0]} queries against the full {nb}-row database, k=32, "
                  f"on {cores} threads ({dt_all:.1f} s); single thread: {n_one} queries "
                  f"({dt_one:.1f} s). float64 direct-form distances + full sort per query",
    }


HBM_PEAK_GBS = 8000.0


T_START = time.perf_counter()


def progress(msg: str) -> None:
    print(f"[bench {time.perf_counter() - T_START:7.1f}s] {msg}", file=sys.stderr, flush=True)


def _timed(torch, fn, reps=5, warmup=1):
    """Warm-up, then `reps` timed calls each bracketed by device syncs:
    (median seconds, min seconds)."""
    import statistics
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts), min(ts)


def kselect_section(api, synth, torch):
    """Row-wise k-selection of 10,000 U[0,1) rows of length l (HBM-bound)."""
    progress("kselect: generating 10,000 x 128,000 rows")
    full = torch.from_numpy(synth.kselect_rows(10_000, 128_000)).cuda()
    res = {"rows": 10_000, "lengths": {}}
    for length in (1_000, 8_000, 32_000, 128_000):
        a = full[:, :length].contiguous() if length < full.shape[1] else full
        row = {"input_gb": round(a.numel() * 4 / 1e9, 3)}
        for k in (100, 1000):
            if k > length:
                continue
            dt, dmin = _timed(torch, lambda: api.kselect(a, k))
            gbs = (a.numel() * 4 + a.shape[0] * k * 12) / dt / 1e9
            row[f"k{k}"] = {"ms": round(dt * 1e3, 3), "ms_min": round(dmin * 1e3, 3),
                            "GB/s": round(gbs, 1),
                            "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
        res["lengths"][str(length)] = row
        del a
    return res


def small_exact_section(api, synth, torch):
    """Latency of one exact search on the 50,000 x 64 N(0,1) database with
    500 queries, k = 10 (launch-bound: 3.2 GFLOP)."""
    w = synth.exact_small()
    xb = torch.from_numpy(w["xb"]).cuda()
    xq = torch.from_numpy(w["xq"]).cuda()
    dt, dmin = _timed(torch, lambda: api.knn_search(xq, xb, w["k"]), 20, 3)
    return {"workload": "50,000 x 64 N(0,1), 500 queries, k = 10, L2",
            "latency_ms": round(dt * 1e3, 3), "latency_ms_min": round(dmin * 1e3, 3),
            "TFLOP/s": round(2 * 500 * 50_000 * 64 / dt / 1e12, 2)}


def rotate_section(api, synth, torch):
    """Row rotation (OPQ-style pre-processing): 10,000,000 x 128 FP32 rows
    times a 128 x 128 orthogonal matrix; 2 n d^2 flop against 2 n d 4 bytes,
    so the FP32 matrix cores bound it (0.34 TFLOP: 2.1 ms at 157.3 TFLOP/s;
    10.2 GB: 1.3 ms at 8 TB/s)."""
    import numpy as np
    n, d = 10_000_000, 128
    g = torch.Generator(device="cuda")
    g.manual_seed(41)
    x = torch.randn((n, d), generator=g, device="cuda", dtype=torch.float32)
    q, _ = np.linalg.qr(np.random.default_rng(41).standard_normal((d, d)))
    rot = torch.from_numpy(q.astype(np.float32)).cuda()
    dt, dmin = _timed(torch, lambda: api.rotate_rows(x, rot))
    flop = 2.0 * n * d * d
    tf = flop / dt / 1e12
    del x
    torch.cuda.empty_cache()
    return {"workload": "10,000,000 x 128 float32 rows times a 128 x 128 rotation",
            "ms": round(dt * 1e3, 3), "ms_min": round(dmin * 1e3, 3), "TFLOP/s": round(tf, 2),
            "frac_fp32_mfma_peak": round(tf / FP32_MFMA_PEAK_TFLOPS, 4),
            "GB/s": round(2 * n * d * 4 / dt / 1e9, 1)}


def lowp_section(api, synth, torch, oracle_queries=32):
    """BF16 / FP8-E4M3 brute force on the matrix cores with an exact FP32
    re-rank of the R = 4k best against FP32 brute force: 20,000,000 x 96
    unit-norm rows of a 2,000-component mixture, 10,000 queries, k = 100.
    Every variant: one warm-up, 5 timed runs (median, min).  Recall@100 and
    the relative distance error of the returned distances are taken against
    the float64 oracle on a sample of queries."""
    import numpy as np
    import oracle
    w = synth.lowp_workload()
    progress("lowp: generating 20,000,000 x 96 unit-norm mixture")
    xb_h, xq_h = w["xb"], w["xq"]
    xb = torch.from_numpy(xb_h).cuda()
    xq = torch.from_numpy(xq_h).cuda()
    k, R = w["k"], w["R"]
    nq, nb, d = xq.shape[0], xb.shape[0], xb.shape[1]
    flop = 2.0 * nq * nb * d
    sample = np.linspace(0, nq - 1, oracle_queries).astype(np.int64)
    res = {"workload": "20,000,000 x 96 unit-norm 2,000-component mixture, 10,000 queries, "
                       f"k = {k}, re-rank R = {R}",
           "oracle_sample": f"{oracle_queries} queries (evenly spaced) against the full database, "
                            "float64 direct form, full sort", "metrics": {}}

    def vs_oracle(D, I, Do, Io):
        D = D.cpu().numpy()[sample].astype(np.float64)
        I = I.cpu().numpy()[sample]
        rec = float(np.mean([len(set(I[j]) & set(Io[j])) / k for j in range(len(sample))]))
        # float64 value of the returned rows, the same index's oracle distance
        x = xq_h[sample].astype(np.float64)
        y = xb_h[I].astype(np.float64)
        if metric == "l2":
            ref = ((y - x[:, None, :]) ** 2).sum(-1)
        else:
            ref = (y * x[:, None, :]).sum(-1)
        err = np.abs(D - ref) / np.maximum(np.abs(ref), 1e-30)
        return rec, float(err.max()), float(err.mean())

    for metric in w["metrics"]:
        progress(f"lowp: oracle on {oracle_queries} queries ({metric})")
        Do, Io = oracle.knn(xq_h[sample], xb_h, k,
                            oracle.METRIC_L2 if metric == "l2" else oracle.METRIC_IP)
        progress(f"lowp: fp32 {metric}")
        t32, t32min = _timed(torch, lambda: api.knn_search(xq, xb, k, metric))
        D, I = api.knn_search(xq, xb, k, metric)
        rec, emax, emean = vs_oracle(D, I, Do, Io)
        row = {"fp32": {"ms": round(t32 * 1e3, 1), "ms_min": round(t32min * 1e3, 1),
                        "TFLOP/s": round(flop / t32 / 1e12, 2),
                        "recall_at_100_vs_oracle": round(rec, 4),
                        "max_rel_dist_err": emax, "mean_rel_dist_err": emean}}
        for prec in ("bf16", "fp8"):
            progress(f"lowp: {prec} {metric}")
            lp, inv = api.quantize_rows(xb, prec)
            dt, dmin = _timed(torch, lambda: api.knn_search_lowp(xq, xb, lp, inv, k, R, prec,
                                                                 metric))
            D, I = api.knn_search_lowp(xq, xb, lp, inv, k, R, prec, metric)
            rec, emax, emean = vs_oracle(D, I, Do, Io)
            # distances are the exact FP32 direct form of the returned rows
            row[prec] = {"ms": round(dt * 1e3, 1), "ms_min": round(dmin * 1e3, 1),
                         "TFLOP/s": round(flop / dt / 1e12, 2),
                         "frac_mfma_peak": round(flop / dt / 1e12 /
                                                 (BF16_MFMA_PEAK_TFLOPS if prec == "bf16"
                                                  else FP8_MFMA_PEAK_TFLOPS), 4),
                         "speedup_vs_fp32": round(t32 / dt, 2),
                         "recall_at_100_vs_oracle": round(rec, 4),
                         "max_rel_dist_err": emax, "mean_rel_dist_err": emean}
            del lp, inv
            torch.cuda.empty_cache()
        res["metrics"][metric] = row
    return res


def ivfpq_section(api, synth, torch):
    import numpy as np
    progress("ivfpq: generating 10,000,000 x 128 mixture")
    w = synth.ivfpq_workload()
    xb = torch.from_numpy(w["xb"]).cuda()
    xq = torch.from_numpy(w["xq"]).cuda()
    xt = xb[torch.from_numpy(w["sample"]).cuda()].contiguous()
    ix = api.IVFPQ(128, w["nlist"], w["M"])
    progress("ivfpq: training")
    t0 = time.perf_counter()
    ix.train(xt, 20, w["coarse_init"], w["pq_init"])
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    progress("ivfpq: adding")
    t0 = time.perf_counter()
    ix.add(xb)
    torch.cuda.synchronize()
    t_add = time.perf_counter() - t0
    offs, _, _ = ix.get_lists()
    sizes = np.diff(offs)
    _, gt = api.knn_search(xq, xb, 10)
    gt = gt.cpu().numpy()
    del xt
    torch.cuda.empty_cache()
    nq, k = xq.shape[0], w["k"]
    _, probe = api.knn_search(xq, torch.from_numpy(ix.get_quantizers()[0]).cuda(),
                              max(w["nprobes"]))
    probe = probe.cpu().numpy()

    def recalls(I):
        I = I.cpu().numpy()[:, :10]
        r1 = float(np.mean([gt[j, 0] in I[j] for j in range(nq)]))
        r2 = float(np.mean([len(set(gt[j]) & set(I[j])) / 10 for j in range(nq)]))
        return round(r1, 4), round(r2, 4)

    curve, rerank = [], []
    for nprobe in w["nprobes"]:
        progress(f"ivfpq: nprobe {nprobe}")
        api.profile_enable(True)
        dt, dmin = _timed(torch, lambda: ix.search(xq, k, nprobe))
        api.profile_enable(False)
        scan_ms, scan_n = api.profile_read("ivf_scan")
        r1, r2 = recalls(ix.search(xq, k, nprobe)[1])
        # algorithmic bytes: the probed lists' codes (M bytes per entry)
        scanned = int(sizes[probe[:, :nprobe]].sum())
        code_bytes = scanned * w["M"]
        scan_s = scan_ms / max(scan_n, 1) / 1e3
        curve.append({"nprobe": nprobe, "ms": round(dt * 1e3, 3), "ms_min": round(dmin * 1e3, 3),
                      "qps": round(nq / dt, 1),
                      "recall_at_10": r1, "ten_intersection": r2,
                      "scanned_codes": scanned,
                      "scan_GB/s": round(code_bytes / scan_s / 1e9, 1) if scan_s > 0 else None,
                      "scan_frac_hbm": round(code_bytes / scan_s / 1e9 / HBM_PEAK_GBS, 4)
                      if scan_s > 0 else None})
        for R in w["rerank"]:
            dt, dmin = _timed(torch, lambda: ix.search_rerank(xq, 10, nprobe, R, xb))
            r1, r2 = recalls(ix.search_rerank(xq, 10, nprobe, R, xb)[1])
            rerank.append({"nprobe": nprobe, "R": R, "ms": round(dt * 1e3, 3),
                           "ms_min": round(dmin * 1e3, 3),
                           "qps": round(nq / dt, 1), "recall_at_10": r1,
                           "ten_intersection": r2})
    scan_options = scan_options_section(api, torch, ix, xq, w, sizes, probe)
    graph = graph_section(api, torch, ix, xb, w, t_train + t_add)
    learned = learned_probe_section(api, synth, torch, ix, xb, xq, w, recalls)
    serving = serving_section(api, synth, torch, ix, xb, xq, w, learned)
    del xb
    torch.cuda.empty_cache()
    best = [c for c in curve if c["recall_at_10"] >= 0.9]
    best_rr = sorted((c for c in rerank if c["recall_at_10"] >= 0.9), key=lambda c: -c["qps"])
    return {"learned_probe": learned, "serving": serving, "knn_graph": graph,
            "scan_options": scan_options,
            "workload": "10,000,000 x 128 mixture, nlist 4096, PQ 16 x 8 bit, 10,000 queries, "
                        "k = 100 (ADC) / k = 10 after exact re-rank of R, "
                        "train 500,000 rows x 20 iterations",
            "train_s": round(t_train, 2), "add_s": round(t_add, 2),
            "list_size_mean": float(sizes.mean()), "list_size_max": int(sizes.max()),
            "curve": curve, "rerank_curve": rerank,
            "qps_at_recall10_0.9_fixed_nprobe": best[0]["qps"] if best else None,
            "nprobe_at_recall10_0.9": best[0]["nprobe"] if best else None,
            "qps_at_recall10_0.9_rerank": best_rr[0]["qps"] if best_rr else None,
            "rerank_setting_at_recall10_0.9": ({"nprobe": best_rr[0]["nprobe"],
                                                 "R": best_rr[0]["R"]} if best_rr else None)}


def scan_options_section(api, torch, ix, xq, w, sizes, probe):
    """The list scan with its options side by side at k = 100: the automatic
    grouping (as many probed lists per workgroup as keep 2048+ workgroups),
    fixed groups of 16 lists, the per-query fused scan (one workgroup per
    query over all its lists, Section 5.3), and 16-bit lookup tables; scan
    kernel time and algorithmic bytes (codes + stored term 1) per second."""
    nq, k = xq.shape[0], w["k"]
    rows = []
    for nprobe in (8, 32, 128):
        alg = int(sizes[probe[:, :nprobe]].sum()) * (w["M"] + 4)
        for label, lut, group in (("automatic", "fp32", 0), ("groups of 16", "fp32", 16),
                                  ("per-query fused", "fp32", -1), ("fp16 tables", "fp16", 0)):
            ix.set_scan_options(lut, group)
            api.profile_enable(True)
            dt, dmin = _timed(torch, lambda: ix.search(xq, k, nprobe))
            api.profile_enable(False)
            name = "ivf_scan_lut16" if lut == "fp16" else "ivf_scan"
            ms, n = api.profile_read(name)
            scan_s = ms / max(n, 1) / 1e3
            rows.append({"nprobe": nprobe, "variant": label, "search_ms": round(dt * 1e3, 3),
                         "qps": round(nq / dt, 1), "scan_ms": round(scan_s * 1e3, 3),
                         "scan_GB/s": round(alg / scan_s / 1e9, 1) if scan_s > 0 else None})
    ix.set_scan_options("fp32", 0)
    return {"k": k, "rows": rows}


def host_db_section(api, synth, torch):
    """Exact search against a database held in pinned host memory, streamed
    in chunks (copies overlapping the fused search of the previous chunk),
    next to the same search on a device-resident copy: the 10,000,000 x 128
    mixture of the IVFADC workload (5.1 GB), k = 10."""
    w = synth.ivfpq_workload(nq=10_000)
    xb_h = torch.from_numpy(w["xb"])
    pinned = torch.empty(xb_h.shape, dtype=torch.float32, pin_memory=True)
    pinned.copy_(xb_h)
    del xb_h
    xq = torch.from_numpy(w["xq"]).cuda()
    gb = pinned.numel() * 4 / 1e9
    # plain host-to-device copy rate of the same bytes
    dev = torch.empty_like(pinned, device="cuda")
    dt_copy, _ = _timed(torch, lambda: dev.copy_(pinned, non_blocking=True), 3)
    rows = []
    for nq in (1_000, 10_000):
        q = xq[:nq].contiguous()
        dt_dev, _ = _timed(torch, lambda: api.knn_search(q, dev, 10), 3)
        for chunk in (1 << 20, 1 << 21):
            progress(f"host db: nq {nq}, chunk {chunk}")
            dt, dmin = _timed(torch, lambda: api.knn_search_host(q, pinned, 10, "l2", chunk), 3)
            rows.append({"nq": nq, "chunk_rows": chunk, "ms": round(dt * 1e3, 1),
                         "ms_min": round(dmin * 1e3, 1), "device_resident_ms": round(dt_dev * 1e3, 1),
                         "effective_GB/s": round(gb / dt, 1)})
    del dev, pinned
    torch.cuda.empty_cache()
    return {"workload": "10,000,000 x 128 float32 mixture in pinned host memory (5.12 GB), k = 10",
            "h2d_copy_GB/s": round(gb / dt_copy, 1), "rows": rows}


def graph_section(api, torch, ix, xb, w, build_s):
    """k-NN graph (k = 10, a node is not its own neighbour) of every database
    vector searched against the IVFADC index, as in Section 6.5: build time
    (train + add) plus search time, and the 10-intersection with the exact
    graph on 10,000 nodes (the first 10,000 rows; the rows are i.i.d. draws).
    Settings (nprobe, R): R = 0 is the paper's ADC-only graph, R > 0 re-ranks
    an R-entry ADC short list exactly."""
    import numpy as np
    n, k, ns = xb.shape[0], 10, 10_000
    progress("knn graph: exact rows of 10,000 sample nodes")
    ge = api.knn_graph(xb, k, "l2", 0, ns)[1].cpu().numpy()
    rows = []
    for nprobe, R in w["graph_settings"]:
        progress(f"knn graph: all {n} nodes, nprobe {nprobe}, R {R}")
        ix.knn_graph(xb, k, nprobe, 0, 1_000_000, R=R)  # warm-up on a tenth
        dt, dmin = _timed(torch, lambda: ix.knn_graph(xb, k, nprobe, R=R), 3, warmup=0)
        I = ix.knn_graph(xb, k, nprobe, 0, ns, R=R)[1].cpu().numpy()
        inter = float(np.mean([len(set(I[j]) & set(ge[j])) / k for j in range(ns)]))
        rows.append({"nprobe": nprobe, "R": R, "search_s": round(dt, 3),
                     "search_s_min": round(dmin, 3), "nodes_per_s": round(n / dt, 1),
                     "end_to_end_s": round(build_s + dt, 3),
                     "ten_intersection": round(inter, 4)})
    return {"nodes": n, "k": k, "build_s": round(build_s, 3), "curve": rows,
            "quality": "10-intersection with the exact graph on 10,000 nodes",
            "timing": "one warm-up on 1,000,000 nodes, then 3 timed builds of the whole graph "
                      "(median, min)"}


def learned_probe_section(api, synth, torch, ix, xb, xq, w, recalls):
    """Learned per-query probe count vs the best fixed probe count, both with
    the same exact re-rank depth, at recall@10 >= 0.9 (true nearest
    neighbour among the 10 returned)."""
    import numpy as np
    R, cap, k, nq = w["learn_rerank"], w["learn_cap"], 10, xq.shape[0]
    # fixed probe counts with the same re-rank depth
    fixed = []
    for nprobe in w["learn_fixed_nprobes"]:
        dt, dmin = _timed(torch, lambda: ix.search_rerank(xq, k, nprobe, R, xb))
        r1, r2 = recalls(ix.search_rerank(xq, k, nprobe, R, xb)[1])
        fixed.append({"nprobe": nprobe, "ms": round(dt * 1e3, 3), "ms_min": round(dmin * 1e3, 3),
                      "qps": round(nq / dt, 1),
                      "recall_at_10": r1, "ten_intersection": r2})
    progress("learned probe: labels for training queries")
    base = w["base"]
    mix = synth.Mixture(*w["mix"])
    xtr = torch.from_numpy(mix.sample(w["learn_train"], (base, 20))).cuda()
    nn = torch.cat([api.knn_search(xtr[i:i + 20000], xb, 1)[1][:, 0]
                    for i in range(0, xtr.shape[0], 20000)]).contiguous()
    F = ix.probe_features(xtr)
    target, label = ix.probe_labels(xtr, nn, cap)
    net = api.MLP(128 + 32, 256, "bf16")
    net.set_params(synth.mlp_init(160, 256, (base, 21)))
    net.fit_standardization(F)
    progress("learned probe: training")
    t0 = time.perf_counter()
    losses = []
    for ep in range(w["learn_epochs"]):
        perm = torch.from_numpy(synth.permutation(F.shape[0], (base, 22, ep))).cuda()
        losses.append(float(net.train_epoch(F, target, perm, 1024, 1e-3).mean().item()))
    t_train = time.perf_counter() - t0
    # calibrate the offset on held-out queries: smallest delta reaching 0.9
    progress("learned probe: calibration")
    xcal = torch.from_numpy(mix.sample(10_000, (base, 23))).cuda()
    gcal = api.knn_search(xcal, xb, 1)[1][:, 0].cpu().numpy()
    def cal_recall(dlt):
        I = ix.search_learned(net, float(dlt), xcal, k, cap, R, xb)[1].cpu().numpy()
        return np.mean([gcal[j] in I[j] for j in range(len(gcal))])

    delta = None
    for dlt in np.arange(-1.0, 4.01, 0.25):
        if cal_recall(dlt) >= 0.9:
            delta = float(dlt)
            break
    if delta is not None:  # then in steps of 0.05 below it
        for dlt in np.arange(delta - 0.2, delta - 0.01, 0.05):
            if cal_recall(dlt) >= 0.9:
                delta = round(float(dlt), 2)
                break
    out = {"train_queries": int(xtr.shape[0]), "epochs": w["learn_epochs"],
           "epoch_loss": [round(v, 4) for v in losses], "train_s": round(t_train, 2),
           "label_mean": round(float(label.float().mean().item()), 2), "R": R, "cap": cap,
           "fixed": fixed, "delta": delta}
    best_fixed = [c for c in fixed if c["recall_at_10"] >= 0.9]
    out["qps_fixed_at_0.9"] = max((c["qps"] for c in best_fixed), default=None)
    if delta is not None:
        dt, dmin = _timed(torch, lambda: ix.search_learned(net, delta, xq, k, cap, R, xb))
        _, I, tau = ix.search_learned(net, delta, xq, k, cap, R, xb)
        r1, r2 = recalls(I)
        out.update({"ms": round(dt * 1e3, 3), "ms_min": round(dmin * 1e3, 3),
                    "qps_learned": round(nq / dt, 1),
                    "recall_at_10": r1, "ten_intersection": r2,
                    "mean_nprobe": round(float(tau.float().mean().item()), 2)})
    # device time per kernel of one search at the fixed count reaching 0.9 and
    # of one learned search (the rest of the wall time is launches and syncs)
    names = ("knn_fused", "knn_merge_rerank", "ivf_term3", "ivf_scan", "ivf_merge", "rerank",
             "mlp_forward")

    def breakdown(fn):
        fn()
        torch.cuda.synchronize()
        api.profile_enable(True)
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        api.profile_enable(False)
        b = {n: round(api.profile_read(n)[0], 3) for n in names}
        b["wall_ms"] = round(wall * 1e3, 3)
        return b

    if best_fixed:
        tau0 = min(c["nprobe"] for c in best_fixed)
        out["fixed_breakdown_ms"] = breakdown(lambda: ix.search_rerank(xq, k, tau0, R, xb))
    if delta is not None:
        out["learned_breakdown_ms"] = breakdown(
            lambda: ix.search_learned(net, delta, xq, k, cap, R, xb))
    out["net"] = net
    return out


def serving_section(api, synth, torch, ix, xb, xq, w, learned):
    """Continuous batching under Poisson arrivals: requests of log-uniform size
    in [1, 1024] rows, k = 10, exact re-rank; latency percentiles per rate."""
    import threading
    import numpy as np
    net = learned.pop("net", None)
    R, k = w["learn_rerank"], 10
    delta = learned.get("delta")
    cfg = {"R": R, "xb": xb, "max_batch": 1024, "nstreams": 2}
    if net is not None and delta is not None:
        cfg.update({"net": net, "delta": delta, "cap": w["learn_cap"]})
        mode = "learned probe count"
    else:
        best = [c for c in learned["fixed"] if c["recall_at_10"] >= 0.9]
        cfg["nprobe"] = best[0]["nprobe"] if best else max(w["learn_fixed_nprobes"])
        mode = f"fixed probe count {cfg['nprobe']}"
    xq_h = xq.cpu().numpy()
    nreq = w["serve_requests"]
    rng = np.random.default_rng(np.random.SeedSequence((w["base"], 24)))
    sizes = np.clip(np.floor(np.exp(rng.random(nreq) * np.log(1025))), 1, 1024).astype(int)
    starts = rng.integers(0, xq_h.shape[0] - 1024, nreq)
    gaps = rng.exponential(1.0, nreq)
    # saturated throughput: everything submitted at once
    srv = api.Server(ix, k, **cfg)
    t0 = time.perf_counter()
    tk = [srv.submit(xq_h[s:s + n]) for s, n in zip(starts, sizes)]
    for t in tk:
        srv.wait(t)
    peak_rows = sizes.sum() / (time.perf_counter() - t0)
    srv.close()
    res = {"mode": mode, "requests": nreq, "mean_rows": round(float(sizes.mean()), 1),
           "saturated_rows_per_s": round(float(peak_rows), 1), "rates": []}
    for frac in w["serve_load"]:
        progress(f"serving: load {frac}")
        lam = frac * peak_rows / sizes.mean()  # requests per second
        srv = api.Server(ix, k, **cfg)
        tickets = [None] * nreq
        lat = [0.0] * nreq
        done = threading.Event()

        def collect():
            for i in range(nreq):
                while tickets[i] is None:
                    time.sleep(1e-4)
                lat[i] = srv.wait(tickets[i])[2]
            done.set()

        th = threading.Thread(target=collect)
        th.start()
        t0 = time.perf_counter()
        t_arr = t0
        for i in range(nreq):
            t_arr += gaps[i] / lam
            pause = t_arr - time.perf_counter()
            if pause > 0:
                time.sleep(pause)
            tickets[i] = srv.submit(xq_h[starts[i]:starts[i] + sizes[i]])
        th.join()
        wall = time.perf_counter() - t0
        nb, _ = srv.stats()
        srv.close()
        ms = np.array(lat) * 1e3
        res["rates"].append({"load": frac, "offered_rows_per_s": round(float(lam * sizes.mean()), 1),
                             "achieved_rows_per_s": round(float(sizes.sum() / wall), 1),
                             "batches": nb, "p50_ms": round(float(np.percentile(ms, 50)), 3),
                             "p99_ms": round(float(np.percentile(ms, 99)), 3)})
    return res


def build_large_index(api, synth, torch):
    """The 50,000,000 x 128 IVFADC index (16,384 lists, PQ 16 x 8 bit) with its
    database and queries resident on the device."""
    progress("ivf-large: generating 50,000,000 x 128 mixture")
    w = synth.ivfpq_large_workload()
    xb = torch.from_numpy(w["xb"]).cuda()
    del w["xb"]
    xq = torch.from_numpy(w["xq"]).cuda()
    xt = xb[torch.from_numpy(w["sample"]).cuda()].contiguous()
    ix = api.IVFPQ(128, w["nlist"], w["M"])
    progress("ivf-large: training")
    t0 = time.perf_counter()
    ix.train(xt, 20, w["coarse_init"], w["pq_init"])
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del xt
    progress("ivf-large: adding")
    t0 = time.perf_counter()
    ix.add(xb)
    torch.cuda.synchronize()
    t_add = time.perf_counter() - t0
    return w, ix, xb, xq, t_train, t_add


def ivf_large_run(api, synth, torch):
    """IVFADC at 50,000,000 x 128 (16,384 lists, PQ 16): the ADC scan curve
    (codes 800 MB, more than the 256 MB last-level cache, so list scans read
    HBM), fixed vs learned probe count at R@10 >= 0.9 with the same exact
    re-rank depth, and serving latencies."""
    import numpy as np
    w, ix, xb, xq, t_train, t_add = build_large_index(api, synth, torch)
    progress("ivf-large: ground truth")
    gt = api.knn_search(xq, xb, 10)[1].cpu().numpy()
    nq = xq.shape[0]
    offs, _, _ = ix.get_lists()
    sizes = np.diff(offs)
    _, probe = api.knn_search(xq, torch.from_numpy(ix.get_quantizers()[0]).cuda(), 64)
    probe = probe.cpu().numpy()

    def recalls(I):
        I = I.cpu().numpy()[:, :10]
        r1 = float(np.mean([gt[j, 0] in I[j] for j in range(nq)]))
        r2 = float(np.mean([len(set(gt[j]) & set(I[j])) / 10 for j in range(nq)]))
        return round(r1, 4), round(r2, 4)

    curve = []
    for nprobe in (8, 32, 64):
        progress(f"ivf-large: ADC scan nprobe {nprobe}")
        api.profile_enable(True)
        dt, dmin = _timed(torch, lambda: ix.search(xq, 100, nprobe))
        api.profile_enable(False)
        scan_ms, scan_n = api.profile_read("ivf_scan")
        scanned = int(sizes[probe[:, :nprobe]].sum())
        alg = scanned * (w["M"] + 4)  # code bytes + stored term 1 per entry
        scan_s = scan_ms / max(scan_n, 1) / 1e3
        r1, r2 = recalls(ix.search(xq, 100, nprobe)[1])
        curve.append({"nprobe": nprobe, "k": 100, "ms": round(dt * 1e3, 3),
                      "ms_min": round(dmin * 1e3, 3), "qps": round(nq / dt, 1),
                      "recall_at_10": r1, "ten_intersection": r2, "scanned_entries": scanned,
                      "scan_ms": round(scan_s * 1e3, 3),
                      "scan_GB/s": round(alg / scan_s / 1e9, 1) if scan_s > 0 else None,
                      "scan_frac_hbm": round(alg / scan_s / 1e9 / HBM_PEAK_GBS, 4)
                      if scan_s > 0 else None})
    learned = learned_probe_section(api, synth, torch, ix, xb, xq, w, recalls)
    serving = serving_section(api, synth, torch, ix, xb, xq, w, learned)
    del xb
    torch.cuda.empty_cache()
    return {"metric": "IVFADC queries/s at R@10 >= 0.9 (learned vs fixed probe count, exact re-rank)",
            "workload": "50,000,000 x 128 1,000-component mixture, nlist 16384, PQ 16 x 8 bit, "
                        f"10,000 queries, k = 10, re-rank R = {w['learn_rerank']}",
            "train_s": round(t_train, 2), "add_s": round(t_add, 2),
            "list_size_mean": float(sizes.mean()), "list_size_max": int(sizes.max()),
            "adc_curve": curve, "learned_probe": learned, "serving": serving}


def ivf_large_scan_profile(api, synth, torch):
    """Only the ADC list scans of the 50,000,000-vector index at nprobe 16
    and 64 (for hardware-counter runs restricted to the scan kernel)."""
    import numpy as np
    w, ix, xb, xq, _, _ = build_large_index(api, synth, torch)
    offs, _, _ = ix.get_lists()
    sizes = np.diff(offs)
    _, probe = api.knn_search(xq, torch.from_numpy(ix.get_quantizers()[0]).cuda(), 64)
    probe = probe.cpu().numpy()
    out = {"profiled": "ivf_scan at nprobe 16 and 64, 3 searches each, 10,000 queries, k = 100",
           "algorithmic_bytes_per_search": {}}
    for nprobe in (16, 64):
        progress(f"ivf-large scan profile: nprobe {nprobe}")
        for _ in range(3):
            ix.search(xq, 100, nprobe)
        torch.cuda.synchronize()
        scanned = int(sizes[probe[:, :nprobe]].sum())
        out["algorithmic_bytes_per_search"][str(nprobe)] = {
            "scanned_entries": scanned, "bytes": scanned * (w["M"] + 4)}
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--skip-extra", action="store_true",
                    help="only the exact-search measurement (for profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 1 GiB device to device (HBM byte-counter calibration)")
    ap.add_argument("--ivf-large", action="store_true",
                    help="only the 50,000,000-vector IVFADC learned-probe and serving run")
    ap.add_argument("--ivf-large-scan", action="store_true",
                    help="only the list scans of the 50,000,000-vector index (profiling)")
    ap.add_argument("--skip-large", action="store_true",
                    help="leave out the 50,000,000-vector IVFADC section")
    ap.add_argument("--section", default=None,
                    help="only this extra section (small_exact, kselect, ivfpq, lowp, ivf_large, host_db, "
                         "rotate), "
                         "for profiling runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); multi-GPU runs are "
              "not part of this build", file=sys.stderr)
        return 2

    import torch
    if args.copy_calibration:
        x = torch.ones(1 << 28, device="cuda")  # 1 GiB read + 1 GiB written by one copy
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4}))
        return 0
    from paper_1702_08734_amd import api, synth

    if args.ivf_large:
        print(json.dumps(ivf_large_run(api, synth, torch)), flush=True)
        return 0
    if args.ivf_large_scan:
        print(json.dumps(ivf_large_scan_profile(api, synth, torch)), flush=True)
        return 0
    if args.section:
        fns = {"small_exact": small_exact_section, "kselect": kselect_section,
               "ivfpq": ivfpq_section, "lowp": lowp_section, "ivf_large": ivf_large_run,
               "host_db": host_db_section, "rotate": rotate_section}
        print(json.dumps({args.section: fns[args.section](api, synth, torch)}), flush=True)
        return 0

    progress("exact: generating 1,000,000 x 128 mixture")
    w = synth.exact_large()
    xq_h, xb_h = w["xq"], w["xb"]
    nq, d = xq_h.shape
    nb = xb_h.shape[0]
    xq = torch.from_numpy(xq_h).cuda()
    xb = torch.from_numpy(xb_h).cuda()
    torch.cuda.synchronize()

    def step():
        for k in KS:
            api.knn_search(xq, xb, k)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # per-k timing (not part of the reported value)
    per_k = {}
    for k in KS:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        api.knn_search(xq, xb, k)
        torch.cuda.synchronize()
        per_k[str(k)] = round((time.perf_counter() - t0) * 1e3, 3)

    api.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    api.profile_enable(False)
    tile_ms, tile_n = api.profile_read("knn_fused")
    merge_ms, merge_n = api.profile_read("knn_merge_rerank")

    flops_search = 2.0 * nq * nb * d
    flops_step = flops_search * len(KS)
    value = flops_step * args.steps / elapsed / 1e12
    achieved = flops_search * tile_n / (tile_ms / 1e3) / 1e12 if tile_ms > 0 else None
    traffic = traffic_from_counters()
    out = {
        "metric": "brute-force k-NN TFLOP/s (exact L2, fused MFMA distance + k-selection)",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "exact_large: 1,000,000 x 128 float32 database from a 1,000-component "
                        "Gaussian mixture, 10,000 queries, L2, one search per k in "
                        "{1, 32, 256, 1024}",
            "nb": nb, "nq": nq, "d": d, "ks": list(KS),
        },
        "roofline": {
            "bound": "mfma",
            "kernel": "knn_fused",
            "achieved": round(achieved, 3) if achieved else None,
            "peak": FP32_MFMA_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / FP32_MFMA_PEAK_TFLOPS, 4) if achieved else None,
            "traffic": traffic,
            "launch_ms_avg": round(tile_ms / max(tile_n, 1), 4),
            "launches": tile_n,
        },
        "extra": {
            "per_k_ms": per_k,
            "merge_rerank_ms_avg": round(merge_ms / max(merge_n, 1), 4),
        },
    }
    progress(f"exact: {value:.2f} TFLOP/s")
    if not args.no_cpu_baseline:
        progress("cpu baseline")
        out["cpu_baseline"] = cpu_baseline(xq_h, xb_h, args.cpu_seconds)
    del xq, xb
    torch.cuda.empty_cache()
    if not args.skip_extra:
        sections = [("small_exact", small_exact_section), ("kselect", kselect_section),
                    ("ivfpq", ivfpq_section), ("lowp", lowp_section),
                    ("host_db", host_db_section), ("rotate", rotate_section)]
        if not args.skip_large:
            sections.append(("ivf_large", ivf_large_run))
        for name, fn in sections:
            try:
                out["extra"][name] = fn(api, synth, torch)
            except Exception as e:  # the headline value stands on its own
                out["extra"][name] = {"error": repr(e)[:300]}
            torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
