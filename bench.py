#!/usr/bin/env python3
"""Benchmark: exact k-NN queries/s on one MI355X (plain float32 path).

Workload (the plain-FP32 configuration): 10,000,000 z-normalised random-walk
series of length 256 (float32, ~10 GB resident in HBM), 300 queries -- 100
each built from dataset series with 1 %, 5 % and 10 % Gaussian noise (variance
labels), re-normalised -- iSAX w = 16 at alphabet 256, leaves of 10,000
series, k = 10 (k = 1 reported beside it).  One step answers the whole
300-query batch through the C ABI; inputs are resident in HBM before timing.

The JSON line also carries:
  roofline      the leaf-scan kernel (LB_SAX filter + refinement, the dominant
                kernel): algorithmic bytes it must read per launch (iSAX words
                of the series it filters, 256-byte chunks of the series it
                refines) over its average launch duration, timed with HIP
                events on the stream it runs on, against the 8 TB/s HBM peak;
  cpu_baseline  the FP64 oracle (C/OpenMP brute force) timed on the host cores
                on a bounded sample of the same queries;
  latency_ms    p50/p99 of single-query calls.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "exact k-NN queries/s at 1 GPU (plain FP32 vs BF16-bound+FP32 refine) + p99 latency"
HBM_PEAK_GBS = 8000.0
COPY_CAL_BYTES = 1 << 30


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


# HBM byte counters of the scan kernels, taken with rocprofv3 --pmc and scaled by
# a plain copy kernel (the summary holds the commands and the raw figures).  They
# count only while the kernel's sources hash to the recorded value.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_scan_kernels_random_walk_10Mx256.txt")
KERNEL_SOURCES = {
    "k_filter": ["hs_filter.hip", "hs_device.h", "hs_internal.h"],
    "k_refine": ["hs_refine.hip", "hs_device.h", "hs_internal.h"],
    "k_bound": ["hs_precision.hip", "hs_device.h", "hs_internal.h"],
}


def kernel_source_hash(kernel):
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2212_13297_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None."""
    if kernel not in KERNEL_SOURCES or not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if "=" in line and not line.lstrip().startswith("#"):
                key, val = line.split("=", 1)
                kv[key.strip()] = val.strip()
    if any(kv.get(f"workload.{key}") != str(val) for key, val in workload.items()):
        return None
    if kv.get(f"{kernel}.source_sha256") != kernel_source_hash(kernel):
        return None
    try:
        fetch = int(kv[f"{kernel}.fetch_bytes_per_launch"])
        write = int(kv[f"{kernel}.write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None
    return {"bytes_per_launch": fetch + write, "fetch": fetch, "write": write,
            "copy_scale": float(kv.get("copy.scale", "nan")), "source": os.path.basename(TRAFFIC_FILE)}


MFMA_PEAK_TFLOPS = {"bf16": 2500.0, "fp16": 2500.0}
# LDS: 256 compute units x 32 banks x one 4-byte access per bank per clock x 2.4 GHz
LDS_PEAK_TLOOKUPS = 256 * 32 * 2.4e9 / 1e12
_LDS_PROBE = {}


def lds_probe(hs):
    """Achievable LDS lookup rates (T/s), measured once per process: 16 lookups
    per round into a 16 x 256 table, conflict-free and at random symbols."""
    if not _LDS_PROBE:
        _LDS_PROBE["conflict_free"] = round(hs.lds_probe_tps(0) / 1e12, 3)
        _LDS_PROBE["random"] = round(hs.lds_probe_tps(1) / 1e12, 3)
        log(f"LDS lookup probe: {_LDS_PROBE} T/s")
    return dict(_LDS_PROBE)


def run_mixed(hs, torch, idx, qt, k, steps, warmup, wl, plain_ids, plain_d2, build=True):
    """Precision form on the same index and batch: bf16 copy of the series
    (unless the caller built a copy already), matrix-core bounding pass,
    compensated float32 refinement."""
    Q = qt.shape[0]
    t0 = time.time()
    if build:
        idx.build_shadow(hs.HS_SHADOW_BF16)
    torch.cuda.synchronize()
    shadow_s = time.time() - t0
    for _ in range(warmup):
        idx.knn_mixed(qt, k)
    torch.cuda.synchronize()
    hs.profile_read_all(reset=True)
    hs.hs_profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        ids, d2, err, st = idx.knn_mixed(qt, k, stats=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hs.hs_profile_enable(False)
    prof = hs.profile_read_all(reset=True)
    ms = (t1 - t0) * 1000.0 / steps
    qps = Q / (ms / 1000.0)
    log(f"precision form: {ms:.3f} ms/step, {qps:.0f} queries/s; kernels {prof}")
    same = int((ids == plain_ids).all(dim=1).sum().item())
    same_d = bool(torch.equal(d2.view(torch.int32), plain_d2.view(torch.int32)))
    stats = {f: v.cpu().numpy().astype(np.int64) for f, v in st.items()}
    info = idx.info
    K = info.row_stride
    kern = {}
    bms, bl = prof["bound"]
    if bl:
        avg = bms / bl
        # algorithmic work of the bounding pass: one q~.x~ (2K flop) per bounded
        # (query, series) pair; the low-precision rows and norms it must read once
        flops = 2.0 * K * float(stats["rows_bounded"].sum()) / (bl / steps)
        # what the matrix cores computed: every (query, series) pair of the
        # tiles each wavefront of 32 queries took (padding queries not counted)
        xflops = 2.0 * K * float(stats["bound_pairs"].sum()) / (bl / steps)
        kern["bound"] = {"avg_launch_ms": round(avg, 4), "launches_per_step": bl / steps,
                         "flops_per_launch": int(flops),
                         "TFLOP_s": round(flops / (avg / 1e3) / 1e12, 2),
                         "executed_flops_per_launch": int(xflops),
                         "executed_TFLOP_s": round(xflops / (avg / 1e3) / 1e12, 2),
                         "shadow_bytes": int(info.n_series * (2 * K + 16)),
                         "shadow_GB_s": round(info.n_series * (2 * K + 16) / (avg / 1e3) / 1e9, 2)}
    rms, rl = prof["refine"]
    if rl:
        avg = rms / rl
        nbytes = (int(stats["chunks_read"].sum()) * 256 + int(stats["candidates"].sum()) * 12) / (rl / steps)
        kern["refine"] = {"avg_launch_ms": round(avg, 4), "launches_per_step": rl / steps,
                          "bytes_per_launch": int(nbytes), "GB_s": round(nbytes / (avg / 1e3) / 1e9, 2)}
    traffic = measured_traffic("k_bound", wl)
    low = "fp16" if idx.shadow_kind == hs.HS_SHADOW_FP16 else "bf16"
    out = {"value": round(qps, 2), "unit": "queries/s", "ms_per_step": round(ms, 4),
           "dtype": f"{low} bound, f32 compensated refine",
           "identical_id_lists_vs_plain": same, "identical_distances_vs_plain": same_d, "queries": Q,
           "max_err_bound_rel": float((err / d2.double()).max().item()),
           "shadow_build_s": round(shadow_s, 2),
           "kernels": kern,
           "roofline": ({"bound": "mfma", "achieved": kern["bound"]["TFLOP_s"], "peak": MFMA_PEAK_TFLOPS[low],
                         "unit": "TFLOP/s", "frac": round(kern["bound"]["TFLOP_s"] / MFMA_PEAK_TFLOPS[low], 4),
                         "executed_frac": round(kern["bound"]["executed_TFLOP_s"] / MFMA_PEAK_TFLOPS[low], 4),
                         "kernel": "k_bound", "traffic": traffic.get("bytes_per_launch") if traffic else None,
                         "traffic_detail": traffic} if "bound" in kern else None),
           "pruning": {"rows_bounded_mean": float(stats["rows_bounded"].mean()),
                       "rows_filtered_mean": float(stats["rows_filtered"].mean()),
                       "candidates_mean": float(stats["candidates"].mean()),
                       "rows_refined_mean": float(stats["rows_refined"].mean()),
                       "rounds_max": int(stats["rounds"].max())}}
    log(f"precision form: {out}")
    return out


def measure_plain(hs, torch, idx, qt, k, steps, warmup, w, wl, read_gbs):
    """The plain form's timed steps (inputs resident in HBM), the scan kernels'
    event-timed launches, and the algorithmic bytes both per (query, unit)
    pair and as the batch union (distinct units read, one untimed call with
    the marking kernels)."""
    Q = qt.shape[0]
    info = idx.info
    for _ in range(warmup):
        idx.knn(qt, k)
    torch.cuda.synchronize()
    hs.profile_read_all(reset=True)
    hs.hs_profile_enable(True)
    log(f"timing {steps} steps, Q={Q}, k={k}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ids, d2, st = idx.knn(qt, k, stats=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hs.hs_profile_enable(False)
    prof = hs.profile_read_all(reset=True)
    ms_per_step = (t1 - t0) * 1000.0 / steps
    qps = Q / (ms_per_step / 1000.0)
    log(f"{ms_per_step:.3f} ms/step, {qps:.0f} queries/s; scan kernels {prof}")
    stats = {f: v.cpu().numpy().astype(np.int64) for f, v in st.items()}
    # per pair: what each (query, unit) pair reads (the seed step's series included)
    word_bytes = int(stats["rows_filtered"].sum()) * w + int(stats["chunks_tested"].sum()) * w * 16
    sig_bytes = int(stats["rows_sigma"].sum()) * w  # deviation codes of the LB_SAX survivors
    cand_bytes = int(stats["candidates"].sum()) * 12
    raw_bytes = int(stats["chunks_read"].sum()) * 64 * 4
    # batch union: distinct (series, chunk) pairs the refine reads, distinct
    # words and chunk envelopes the filter reads; deviation codes and candidate
    # entries are counted per pair
    ust = {}

    def ucall():
        ust["st"] = idx.knn(qt, k, stats=True)[2]

    u_raw, u_words, u_env = hs.union_counts(idx, ucall)
    u_cand = int(ust["st"]["candidates"].sum().item()) * 12
    u_sig = int(ust["st"]["rows_sigma"].sum().item()) * w
    union = {"filter": u_words * w + u_env * w * 16 + u_sig + u_cand, "refine": u_raw * 256 + u_cand}
    pair = {"filter": word_bytes + sig_bytes + cand_bytes, "refine": raw_bytes + cand_bytes}
    log(f"batch union: {u_raw} raw chunk pairs, {u_words} words, {u_env} envelopes "
        f"(per pair: {stats['chunks_read'].sum()}, {stats['rows_filtered'].sum()}, {stats['chunks_tested'].sum()})")
    kern = {}
    for name in ("filter", "refine"):
        kms, launches = prof[name]
        if launches:
            avg = kms / launches
            per = launches / steps
            ub, pb = union[name] / per, pair[name] / per
            kern[name] = {"avg_launch_ms": round(avg, 4), "launches_per_step": per,
                          "bytes_per_launch": int(ub), "GB_s": round(ub / (avg / 1e3) / 1e9, 2),
                          "bytes_per_launch_per_pair": int(pb), "GB_s_per_pair": round(pb / (avg / 1e3) / 1e9, 2)}
    if "filter" in kern:
        # its words (w B per series) and chunk envelopes come back for every query
        # that keeps their leaf and are served mostly from the 256 MB Infinity
        # Cache; its time goes to the LB_SAX table lookups in LDS (one 4-byte
        # lookup per segment per filtered (query, series) pair) and VALU work
        kms, launches = prof["filter"]
        avg = kms / launches
        lookups = int(stats["rows_filtered"].sum()) * w / (launches / steps)
        probe = lds_probe(hs)
        tps = lookups / (avg / 1e3) / 1e12
        kern["filter"].update({"bound": "lds", "lds_lookups_per_launch": int(lookups),
                               "lds_lookups_T_s": round(tps, 3),
                               "lds_frac": round(tps / LDS_PEAK_TLOOKUPS, 4),
                               "achievable_lookups_T_s": probe,
                               "frac_of_achievable_random": round(tps / probe["random"], 4)})
    if "refine" in kern:
        kern["refine"]["bound"] = "hbm"
    dom = max(kern, key=lambda n: kern[n]["avg_launch_ms"] * kern[n]["launches_per_step"]) if kern else None
    traffic = measured_traffic(f"k_{dom}", wl) if dom else None
    env_union = info.n_leaves * w * 16              # leaf envelopes: read once per batch
    out_bytes = Q * k * 12
    path_union = union["filter"] + union["refine"] + env_union + out_bytes
    path_pair = word_bytes + sig_bytes + raw_bytes + Q * info.n_leaves * w * 16 + out_bytes
    if dom == "filter":
        kf = kern["filter"]
        roof = {**kf, "bound": "lds", "achieved": kf["lds_lookups_T_s"], "peak": LDS_PEAK_TLOOKUPS,
                "unit": "T lookups/s", "frac": kf["lds_frac"],
                "work": "one 4-byte LB_SAX table lookup per segment per filtered (query, series) pair",
                "hbm_union_GB_s": kf["GB_s"], "hbm_union_frac": round(kf["GB_s"] / HBM_PEAK_GBS, 4),
                "traffic": traffic.get("bytes_per_launch") if traffic else None, "traffic_detail": traffic,
                "kernel": "k_filter"}
    elif dom == "refine":
        kr = kern["refine"]
        roof = {**kr, "bound": "hbm", "achieved": kr["GB_s"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(kr["GB_s"] / HBM_PEAK_GBS, 4),
                "bytes": "batch union: distinct (series, 64-point chunk) pairs x 256 B + 12 B per candidate entry",
                "per_pair": {"achieved": kr["GB_s_per_pair"], "frac": round(kr["GB_s_per_pair"] / HBM_PEAK_GBS, 4)},
                "achievable_read_GB_s": round(read_gbs, 1),
                "frac_of_achievable": round(kr["GB_s"] / read_gbs, 4),
                "traffic": traffic.get("bytes_per_launch") if traffic else None, "traffic_detail": traffic,
                "kernel": "k_refine"}
    else:
        roof = None
    return {
        "ids": ids, "d2": d2, "stats": stats, "ms_per_step": ms_per_step, "qps": qps, "kern": kern, "roofline": roof,
        "algorithmic_bytes_per_step": {"union": {"raw_chunk_pairs": u_raw, "words": u_words, "envelopes": u_env,
                                                 "deviation_code_bytes": u_sig, "total": path_union},
                                       "per_pair": {"words": word_bytes, "deviation_codes": sig_bytes,
                                                    "raw": raw_bytes, "total": path_pair}},
        "path_frac_of_hbm_peak": round(path_union / (ms_per_step / 1000.0) / 1e9 / HBM_PEAK_GBS, 4),
        "path_frac_of_hbm_peak_per_pair": round(path_pair / (ms_per_step / 1000.0) / 1e9 / HBM_PEAK_GBS, 4),
    }


def pruning_summary(stats, pct, levels):
    return {"leaves_kept_mean": float(stats["leaves_kept"].mean()),
            "rows_filtered_mean": float(stats["rows_filtered"].mean()),
            "rows_sigma_mean": float(stats["rows_sigma"].mean()),
            "rows_refined_mean": float(stats["rows_refined"].mean()),
            "candidates_mean": float(stats["candidates"].mean()),
            "per_level_refined_mean": [float(stats["rows_refined"][pct == p].mean()) for p in levels],
            "per_level_candidates_mean": [float(stats["candidates"][pct == p].mean()) for p in levels],
            "rounds_max": int(stats["rounds"].max()),
            "queries_on_fallback": int((stats["rounds"] > 1).sum()),
            "candidates_max": int(stats["candidates"].max())}


def cpu_oracle(x, q, sel, k, note):
    """The FP64 oracle (C/OpenMP brute force) on the host cores for the
    queries sel, and parity of the GPU's lists on them (caller compares)."""
    from oracle import brute
    log(f"CPU oracle on {len(sel)} queries ({brute.threads()} threads)")
    t0 = time.perf_counter()
    oids, od = brute.knn(x, q[sel], k)
    cpu_s = time.perf_counter() - t0
    cpu = {"value": round(len(sel) / cpu_s, 4), "unit": "queries/s", "cores": brute.threads(), "kind": "oracle",
           "sample": f"{note}; FP64 brute force over all {x.shape[0]} series; {cpu_s:.1f} s"}
    return cpu, oids, od


def cpu_method(args, hs, torch, G, dev, N=100_000, n=256, nq=10, level=5, k=1, leaf=1000, coll=1):
    """The method on the CPU: the oracle's serial FP64 filter-and-refine
    (leaf pruning by LB_EAPCA, series pruning by LB_SAX, early-abandoning
    refinement) on the small random-walk workload, beside the GPU's plain
    form on the same queries.  The oracle's index over 10M series would take
    minutes to build, so the comparison runs at 100k x 256."""
    from oracle import search
    x = G.random_walks(N, n, coll=coll)
    q, _, _ = G.workload(x, [level], nq, coll=coll)
    t0 = time.perf_counter()
    oix = search.LeafIndex(x, args.w, leaf)
    build_cpu = time.perf_counter() - t0
    t0 = time.perf_counter()
    res = [search.exact_knn(oix, q[i], k, l_max=args.l_max) for i in range(nq)]
    cpu_s = time.perf_counter() - t0
    xt = torch.from_numpy(x).to(dev)
    qt = torch.from_numpy(q).to(dev)
    idx = hs.Index(xt, hs.Params(w=args.w, leaf_size=leaf, l_max=args.l_max, seed_rows=args.seed_rows))
    for _ in range(5):
        idx.knn(qt, k)
    torch.cuda.synchronize()
    calls = 50
    t0 = time.perf_counter()
    for _ in range(calls):
        ids, d2 = idx.knn(qt, k)
    torch.cuda.synchronize()
    gpu_s = (time.perf_counter() - t0) / calls
    g = ids.cpu().numpy()
    same = int(sum(np.array_equal(g[i], res[i][0]) for i in range(nq)))
    idx.close()
    out = {"workload": f"random-walk {N}x{n} f32, {nq} queries at {level}% noise, k={k}, w={args.w}, leaf {leaf}, "
                       f"l_max {args.l_max}",
           "cpu": {"value": round(nq / cpu_s, 3), "unit": "queries/s", "cores": 1,
                   "kind": "oracle filter-and-refine (serial, FP64)", "index_build_s": round(build_cpu, 2)},
           "gpu": {"value": round(nq / gpu_s, 2), "unit": "queries/s", "ms_per_call": round(gpu_s * 1e3, 4),
                   "mode": f"one call of {nq} queries"},
           "identical_id_lists": same}
    log(f"method on the CPU: {out}")
    return out


def parity_of(ids, d2, sel, oids, od):
    g_ids = ids.cpu().numpy()[sel]
    g_d = d2.cpu().numpy()[sel].astype(np.float64)
    same = int((g_ids == oids).all(axis=1).sum())
    rel = float(np.max(np.abs(g_d - od) / np.maximum(od, 1e-30)))
    return {"queries_checked": int(len(sel)), "identical_id_lists": same, "max_rel_d_err": rel}


def run_serving(args, hs, torch, G, idx256, x256):
    """Serving form: three collections (20M x 128, 10M x 256 -- the headline
    index -- and 2M x 1024 at scale 1), a Poisson stream of requests with the
    collection uniform, k ~ U{1..100} and noise variance ~ U[1 %, 10 %];
    latency = completion - scheduled arrival on the server's clock."""
    dev = torch.device("cuda:0")
    scale = args.serve_scale
    specs = [(max(1000, int(20_000_000 * scale)), 128, 16), (None, 256, 16), (max(1000, int(2_000_000 * scale)), 1024, 32)]
    xs, idxs = [], []
    for c, (N, n, w) in enumerate(specs):
        if N is None:
            xs.append(x256)
            idxs.append(idx256)
            continue
        t0 = time.time()
        xc = G.random_walks(N, n, coll=100 + c)
        xt = torch.from_numpy(xc).to(dev)
        ic = hs.Index(xt, hs.Params(w=w, leaf_size=args.leaf, l_max=args.l_max, seed_rows=args.seed_rows))
        torch.cuda.synchronize()
        del xt
        torch.cuda.empty_cache()
        xs.append(xc)
        idxs.append(ic)
        log(f"serving collection {c}: {N} x {n} built in {time.time() - t0:.1f}s")
    budget = int(args.serve_budget_gb * (1 << 30))
    srv = hs.Server(idxs, [0, 0, 0], budget_bytes=budget, streams_per_coll=args.serve_streams, max_slots=8192,
                    max_batch=256)

    rng = np.random.default_rng(G.SEED_ARRIVAL)
    total_s = args.serve_warmup + args.serve_seconds
    arrivals = G.poisson_arrivals(args.serve_rate, total_s, seed=G.SEED_ARRIVAL)
    R = len(arrivals)
    coll = rng.integers(0, 3, R)
    ks = rng.integers(1, 101, R)
    var = rng.uniform(0.01, 0.10, R)
    qs = []
    for i in range(R):
        xc = xs[coll[i]]
        q = xc[rng.integers(0, len(xc))].astype(np.float64) + rng.standard_normal(xc.shape[1]) * np.sqrt(var[i])
        qs.append(((q - q.mean()) / q.std()).astype(np.float32))
    log(f"serving: {R} requests over {total_s:.0f}s at {args.serve_rate:.0f}/s")

    done = {}
    arr_srv = np.empty(R)
    busy = 0
    # the submitting loop is the load generator: Python's cyclic garbage
    # collector (tens of thousands of result dicts) would pause it and delay
    # arrivals, so it is off while requests are generated
    gc.collect()
    gc.disable()
    t0p = time.perf_counter()
    t0s = hs.hs_server_now()
    i = 0
    while i < R or len(done) < R:
        now = time.perf_counter() - t0p
        while i < R and arrivals[i] <= now:
            if srv.submit(int(coll[i]), qs[i], int(ks[i]), i):
                arr_srv[i] = t0s + arrivals[i]
                i += 1
            else:
                busy += 1
                break
        for r in srv.poll():
            done[r["tag"]] = r
        if time.perf_counter() - t0p > total_s + 120:
            raise RuntimeError("serving run did not finish")
    wall = time.perf_counter() - t0p
    gc.enable()
    meas = [t for t in range(R) if arrivals[t] >= args.serve_warmup]
    lat = np.array([(done[t]["t_done"] - arr_srv[t]) * 1000.0 for t in meas])
    # where the time of the slowest 1 % went: before the launch (admission,
    # queueing, graph capture) or on the device
    qwait = np.array([(done[t]["t_launch"] - arr_srv[t]) * 1000.0 for t in meas])
    run = np.array([(done[t]["t_done"] - done[t]["t_launch"]) * 1000.0 for t in meas])
    tail = lat >= np.percentile(lat, 99)
    ok = all(done[t]["status"] == 0 for t in range(R))
    span = max(done[t]["t_done"] for t in meas) - (t0s + args.serve_warmup)
    info = srv.info()
    # spot-check: server results equal the eager entry point on the same query
    same = 0
    checked = list(range(0, R, max(1, R // 50)))
    for t in checked:
        c = int(coll[t])
        qt1 = torch.from_numpy(qs[t][None, :].copy()).to(dev)
        e_ids, e_d2 = idxs[c].knn(qt1, int(ks[t]))
        torch.cuda.synchronize()
        same += int(list(e_ids.cpu().numpy()[0]) == done[t]["ids"] and list(e_d2.cpu().numpy()[0]) == done[t]["d2"])
    # saturation: everything submitted at once, completion rate
    S = min(R, 20000)
    t1 = hs.hs_server_now()
    for t in range(S):
        while not srv.submit(int(coll[t]), qs[t], int(ks[t]), R + t):
            for r in srv.poll():
                done[r["tag"]] = r
    while len([1 for tg in done if tg >= R]) < S:
        for r in srv.poll():
            done[r["tag"]] = r
    sat_s = max(done[R + t]["t_done"] for t in range(S)) - t1
    info2 = srv.info()
    # the same request mix without batching: one eager call per request (plain
    # form, queries already on the device), in submission order
    E = min(S, 3000)
    qdev = [torch.from_numpy(qs[t][None, :].copy()).to(dev) for t in range(E)]
    for t in range(min(E, 50)):
        idxs[int(coll[t])].knn(qdev[t], int(ks[t]))
    torch.cuda.synchronize()
    t0e = time.perf_counter()
    for t in range(E):
        idxs[int(coll[t])].knn(qdev[t], int(ks[t]))
    torch.cuda.synchronize()
    eager_qps = E / (time.perf_counter() - t0e)
    del qdev
    out = {"value": round(len(meas) / span, 2), "unit": "queries/s", "offered_rate": args.serve_rate,
           "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4), "p99": round(float(np.percentile(lat, 99)), 4),
                          "mean": round(float(lat.mean()), 4), "from": "scheduled arrival"},
           "tail_1pct_ms": {"to_launch_mean": round(float(qwait[tail].mean()), 3),
                            "on_device_mean": round(float(run[tail].mean()), 3),
                            "collections": [int(np.sum(coll[np.array(meas)[tail]] == c)) for c in range(3)]},
           "requests_measured": len(meas), "requests_total": R, "all_ok": bool(ok), "busy_retries": busy,
           "batches": info["batches"], "mean_batch": round(info["queries"] / max(1, info["batches"]), 2),
           "graphs": info2["graphs"], "identical_to_eager": f"{same}/{len(checked)}",
           "saturation_queries_per_s": round(S / sat_s, 2), "saturation_requests": S,
           "saturation_mean_batch": round((info2["queries"] - info["queries"]) /
                                          max(1, info2["batches"] - info["batches"]), 2),
           "eager_one_call_per_request_queries_per_s": round(eager_qps, 2), "eager_requests": E,
           "collections": [f"{len(xc)}x{xc.shape[1]}" for xc in xs], "k": "U{1..100}",
           "noise_variance": "U[0.01, 0.10]", "wall_s": round(wall, 1)}
    log(f"serving: {out}")
    srv.close()
    for c, ic in enumerate(idxs):
        if ic is not idx256:
            ic.close()
    return out


def run_ablation(args, torch, variants, q, pct, levels, ref_ids):
    """Plain form per noise level under each access-path variant: queries/s
    (each level's queries as one batch, 3 timed calls after 1 warm-up) and
    whether the id lists equal the default index's."""
    out = {}
    ref = ref_ids.cpu().numpy()
    for name, ix in variants.items():
        row = {}
        for p in levels:
            sel = np.where(pct == p)[0]
            qt = torch.from_numpy(np.ascontiguousarray(q[sel])).to("cuda:0")
            ix.knn(qt, args.k)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                res = ix.knn(qt, args.k)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t0) / 3
            same = int((res[0].cpu().numpy() == ref[sel]).all(axis=1).sum())
            row[f"{p}%"] = {"queries_per_s": round(len(sel) / dt, 1), "ms": round(dt * 1e3, 3),
                            "identical_id_lists": f"{same}/{len(sel)}"}
        out[name] = row
        log(f"ablation {name}: {row}")
    return out


def run_large(args, hs, torch, G, dev):
    """The precision form's own configuration: 100M random walks of length 256
    (102.4 GB float32 plus a 51.2 GB bf16 copy), 1,000 queries at 5 % noise,
    k = 10; plain and precision form on the same index, the oracle on the
    first 50 queries."""
    N, n, k, w = args.large_N, 256, args.large_k, args.w
    log(f"large: generating {N} x {n} random walks")
    t0 = time.time()
    x = G.random_walks(N, n, coll=0)
    q, _, _ = G.workload(x, [args.large_level], args.large_queries)
    log(f"large: generated in {time.time() - t0:.1f}s; uploading")
    xt = torch.from_numpy(x).to(dev)
    qt = torch.from_numpy(q).to(dev)
    torch.cuda.synchronize()
    t0 = time.time()
    idx = hs.Index(xt, hs.Params(w=w, leaf_size=args.leaf, l_max=args.l_max, seed_rows=args.seed_rows))
    torch.cuda.synchronize()
    build_s = time.time() - t0
    log(f"large: built in {build_s:.1f}s, {idx.info.n_leaves} leaves")
    read_gbs = hs.read_probe_gbs(xt, passes=2)
    del xt
    torch.cuda.empty_cache()
    Q = q.shape[0]
    wl = {"N": N, "n": n, "Q": Q, "k": k}
    res = measure_plain(hs, torch, idx, qt, k, args.large_steps, args.large_warmup, w, wl, read_gbs)
    mixed = run_mixed(hs, torch, idx, qt, k, args.large_steps, args.large_warmup, wl, res["ids"], res["d2"])
    out = {"workload": f"random-walk {N}x{n} f32, {Q} queries at {args.large_level}% noise, k={k}, w={w}, "
                       f"card 256, leaf {args.leaf}, l_max {args.l_max}",
           "value": round(res["qps"], 2), "unit": "queries/s", "ms_per_step": round(res["ms_per_step"], 4),
           "steps": args.large_steps, "warmup": args.large_warmup, "n_leaves": int(idx.info.n_leaves),
           "build_s": round(build_s, 2), "roofline": res["roofline"], "scan_kernels": res["kern"],
           "algorithmic_bytes_per_step": res["algorithmic_bytes_per_step"],
           "path_frac_of_hbm_peak": res["path_frac_of_hbm_peak"],
           "pruning": pruning_summary(res["stats"], np.full(Q, args.large_level), [args.large_level]),
           "precision_form": mixed,
           "precision_vs_plain_speedup": round(mixed["value"] / res["qps"], 3)}
    if args.large_cpu > 0:
        sel = np.arange(min(args.large_cpu, Q))
        cpu, oids, od = cpu_oracle(x, q, sel, k, f"the first {len(sel)} of the {Q} queries, k={k}")
        out["cpu_baseline"] = cpu
        out["parity_sample"] = {"plain": parity_of(res["ids"], res["d2"], sel, oids, od)}
        log(f"large: CPU oracle {cpu['value']} q/s; parity {out['parity_sample']}")
    idx.close()
    del idx, x, q, qt
    gc.collect()
    torch.cuda.empty_cache()
    log(f"large: {out['value']} q/s plain, {mixed['value']} q/s precision")
    return out


def run_hard(args, hs, torch, G, dev):
    """The hard-large configuration: 50M random walks of length 1024 (204.8 GB
    float32, generated on the GPU chunk by chunk and built by the streaming
    build, so they are never in device memory twice), w = 32, k = 100, 500
    queries at 10 % noise plus 100 out-of-dataset queries; the plain form, the
    precision form with an fp16 copy of as many series as fit beside them, and
    the serving form over that precision-form collection; the oracle on 50
    sampled queries, its data streamed back chunk by chunk."""
    N, n, w, k = args.hard_N, 1024, 32, 100
    coll = 4
    CH = G.DEV_CHUNK
    src = np.sort(G.query_sources(N, args.hard_queries, coll=coll))
    src_rows = {}

    def chunk(r0):
        rows = min(CH, N - r0)
        x = G.walk_chunk_device(r0 // CH, rows, n, coll=coll, device=dev)
        lo, hi = np.searchsorted(src, [r0, r0 + rows])
        if hi > lo and r0 not in src_rows:
            src_rows[r0] = (src[lo:hi], x[torch.as_tensor(src[lo:hi] - r0, device=dev)].cpu().numpy())
        return x

    log(f"hard: streaming build of {N} x {n} (generated on the device)")
    t0 = time.time()
    params = hs.Params(w=w, leaf_size=args.leaf, l_max=args.l_max, seed_rows=args.seed_rows,
                       cand_per_query=args.hard_cand_per_query)
    idx = hs.Index.from_chunks(chunk, N, n, params, device=dev)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    log(f"hard: built in {build_s:.1f}s, {idx.info.n_leaves} leaves, index {idx.info.index_bytes / 1e9:.1f} GB")
    rows_src = np.concatenate([v[1] for _, v in sorted(src_rows.items())])
    ids_src = np.concatenate([v[0] for _, v in sorted(src_rows.items())])
    assert np.array_equal(ids_src, src)
    q = np.concatenate([G.noisy_queries(rows_src, 10.0, coll=coll), G.ood_queries(args.hard_ood, n, coll=coll)])
    Q = q.shape[0]
    qt = torch.from_numpy(q).to(dev)
    wl = {"N": N, "n": n, "Q": Q, "k": k}
    read_gbs = hs.read_probe_gbs(idx.mem[:idx.info.n_series * idx.info.row_stride * 4], passes=1)
    res = measure_plain(hs, torch, idx, qt, k, args.hard_steps, 1, w, wl, read_gbs)
    ids_plain, d2_plain = res["ids"], res["d2"]
    # the fp16 copy: as many series as fit beside the index, the workspace and
    # the server's budget
    ws_bytes = hs.hs_query_workspace_bytes(idx.h, Q, k)
    budget = int(args.hard_serve_budget_gb * (1 << 30))
    idx._ws = None
    torch.cuda.empty_cache()
    free = torch.cuda.mem_get_info(dev)[0]
    spare = free - 2 * ws_bytes - budget - (4 << 30)
    shadow_rows = int(max(0, min(N, spare // (2 * idx.info.row_stride + 16))))
    log(f"hard: fp16 copy of {shadow_rows} of {N} series ({shadow_rows / N:.1%})")
    t0 = time.time()
    idx.build_shadow(hs.HS_SHADOW_FP16, shadow_rows=shadow_rows)
    torch.cuda.synchronize()
    shadow_s = time.time() - t0
    mixed = run_mixed(hs, torch, idx, qt, k, args.hard_steps, 1, wl, ids_plain, d2_plain, build=False)
    mixed["shadow_rows"] = shadow_rows
    mixed["shadow_build_s"] = round(shadow_s, 2)
    # serving: every query submitted at once to a server over the
    # precision-form collection; results equal the plain form's
    srv = hs.Server([idx], [1], budget_bytes=budget, streams_per_coll=2, max_slots=4096, max_batch=128)
    done = {}
    t1 = hs.hs_server_now()
    for i in range(Q):
        while not srv.submit(0, q[i], k, i):
            for r in srv.poll():
                done[r["tag"]] = r
    while len(done) < Q:
        for r in srv.poll():
            done[r["tag"]] = r
    span = max(r["t_done"] for r in done.values()) - t1
    lat = np.array([(r["t_done"] - r["t_submit"]) * 1e3 for r in done.values()])
    ip = ids_plain.cpu().numpy()
    same_srv = sum(int(done[i]["ids"] == list(ip[i])) for i in range(Q))
    info = srv.info()
    srv.close()
    serving = {"value": round(Q / span, 2), "unit": "queries/s", "mode": "all queries submitted at once",
               "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                              "p99": round(float(np.percentile(lat, 99)), 3), "from": "submission"},
               "batches": info["batches"], "identical_id_lists_vs_plain": same_srv}
    log(f"hard: serving {serving}")
    out = {"workload": f"random-walk {N}x{n} f32 (generated on the device), {args.hard_queries} queries at 10% noise "
                       f"+ {args.hard_ood} out-of-dataset, k={k}, w={w}, card 256, leaf {args.leaf}, "
                       f"l_max {args.l_max}",
           "value": round(res["qps"], 2), "unit": "queries/s", "ms_per_step": round(res["ms_per_step"], 4),
           "steps": args.hard_steps, "n_leaves": int(idx.info.n_leaves), "build_s": round(build_s, 2),
           "index_GB": round(idx.info.index_bytes / 1e9, 2),
           "roofline": res["roofline"], "scan_kernels": res["kern"],
           "algorithmic_bytes_per_step": res["algorithmic_bytes_per_step"],
           "pruning": pruning_summary(res["stats"], np.concatenate([np.full(args.hard_queries, 10),
                                                                     np.full(args.hard_ood, -1)]), [10, -1]),
           "precision_form": mixed, "serving_form": serving}
    if args.hard_cpu > 0:
        sel = np.unique(np.concatenate([np.linspace(0, args.hard_queries - 1, args.hard_cpu - args.hard_cpu // 5),
                                        args.hard_queries + np.arange(args.hard_cpu // 5)]).round().astype(np.int64))
        from oracle import brute
        log(f"hard: CPU oracle on {len(sel)} queries, the collection streamed back chunk by chunk")
        t0 = time.perf_counter()

        def host_chunks():
            for c in range((N + CH - 1) // CH):
                rows = min(CH, N - c * CH)
                yield G.walk_chunk_device(c, rows, n, coll=coll, device=dev).cpu().numpy()

        oids, od = brute.knn_chunked(host_chunks(), q[sel], k)
        cpu_s = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(len(sel) / cpu_s, 4), "unit": "queries/s", "cores": brute.threads(),
                               "kind": "oracle",
                               "sample": f"{len(sel)} of the {Q} queries, k={k}; FP64 brute force over all {N} "
                                         f"series; {cpu_s:.1f} s (including regenerating the chunks)"}
        out["parity_sample"] = {"plain": parity_of(ids_plain, d2_plain, sel, oids, od)}
        mids = torch.from_numpy(np.array([done[i]["ids"] for i in range(Q)]))
        md2 = torch.from_numpy(np.array([done[i]["d2"] for i in range(Q)], dtype=np.float32))
        out["parity_sample"]["serving_precision"] = parity_of(mids, md2, sel, oids, od)
        log(f"hard: parity {out['parity_sample']}")
    idx.close()
    del idx, qt
    gc.collect()
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--N", type=int, default=10_000_000)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--per-level", type=int, default=100)
    ap.add_argument("--levels", default="1,5,10", help="noise levels (variance, percent) of the queries")
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--w", type=int, default=16)
    ap.add_argument("--leaf", type=int, default=10_000)
    ap.add_argument("--l-max", type=int, default=4)
    ap.add_argument("--seed-rows", type=int, default=256)
    ap.add_argument("--cpu-sample", type=int, default=180, help="queries timed on the CPU oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-queries", type=int, default=300)
    ap.add_argument("--forms", default="plain,mixed,serving,large",
                    help="plain: the paper's filter-and-refine (always timed, the headline value); mixed: also "
                         "the precision form (bf16 copy, matrix-core bound, compensated refine) on the same index; "
                         "serving: the continuous-batching server over three collections under Poisson arrivals; "
                         "large: the precision form's own configuration (100M x 256, 1,000 queries at 5 %%, "
                         "k = 10), plain and precision form, after the headline index is freed; "
                         "hard: the hard-large configuration (50M x 1024 generated on the device, streaming "
                         "build, 500 queries at 10 %% + 100 ood, k = 100, w = 32; plain, partial fp16 copy, "
                         "serving); "
                         "ablation: the plain form per noise level with the LB_SAX filter always on (the default), "
                         "skipped (NoSAX) and skipped below the paper's leaf-pruning threshold 0.25")
    ap.add_argument("--large-N", type=int, default=100_000_000)
    ap.add_argument("--large-queries", type=int, default=1000)
    ap.add_argument("--large-level", type=int, default=5)
    ap.add_argument("--large-k", type=int, default=10)
    ap.add_argument("--large-steps", type=int, default=5)
    ap.add_argument("--large-warmup", type=int, default=2)
    ap.add_argument("--large-cpu", type=int, default=50, help="queries of the large workload timed on the oracle")
    ap.add_argument("--hard-N", type=int, default=50_000_000)
    ap.add_argument("--hard-queries", type=int, default=500)
    ap.add_argument("--hard-ood", type=int, default=100)
    ap.add_argument("--hard-steps", type=int, default=3)
    ap.add_argument("--hard-cpu", type=int, default=50, help="queries of the hard workload checked on the oracle")
    ap.add_argument("--hard-cand-per-query", type=int, default=2_000_000)
    ap.add_argument("--hard-serve-budget-gb", type=float, default=8.0)
    ap.add_argument("--serve-rate", type=float, default=2000.0, help="Poisson arrival rate (queries/s)")
    ap.add_argument("--serve-seconds", type=float, default=30.0, help="measured arrival window (s)")
    ap.add_argument("--serve-warmup", type=float, default=5.0, help="arrivals before the measured window (s)")
    ap.add_argument("--serve-scale", type=float, default=1.0,
                    help="fraction of the serving collections' sizes (1.0 = 20M x 128, 10M x 256, 2M x 1024)")
    ap.add_argument("--serve-budget-gb", type=float, default=48.0, help="device budget of the server (GB)")
    ap.add_argument("--serve-streams", type=int, default=3, help="server streams per collection")
    ap.add_argument("--profile-run", action="store_true",
                    help="only the warmup and timed k-NN steps (no k=1 pass, latency or CPU oracle), so a "
                         "profiler's per-kernel averages cover exactly the launches timed here; also copies "
                         "a 1 GiB buffer once, the calibration kernel for HBM byte counters")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the leaf-sharded design is described in DESIGN.md); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    forms = args.forms.split(",")
    if "serving" in forms:
        # the server runs streams_per_coll streams per collection; give each its
        # own hardware queue (set before the HIP runtime starts)
        os.environ.setdefault("GPU_MAX_HW_QUEUES", str(min(16, 3 * args.serve_streams + 1)))

    import torch
    from paper_2212_13297_amd import datagen as G
    from paper_2212_13297_amd import hs

    dev = torch.device("cuda:0")
    levels = [int(v) for v in args.levels.split(",")]
    log(f"generating {args.N} x {args.n} random walks")
    t0 = time.time()
    x = G.random_walks(args.N, args.n)
    q, src, pct = G.workload(x, levels, args.per_level)
    Q = q.shape[0]
    log(f"generated in {time.time() - t0:.1f}s; uploading")
    xt = torch.from_numpy(x).to(dev)
    qt = torch.from_numpy(q).to(dev)
    torch.cuda.synchronize()
    params = hs.Params(w=args.w, leaf_size=args.leaf, l_max=args.l_max, seed_rows=args.seed_rows)
    t0 = time.time()
    idx = hs.Index(xt, params)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    info = idx.info
    log(f"built index in {build_s:.1f}s: {info.n_leaves} leaves, max leaf {info.max_leaf}")
    # an achievable read-stream rate on this GPU, beside the nominal peak: the
    # library's read probe over the input (5 passes)
    read_gbs = hs.read_probe_gbs(xt, passes=5)
    log(f"read stream (probe over {xt.numel() * 4 / 1e9:.2f} GB): {read_gbs:.0f} GB/s")
    # ablation indexes: same data and leaves, other access-path thresholds (eapca_th)
    abl_idx = {}
    if "ablation" in forms and not args.profile_run:
        for name, th in (("nosax", 1.1), ("thresh_0.25", 0.25)):
            abl_idx[name] = hs.Index(xt, hs.Params(w=args.w, leaf_size=args.leaf, l_max=args.l_max,
                                                   seed_rows=args.seed_rows, eapca_th=th))
        torch.cuda.synchronize()
    del xt
    torch.cuda.empty_cache()

    if args.profile_run:
        # a plain 1 GiB device-to-device copy: the known-size kernel against which
        # the HBM byte counters (FETCH_SIZE / WRITE_SIZE) are scaled
        src_buf = torch.ones(COPY_CAL_BYTES // 4, dtype=torch.float32, device=dev)
        dst_buf = torch.empty_like(src_buf)
        torch.cuda.synchronize()
        dst_buf.copy_(src_buf)
        torch.cuda.synchronize()
        del src_buf, dst_buf
        torch.cuda.empty_cache()

    def run(k, steps, stats=False):
        out = None
        for _ in range(steps):
            out = idx.knn(qt, k, stats=stats)
        return out

    wl = {"N": args.N, "n": args.n, "Q": Q, "k": args.k}
    if args.profile_run:
        # warmup and timed steps only (plain form, then the precision form when
        # asked for): the profiler's averages cover exactly these launches, and
        # the HIP-event timing of the same launches is logged beside them
        out = {"profile_run": True, "queries": Q}
        for form in ("plain", "mixed"):
            if form not in forms:
                continue
            if form == "mixed":
                idx.build_shadow(hs.HS_SHADOW_BF16)
            call = (lambda st: idx.knn(qt, args.k, stats=st)) if form == "plain" else \
                (lambda st: idx.knn_mixed(qt, args.k, stats=st))
            for _ in range(args.warmup):
                call(False)
            torch.cuda.synchronize()
            hs.profile_read_all(reset=True)
            hs.hs_profile_enable(True)
            t0 = time.perf_counter()
            for _ in range(args.steps):
                call(True)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1000.0 / args.steps
            hs.hs_profile_enable(False)
            prof = hs.profile_read_all(reset=True)
            log(f"profile run, {form} form: {ms:.3f} ms/step; scan kernels {prof}")
            out[form] = {"ms_per_step": round(ms, 4),
                         "kernel_avg_ms": {kk: round(v[0] / v[1], 4) for kk, v in prof.items() if v[1]}}
        print(json.dumps(out), flush=True)
        idx.close()
        return

    res = measure_plain(hs, torch, idx, qt, args.k, args.steps, args.warmup, args.w, wl, read_gbs)
    ids, d2, stats = res["ids"], res["d2"], res["stats"]
    ms_per_step, qps = res["ms_per_step"], res["qps"]

    # k = 1 on the same batch
    run(1, max(1, args.warmup // 2))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(1, args.steps)
    torch.cuda.synchronize()
    qps_k1 = round(Q * args.steps / (time.perf_counter() - t0), 2)
    log(f"k=1: {qps_k1:.0f} queries/s")

    # single-query latency
    lat = []
    nl = min(args.latency_queries, Q)
    for i in range(nl):
        qi = qt[i:i + 1]
        torch.cuda.synchronize()
        a = time.perf_counter()
        idx.knn(qi, args.k)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1000.0)
    lat = np.asarray(lat if lat else [float("nan")])
    log(f"single-query latency p50 {np.percentile(lat, 50):.3f} ms p99 {np.percentile(lat, 99):.3f} ms")

    mixed = None
    if "mixed" in forms:
        mixed = run_mixed(hs, torch, idx, qt, args.k, args.steps, args.warmup, wl, ids, d2)
    serving = None
    if "serving" in forms:
        serving = run_serving(args, hs, torch, G, idx, x)

    ablation = None
    if abl_idx:
        ablation = run_ablation(args, torch, {"sax": idx, **abl_idx}, q, pct, levels, ids)
        for v in abl_idx.values():
            v.close()

    cpu = None
    parity = None
    method = None
    if not args.no_cpu_baseline and args.cpu_sample > 0:
        sel = np.linspace(0, Q - 1, min(args.cpu_sample, Q)).round().astype(np.int64)
        cpu, oids, od = cpu_oracle(x, q, sel, args.k,
                                   f"{len(sel)} of the {Q} queries (evenly spaced over the "
                                   f"{'/'.join(map(str, levels))}% levels), k={args.k}")
        parity = parity_of(ids, d2, sel, oids, od)
        log(f"CPU oracle {cpu['value']} q/s; parity {parity}")
        method = cpu_method(args, hs, torch, G, dev)

    ids_cpu = ids.cpu()
    idx.close()
    del idx, qt, x
    gc.collect()
    torch.cuda.empty_cache()
    large = None
    if "large" in forms and args.large_N > 0:
        large = run_large(args, hs, torch, G, dev)
    hard = None
    if "hard" in forms and args.hard_N > 0:
        hard = run_hard(args, hs, torch, G, dev)

    out = {
        "metric": METRIC,
        "value": round(qps, 2),
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"random-walk {args.N}x{args.n} f32, {Q} queries ({args.per_level} each at "
                        f"{'/'.join(map(str, levels))}% noise), k={args.k}, w={args.w}, card 256, "
                        f"leaf {args.leaf}, l_max {args.l_max}",
            "N": args.N, "n": args.n, "queries": Q, "k": args.k, "w": args.w, "leaf_size": args.leaf,
            "l_max": args.l_max, "n_leaves": int(info.n_leaves), "form": "plain fp32",
        },
        "queries_per_s_k1": qps_k1,
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 4),
                       "p99": round(float(np.percentile(lat, 99)), 4), "mode": "one query per call",
                       "queries": int(nl)},
        "roofline": res["roofline"],
        "scan_kernels": res["kern"],
        "algorithmic_bytes_per_step": res["algorithmic_bytes_per_step"],
        "path_frac_of_hbm_peak": res["path_frac_of_hbm_peak"],
        "path_frac_of_hbm_peak_per_pair": res["path_frac_of_hbm_peak_per_pair"],
        "pruning": pruning_summary(stats, pct, levels),
        "build_s": round(build_s, 2),
        "cpu_baseline": cpu,
        "cpu_method": method,
        "parity_sample": parity,
        "precision_form": mixed,
        "serving_form": serving,
        "ablation": ablation,
        "large_config": large,
        "hard_config": hard,
    }
    del ids_cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
