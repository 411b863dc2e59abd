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


def run_mixed(args, hs, torch, idx, qt, Q, plain_ids, plain_stats):
    """Precision form on the same index and batch: bf16 copy of the series,
    matrix-core bounding pass, compensated float32 refinement."""
    t0 = time.time()
    idx.build_shadow(hs.HS_SHADOW_BF16)
    torch.cuda.synchronize()
    shadow_s = time.time() - t0
    for _ in range(args.warmup):
        idx.knn_mixed(qt, args.k)
    torch.cuda.synchronize()
    hs.profile_read_all(reset=True)
    hs.hs_profile_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ids, d2, err, st = idx.knn_mixed(qt, args.k, stats=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hs.hs_profile_enable(False)
    prof = hs.profile_read_all(reset=True)
    ms = (t1 - t0) * 1000.0 / args.steps
    qps = Q / (ms / 1000.0)
    log(f"precision form: {ms:.3f} ms/step, {qps:.0f} queries/s; kernels {prof}")
    same = int((ids == plain_ids).all(dim=1).sum().item())
    stats = {f: v.cpu().numpy().astype(np.int64) for f, v in st.items()}
    info = idx.info
    K = info.row_stride
    kern = {}
    bms, bl = prof["bound"]
    if bl:
        avg = bms / bl
        # algorithmic work of the bounding pass: one q~.x~ (2K flop) per bounded
        # (query, series) pair; the low-precision rows and norms it must read once
        flops = 2.0 * K * float(stats["rows_filtered"].sum()) / (bl / args.steps)
        kern["bound"] = {"avg_launch_ms": round(avg, 4), "launches_per_step": bl / args.steps,
                         "flops_per_launch": int(flops),
                         "TFLOP_s": round(flops / (avg / 1e3) / 1e12, 2),
                         "shadow_bytes": int(info.n_series * (2 * K + 8)),
                         "shadow_GB_s": round(info.n_series * (2 * K + 8) / (avg / 1e3) / 1e9, 2)}
    rms, rl = prof["refine"]
    if rl:
        avg = rms / rl
        nbytes = (int(stats["chunks_read"].sum()) * 256 + int(stats["candidates"].sum()) * 12) / (rl / args.steps)
        kern["refine"] = {"avg_launch_ms": round(avg, 4), "launches_per_step": rl / args.steps,
                          "bytes_per_launch": int(nbytes), "GB_s": round(nbytes / (avg / 1e3) / 1e9, 2)}
    out = {"value": round(qps, 2), "unit": "queries/s", "ms_per_step": round(ms, 4), "dtype": "bf16 bound, f32 refine",
           "identical_id_lists_vs_plain": same, "queries": Q,
           "max_err_bound_rel": float((err / d2.double()).max().item()),
           "shadow_build_s": round(shadow_s, 2),
           "kernels": kern,
           "roofline": ({"bound": "mfma", "achieved": kern["bound"]["TFLOP_s"], "peak": MFMA_PEAK_TFLOPS["bf16"],
                         "unit": "TFLOP/s", "frac": round(kern["bound"]["TFLOP_s"] / MFMA_PEAK_TFLOPS["bf16"], 4),
                         "kernel": "k_bound"} if "bound" in kern else None),
           "pruning": {"rows_bounded_mean": float(stats["rows_filtered"].mean()),
                       "candidates_mean": float(stats["candidates"].mean()),
                       "rows_refined_mean": float(stats["rows_refined"].mean()),
                       "rounds_max": int(stats["rounds"].max())}}
    log(f"precision form: {out}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--N", type=int, default=10_000_000)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--per-level", type=int, default=100)
    ap.add_argument("--k", type=int, default=10)
    ap.add_argument("--w", type=int, default=16)
    ap.add_argument("--leaf", type=int, default=10_000)
    ap.add_argument("--l-max", type=int, default=4)
    ap.add_argument("--seed-rows", type=int, default=256)
    ap.add_argument("--cpu-sample", type=int, default=180, help="queries timed on the CPU oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--latency-queries", type=int, default=300)
    ap.add_argument("--forms", default="plain,mixed",
                    help="plain: the paper's filter-and-refine (always timed, the headline value); mixed: also "
                         "the precision form (bf16 copy, matrix-core bound, compensated refine) on the same index")
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

    import torch
    from paper_2212_13297_amd import datagen as G
    from paper_2212_13297_amd import hs

    dev = torch.device("cuda:0")
    levels = [1, 5, 10]
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
    del xt
    torch.cuda.empty_cache()

    def run(k, steps, stats=False):
        out = None
        for _ in range(steps):
            out = idx.knn(qt, k, stats=stats)
        return out

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

    log(f"warmup {args.warmup} steps")
    run(args.k, args.warmup)
    torch.cuda.synchronize()
    hs.profile_read_all(reset=True)
    hs.hs_profile_enable(True)
    log(f"timing {args.steps} steps, Q={Q}, k={args.k}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ids, d2, st = run(args.k, args.steps, stats=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hs.hs_profile_enable(False)
    prof = hs.profile_read_all(reset=True)
    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    qps = Q / (ms_per_step / 1000.0)
    log(f"{ms_per_step:.3f} ms/step, {qps:.0f} queries/s; scan kernels {prof}")

    stats = {f: v.cpu().numpy().astype(np.int64) for f, v in st.items()}
    # algorithmic bytes (the seed step's few thousand series per query are included)
    word_bytes = int(stats["rows_filtered"].sum()) * args.w + int(stats["chunks_tested"].sum()) * args.w * 16
    cand_bytes = int(stats["candidates"].sum()) * 12
    raw_bytes = int(stats["chunks_read"].sum()) * 64 * 4
    kern = {}
    for name, nbytes in (("filter", word_bytes + cand_bytes), ("refine", raw_bytes + cand_bytes)):
        ms, launches = prof[name]
        if launches:
            avg = ms / launches
            per_launch = nbytes / (launches / args.steps)
            kern[name] = {"avg_launch_ms": round(avg, 4), "launches_per_step": launches / args.steps,
                          "bytes_per_launch": int(per_launch), "GB_s": round(per_launch / (avg / 1e3) / 1e9, 2)}
    dom = max(kern, key=lambda n: kern[n]["avg_launch_ms"] * kern[n]["launches_per_step"]) if kern else None
    achieved = kern[dom]["GB_s"] if dom else 0.0
    traffic = measured_traffic(f"k_{dom}", {"N": args.N, "n": args.n, "Q": Q, "k": args.k}) if dom else None
    env_bytes = Q * info.n_leaves * args.w * 16
    path_bytes_step = word_bytes + raw_bytes + env_bytes + Q * args.k * 12

    # k = 1 on the same batch
    qps_k1 = None
    if not args.profile_run:
        run(1, max(1, args.warmup // 2))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(1, args.steps)
        torch.cuda.synchronize()
        qps_k1 = round(Q * args.steps / (time.perf_counter() - t0), 2)
        log(f"k=1: {qps_k1:.0f} queries/s")

    # single-query latency
    lat = []
    nl = 0 if args.profile_run else min(args.latency_queries, Q)
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
    if "mixed" in args.forms.split(","):
        mixed = run_mixed(args, hs, torch, idx, qt, Q, ids, st)

    cpu = None
    parity = None
    if not args.no_cpu_baseline and not args.profile_run and args.cpu_sample > 0:
        from oracle import brute
        sel = np.linspace(0, Q - 1, min(args.cpu_sample, Q)).round().astype(np.int64)
        log(f"CPU oracle on {len(sel)} queries ({brute.threads()} threads)")
        t0 = time.perf_counter()
        oids, od = brute.knn(x, q[sel], args.k)
        cpu_s = time.perf_counter() - t0
        cpu = {"value": round(len(sel) / cpu_s, 4), "unit": "queries/s", "cores": brute.threads(),
               "kind": "oracle",
               "sample": f"{len(sel)} of the {Q} queries (evenly spaced over the 1/5/10% levels), k={args.k}, "
                         f"FP64 brute force over all {args.N} series; {cpu_s:.1f} s"}
        g_ids = ids.cpu().numpy()[sel]
        g_d = d2.cpu().numpy()[sel].astype(np.float64)
        same = int((g_ids == oids).all(axis=1).sum())
        rel = float(np.max(np.abs(g_d - od) / np.maximum(od, 1e-30)))
        parity = {"queries_checked": int(len(sel)), "identical_id_lists": same, "max_rel_d_err": rel}
        log(f"CPU oracle {cpu['value']} q/s; parity {parity}")

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
        "roofline": {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic.get("bytes_per_launch") if traffic else None,
                     "traffic_detail": traffic,
                     "kernel": f"k_{dom}" if dom else None, **(kern.get(dom, {}))},
        "scan_kernels": kern,
        "algorithmic_bytes_per_step": {"words": word_bytes, "raw": raw_bytes, "envelopes": env_bytes,
                                       "total": path_bytes_step},
        "path_frac_of_hbm_peak": round(path_bytes_step / (ms_per_step / 1000.0) / 1e9 / HBM_PEAK_GBS, 4),
        "pruning": {"leaves_kept_mean": float(stats["leaves_kept"].mean()),
                    "rows_filtered_mean": float(stats["rows_filtered"].mean()),
                    "rows_refined_mean": float(stats["rows_refined"].mean()),
                    "candidates_mean": float(stats["candidates"].mean()),
                    "per_level_refined_mean": [float(stats["rows_refined"][pct == p].mean()) for p in levels],
                    "per_level_candidates_mean": [float(stats["candidates"][pct == p].mean()) for p in levels],
                    "rounds_max": int(stats["rounds"].max()),
                    "queries_on_fallback": int((stats["rounds"] > 1).sum()),
                    "candidates_max": int(stats["candidates"].max())},
        "build_s": round(build_s, 2),
        "cpu_baseline": cpu,
        "parity_sample": parity,
        "precision_form": mixed,
    }
    print(json.dumps(out), flush=True)
    idx.close()


if __name__ == "__main__":
    main()
