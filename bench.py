#!/usr/bin/env python3
"""Throughput of the HyperOMS hot path on one MI355X.

Workload (default "large"): a synthetic library of 1,000,000 references plus
1,000,000 decoys and 100,000 queries shaped like the paper's workloads
(Section 4.1, Table 1), D = 8192, 16 levels, 0.05 Da bins, open window
+-500 Da with charge matching. The library is preprocessed, uploaded and
encoded once before timing (reference hypervectors are encoded once and
reused, Section 3.3). One step = encode all query spectrum vectors (already
resident in HBM) + open-window Hamming top-1 search of every query.

Prints one JSON line: comparisons/s (sum of candidate-window sizes per
second), queries/s, the roofline of the search kernel measured with HIP
events inside the library, and the oracle timed on the host cores on a
bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "query-ref Hamming comparisons/s and queries/s at ±500 Da, D=8192"
# issue model: 256 CUs x 4 SIMD16 units (64 lanes per clock) x 2.4 GHz. The
# xor + popcount pair the search is made of runs faster than this model on
# MI355X, so the roofline uses the rate measured live on the box
# (homs_measure_xor_popcount_rate) and reports the model beside it.
VALU_MODEL_TOPS = 256 * 64 * 2.4e9 / 1e12
MFMA_PEAK_TOPS = 5000.0  # dense fp8 / int8 matrix peak of MI355X, TFLOP/s (TOP/s)

# HBM bytes per launch of the search kernel on the default large workload, from
# rocprofv3 FETCH_SIZE and WRITE_SIZE runs scaled by a 1 GiB copy kernel
# (profiles/search_popcount_large.md). Valid only while the kernel source has
# the hash it was measured on.
MEASURED_TRAFFIC = {"a5ee47bd0896dc11": 4.868e12}


VALU_PEAK_TOPS = VALU_MODEL_TOPS  # replaced by the live measurement in main()


def kernel_source_hash() -> str:
    import hashlib
    digest = hashlib.sha256()
    for name in ("search_popc.hip", "popcount_tile.h"):
        with open(os.path.join(ROOT, "paper_2211_16422_amd", "csrc", name), "rb") as fh:
            digest.update(fh.read())
    return digest.hexdigest()[:16]


def log(msg: str):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large", choices=["tiny", "large", "batched"])
    ap.add_argument("--n-ref", type=int, default=None, help="override reference count")
    ap.add_argument("--n-query", type=int, default=None, help="override query count")
    ap.add_argument("--cpu-sample", type=int, default=512,
                    help="queries in the oracle's timed sample (0 = skip)")
    ap.add_argument("--profile-only", action="store_true",
                    help="skip the CPU baseline (for profiler runs)")
    ap.add_argument("--skip-mfma", action="store_true",
                    help="do not time the matrix-core (precision) form")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="also run one device-to-device copy of BYTES bytes (a reference "
                         "kernel for scaling hardware byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(queries would be sharded across GPUs with the library replicated); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2211_16422_amd.hyperoms as h
    from synth import WORKLOADS, make_workload

    global VALU_PEAK_TOPS
    VALU_PEAK_TOPS = h.measure_xor_popcount_rate(0) / 1e12
    log(f"measured xor+popcount rate {VALU_PEAK_TOPS:.2f} T lane-ops/s "
        f"(issue model {VALU_MODEL_TOPS:.2f})")
    w = WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    if w.name == "batched":
        return bench_batched(args, w, dev)
    t0 = time.time()
    g = make_workload(w, n_ref=args.n_ref, n_query=args.n_query)
    lib, q = g.library, g.queries
    log(f"generated {lib.n} library + {q.n} query spectra in {time.time() - t0:.1f}s")

    hp = h.Params(dim=w.dim, n_levels=w.n_levels, bins_per_da=w.bins_per_da)
    t0 = time.time()
    l_csr = h.preprocess(hp, lib.offsets, lib.mz, lib.intensity)
    q_csr = h.preprocess(hp, q.offsets, q.mz, q.intensity)
    log(f"host preprocessing {time.time() - t0:.1f}s; "
        f"{l_csr[0][-1] / lib.n:.1f} peaks per library spectrum")

    ctx = h.Context(hp, device=0)
    l_dev = h.to_device_csr(*l_csr, dev)
    q_dev = h.to_device_csr(*q_csr, dev)
    l_pmz = torch.from_numpy(lib.pmz).to(dev)
    l_ch = torch.from_numpy(lib.charge).to(dev)
    q_pmz = torch.from_numpy(q.pmz).to(dev)
    q_ch = torch.from_numpy(q.charge).to(dev)
    torch.cuda.synchronize()
    t0 = time.time()
    ctx.encode_library(*l_dev, l_pmz, l_ch)
    torch.cuda.synchronize()
    lib_encode_s = time.time() - t0
    log(f"library encoded and sorted on the GPU in {lib_encode_s:.3f}s")
    del l_dev

    lo, hi = ctx.window_bounds(q_pmz, q_ch, h.TOL_DA, 500.0)
    pairs = int((hi - lo).sum().item())
    log(f"candidate pairs per step: {pairs:.4e} ({pairs / q.n:.0f} per query)")

    q_hv = torch.empty((q.n, ctx.words), dtype=torch.int32, device=dev)
    out_idx = torch.empty(q.n, dtype=torch.int64, device=dev)
    out_dist = torch.empty(q.n, dtype=torch.int32, device=dev)

    def step():
        ctx.encode_queries(*q_dev, out=q_hv)
        ctx.search_window(q_hv, q_pmz, q_ch, h.TOL_DA, 500.0, h.ENGINE_POPCOUNT,
                          out_idx=out_idx, out_dist=out_dist)

    if args.copy_calibration > 0:
        n = args.copy_calibration // 4
        src = torch.ones(n, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {4 * n} bytes read and written")
        del src, dst

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    ctx.profile_enable(True)
    ctx.profile_read()  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    log(f"timed {args.steps} steps in {elapsed:.3f}s; search kernel "
        f"{prof['search_ms'] / max(prof['search_launches'], 1):.2f} ms per launch")

    ms_per_step = 1e3 * elapsed / args.steps
    value = pairs * args.steps / elapsed
    qps = q.n * args.steps / elapsed
    words = w.dim // 32
    search_ms = prof["search_ms"] / max(prof["search_launches"], 1)
    ops_per_launch = 2.0 * words * pairs  # v_xor_b32 + v_bcnt_u32_b32 per word per pair
    achieved = ops_per_launch / (search_ms * 1e-3) / 1e12
    default_shape = args.n_ref is None and args.n_query is None and w.name == "large"
    traffic = MEASURED_TRAFFIC.get(kernel_source_hash()) if default_shape else None
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(VALU_PEAK_TOPS, 3),
                "unit": "TOP/s", "frac": round(achieved / VALU_PEAK_TOPS, 4), "traffic": traffic,
                "peak_kind": "measured xor+popcount issue rate (homs_measure_xor_popcount_rate)",
                "peak_issue_model": round(VALU_MODEL_TOPS, 3),
                "kernel": "search_popcount_kernel", "kernel_ms": round(search_ms, 3),
                "ops_per_pair": 2 * words}

    res_idx = out_idx.cpu().numpy()
    res_dist = out_dist.cpu().numpy()

    # precision form: the same search on matrix cores (fp8 e4m3 and int8 +-1)
    forms = {}
    if not args.skip_mfma:
        for name, engine in (("mfma_fp8", h.ENGINE_MFMA_F8), ("mfma_int8", h.ENGINE_MFMA_I8)):
            m_idx = torch.empty_like(out_idx)
            m_dist = torch.empty_like(out_dist)
            ctx.search_window(q_hv, q_pmz, q_ch, h.TOL_DA, 500.0, engine, m_idx, m_dist)
            torch.cuda.synchronize()
            ctx.profile_enable(True)
            ctx.profile_read()
            reps = max(1, args.steps)
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.search_window(q_hv, q_pmz, q_ch, h.TOL_DA, 500.0, engine, m_idx, m_dist)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            pm = ctx.profile_read()
            ctx.profile_enable(False)
            kms = pm["search_ms"] / max(pm["search_launches"], 1)
            same = bool(np.array_equal(m_idx.cpu().numpy(), res_idx) and
                        np.array_equal(m_dist.cpu().numpy(), res_dist))
            tops = 2.0 * w.dim * pairs / (kms * 1e-3) / 1e12
            forms[name] = {"comparisons_per_s": pairs * reps / el, "kernel_ms": round(kms, 3),
                           "achieved": round(tops, 1), "peak": MFMA_PEAK_TOPS,
                           "unit": "TOP/s", "frac": round(tops / MFMA_PEAK_TOPS, 4),
                           "vs_popcount_valu_roofline": round(
                               pairs / (kms * 1e-3) / (VALU_PEAK_TOPS * 1e12 / (2 * words)), 3),
                           "bit_exact_vs_popcount": same}
            log(f"{name}: search kernel {kms:.2f} ms ({tops:.0f} TOP/s, "
                f"{tops / MFMA_PEAK_TOPS:.1%} of peak), identical to popcount: {same}")
    cpu = None
    parity = None
    if args.cpu_sample > 0 and not args.profile_only:
        cpu, parity = cpu_baseline(args.cpu_sample, w, g, l_csr, q_csr, res_idx, res_dist)

    line = {
        "metric": METRIC, "value": value, "unit": "comparisons/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {g.meta['n_ref']} references + {g.meta['n_decoy']} "
                               f"decoys, {q.n} queries, D={w.dim}, Q={w.n_levels}, "
                               f"0.05 Da bins, +-500 Da, charge-matched",
                   "library": lib.n, "queries": q.n, "dim": w.dim, "pairs_per_step": pairs,
                   "step": "encode queries + open-window Hamming top-1 (XOR+popcount)"},
        "queries_per_s": qps,
        "library_encode_s": lib_encode_s,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity_sample": parity,
        "precision_form": forms,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def bench_batched(args, w, dev):
    """Mixed stream: 70% +-20 ppm and 30% +-500 Da windows, charges 2-4, one
    persistent launch per batch, autotuned, replayed from a hipGraph."""
    import torch

    import paper_2211_16422_amd.hyperoms as h
    from synth import make_workload

    t0 = time.time()
    g = make_workload(w, n_ref=args.n_ref, n_query=args.n_query)
    lib, q = g.library, g.queries
    log(f"generated {lib.n} library + {q.n} query spectra in {time.time() - t0:.1f}s")
    hp = h.Params(dim=w.dim, n_levels=w.n_levels, bins_per_da=w.bins_per_da)
    l_csr = h.preprocess(hp, lib.offsets, lib.mz, lib.intensity)
    q_csr = h.preprocess(hp, q.offsets, q.mz, q.intensity)
    ctx = h.Context(hp, device=0)
    l_dev = h.to_device_csr(*l_csr, dev)
    t0 = time.time()
    ctx.encode_library(*l_dev, torch.from_numpy(lib.pmz).to(dev),
                       torch.from_numpy(lib.charge).to(dev))
    torch.cuda.synchronize()
    lib_encode_s = time.time() - t0
    del l_dev
    q_pmz = torch.from_numpy(q.pmz).to(dev)
    q_ch = torch.from_numpy(q.charge).to(dev)
    kinds = torch.from_numpy(g.tol_kind).to(dev)
    values = torch.from_numpy(g.tol_value).to(dev)
    q_hv = ctx.encode_queries(*h.to_device_csr(*q_csr, dev))

    # window sizes (per-query windows), for the pair count and the histogram
    sizes = np.zeros(q.n, dtype=np.int64)
    for kind in (h.TOL_DA, h.TOL_PPM):
        sel = np.flatnonzero(g.tol_kind == kind)
        if len(sel) == 0:
            continue
        val = float(g.tol_value[sel[0]])
        lo, hi = ctx.window_bounds(q_pmz[torch.from_numpy(sel).to(dev)].contiguous(),
                                   q_ch[torch.from_numpy(sel).to(dev)].contiguous(), kind, val)
        sizes[sel] = (hi - lo).cpu().numpy()
    pairs = int(sizes.sum())
    edges = [0, 1, 10, 100, 1000, 10_000, 100_000, 1_000_000, 10_000_000]
    hist = {f"[{a},{b})": int(((sizes >= a) & (sizes < b)).sum()) for a, b in zip(edges, edges[1:])}
    log(f"pairs per batch {pairs:.4e}; window histogram {hist}")

    out_idx = torch.empty(q.n, dtype=torch.int64, device=dev)
    out_dist = torch.empty(q.n, dtype=torch.int32, device=dev)
    t0 = time.time()
    best, best_ms = ctx.autotune_batched(q_hv, q_pmz, q_ch, kinds, values, reps=1,
                                         out_idx=out_idx, out_dist=out_dist)
    log(f"autotune {time.time() - t0:.1f}s: {best} at {best_ms:.1f} ms per batch")
    # reference: one search_window per window kind with the plain kernel
    ref_idx = torch.empty_like(out_idx)
    ref_dist = torch.empty_like(out_dist)
    for kind in (h.TOL_DA, h.TOL_PPM):
        sel = torch.from_numpy(np.flatnonzero(g.tol_kind == kind)).to(dev)
        if sel.numel() == 0:
            continue
        val = float(g.tol_value[int(sel[0])])
        i, d = ctx.search_window(q_hv[sel].contiguous(), q_pmz[sel].contiguous(),
                                 q_ch[sel].contiguous(), kind, val)
        ref_idx[sel] = i
        ref_dist[sel] = d
    for _ in range(args.warmup):
        ctx.search_batched(q_hv, q_pmz, q_ch, kinds, values, True, out_idx, out_dist)
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    ctx.profile_read()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.search_batched(q_hv, q_pmz, q_ch, kinds, values, True, out_idx, out_dist)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = ctx.profile_read()
    same = bool(torch.equal(out_idx, ref_idx) and torch.equal(out_dist, ref_dist))
    words = w.dim // 32
    ms = prof["search_ms"] / max(prof["search_launches"], 1)
    tops = 2.0 * words * pairs / (ms * 1e-3) / 1e12
    line = {
        "metric": "mixed-window (70% +-20 ppm, 30% +-500 Da) Hamming comparisons/s and "
                  "queries/s, D=8192, one persistent hipGraph launch per batch",
        "value": pairs * args.steps / el, "unit": "comparisons/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": f"batched: {g.meta['n_ref']} references + {g.meta['n_decoy']} "
                               f"decoys, {q.n} queries (70% 20 ppm, 30% 500 Da), charges 2-4, "
                               f"D={w.dim}", "pairs_per_step": pairs, "window_histogram": hist,
                   "autotuned": best},
        "queries_per_s": q.n * args.steps / el,
        "library_encode_s": lib_encode_s,
        "roofline": {"bound": "alu", "achieved": round(tops, 3), "peak": round(VALU_PEAK_TOPS, 3),
                     "unit": "TOP/s", "frac": round(tops / VALU_PEAK_TOPS, 4), "traffic": None,
                     "peak_kind": "measured xor+popcount issue rate",
                     "kernel": "batched graph (persistent_search_kernel + planning)",
                     "kernel_ms": round(ms, 3)},
        "bit_exact_vs_search_window": same,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def cpu_baseline(sample, w, g, l_csr, q_csr, gpu_idx, gpu_dist):
    """The oracle on the host cores over `sample` queries of the same workload:
    the lowest-m/z queries of charge 2 with their candidate sub-library."""
    import oracle

    lib, q = g.library, g.queries
    op = oracle.Params(dim=w.dim, n_levels=w.n_levels, bins_per_da=w.bins_per_da)
    cand = np.flatnonzero(q.charge == 2)
    cand = cand[np.argsort(q.pmz[cand], kind="stable")][:sample]
    lo_m, hi_m = q.pmz[cand].min() - 500.0, q.pmz[cand].max() + 500.0
    rows = np.flatnonzero((lib.charge == 2) & (lib.pmz >= lo_m) & (lib.pmz <= hi_m))
    log(f"cpu baseline: {len(cand)} queries, sub-library of {len(rows)} spectra")
    from synth import subset
    t0 = time.time()
    idt, lvt = oracle.codebook(op)
    sub = subset(lib, rows)
    s_off, s_bin, s_lv = oracle.preprocess(sub.offsets, sub.mz, sub.intensity, op)
    sub_hv = oracle.encode(op, idt, lvt, s_off, s_bin, s_lv)
    qs = subset(q, cand)
    qo, qb, ql = oracle.preprocess(qs.offsets, qs.mz, qs.intensity, op)
    log(f"cpu baseline: oracle library side ready in {time.time() - t0:.1f}s")
    t0 = time.perf_counter()
    q_hv = oracle.encode(op, idt, lvt, qo, qb, ql)
    o_idx, o_dist = oracle.search(op, sub_hv, sub.pmz, sub.charge, q_hv, qs.pmz, qs.charge,
                                  0, 500.0)
    t = time.perf_counter() - t0
    cnt = oracle.window_counts(sub.pmz, sub.charge, qs.pmz, qs.charge, 0, 500.0)
    pairs = int(cnt.sum())
    full_idx = np.where(o_idx >= 0, rows[np.maximum(o_idx, 0)], -1)
    match = bool(np.array_equal(full_idx, gpu_idx[cand]) and np.array_equal(o_dist, gpu_dist[cand]))
    log(f"cpu baseline: {pairs:.3e} pairs in {t:.2f}s; GPU results match oracle: {match}")
    cores = oracle.max_threads()
    return ({"value": pairs / t, "unit": "comparisons/s", "cores": cores, "kind": "oracle",
             "sample": f"{len(cand)} lowest-m/z charge-2 queries of the same workload "
                       f"({pairs} candidate pairs; oracle encode of those queries + search)",
             "seconds": t},
            {"queries": int(len(cand)), "pairs": pairs, "bit_exact": match})


if __name__ == "__main__":
    main()
