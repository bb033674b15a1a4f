#!/usr/bin/env python3
"""Throughput of the HyperOMS hot path on one MI355X.

Workload (default "large"): a synthetic library of 1,000,000 references plus
1,000,000 decoys and 100,000 queries shaped like the paper's workloads
(Section 4.1, Table 1), D = 8192, 16 levels, 0.05 Da bins, open window
+-500 Da with charge matching. The library is preprocessed, uploaded and
encoded once before timing (reference hypervectors are encoded once and
reused, Section 3.3). One step = encode all query spectrum vectors (already
resident in HBM) + open-window Hamming top-1 search of every query. The
search is exact with every engine; the default engine computes the bipolar
dot products on matrix cores (fp4 e2m1 operands encoding the bits, fp32
accumulation, which is exact for these integers), and the fp8, XOR + popcount
and int8 engines are timed beside it on the same queries.

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

METRIC = "query-ref Hamming comparisons/s and queries/s at ±500 Da, D={dim}"
# issue model: 256 CUs x 4 SIMD16 units (64 lanes per clock) x 2.4 GHz. The
# xor + popcount pair the search is made of runs faster than this model on
# MI355X, so the roofline uses the rate measured live on the box
# (homs_measure_xor_popcount_rate) and reports the model beside it.
VALU_MODEL_TOPS = 256 * 64 * 2.4e9 / 1e12
MFMA_PEAK_TOPS = 5000.0  # dense fp8 / int8 matrix peak of MI355X, TFLOP/s (TOP/s)
MFMA_F4_PEAK_TOPS = 10100.0  # dense fp4 (and fp6) matrix peak of MI355X, TFLOP/s

# HBM bytes per launch of each search kernel on the default large workload,
# from rocprofv3 FETCH_SIZE and WRITE_SIZE runs scaled by a 1 GiB copy kernel
# (profiles/search_kernels_large.md). Keyed by engine and the hash of the
# kernel's sources: valid only while the source is the one measured.
MEASURED_TRAFFIC = {("popcount", "a5ee47bd0896dc11"): 4.868e12,
                    ("mfma_fp4", "cee04aab8d424ae0"): 2.6084e+11}

ENGINE_SOURCES = {"popcount": ("search_popc.hip", "popcount_tile.h"),
                  "mfma_fp8": ("search_mfma.hip", "mfma_direct.h"),
                  "mfma_fp4": ("search_mfma.hip", "mfma_direct.h"),
                  "mfma_int8": ("search_mfma.hip",)}

# per engine: element format, dense matrix peak (TFLOP/s or TOP/s), kernel name, JSON dtype
MFMA_ENGINES = {"mfma_fp8": ("fp8 e4m3", MFMA_PEAK_TOPS, "mfma_direct_kernel<0> (fp8 e4m3)",
                             "fp8e4m3(+-1)->f32"),
                "mfma_fp4": ("fp4 e2m1", MFMA_F4_PEAK_TOPS, "mfma_direct_kernel<4> (fp4 e2m1)",
                             "fp4e2m1(+-1)->f32"),
                "mfma_int8": ("int8", MFMA_PEAK_TOPS, "mfma_search_kernel (int8)",
                              "i8(+-1)->i32")}


VALU_PEAK_TOPS = VALU_MODEL_TOPS  # replaced by the live measurement in main()


def kernel_source_hash(engine: str = "popcount") -> str:
    import hashlib
    digest = hashlib.sha256()
    for name in ENGINE_SOURCES[engine]:
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
    ap.add_argument("--workload", default="large",
                    choices=["tiny", "large", "large16k", "cascade", "batched", "learned"])
    ap.add_argument("--n-ref", type=int, default=None, help="override reference count")
    ap.add_argument("--n-query", type=int, default=None, help="override query count")
    ap.add_argument("--cpu-sample", type=int, default=512,
                    help="queries in the oracle's timed sample (0 = skip)")
    ap.add_argument("--profile-only", action="store_true",
                    help="skip the CPU baseline (for profiler runs)")
    ap.add_argument("--engine", default="mfma_fp4", choices=list(ENGINE_SOURCES),
                    help="search engine of the timed step (all are bit-exact)")
    ap.add_argument("--skip-mfma", action="store_true",
                    help="time only the step's engine (no side-by-side engine timings)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="also run one device-to-device copy of BYTES bytes (a reference "
                         "kernel for scaling hardware byte counters)")
    ap.add_argument("--n-train", type=int, default=None, help="learned: training queries")
    ap.add_argument("--k", type=int, default=64, help="learned: shortlist size")
    ap.add_argument("--epochs", type=int, default=2, help="learned: training epochs")
    ap.add_argument("--batch", type=int, default=1024, help="learned: training pairs per step")
    ap.add_argument("--lr", type=float, default=3e-5, help="learned: Adam learning rate")
    ap.add_argument("--tau", type=float, default=0.02, help="learned: InfoNCE temperature")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
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
    if w.name == "learned":
        return bench_learned(args, w, dev)
    if w.name == "cascade":
        return bench_cascade(args, w, dev)
    t0 = time.time()
    g = make_workload(w, n_ref=args.n_ref, n_query=args.n_query)
    lib, q = g.library, g.queries
    log(f"generated {lib.n} library + {q.n} query spectra in {time.time() - t0:.1f}s")

    hp = h.Params(dim=w.dim, n_levels=w.n_levels, bins_per_da=w.bins_per_da)
    t0 = time.time()
    l_csr = h.preprocess(hp, lib.offsets, lib.mz, lib.intensity)
    q_csr = h.preprocess(hp, q.offsets, q.mz, q.intensity)
    host_prep_s = time.time() - t0
    log(f"host preprocessing {host_prep_s:.1f}s; "
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
    prep = prep_device_measure(ctx, lib, l_csr, dev, host_prep_s)
    encodings = encodings_measure(w, l_csr, l_pmz, l_ch, dev, lib_encode_s)

    lo, hi = ctx.window_bounds(q_pmz, q_ch, h.TOL_DA, 500.0)
    pairs = int((hi - lo).sum().item())
    log(f"candidate pairs per step: {pairs:.4e} ({pairs / q.n:.0f} per query)")

    q_hv = torch.empty((q.n, ctx.words), dtype=torch.int32, device=dev)
    out_idx = torch.empty(q.n, dtype=torch.int64, device=dev)
    out_dist = torch.empty(q.n, dtype=torch.int32, device=dev)

    engines = {"popcount": h.ENGINE_POPCOUNT, "mfma_fp8": h.ENGINE_MFMA_F8,
               "mfma_fp4": h.ENGINE_MFMA_F4, "mfma_int8": h.ENGINE_MFMA_I8}
    engine = engines[args.engine]

    def step():
        ctx.encode_queries(*q_dev, out=q_hv)
        ctx.search_window(q_hv, q_pmz, q_ch, h.TOL_DA, 500.0, engine,
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
    log(f"timed {args.steps} steps in {elapsed:.3f}s; {args.engine} search kernel "
        f"{prof['search_ms'] / max(prof['search_launches'], 1):.2f} ms per launch")

    ms_per_step = 1e3 * elapsed / args.steps
    value = pairs * args.steps / elapsed
    qps = q.n * args.steps / elapsed
    words = w.dim // 32
    default_shape = args.n_ref is None and args.n_query is None and w.name == "large"

    def roofline_of(name, kernel_ms):
        traffic = (MEASURED_TRAFFIC.get((name, kernel_source_hash(name)))
                   if default_shape else None)
        if name == "popcount":
            ops = 2.0 * words * pairs  # v_xor_b32 + v_bcnt_u32_b32 per word per pair
            ach = ops / (kernel_ms * 1e-3) / 1e12
            return {"bound": "alu", "achieved": round(ach, 3), "peak": round(VALU_PEAK_TOPS, 3),
                    "unit": "TOP/s", "frac": round(ach / VALU_PEAK_TOPS, 4), "traffic": traffic,
                    "peak_kind": "measured xor+popcount issue rate "
                                 "(homs_measure_xor_popcount_rate)",
                    "peak_issue_model": round(VALU_MODEL_TOPS, 3),
                    "kernel": "search_popcount_kernel", "kernel_ms": round(kernel_ms, 3),
                    "ops_per_pair": 2 * words}
        ops = 2.0 * w.dim * pairs  # one multiply-add per component per pair
        ach = ops / (kernel_ms * 1e-3) / 1e12
        fmt, peak, kernel, _ = MFMA_ENGINES[name]
        return {"bound": "mfma", "achieved": round(ach, 1), "peak": peak,
                "unit": "TOP/s" if name == "mfma_int8" else "TFLOP/s",
                "frac": round(ach / peak, 4), "traffic": traffic,
                "peak_kind": f"dense {fmt} matrix peak of MI355X",
                "kernel": kernel, "kernel_ms": round(kernel_ms, 3),
                "ops_per_pair": 2 * w.dim}

    search_ms = prof["search_ms"] / max(prof["search_launches"], 1)
    roofline = roofline_of(args.engine, search_ms)
    res_idx = out_idx.cpu().numpy()
    res_dist = out_dist.cpu().numpy()

    # the other engines on the same queries: same results, their own rooflines
    forms = {}
    if not args.skip_mfma:
        for name, eng in engines.items():
            if name == args.engine:
                continue
            m_idx = torch.empty_like(out_idx)
            m_dist = torch.empty_like(out_dist)
            ctx.search_window(q_hv, q_pmz, q_ch, h.TOL_DA, 500.0, eng, m_idx, m_dist)
            torch.cuda.synchronize()
            ctx.profile_enable(True)
            ctx.profile_read()
            reps = max(1, args.steps)
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.search_window(q_hv, q_pmz, q_ch, h.TOL_DA, 500.0, eng, m_idx, m_dist)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            pm = ctx.profile_read()
            ctx.profile_enable(False)
            kms = pm["search_ms"] / max(pm["search_launches"], 1)
            same = bool(np.array_equal(m_idx.cpu().numpy(), res_idx) and
                        np.array_equal(m_dist.cpu().numpy(), res_dist))
            forms[name] = {"comparisons_per_s": pairs * reps / el,
                           "roofline": roofline_of(name, kms),
                           f"bit_exact_vs_{args.engine}": same}
            log(f"{name}: search kernel {kms:.2f} ms, identical to {args.engine}: {same}")
    cpu = None
    parity = None
    if args.cpu_sample > 0 and not args.profile_only:
        cpu, parity = cpu_baseline(args.cpu_sample, w, g, l_csr, q_csr, res_idx, res_dist)

    line = {
        "metric": METRIC.format(dim=w.dim), "value": value, "unit": "comparisons/s",
        "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32" if args.engine == "popcount" else MFMA_ENGINES[args.engine][3],
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {g.meta['n_ref']} references + {g.meta['n_decoy']} "
                               f"decoys, {q.n} queries, D={w.dim}, Q={w.n_levels}, "
                               f"0.05 Da bins, +-500 Da, charge-matched",
                   "library": lib.n, "queries": q.n, "dim": w.dim, "pairs_per_step": pairs,
                   "engine": args.engine,
                   "step": "encode queries + open-window Hamming top-1 (exact; "
                           f"{args.engine} engine)"},
        "queries_per_s": qps,
        "library_encode_s": lib_encode_s,
        "prep_device": prep,
        "library_encode_s_by_encoding": encodings,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity_sample": parity,
        "other_engines": forms,
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
    if best["engine"] in (h.ENGINE_MFMA_F8, h.ENGINE_MFMA_F4):
        name = "mfma_fp8" if best["engine"] == h.ENGINE_MFMA_F8 else "mfma_fp4"
        fmt, peak, _, dtype = MFMA_ENGINES[name]
        tops = 2.0 * w.dim * pairs / (ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(tops, 1), "peak": peak,
                "unit": "TFLOP/s", "frac": round(tops / peak, 4), "traffic": None,
                "peak_kind": f"dense {fmt} matrix peak of MI355X (wide tiles; narrow "
                             "windows are scored by popcount in the same launch)",
                "kernel": f"batched graph (persistent_search_kernel<{fmt}> + planning)",
                "kernel_ms": round(ms, 3)}
    else:
        tops = 2.0 * words * pairs / (ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(tops, 3), "peak": round(VALU_PEAK_TOPS, 3),
                "unit": "TOP/s", "frac": round(tops / VALU_PEAK_TOPS, 4), "traffic": None,
                "peak_kind": "measured xor+popcount issue rate",
                "kernel": "batched graph (persistent_search_kernel<popcount> + planning)",
                "kernel_ms": round(ms, 3)}
    line = {
        "metric": "mixed-window (70% +-20 ppm, 30% +-500 Da) Hamming comparisons/s and "
                  "queries/s, D=8192, one persistent hipGraph launch per batch",
        "value": pairs * args.steps / el, "unit": "comparisons/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype if best["engine"] != h.ENGINE_POPCOUNT else "u32",
        "data": "synthetic",
        "config": {"workload": f"batched: {g.meta['n_ref']} references + {g.meta['n_decoy']} "
                               f"decoys, {q.n} queries (70% 20 ppm, 30% 500 Da), charges 2-4, "
                               f"D={w.dim}", "pairs_per_step": pairs, "window_histogram": hist,
                   "autotuned": best},
        "queries_per_s": q.n * args.steps / el,
        "library_encode_s": lib_encode_s,
        "roofline": roof,
        "bit_exact_vs_search_window": same,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def bench_learned(args, w, dev):
    """Learned shortlist: MLP D -> 1024 -> 256 trained on the GPU on (training
    query, exact top-1) pairs; per query the top-k window candidates by
    embedding score are rescored exactly, with exhaustive fallback. Reports
    queries/s and window comparisons covered per second, top-1 agreement
    with the exhaustive search and the speedup over it."""
    import torch

    import paper_2211_16422_amd.hyperoms as h
    from synth import make_workload

    t0 = time.time()
    g = make_workload(w, n_ref=args.n_ref, n_query=args.n_query, n_train=args.n_train)
    lib, q, tr = g.library, g.queries, g.train
    log(f"generated {lib.n} library + {q.n} query + {tr.n} training spectra in "
        f"{time.time() - t0:.1f}s")
    hp = h.Params(dim=w.dim, n_levels=w.n_levels, bins_per_da=w.bins_per_da)
    ctx = h.Context(hp, device=0)
    l_dev = h.to_device_csr(*h.preprocess(hp, lib.offsets, lib.mz, lib.intensity), dev)
    ctx.encode_library(*l_dev, torch.from_numpy(lib.pmz).to(dev),
                       torch.from_numpy(lib.charge).to(dev))
    del l_dev
    q_hv = ctx.encode_queries(*h.to_device_csr(*h.preprocess(hp, q.offsets, q.mz,
                                                             q.intensity), dev))
    t_hv = ctx.encode_queries(*h.to_device_csr(*h.preprocess(hp, tr.offsets, tr.mz,
                                                             tr.intensity), dev))
    q_pmz, q_ch = torch.from_numpy(q.pmz).to(dev), torch.from_numpy(q.charge).to(dev)
    t_pmz, t_ch = torch.from_numpy(tr.pmz).to(dev), torch.from_numpy(tr.charge).to(dev)
    lo, hi = ctx.window_bounds(q_pmz, q_ch, h.TOL_DA, 500.0)
    pairs = int((hi - lo).sum().item())
    torch.cuda.synchronize()
    log(f"encoded; {pairs:.4e} window pairs for {q.n} queries")

    # exhaustive reference (and timing) on the evaluation queries
    ctx.profile_enable(True)
    ctx.profile_read()
    ex = {}
    for name, engine in (("popcount", h.ENGINE_POPCOUNT), ("mfma_fp8", h.ENGINE_MFMA_F8),
                         ("mfma_fp4", h.ENGINE_MFMA_F4)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e_idx, e_dist = ctx.search_window(q_hv, q_pmz, q_ch, h.TOL_DA, 500.0, engine)
        torch.cuda.synchronize()
        ex[name] = time.perf_counter() - t0
    ctx.profile_read()
    log(f"exhaustive search: popcount {ex['popcount']:.2f}s, fp8 {ex['mfma_fp8']:.2f}s, "
        f"fp4 {ex['mfma_fp4']:.2f}s")

    # training pairs: exact top-1 of the training queries, batched in m/z order
    t0 = time.perf_counter()
    t_idx, _ = ctx.search_window(t_hv, t_pmz, t_ch, h.TOL_DA, 500.0, h.ENGINE_MFMA_F4)
    lib_rows = ctx.library_export()
    order = torch.from_numpy(np.lexsort((tr.pmz, tr.charge))).to(dev)
    order = order[t_idx[order] >= 0]
    B = args.batch
    nb = order.numel() // B
    order = order[:nb * B]
    tq = t_hv[order].contiguous()
    tr_rows = lib_rows[t_idx[order]].contiguous()
    del lib_rows
    torch.cuda.synchronize()
    label_s = time.perf_counter() - t0
    log(f"training labels: {order.numel()} pairs in {label_s:.1f}s")

    rng = np.random.default_rng(12345)
    H, E, D = 1024, 256, w.dim
    wts = {"W1": (rng.uniform(-1, 1, (H, D)) / np.sqrt(D)).astype(np.float32),
           "b1": np.zeros(H, np.float32),
           "W2": (rng.uniform(-1, 1, (E, H)) / np.sqrt(H)).astype(np.float32),
           "b2": np.zeros(E, np.float32)}
    model = h.Model(ctx, wts)
    has = e_idx >= 0

    def evaluate(tag):
        model.embed_library()
        idx, dist, fb = model.search(q_hv, q_pmz, q_ch, args.k)
        agree = float(((idx == e_idx) & (dist == e_dist))[has].float().mean().item())
        fbr = float(fb.float().mean().item())
        log(f"{tag}: top-1 agreement {agree:.4f}, fallback {fbr:.4f}")
        return agree, fbr

    agree0, _ = evaluate("untrained")
    t0 = time.perf_counter()
    losses = []
    gen = torch.Generator().manual_seed(0)
    for ep in range(args.epochs):
        for b in torch.randperm(nb, generator=gen).tolist():
            sl = slice(b * B, (b + 1) * B)
            losses.append(model.train_step(tq[sl], tr_rows[sl], args.tau, args.lr).clone())
        torch.cuda.synchronize()
        log(f"epoch {ep + 1}/{args.epochs}: mean loss "
            f"{torch.cat(losses[-nb:]).mean().item():.4f}")
    train_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    model.embed_library()
    torch.cuda.synchronize()
    embed_lib_s = time.perf_counter() - t0
    agree, fbr = evaluate("trained")

    for _ in range(args.warmup):
        model.search(q_hv, q_pmz, q_ch, args.k)
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    ctx.profile_read()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        idx, dist, fb = model.search(q_hv, q_pmz, q_ch, args.k)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    step_s = el / args.steps
    score_ms = prof["score_ms"] / args.steps
    flops = 2.0 * E * pairs  # one E-dim dot product per window pair
    tflops = flops / (score_ms * 1e-3) / 1e12
    line = {
        "metric": "learned-shortlist open search: queries/s and window comparisons covered/s "
                  f"at +-500 Da, D={D}, k={args.k}",
        "value": q.n / step_s, "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * step_s, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"learned: {g.meta['n_ref']} references + {g.meta['n_decoy']} "
                               f"decoys, {q.n} queries, {order.numel()} training pairs, "
                               f"D={D}, MLP {D}-{H}-{E}, k={args.k}",
                   "pairs_per_step": pairs, "epochs": args.epochs, "batch": B,
                   "lr": args.lr, "tau": args.tau},
        "comparisons_covered_per_s": pairs / step_s,
        "top1_agreement": agree, "top1_agreement_untrained": agree0, "fallback_rate": fbr,
        "exhaustive_s": ex, "speedup_vs_popcount": ex["popcount"] / step_s,
        "speedup_vs_mfma_fp8": ex["mfma_fp8"] / step_s,
        "speedup_vs_mfma_fp4": ex["mfma_fp4"] / step_s,
        "train_s": train_s, "train_steps": len(losses), "label_s": label_s,
        "embed_library_s": embed_lib_s,
        "roofline": {"bound": "mfma", "achieved": round(tflops, 1), "peak": 2500.0,
                     "unit": "TFLOP/s", "frac": round(tflops / 2500.0, 4), "traffic": None,
                     "kernel": "collect_kernel (bf16 scoring)", "kernel_ms": round(score_ms, 3),
                     "flops_per_pair": 2 * E},
        "phase_ms": {"search": prof["search_ms"] / args.steps,
                     "prep_and_embed": prof["prep_ms"] / args.steps},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    model.close()
    ctx.close()


def encodings_measure(w, l_csr, l_pmz, l_ch, dev, id_level_s):
    """Library encode + sort time with the encoding baselines of Section 4.2
    (random position vectors; random-projection LSH) beside the paper's."""
    import torch

    import paper_2211_16422_amd.hyperoms as h
    out = {"id_level": round(id_level_s, 4)}
    for name, enc in (("random_id", h.ENCODING_RANDOM_ID), ("lsh", h.ENCODING_LSH)):
        c2 = h.Context(h.Params(dim=w.dim, n_levels=w.n_levels, bins_per_da=w.bins_per_da,
                                encoding=enc), device=0)
        l_dev = h.to_device_csr(*l_csr, dev)
        c2.encode_library(*l_dev, l_pmz, l_ch)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c2.encode_library(*l_dev, l_pmz, l_ch)
        torch.cuda.synchronize()
        out[name] = round(time.perf_counter() - t0, 4)
        c2.close()
        del l_dev
    log(f"library encode + sort by encoding (s): {out}")
    return out


def prep_device_measure(ctx, lib, l_csr, dev, host_prep_s):
    """Device preprocessing (homs_preprocess_device) of the library's raw peaks,
    already in HBM: time, identity with the host path, and HBM roofline over
    the algorithmic bytes (raw m/z and intensity read once, offsets, output
    bins and levels written once)."""
    import torch

    off = torch.from_numpy(lib.offsets).to(dev)
    mz = torch.from_numpy(lib.mz).to(dev)
    inten = torch.from_numpy(lib.intensity).to(dev)
    ctx.preprocess_device(off, mz, inten)  # warm-up (workspace, code objects)
    torch.cuda.synchronize()
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        o, b, lv = ctx.preprocess_device(off, mz, inten)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    same = bool(np.array_equal(o.cpu().numpy(), l_csr[0]) and
                np.array_equal(b.cpu().numpy(), l_csr[1]) and
                np.array_equal(lv.cpu().numpy(), l_csr[2]))
    raw = int(lib.offsets[-1])
    entries = int(l_csr[0][-1])
    nbytes = 16 * raw + 8 * 2 * (lib.n + 1) + 5 * entries
    gbs = nbytes / (ms * 1e-3) / 1e9
    log(f"device preprocessing of {lib.n} library spectra ({raw} raw peaks): {ms:.2f} ms, "
        f"identical to the host path: {same}")
    del off, mz, inten
    return {"spectra": lib.n, "raw_peaks": raw, "ms": round(ms, 3),
            "spectra_per_s": lib.n / (ms * 1e-3), "identical_to_host": same,
            "host_prep_s_library_and_queries": round(host_prep_s, 3),
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0,
                         "unit": "GB/s", "frac": round(gbs / 8000.0, 4),
                         "algorithmic_bytes": nbytes,
                         "kernel": "preprocess_wave_kernel (one staged pass) + scan "
                                   "+ compaction",
                         "note": "bounded by the per-spectrum rank counting in LDS "
                                 "(O(peaks^2) double compares), not by HBM"}}


def bench_cascade(args, w, dev):
    """Cascade search (Section 3.4) with 1% target-decoy FDR (Sections 2.1,
    4.1) on the large workload's data: a step encodes the queries and runs
    homs_cascade_search (+-20 ppm standard search, FDR, +-500 Da open search
    of the unidentified queries, FDR) on the fp4 engine."""
    import torch

    import paper_2211_16422_amd.hyperoms as h
    from synth import make_workload

    t0 = time.time()
    g = make_workload(w, n_ref=args.n_ref, n_query=args.n_query)
    lib, q = g.library, g.queries
    n_ref = g.meta["n_ref"]
    log(f"generated {lib.n} library + {q.n} query spectra in {time.time() - t0:.1f}s")
    hp = h.Params(dim=w.dim, n_levels=w.n_levels, bins_per_da=w.bins_per_da)
    l_csr = h.preprocess(hp, lib.offsets, lib.mz, lib.intensity)
    q_csr = h.preprocess(hp, q.offsets, q.mz, q.intensity)
    ctx = h.Context(hp, device=0)
    l_dev = h.to_device_csr(*l_csr, dev)
    ctx.encode_library(*l_dev, torch.from_numpy(lib.pmz).to(dev),
                       torch.from_numpy(lib.charge).to(dev))
    del l_dev
    q_dev = h.to_device_csr(*q_csr, dev)
    q_pmz = torch.from_numpy(q.pmz).to(dev)
    q_ch = torch.from_numpy(q.charge).to(dev)
    decoy = torch.from_numpy((np.arange(lib.n) >= n_ref).astype(np.uint8)).to(dev)
    q_hv = torch.empty((q.n, ctx.words), dtype=torch.int32, device=dev)
    narrow, wide, level = (h.TOL_PPM, 20.0), (h.TOL_DA, 500.0), 0.01

    def step():
        ctx.encode_queries(*q_dev, out=q_hv)
        return ctx.cascade_search(q_hv, q_pmz, q_ch, decoy, narrow, wide, h.ENGINE_MFMA_F4,
                                  level)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    ctx.profile_read()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    idx, dist, stage, qv = (t.cpu().numpy() for t in out)
    n1, n2 = int(np.sum(stage == 1)), int(np.sum(stage == 2))
    # candidate pairs searched per step: every query narrow, the rest open
    lo, hi = ctx.window_bounds(q_pmz, q_ch, *narrow)
    pairs_narrow = int((hi - lo).sum().item())
    rest = torch.from_numpy(np.flatnonzero(stage != 1)).to(dev)
    lo, hi = ctx.window_bounds(q_pmz[rest].contiguous(), q_ch[rest].contiguous(), *wide)
    pairs_open = int((hi - lo).sum().item())
    pairs = pairs_narrow + pairs_open
    search_ms = prof["search_ms"] / max(args.steps, 1)  # both stages' search kernels
    tflops = 2.0 * w.dim * pairs / (search_ms * 1e-3) / 1e12
    log(f"stage 1: {n1}, stage 2: {n2}, unidentified {q.n - n1 - n2}; pairs narrow "
        f"{pairs_narrow:.3e}, open {pairs_open:.3e}; search kernels {search_ms:.1f} ms per step")
    cpu = None
    if args.cpu_sample > 0 and not args.profile_only:
        cpu = cascade_cpu_baseline(args.cpu_sample, w, g, n_ref, idx, dist, stage)
    line = {
        "metric": "cascade search queries/s (+-20 ppm standard search, 1% FDR, +-500 Da open "
                  f"search of the unidentified queries, 1% FDR), D={w.dim}",
        "value": q.n * args.steps / el, "unit": "queries/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": MFMA_ENGINES["mfma_fp4"][3], "data": "synthetic",
        "config": {"workload": f"cascade: {n_ref} references + {g.meta['n_decoy']} decoys, "
                               f"{q.n} queries (half with a precursor mass shift), D={w.dim}, "
                               "fp4 engine", "pairs_per_step": pairs,
                   "pairs_narrow": pairs_narrow, "pairs_open": pairs_open},
        "identified_stage1": n1, "identified_stage2": n2,
        "comparisons_per_s": pairs * args.steps / el,
        "roofline": {"bound": "mfma", "achieved": round(tflops, 1), "peak": MFMA_F4_PEAK_TOPS,
                     "unit": "TFLOP/s", "frac": round(tflops / MFMA_F4_PEAK_TOPS, 4),
                     "traffic": None,
                     "peak_kind": "dense fp4 e2m1 matrix peak of MI355X",
                     "kernel": "mfma_direct_kernel<4> (both stages)",
                     "kernel_ms": round(search_ms, 3), "ops_per_pair": 2 * w.dim},
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def cascade_cpu_baseline(sample, w, g, n_ref, gpu_idx, gpu_dist, gpu_stage):
    """The oracle cascade on the host cores over `sample` queries (the lowest
    m/z queries of charge 2, their candidate sub-library). Its FDR is over the
    sample's PSMs only, so stages may differ from the full run; each query's
    matches are checked instead: the GPU's stage-1 identifications against
    the oracle's narrow top-1, the others against its open top-1."""
    import oracle
    from oracle import fdr

    lib, q = g.library, g.queries
    op = oracle.Params(dim=w.dim, n_levels=w.n_levels, bins_per_da=w.bins_per_da)
    cand = np.flatnonzero(q.charge == 2)
    cand = cand[np.argsort(q.pmz[cand], kind="stable")][:sample]
    lo_m, hi_m = q.pmz[cand].min() - 500.0, q.pmz[cand].max() + 500.0
    rows = np.flatnonzero((lib.charge == 2) & (lib.pmz >= lo_m) & (lib.pmz <= hi_m))
    from synth import subset
    idt, lvt = oracle.codebook(op)
    sub = subset(lib, rows)
    sub_hv = oracle.encode_raw(op, idt, lvt, sub)
    qs = subset(q, cand)
    qo, qb, ql = oracle.preprocess(qs.offsets, qs.mz, qs.intensity, op)
    t0 = time.perf_counter()
    q_hv = oracle.encode(op, idt, lvt, qo, qb, ql)
    fdr.cascade(op, sub_hv, sub.pmz, sub.charge, rows >= n_ref, q_hv, qs.pmz, qs.charge,
                (1, 20.0), (0, 500.0), 0.01)
    t = time.perf_counter() - t0
    n_idx, n_dist = oracle.search(op, sub_hv, sub.pmz, sub.charge, q_hv, qs.pmz, qs.charge,
                                  1, 20.0)
    o_idx, o_dist = oracle.search(op, sub_hv, sub.pmz, sub.charge, q_hv, qs.pmz, qs.charge,
                                  0, 500.0)
    s1 = gpu_stage[cand] == 1
    want_idx = np.where(s1, n_idx, o_idx)
    want_dist = np.where(s1, n_dist, o_dist)
    want_idx = np.where(want_idx >= 0, rows[np.maximum(want_idx, 0)], -1)
    match = bool(np.array_equal(want_idx, gpu_idx[cand]) and
                 np.array_equal(want_dist, gpu_dist[cand]))
    log(f"cpu baseline: cascade of {len(cand)} queries in {t:.2f}s; GPU matches agree: {match}")
    return {"value": len(cand) / t, "unit": "queries/s", "cores": oracle.max_threads(),
            "kind": "oracle",
            "sample": f"{len(cand)} lowest-m/z charge-2 queries of the same workload with their "
                      f"{len(rows)}-spectrum candidate sub-library (oracle encode of the queries + "
                      "cascade with FDR over the sample's PSMs)",
            "seconds": t, "matches_bit_exact": match}


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
