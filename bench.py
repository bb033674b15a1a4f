#!/usr/bin/env python3
"""Throughput of the HyperOMS hot path on one MI355X.

Default workload ("large"): a synthetic library of 1,000,000 references plus
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

The default run also measures, under extra keys of the same line, the batched
form ("batched": 2M + 2M library, 200,000 queries of mixed narrow and open
windows in one persistent hipGraph launch) and the learned form at a moderate
size ("learned": the large workload's library and queries, a D-1024-256 MLP
trained on the GPU on 300,000 labelled training queries, k = 64 shortlists)
and the cascade ("cascade": the same library and queries, +-20 ppm standard
search, 1% FDR, +-500 Da open search of the unidentified queries, 1% FDR).

Prints one JSON line: comparisons/s (sum of candidate-window sizes per
second), queries/s, the roofline of each kernel measured with HIP events
inside the library, and the oracle timed on the host cores on a random
sample of each workload, whose results are also the parity sample.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
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
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of each search kernel on the default large workload,
# from rocprofv3 FETCH_SIZE and WRITE_SIZE runs scaled by a 1 GiB copy kernel
# (profiles/search_kernels_large.md). Keyed by engine and the hash of the
# kernel's sources: valid only while the source is the one measured.
MEASURED_TRAFFIC = {("popcount", "8a0818167cd6a169"): 4.868e12,
                    ("mfma_fp4", "6cc7539ab6528dd9"): 2.5363e+11}

ENGINE_SOURCES = {"popcount": ("search_popc.hip", "popcount_tile.h"),
                  "mfma_fp8": ("search_mfma.hip", "mfma_direct.h"),
                  "mfma_fp4": ("search_mfma.hip", "mfma_direct.h"),
                  "mfma_int8": ("search_mfma.hip", "mfma_direct.h")}

# per engine: element format, dense matrix peak (TFLOP/s or TOP/s), kernel name, JSON dtype
MFMA_ENGINES = {"mfma_fp8": ("fp8 e4m3", MFMA_PEAK_TOPS, "mfma_direct_kernel<0> (fp8 e4m3)",
                             "fp8e4m3(+-1)->f32"),
                "mfma_fp4": ("fp4 e2m1", MFMA_F4_PEAK_TOPS, "mfma_direct_kernel<4> (fp4 e2m1)",
                             "fp4e2m1->f32"),
                "mfma_int8": ("int8", MFMA_PEAK_TOPS, "mfma_direct_kernel<8> (int8 +-64)",
                              "i8(+-64)->i32")}

SAMPLE_SEED = 2024  # seed of every oracle sample (queries drawn without replacement)
N_TRAIN_MODERATE = 300_000  # training queries of the learned leg of the default run

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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def random_sample(n: int, size: int, seed: int = SAMPLE_SEED) -> np.ndarray:
    """`size` distinct query indices drawn at random, ascending."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=min(size, n), replace=False))


# ---------------------------------------------------------------------------
# oracle side: untimed set-up on a background thread, timed runs at the end

class OracleJobs:
    """Runs the oracle's untimed set-up (its codebook and its encoding of the
    library rows a sample can reach) on one background thread while the GPU
    legs run; the oracle's C code releases the interpreter lock. The timed
    oracle runs happen only after every job has finished."""

    def __init__(self):
        self._ex = cf.ThreadPoolExecutor(max_workers=1)

    def submit(self, fn, *a):
        return self._ex.submit(fn, *a)

    def close(self):
        self._ex.shutdown(wait=True)


def tolerances(pmz, kinds, values):
    """Per-query tolerance in Da (kind 0 = Da, 1 = ppm), as the window rule."""
    pmz = np.asarray(pmz, np.float64)
    k = np.broadcast_to(np.asarray(kinds), pmz.shape)
    v = np.broadcast_to(np.asarray(values, np.float64), pmz.shape)
    return np.where(k == 0, v, pmz * v / 1e6)


def oracle_library_side(w, lib, q_pmz, q_charge, kinds, values):
    """Untimed: the oracle's codebook and its encoding (from the raw peaks) of
    every library row of a charge in the sample whose precursor lies within
    the sample's widest reach for that charge (a superset of the union of the
    sampled queries' windows; the oracle applies the window rule itself)."""
    import oracle
    from synth import subset

    t0 = time.time()
    op = oracle.Params(dim=w.dim, n_levels=w.n_levels, bins_per_da=w.bins_per_da)
    tol = tolerances(q_pmz, kinds, values)
    mask = np.zeros(lib.n, dtype=bool)
    for c in np.unique(q_charge):
        sel = q_charge == c
        lo = float(np.min(q_pmz[sel] - tol[sel])) - 1.0
        hi = float(np.max(q_pmz[sel] + tol[sel])) + 1.0
        mask |= (lib.charge == c) & (lib.pmz >= lo) & (lib.pmz <= hi)
    rows = np.flatnonzero(mask)
    idt, lvt = oracle.codebook(op)
    sub = subset(lib, rows)
    sub_hv = oracle.encode_raw(op, idt, lvt, sub)
    log(f"oracle set-up: {len(rows)} library rows encoded in {time.time() - t0:.1f}s "
        f"(untimed, background)")
    return {"op": op, "idt": idt, "lvt": lvt, "rows": rows, "pmz": sub.pmz,
            "charge": sub.charge, "hv": sub_hv}


def oracle_timed_search(side, qs, kinds, values):
    """Timed: the oracle encodes the sampled queries (preprocessed untimed)
    and searches them over its sub-library. Returns seconds, top-1 in full
    library indices, distances, the oracle's query rows and the pair count."""
    import oracle
    op = side["op"]
    qo, qb, ql = oracle.preprocess(qs.offsets, qs.mz, qs.intensity, op)
    t0 = time.perf_counter()
    q_hv = oracle.encode(op, side["idt"], side["lvt"], qo, qb, ql)
    o_idx, o_dist = oracle.search(op, side["hv"], side["pmz"], side["charge"], q_hv, qs.pmz,
                                  qs.charge, kinds, values)
    t = time.perf_counter() - t0
    cnt = oracle.window_counts(side["pmz"], side["charge"], qs.pmz, qs.charge, kinds, values)
    rows = side["rows"]
    full_idx = np.where(o_idx >= 0, rows[np.maximum(o_idx, 0)], -1)
    return t, full_idx, o_dist, q_hv, int(cnt.sum())


def cpu_entry(value, unit, sample_desc, seconds):
    import oracle
    return {"value": value, "unit": unit, "cores": oracle.max_threads(), "kind": "oracle",
            "sample": sample_desc, "seconds": round(seconds, 3), "cpu_model": cpu_model()}


# ---------------------------------------------------------------------------

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
                    help="skip the CPU baselines and the extra legs (for profiler runs)")
    ap.add_argument("--no-extra", action="store_true",
                    help="large workload only: skip the learned, cascade and batched legs")
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
    ap.add_argument("--init", default="random", choices=["random", "sketch"],
                    help="learned: initial weights of training (random, or the centred "
                         "training-free sketch)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(queries would be sharded across GPUs with the library replicated); "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2211_16422_amd.hyperoms as h
    from synth import WORKLOADS

    global VALU_PEAK_TOPS
    VALU_PEAK_TOPS = h.measure_xor_popcount_rate(0) / 1e12
    log(f"measured xor+popcount rate {VALU_PEAK_TOPS:.2f} T lane-ops/s "
        f"(issue model {VALU_MODEL_TOPS:.2f})")
    w = WORKLOADS[args.workload]
    dev = torch.device("cuda", 0)
    jobs = OracleJobs()
    try:
        if w.name == "batched":
            line, finish = batched_leg(args, w, dev, jobs)
            jobs.close()
            finish()
        elif w.name == "learned":
            line = bench_learned_full(args, w, dev, jobs)
        elif w.name == "cascade":
            line = bench_cascade(args, w, dev, jobs)
        else:
            line = bench_large(args, w, dev, jobs)
    finally:
        jobs.close()
    print(json.dumps(line), flush=True)


def bench_large(args, w, dev, jobs):
    import torch

    import paper_2211_16422_amd.hyperoms as h
    from synth import WORKLOADS, make_workload, subset

    t0 = time.time()
    g = make_workload(w, n_ref=args.n_ref, n_query=args.n_query)
    lib, q = g.library, g.queries
    log(f"generated {lib.n} library + {q.n} query spectra in {time.time() - t0:.1f}s")
    want_cpu = args.cpu_sample > 0 and not args.profile_only
    sample = random_sample(q.n, args.cpu_sample) if want_cpu else None
    side = (jobs.submit(oracle_library_side, w, lib, q.pmz[sample], q.charge[sample], 0, 500.0)
            if want_cpu else None)

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
    ctx.profile_enable(True)
    ctx.profile_read()
    t0 = time.time()
    ctx.encode_library(*l_dev, l_pmz, l_ch)
    torch.cuda.synchronize()
    lib_encode_s = time.time() - t0
    pe = ctx.profile_read()
    ctx.profile_enable(False)
    log(f"library encoded and sorted on the GPU in {lib_encode_s:.3f}s (encode kernels "
        f"{pe['encode_ms']:.2f} ms, sort {pe['prep_ms']:.2f} ms)")
    encode = encode_roofline(w, l_csr, lib.n, pe["encode_ms"], pe["prep_ms"])
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
            reps = max(1, min(args.steps, 5))
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
        "encode": encode,
        "prep_device": prep,
        "library_encode_s_by_encoding": encodings,
        "roofline": roofline,
        "cpu_baseline": None,
        "parity_sample": None,
        "other_engines": forms,
    }

    learned_state = None
    extra = (w.name == "large" and default_shape and not args.no_extra and not args.profile_only)
    if extra:
        # the learned workload at a moderate size has exactly this library and
        # these queries (same seed and generator); its training queries are
        # the learned workload's own stream
        side_ready = side.result() if side is not None else None  # no oracle load while timing
        del side_ready
        from synth import make_training_queries
        tr = make_training_queries(g, N_TRAIN_MODERATE)
        lw = WORKLOADS["learned"]
        desc = (f"learned (moderate): {g.meta['n_ref']} references + {g.meta['n_decoy']} "
                f"decoys, {q.n} queries, {N_TRAIN_MODERATE} training queries, D={w.dim}")
        learned, learned_state = learned_leg(args, lw, ctx, dev, q_hv, q_pmz, q_ch, tr, desc,
                                             args.k)
        line["learned"] = learned
        del tr
    cascade_result = None
    if extra:
        # the cascade (narrow search, FDR, open search of the rest) on the same
        # library and queries
        line["cascade"], cascade_result = cascade_leg(args, w, g, ctx, dev, q_dev, q_pmz, q_ch)
    ctx.close()
    del q_dev, l_pmz, l_ch, q_pmz, q_ch, q_hv, out_idx, out_dist
    torch.cuda.empty_cache()

    finish_batched = None
    if extra:
        batched, finish_batched = batched_leg(args, WORKLOADS["batched"], dev, jobs)
        line["batched"] = batched

    # timed oracle runs, after every background job has finished
    jobs.close()
    if side is not None:
        s = side.result()
        qs = subset(q, sample)
        t, o_idx, o_dist, o_qhv, spairs = oracle_timed_search(s, qs, 0, 500.0)
        match = bool(np.array_equal(o_idx, res_idx[sample]) and
                     np.array_equal(o_dist, res_dist[sample]))
        log(f"cpu baseline: {len(sample)} random queries, {spairs:.3e} pairs in {t:.2f}s; GPU "
            f"results match the oracle: {match}")
        desc = (f"{len(sample)} queries drawn at random (seed {SAMPLE_SEED}, across charges and "
                f"precursor m/z) from the {q.n} of the same workload ({spairs} candidate pairs; "
                "oracle encode of those queries + search; its library rows encoded untimed)")
        line["cpu_baseline"] = cpu_entry(spairs / t, "comparisons/s", desc, t)
        line["parity_sample"] = {"queries": int(len(sample)), "pairs": spairs,
                                 "sampling": f"random, seed {SAMPLE_SEED}", "bit_exact": match}
        if learned_state is not None:
            finish_learned(line["learned"], learned_state, sample, s, o_idx, o_dist, o_qhv, t,
                           desc)
        if cascade_result is not None:
            line["cascade"]["cpu_baseline"] = cascade_cpu_baseline(s, sample, g, *cascade_result)
    if finish_batched is not None:
        finish_batched()
    return line


def encode_roofline(w, l_csr, n, encode_ms, sort_ms):
    """Library encode (Eq. 1) against two models. Ops: binding and bundling
    cost one 32-bit operation each per peak and packed word (2 * n_peaks *
    D/32 per spectrum, as the search's 2 ops per word per pair), against the
    VALU issue model. HBM: CSR entries read (5 bytes per peak), packed rows
    written (D/8 per spectrum); the position-vector rows gathered per peak
    come from the 27 MiB table held in cache, not HBM."""
    peaks = int(l_csr[0][-1])
    words = w.dim // 32
    ops = 2.0 * peaks * words
    s = encode_ms * 1e-3
    tops = ops / s / 1e12
    hbm = 5.0 * peaks + (w.dim // 8) * n + 8.0 * (n + 1)
    gbs = hbm / s / 1e9
    gather = 2.0 * peaks * (w.dim // 8) / s / 1e9
    return {"spectra": n, "peaks": peaks, "kernel_ms": round(encode_ms, 3),
            "sort_ms": round(sort_ms, 3), "spectra_per_s": n / s,
            "roofline": {"bound": "alu", "achieved": round(tops, 3),
                         "peak": round(VALU_MODEL_TOPS, 3), "unit": "TOP/s",
                         "frac": round(tops / VALU_MODEL_TOPS, 4), "traffic": None,
                         "ops_model": "2 ops (bind + bundle) per peak per 32-bit word",
                         "kernel": "encode_kernel (all peak-count classes)"},
            "hbm": {"achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(gbs / HBM_PEAK_GBS, 5), "algorithmic_bytes": hbm},
            "cache_gather_GBs": round(gather, 1)}


def exhaustive_times(ctx, h, q_hv, q_pmz, q_ch, reps=3):
    """Warm timings (median of `reps` after one warm-up) of the exhaustive
    search engines on the same queries, and the fp4 engine's results."""
    import torch
    out, res = {}, None
    for name, engine in (("popcount", h.ENGINE_POPCOUNT), ("mfma_fp8", h.ENGINE_MFMA_F8),
                         ("mfma_fp4", h.ENGINE_MFMA_F4)):
        r = ctx.search_window(q_hv, q_pmz, q_ch, h.TOL_DA, 500.0, engine)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            r = ctx.search_window(q_hv, q_pmz, q_ch, h.TOL_DA, 500.0, engine)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        out[name] = float(np.median(ts))
        if name == "mfma_fp4":
            res = r
    return out, res


def mean_bipolar(ctx, dim, n_sample=65536, seed=3):
    """Mean bipolar hypervector (bit 0 -> +1, bit 1 -> -1) of a random sample
    of library rows: the centre of the training-free sketch baseline."""
    import torch
    rows = ctx.library_export()
    n = rows.shape[0]
    pick = np.sort(np.random.default_rng(seed).choice(n, size=min(n_sample, n), replace=False))
    sub = rows[torch.from_numpy(pick).to(rows.device)].cpu().numpy().view(np.uint8)
    del rows
    bits = np.unpackbits(sub, axis=1, bitorder="little")[:, :dim]
    return 1.0 - 2.0 * bits.mean(axis=0)


def learned_leg(args, w, ctx, dev, q_hv, q_pmz, q_ch, train, desc, k):
    """Learned shortlist (an MLP D -> 1024 -> 256 trained on the GPU through
    homs_model_train on (training query, exact top-1) pairs; per query the
    top-k window candidates by embedding score are rescored exactly, with
    exhaustive fallback) on an encoded context. Reports queries/s, window
    comparisons covered per second, top-1 agreement with the exhaustive search
    beside two untrained shortlists (the random initial network and a
    training-free sketch), and the speedup over the exhaustive engines (warm,
    median of runs). Returns (line, state for the oracle sample)."""
    import torch

    import paper_2211_16422_amd.hyperoms as h

    hp = ctx.params
    nq = q_hv.shape[0]
    t_hv = ctx.encode_queries(*h.to_device_csr(*h.preprocess(hp, train.offsets, train.mz,
                                                             train.intensity), dev))
    t_pmz, t_ch = torch.from_numpy(train.pmz).to(dev), torch.from_numpy(train.charge).to(dev)
    lo, hi = ctx.window_bounds(q_pmz, q_ch, h.TOL_DA, 500.0)
    pairs = int((hi - lo).sum().item())
    torch.cuda.synchronize()
    ex, (e_idx, e_dist) = exhaustive_times(ctx, h, q_hv, q_pmz, q_ch)
    log(f"learned: exhaustive search (warm median) popcount {ex['popcount']:.3f}s, fp8 "
        f"{ex['mfma_fp8']:.3f}s, fp4 {ex['mfma_fp4']:.3f}s over {pairs:.4e} pairs")

    t0 = time.perf_counter()
    t_idx, _ = ctx.search_window(t_hv, t_pmz, t_ch, h.TOL_DA, 500.0, h.ENGINE_MFMA_F4)
    torch.cuda.synchronize()
    label_s = time.perf_counter() - t0

    rng = np.random.default_rng(12345)
    H, E, D = 1024, 256, hp.dim
    init = {"W1": (rng.uniform(-1, 1, (H, D)) / np.sqrt(D)).astype(np.float32),
            "b1": np.zeros(H, np.float32),
            "W2": (rng.uniform(-1, 1, (E, H)) / np.sqrt(H)).astype(np.float32),
            "b2": np.zeros(E, np.float32)}
    model = h.Model(ctx, init)
    has = e_idx >= 0

    def evaluate(tag):
        model.embed_library()
        idx, dist, fb = model.search(q_hv, q_pmz, q_ch, k)
        agree = float(((idx == e_idx) & (dist == e_dist))[has].float().mean().item())
        fbr = float((fb != 0).float().mean().item())
        log(f"learned {tag}: top-1 agreement {agree:.5f}, fallback {fbr:.5f}")
        return agree, fbr

    agree0, _ = evaluate("untrained")
    model.set_weights(h.sketch_weights(D, H, E, seed=7))
    agree_sketch0, _ = evaluate("training-free sketch (uncentred)")
    sketch = h.sketch_weights(D, H, E, seed=7, center=mean_bipolar(ctx, D))
    model.set_weights(sketch)
    agree_sketch, fb_sketch = evaluate("training-free sketch (centred)")
    if args.init == "random":
        model.set_weights(init)
    t0 = time.perf_counter()
    steps, losses = model.train(t_hv, t_idx, epochs=args.epochs, batch=args.batch, lr=args.lr,
                                tau=args.tau, seed=0, losses=True)
    train_s = time.perf_counter() - t0
    nb = steps // args.epochs
    log(f"learned: {steps} training steps in {train_s:.2f}s (labels {label_s:.2f}s); mean loss "
        f"first epoch {losses[:nb].mean().item():.4f}, last {losses[-nb:].mean().item():.4f}")
    t0 = time.perf_counter()
    model.embed_library()
    torch.cuda.synchronize()
    embed_lib_s = time.perf_counter() - t0
    agree, fbr = evaluate("trained")

    for _ in range(args.warmup):
        model.search(q_hv, q_pmz, q_ch, k)
    torch.cuda.synchronize()
    ctx.profile_enable(True)
    ctx.profile_read()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        idx, dist, fb = model.search(q_hv, q_pmz, q_ch, k)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    step_s = el / args.steps
    score_ms = prof["score_ms"] / args.steps
    tflops = 2.0 * E * pairs / (score_ms * 1e-3) / 1e12
    line = {
        "metric": "learned-shortlist open search: queries/s and window comparisons covered/s "
                  f"at +-500 Da, D={D}, k={k}",
        "value": nq / step_s, "unit": "queries/s", "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * step_s, "higher_is_better": True,
        "dtype": "fp8e4m3->f32 (scoring), bf16 (MLP)", "data": "synthetic",
        "config": {"workload": desc + f", MLP {D}-{H}-{E}, k={k}", "pairs_per_step": pairs,
                   "training_pairs": int((t_idx >= 0).sum().item()), "epochs": args.epochs,
                   "batch": args.batch, "lr": args.lr, "tau": args.tau,
                   "init": args.init},
        "comparisons_covered_per_s": pairs / step_s,
        "top1_agreement": agree, "top1_agreement_untrained": agree0,
        "top1_agreement_training_free_sketch": agree_sketch,
        "top1_agreement_training_free_sketch_uncentred": agree_sketch0, "fallback_rate": fbr,
        "fallback_rate_sketch": fb_sketch,
        "fallback_reasons": {r: int((fb == c).sum().item()) for c, r in
                             ((1, "buffer_overflow"), (2, "too_few_kept"),
                              (3, "kth_below_threshold"))},
        "exhaustive_s_warm_median": ex, "speedup_vs_popcount": ex["popcount"] / step_s,
        "speedup_vs_mfma_fp8": ex["mfma_fp8"] / step_s,
        "speedup_vs_mfma_fp4": ex["mfma_fp4"] / step_s,
        "train_s": train_s, "train_steps": steps, "label_s": label_s,
        "embed_library_s": embed_lib_s,
        "roofline": {"bound": "mfma", "achieved": round(tflops, 1), "peak": MFMA_PEAK_TOPS,
                     "unit": "TFLOP/s", "frac": round(tflops / MFMA_PEAK_TOPS, 4),
                     "traffic": None, "peak_kind": "dense fp8 e4m3 matrix peak of MI355X",
                     "kernel": "collect_kernel (E4M3 scoring embeddings)",
                     "kernel_ms": round(score_ms, 3), "flops_per_pair": 2 * E},
        "phase_ms": {"search": prof["search_ms"] / args.steps,
                     "prep_and_embed": prof["prep_ms"] / args.steps},
        "cpu_baseline": None, "parity_sample": None,
    }
    state = {"idx": idx.cpu().numpy(), "dist": dist.cpu().numpy(), "fb": fb.cpu().numpy(),
             "nq": nq}
    model.close()
    return line, state


def finish_learned(line, state, sample, side, o_idx, o_dist, o_qhv, t, desc):
    """The learned leg's oracle baseline and parity sample: the oracle's
    exhaustive search (the reference answer for top-1 agreement) on the sampled queries;
    the learned answers must agree with it at the rate measured on the GPU,
    and every returned distance must be the exact Hamming distance of the
    returned reference, computed from the oracle's own rows."""
    idx, dist, fb = state["idx"][sample], state["dist"][sample], state["fb"][sample]
    agree = float(np.mean((idx == o_idx) & (dist == o_dist)))
    pos = np.searchsorted(side["rows"], idx)
    ok = idx >= 0
    exact = True
    if ok.any():
        rows = side["hv"][np.minimum(pos[ok], len(side["rows"]) - 1)]
        found = side["rows"][np.minimum(pos[ok], len(side["rows"]) - 1)] == idx[ok]
        ham = np.bitwise_count(rows ^ o_qhv[ok]).sum(axis=1)
        exact = bool(found.all() and np.array_equal(ham, dist[ok]))
    line["cpu_baseline"] = cpu_entry(len(sample) / t, "queries/s",
                                     "oracle exhaustive top-1 (the reference answer) of " + desc, t)
    line["parity_sample"] = {"queries": int(len(sample)), "sampling": f"random, seed {SAMPLE_SEED}",
                             "top1_agreement_vs_oracle": agree,
                             "fallback_in_sample": int((fb != 0).sum()),
                             "rescored_distances_exact": exact}
    log(f"learned sample: agreement with the oracle {agree:.4f}, rescoring exact: {exact}")


def bench_learned_full(args, w, dev, jobs):
    """The learned workload at full size (3M + 3M library, 500,000 queries,
    1,000,000 training queries) in its own line."""
    import torch

    import paper_2211_16422_amd.hyperoms as h
    from synth import make_workload, subset

    t0 = time.time()
    g = make_workload(w, n_ref=args.n_ref, n_query=args.n_query, n_train=args.n_train)
    lib, q, tr = g.library, g.queries, g.train
    log(f"generated {lib.n} library + {q.n} query + {tr.n} training spectra in "
        f"{time.time() - t0:.1f}s")
    want_cpu = args.cpu_sample > 0 and not args.profile_only
    sample = random_sample(q.n, args.cpu_sample) if want_cpu else None
    side = (jobs.submit(oracle_library_side, w, lib, q.pmz[sample], q.charge[sample], 0, 500.0)
            if want_cpu else None)
    hp = h.Params(dim=w.dim, n_levels=w.n_levels, bins_per_da=w.bins_per_da)
    ctx = h.Context(hp, device=0)
    l_dev = h.to_device_csr(*h.preprocess(hp, lib.offsets, lib.mz, lib.intensity), dev)
    ctx.encode_library(*l_dev, torch.from_numpy(lib.pmz).to(dev),
                       torch.from_numpy(lib.charge).to(dev))
    del l_dev
    q_hv = ctx.encode_queries(*h.to_device_csr(*h.preprocess(hp, q.offsets, q.mz,
                                                             q.intensity), dev))
    q_pmz, q_ch = torch.from_numpy(q.pmz).to(dev), torch.from_numpy(q.charge).to(dev)
    desc = (f"learned: {g.meta['n_ref']} references + {g.meta['n_decoy']} decoys, {q.n} "
            f"queries, {tr.n} training queries, D={w.dim}")
    line, state = learned_leg(args, w, ctx, dev, q_hv, q_pmz, q_ch, tr, desc, args.k)
    line.update({"n_gpus": 1, "scaling": "weak", "vs_baseline": None})
    ctx.close()
    jobs.close()
    if side is not None:
        s = side.result()
        t, o_idx, o_dist, o_qhv, _ = oracle_timed_search(s, subset(q, sample), 0, 500.0)
        finish_learned(line, state, sample, s, o_idx, o_dist, o_qhv, t,
                       f"{len(sample)} queries drawn at random (seed {SAMPLE_SEED}) from the "
                       f"{q.n} of the same workload")
    return line


def batched_leg(args, w, dev, jobs):
    """Mixed stream (70% +-20 ppm and 30% +-500 Da windows, charges 2-4), one
    persistent launch per batch, autotuned, replayed from a hipGraph. Returns
    the line and a function that adds the oracle baseline and parity sample
    once the background jobs are done."""
    import torch

    import paper_2211_16422_amd.hyperoms as h
    from synth import make_workload, subset

    t0 = time.time()
    g = make_workload(w, n_ref=args.n_ref if w.name == args.workload else None,
                      n_query=args.n_query if w.name == args.workload else None)
    lib, q = g.library, g.queries
    log(f"batched: generated {lib.n} library + {q.n} query spectra in {time.time() - t0:.1f}s")
    want_cpu = args.cpu_sample > 0 and not args.profile_only
    sample = random_sample(q.n, args.cpu_sample // 2) if want_cpu else None
    side = (jobs.submit(oracle_library_side, w, lib, q.pmz[sample], q.charge[sample],
                        g.tol_kind[sample], g.tol_value[sample]) if want_cpu else None)
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
    del l_dev, l_csr
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
    log(f"batched: pairs per batch {pairs:.4e}; window histogram {hist}")

    out_idx = torch.empty(q.n, dtype=torch.int64, device=dev)
    out_dist = torch.empty(q.n, dtype=torch.int32, device=dev)
    t0 = time.time()
    best, best_ms = ctx.autotune_batched(q_hv, q_pmz, q_ch, kinds, values, reps=1,
                                         out_idx=out_idx, out_dist=out_dist)
    log(f"batched: autotune {time.time() - t0:.1f}s: {best} at {best_ms:.1f} ms per batch")
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
                "kernel_ms": round(ms, 3), "ops_per_pair": 2 * w.dim}
    else:
        dtype = "u32"
        tops = 2.0 * words * pairs / (ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": round(tops, 3), "peak": round(VALU_PEAK_TOPS, 3),
                "unit": "TOP/s", "frac": round(tops / VALU_PEAK_TOPS, 4), "traffic": None,
                "peak_kind": "measured xor+popcount issue rate",
                "kernel": "batched graph (persistent_search_kernel<popcount> + planning)",
                "kernel_ms": round(ms, 3), "ops_per_pair": 2 * words}
    line = {
        "metric": "mixed-window (70% +-20 ppm, 30% +-500 Da) Hamming comparisons/s and "
                  "queries/s, D=8192, one persistent hipGraph launch per batch",
        "value": pairs * args.steps / el, "unit": "comparisons/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * el / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": dtype, "data": "synthetic",
        "config": {"workload": f"batched: {g.meta['n_ref']} references + {g.meta['n_decoy']} "
                               f"decoys, {q.n} queries (70% 20 ppm, 30% 500 Da), charges 2-4, "
                               f"D={w.dim}", "pairs_per_step": pairs, "window_histogram": hist,
                   "autotuned": best},
        "queries_per_s": q.n * args.steps / el,
        "library_encode_s": lib_encode_s,
        "roofline": roof,
        "bit_exact_vs_search_window": same,
        "cpu_baseline": None, "parity_sample": None,
    }
    res_idx, res_dist = out_idx.cpu().numpy(), out_dist.cpu().numpy()
    ctx.close()
    del q_hv, q_pmz, q_ch, kinds, values, out_idx, out_dist, ref_idx, ref_dist
    torch.cuda.empty_cache()

    def finish():
        if side is None:
            return
        s = side.result()
        t, o_idx, o_dist, _, spairs = oracle_timed_search(s, subset(q, sample),
                                                          g.tol_kind[sample],
                                                          g.tol_value[sample])
        match = bool(np.array_equal(o_idx, res_idx[sample]) and
                     np.array_equal(o_dist, res_dist[sample]))
        n_open = int(np.sum(g.tol_kind[sample] == h.TOL_DA))
        desc = (f"{len(sample)} queries drawn at random (seed {SAMPLE_SEED}) from the {q.n} "
                f"of the batched workload ({n_open} open, {len(sample) - n_open} narrow; "
                f"{spairs} candidate pairs; oracle encode of those queries + search with "
                "their own windows)")
        log(f"batched cpu baseline: {spairs:.3e} pairs in {t:.2f}s; GPU results match the "
            f"oracle: {match}")
        line["cpu_baseline"] = cpu_entry(spairs / t, "comparisons/s", desc, t)
        line["parity_sample"] = {"queries": int(len(sample)), "pairs": spairs,
                                 "sampling": f"random, seed {SAMPLE_SEED}", "bit_exact": match}

    return line, finish


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
        o, b, lv = ctx.preprocess_device(off, mz, inten, check=False)
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / reps
    if ctx.device_errors():
        raise RuntimeError("device preprocessing raised a device error flag")
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
            "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "algorithmic_bytes": nbytes,
                         "kernel": "preprocess_wave_kernel (one staged pass) + scan "
                                   "+ compaction",
                         "note": "bounded by the per-spectrum rank counting in LDS "
                                 "(O(peaks^2) double compares), not by HBM"}}


def bench_cascade(args, w, dev, jobs):
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
    log(f"generated {lib.n} library + {q.n} query spectra in {time.time() - t0:.1f}s")
    want_cpu = args.cpu_sample > 0 and not args.profile_only
    sample = random_sample(q.n, args.cpu_sample) if want_cpu else None
    side = (jobs.submit(oracle_library_side, w, lib, q.pmz[sample], q.charge[sample], 0, 500.0)
            if want_cpu else None)
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
    line, result = cascade_leg(args, w, g, ctx, dev, q_dev, q_pmz, q_ch)
    ctx.close()
    jobs.close()
    if side is not None:
        line["cpu_baseline"] = cascade_cpu_baseline(side.result(), sample, g, *result)
    return line


def cascade_leg(args, w, g, ctx, dev, q_dev, q_pmz, q_ch):
    """Timed cascade steps on an encoded context: each step encodes the
    queries and runs homs_cascade_search on the fp4 engine. Returns the line
    (cpu_baseline None) and what cascade_cpu_baseline needs besides the
    oracle side: (n_ref, top-1 indices, distances, stages)."""
    import torch

    import paper_2211_16422_amd.hyperoms as h

    lib, q = g.library, g.queries
    n_ref = g.meta["n_ref"]
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
    log(f"cascade: stage 1: {n1}, stage 2: {n2}, unidentified {q.n - n1 - n2}; pairs narrow "
        f"{pairs_narrow:.3e}, open {pairs_open:.3e}; search kernels {search_ms:.1f} ms per step")
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
        "cpu_baseline": None,
    }
    return line, (n_ref, idx, dist, stage)


def cascade_cpu_baseline(side, sample, g, n_ref, gpu_idx, gpu_dist, gpu_stage):
    """The oracle cascade on the host cores over the sampled queries (drawn at
    random; their candidate rows encoded untimed). Its FDR is over the
    sample's PSMs only, so stages may differ from the full run; each query's
    matches are checked instead: the GPU's stage-1 identifications against
    the oracle's narrow top-1, the others against its open top-1."""
    import oracle
    from oracle import fdr
    from synth import subset

    q = g.queries
    op = side["op"]
    qs = subset(q, sample)
    rows = side["rows"]
    qo, qb, ql = oracle.preprocess(qs.offsets, qs.mz, qs.intensity, op)
    t0 = time.perf_counter()
    q_hv = oracle.encode(op, side["idt"], side["lvt"], qo, qb, ql)
    fdr.cascade(op, side["hv"], side["pmz"], side["charge"], rows >= n_ref, q_hv, qs.pmz,
                qs.charge, (1, 20.0), (0, 500.0), 0.01)
    t = time.perf_counter() - t0
    n_idx, n_dist = oracle.search(op, side["hv"], side["pmz"], side["charge"], q_hv, qs.pmz,
                                  qs.charge, 1, 20.0)
    o_idx, o_dist = oracle.search(op, side["hv"], side["pmz"], side["charge"], q_hv, qs.pmz,
                                  qs.charge, 0, 500.0)
    s1 = gpu_stage[sample] == 1
    want_idx = np.where(s1, n_idx, o_idx)
    want_dist = np.where(s1, n_dist, o_dist)
    want_idx = np.where(want_idx >= 0, rows[np.maximum(want_idx, 0)], -1)
    match = bool(np.array_equal(want_idx, gpu_idx[sample]) and
                 np.array_equal(want_dist, gpu_dist[sample]))
    log(f"cpu baseline: cascade of {len(sample)} queries in {t:.2f}s; GPU matches agree: {match}")
    out = cpu_entry(len(sample) / t, "queries/s",
                    f"{len(sample)} queries drawn at random (seed {SAMPLE_SEED}) from the "
                    f"{q.n} of the same workload (oracle encode of the queries + cascade with "
                    "FDR over the sample's PSMs)", t)
    out["matches_bit_exact"] = match
    return out


if __name__ == "__main__":
    main()
