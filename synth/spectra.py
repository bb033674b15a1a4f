"""Seeded generator of raw spectra (fragment m/z, intensity, precursor m/z,
charge) in CSR form.

Shapes follow the paper's workloads (Section 4.1; Table 1): fragment m/z over
[101, 1500], at most 50 peaks kept after preprocessing, libraries of ~1-3 M
references with decoys in the same ratio, and query files of ~16-47 k spectra.
The paper's datasets are not available, so every input here is synthetic:

* references: precursor m/z ~ U[400, 1500], charge uniform over the workload's
  charges, peak count ~ U{20..150}, peak m/z ~ U[101, 1500], intensity ~
  lognormal(0, 1);
* decoys: one per reference, keeping its precursor m/z, charge, peak count
  and intensities, with every fragment peak at a newly drawn m/z from the
  reference peaks' distribution. The workload statement's decoys keep the
  reference's fragment m/z values and only permute them among its peaks; such
  decoys share every peak position with their reference and would win top-1
  so often that no match passes a 1% FDR, so the generator redraws them;
* queries: a random reference with N(0, 0.01) m/z jitter on every fragment,
  each fragment dropped with probability 0.2, round(0.1 * n) noise peaks added,
  and, for half of the queries, a mass shift delta ~ U[-150, 500] Da applied to
  the precursor (as delta / charge on the m/z) and to each fragment with
  probability 0.4.

Nothing here implements any step of the method.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional, Tuple

import numpy as np


@dataclass
class RawSpectra:
    """Raw spectra in CSR form; peaks of spectrum i are [offsets[i], offsets[i+1])."""

    offsets: np.ndarray  # int64 [n + 1]
    mz: np.ndarray  # float64 [P]
    intensity: np.ndarray  # float64 [P]
    pmz: np.ndarray  # float64 [n]
    charge: np.ndarray  # int8 [n]
    source: Optional[np.ndarray] = None  # int64 [n]: reference a query was made from
    is_decoy: Optional[np.ndarray] = None  # bool [n]
    shifted: Optional[np.ndarray] = None  # bool [n]: query carries a mass shift

    @property
    def n(self) -> int:
        return int(self.pmz.shape[0])

    @property
    def n_peaks(self) -> int:
        return int(self.offsets[-1])

    def peaks(self, i: int) -> Tuple[np.ndarray, np.ndarray]:
        a, b = int(self.offsets[i]), int(self.offsets[i + 1])
        return self.mz[a:b], self.intensity[a:b]


def _ranges(starts: np.ndarray, counts: np.ndarray) -> np.ndarray:
    """Concatenation of arange(starts[i], starts[i] + counts[i]) over i."""
    counts = counts.astype(np.int64)
    total = int(counts.sum())
    if total == 0:
        return np.zeros(0, dtype=np.int64)
    seg_start = np.cumsum(counts) - counts
    rep = np.repeat(starts.astype(np.int64) - seg_start, counts)
    return rep + np.arange(total, dtype=np.int64)


def _offsets(counts: np.ndarray) -> np.ndarray:
    off = np.zeros(counts.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    return off


def make_references(n: int, rng: np.random.Generator, charges=(2, 3),
                    peaks=(20, 150), mz_range=(101.0, 1500.0),
                    pmz_range=(400.0, 1500.0)) -> RawSpectra:
    npk = rng.integers(peaks[0], peaks[1] + 1, size=n, dtype=np.int64)
    off = _offsets(npk)
    total = int(off[-1])
    mz = rng.uniform(mz_range[0], mz_range[1], size=total)
    inten = rng.lognormal(0.0, 1.0, size=total)
    pmz = rng.uniform(pmz_range[0], pmz_range[1], size=n)
    ch = np.asarray(charges, dtype=np.int8)[rng.integers(0, len(charges), size=n)]
    return RawSpectra(off, mz, inten, pmz, ch,
                      source=np.full(n, -1, dtype=np.int64),
                      is_decoy=np.zeros(n, dtype=bool),
                      shifted=np.zeros(n, dtype=bool))


def make_decoys(refs: RawSpectra, rng: np.random.Generator,
                mz_range=(101.0, 1500.0)) -> RawSpectra:
    """One decoy per reference, a spectrum that matches no peptide: the
    reference's precursor m/z, charge, peak count and intensities, with every
    fragment peak at a newly drawn m/z (the distribution of reference peaks)."""
    n = refs.n
    mz = rng.uniform(mz_range[0], mz_range[1], size=refs.mz.shape[0])
    return RawSpectra(refs.offsets.copy(), mz, refs.intensity.copy(),
                      refs.pmz.copy(), refs.charge.copy(),
                      source=np.arange(n, dtype=np.int64),
                      is_decoy=np.ones(n, dtype=bool),
                      shifted=np.zeros(n, dtype=bool))


def make_queries(refs: RawSpectra, n: int, rng: np.random.Generator,
                 jitter_sd=0.01, drop=0.2, noise=0.1, shift_frac=0.5,
                 delta_range=(-150.0, 500.0), shift_peak_frac=0.4,
                 mz_range=(101.0, 1500.0)) -> RawSpectra:
    src = rng.integers(0, refs.n, size=n, dtype=np.int64)
    cnt = np.diff(refs.offsets)[src]
    idx = _ranges(refs.offsets[src], cnt)
    qid = np.repeat(np.arange(n, dtype=np.int64), cnt)
    keep = rng.random(idx.shape[0]) >= drop
    mz = refs.mz[idx] + rng.normal(0.0, jitter_sd, size=idx.shape[0])
    inten = refs.intensity[idx]
    shifted = rng.random(n) < shift_frac
    delta = np.where(shifted, rng.uniform(delta_range[0], delta_range[1], size=n), 0.0)
    move = shifted[qid] & (rng.random(idx.shape[0]) < shift_peak_frac)
    mz = np.where(move, mz + delta[qid], mz)
    mz, inten, qid = mz[keep], inten[keep], qid[keep]

    n_noise = np.floor(noise * cnt + 0.5).astype(np.int64)
    nz_q = np.repeat(np.arange(n, dtype=np.int64), n_noise)
    nz_mz = rng.uniform(mz_range[0], mz_range[1], size=nz_q.shape[0])
    nz_in = rng.lognormal(0.0, 1.0, size=nz_q.shape[0])

    all_q = np.concatenate([qid, nz_q])
    order = np.argsort(all_q, kind="stable")  # per query: kept source peaks, then noise
    mz_all = np.concatenate([mz, nz_mz])[order]
    in_all = np.concatenate([inten, nz_in])[order]
    counts = np.bincount(all_q, minlength=n).astype(np.int64)
    ch = refs.charge[src]
    pmz = refs.pmz[src] + delta / ch.astype(np.float64)
    return RawSpectra(_offsets(counts), mz_all, in_all, pmz, ch.copy(), source=src,
                      is_decoy=np.zeros(n, dtype=bool), shifted=shifted)


def concat(a: RawSpectra, b: RawSpectra) -> RawSpectra:
    off = np.concatenate([a.offsets, b.offsets[1:] + a.offsets[-1]])

    def cat(x, y):
        if x is None or y is None:
            return None
        return np.concatenate([x, y])

    return RawSpectra(off, np.concatenate([a.mz, b.mz]),
                      np.concatenate([a.intensity, b.intensity]),
                      np.concatenate([a.pmz, b.pmz]), np.concatenate([a.charge, b.charge]),
                      source=cat(a.source, b.source), is_decoy=cat(a.is_decoy, b.is_decoy),
                      shifted=cat(a.shifted, b.shifted))


def subset(s: RawSpectra, rows: np.ndarray) -> RawSpectra:
    rows = np.asarray(rows, dtype=np.int64)
    cnt = np.diff(s.offsets)[rows]
    idx = _ranges(s.offsets[rows], cnt)

    def pick(x):
        return None if x is None else x[rows]

    return RawSpectra(_offsets(cnt), s.mz[idx], s.intensity[idx], s.pmz[rows],
                      s.charge[rows], source=pick(s.source), is_decoy=pick(s.is_decoy),
                      shifted=pick(s.shifted))


@dataclass(frozen=True)
class Workload:
    """Sizes and search settings of one synthetic workload.

    ``narrow_frac`` of the queries use the narrow tolerance (``narrow_ppm``
    parts per million of the query precursor m/z); the rest use the open
    tolerance of ``wide_da`` Da (Table 1).
    """

    name: str
    n_ref: int
    n_query: int
    dim: int
    charges: Tuple[int, ...] = (2, 3)
    narrow_frac: float = 0.0
    narrow_ppm: float = 20.0
    wide_da: float = 500.0
    n_train: int = 0
    n_levels: int = 16
    bins_per_da: float = 20.0
    seed: int = 0


WORKLOADS = {
    # plain method, every bit and distance checked
    "tiny": Workload("tiny", 2000, 200, 2048),
    # plain method at library scale: the throughput workload
    "large": Workload("large", 1_000_000, 100_000, 8192),
    # the same data in higher-capacity hypervectors (D = 16,384)
    "large16k": Workload("large16k", 1_000_000, 100_000, 16384),
    # the same data searched as a cascade (narrow standard search, FDR, open search)
    "cascade": Workload("cascade", 1_000_000, 100_000, 8192),
    # precision (MFMA) form, same data as tiny
    "precision": Workload("precision", 2000, 200, 2048),
    # mixed narrow/open stream for the batched form
    "batched": Workload("batched", 2_000_000, 200_000, 8192, charges=(2, 3, 4),
                        narrow_frac=0.7),
    # learned shortlist form
    "learned": Workload("learned", 3_000_000, 500_000, 8192, n_train=1_000_000),
}


@dataclass
class Generated:
    library: RawSpectra  # references then decoys; library index = position here
    queries: RawSpectra
    tol_kind: np.ndarray  # int8 [n_query]: 0 = Da, 1 = ppm
    tol_value: np.ndarray  # float64 [n_query]
    train: Optional[RawSpectra] = None
    meta: dict = field(default_factory=dict)


def make_workload(w: Workload, n_ref: Optional[int] = None, n_query: Optional[int] = None,
                  n_train: Optional[int] = None, seed: Optional[int] = None) -> Generated:
    """Generate library (references then decoys), queries and per-query tolerances."""
    n_ref = w.n_ref if n_ref is None else n_ref
    n_query = w.n_query if n_query is None else n_query
    n_train = w.n_train if n_train is None else n_train
    seed = w.seed if seed is None else seed
    ss = np.random.SeedSequence(seed)
    r_ref, r_dec, r_q, r_win, r_train = (np.random.default_rng(s) for s in ss.spawn(5))
    refs = make_references(n_ref, r_ref, charges=w.charges)
    decoys = make_decoys(refs, r_dec)
    lib = concat(refs, decoys)
    q = make_queries(refs, n_query, r_q)
    narrow = r_win.random(n_query) < w.narrow_frac
    tol_kind = narrow.astype(np.int8)
    tol_value = np.where(narrow, w.narrow_ppm, w.wide_da).astype(np.float64)
    train = make_queries(refs, n_train, r_train) if n_train > 0 else None
    return Generated(lib, q, tol_kind, tol_value, train,
                     meta={"workload": w.name, "n_ref": n_ref, "n_decoy": n_ref,
                           "n_query": n_query, "n_train": n_train, "seed": seed})


def make_training_queries(g: Generated, n_train: int) -> RawSpectra:
    """The training queries make_workload draws for the same seed and library
    when asked for n_train of them (its fifth random stream), without
    drawing the library and evaluation queries again."""
    ss = np.random.SeedSequence(g.meta["seed"])
    r_train = np.random.default_rng(ss.spawn(5)[4])
    refs = subset(g.library, np.arange(g.meta["n_ref"]))
    return make_queries(refs, n_train, r_train)
