"""Target-decoy FDR and cascade search oracle — TEST INFRASTRUCTURE ONLY.

Plain numpy/Python, written from the paper: search results are filtered at a
false discovery rate estimated with decoy spectra added to the library
(Section 2.1, following Elias and Gygi), at a fixed 1% threshold (Section
4.1); the search is a cascade (Section 3.4): a standard search with a narrow
precursor tolerance, FDR filtering, then an open search with a wide tolerance
over the spectra the first stage did not identify, filtered in turn.

Readings (the paper does not spell these out):
* A spectrum-spectrum match (PSM) is a query's top-1 candidate; its score is
  the Hamming similarity D - H, so a higher score is a smaller distance. It is
  a decoy match when the matched library entry is a decoy.
* FDR at threshold d (accept every PSM with distance <= d) = number of decoy
  PSMs / number of target PSMs at distance <= d; undefined (never accepted)
  when there is no target PSM.
* A PSM's q-value is the smallest FDR of any threshold that accepts it,
  i.e. the minimum of FDR(d') over d' >= its distance. A target PSM is an
  identification when its q-value is <= the FDR level; decoy PSMs never are.
* Each cascade stage computes its FDR over its own PSMs only. A query
  identified in the narrow stage is not searched again; every other query
  takes the open stage's result.

Only tests/, __graft_entry__.smoke() and the CPU-baseline leg of bench.py may
import this module; it imports nothing from the product library.
"""
from __future__ import annotations

import math
from typing import Tuple

import numpy as np

from . import Params, search


def q_values(dist: np.ndarray, decoy: np.ndarray) -> np.ndarray:
    """q-value of each PSM (float64), by the definition above."""
    dist = np.asarray(dist, dtype=np.int64)
    decoy = np.asarray(decoy, dtype=bool)
    n = dist.shape[0]
    q = np.full(n, math.inf)
    if n == 0:
        return q
    levels = np.unique(dist)  # ascending distances = descending scores
    fdr = {}
    for d in levels:
        accepted = dist <= d
        t = int(np.sum(accepted & ~decoy))
        dc = int(np.sum(accepted & decoy))
        fdr[int(d)] = dc / t if t > 0 else math.inf
    for i in range(n):
        q[i] = min(fdr[int(d)] for d in levels if d >= dist[i])
    return q


def identified(dist: np.ndarray, decoy: np.ndarray, level: float) -> np.ndarray:
    """Target PSMs whose q-value is <= level."""
    q = q_values(dist, decoy)
    return (q <= level) & ~np.asarray(decoy, dtype=bool)


def cascade(p: Params, lib_hv, lib_pmz, lib_charge, lib_decoy, q_hv, q_pmz, q_charge,
            narrow: Tuple[int, float], wide: Tuple[int, float], level: float = 0.01,
            charge_match: bool = True):
    """Two-stage cascade search with FDR filtering of each stage.

    narrow, wide: (kind, value) windows (kind 0: Da, 1: ppm).
    Returns (idx, dist, stage, qvalue) per query: stage 1 or 2 for an
    identification in that stage, 0 otherwise; idx/dist/qvalue are the
    narrow stage's for stage-1 identifications and the open stage's for every
    other query ((-1, -1, inf) when its window is empty).
    """
    lib_decoy = np.asarray(lib_decoy, dtype=bool)
    q_pmz = np.asarray(q_pmz, dtype=np.float64)
    nq = q_pmz.shape[0]
    # stage 1: standard search
    i1, d1 = search(p, lib_hv, lib_pmz, lib_charge, q_hv, q_pmz, q_charge, narrow[0],
                    narrow[1], charge_match)
    has1 = i1 >= 0
    dec1 = np.zeros(nq, dtype=bool)
    dec1[has1] = lib_decoy[i1[has1]]
    q1 = np.full(nq, math.inf)
    q1[has1] = q_values(d1[has1], dec1[has1])
    ok1 = has1 & ~dec1 & (q1 <= level)
    # stage 2: open search of the rest (identified queries get no candidates)
    rest = np.flatnonzero(~ok1)
    i2 = np.full(nq, -1, dtype=np.int64)
    d2 = np.full(nq, -1, dtype=np.int32)
    if rest.size:
        a, b = search(p, lib_hv, lib_pmz, lib_charge, np.asarray(q_hv)[rest], q_pmz[rest],
                      np.asarray(q_charge)[rest], wide[0], wide[1], charge_match)
        i2[rest] = a
        d2[rest] = b
    has2 = i2 >= 0
    dec2 = np.zeros(nq, dtype=bool)
    dec2[has2] = lib_decoy[i2[has2]]
    q2 = np.full(nq, math.inf)
    q2[has2] = q_values(d2[has2], dec2[has2])
    ok2 = has2 & ~dec2 & (q2 <= level)
    idx = np.where(ok1, i1, i2)
    dist = np.where(ok1, d1, d2).astype(np.int32)
    qv = np.where(ok1, q1, q2)
    stage = np.where(ok1, 1, np.where(ok2, 2, 0)).astype(np.int8)
    return idx, dist, stage, qv
