"""HyperOMS oracle — TEST INFRASTRUCTURE ONLY.

A plain, slow CPU implementation of what the HyperOMS hot path computes
(arXiv 2211.16422): preprocessing (Section 3.2, Table 1), position and level
hypervectors (Sections 3.3.1, 3.3.2), Eq. 1 encoding with binarisation
(Section 3.3), the precursor window (Section 3.4) and the Hamming top-1
(Section 3.4). The arithmetic lives in ``hyperoms_oracle.c`` (plain C,
float64, no bit tricks); this module only marshals numpy arrays.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. It shares no code with the product
library and imports nothing from it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hyperoms_oracle.c")
_LIB = os.path.join(_HERE, "_hyperoms_oracle.so")


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP, no FP contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-mpopcnt", "-fopenmp", "-ffp-contract=off", "-fPIC",
               "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, u32, u64, i32, f64 = (ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64,
                                   ctypes.c_int32, ctypes.c_double)
        _lib.oracle_splitmix64.argtypes = [u64, i64, P]
        _lib.oracle_codebook.argtypes = [u32, u32, u32, u32, u64, u32, P, P]
        _lib.oracle_encode_lsh.argtypes = [u32, P, i64, P, P, P, P]
        _lib.oracle_codebook.restype = ctypes.c_int
        _lib.oracle_num_bins.argtypes = [f64, f64, f64]
        _lib.oracle_num_bins.restype = i64
        _lib.oracle_preprocess.argtypes = [i64, P, P, P, f64, f64, f64, f64, u32, u32, P, P, P]
        _lib.oracle_preprocess.restype = i64
        _lib.oracle_encode.argtypes = [u32, P, P, i64, P, P, P, P]
        _lib.oracle_search.argtypes = [u32, i64, P, P, P, i64, P, P, P, P, P, i32, P, P]
        _lib.oracle_window_counts.argtypes = [i64, P, P, i64, P, P, P, P, i32, P]
        _lib.oracle_window_distances.argtypes = [u32, i64, P, P, P, i64, P, P, P, P, P, i32,
                                                 P, P, P]
        _lib.oracle_max_threads.restype = i32
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=dtype)


@dataclass(frozen=True)
class Params:
    """Method parameters (Table 1; Section 4.2: D = 8192, alpha = D/2, Q = 16)."""

    dim: int = 8192
    n_levels: int = 16
    top_n: int = 50
    mz_min: float = 101.0
    mz_max: float = 1500.0
    bins_per_da: float = 20.0  # 0.05 Da bins; 25.0 for 0.04 Da
    noise_frac: float = 0.01
    id_flips: int = 0  # alpha; 0 means D/2
    seed: int = 0
    # 0: the paper's ID-level encoding with locality (Section 3.3); the
    # baselines of Section 4.2: 1 random (independent) position vectors,
    # 2 random-projection LSH
    encoding: int = 0

    @property
    def alpha(self) -> int:
        return self.dim // 2 if self.id_flips == 0 else self.id_flips

    @property
    def words(self) -> int:
        return self.dim // 32


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def splitmix64(seed: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.uint64)
    _load().oracle_splitmix64(ctypes.c_uint64(seed), n, _p(out))
    return out


def num_bins(p: Params) -> int:
    return int(_load().oracle_num_bins(p.mz_min, p.mz_max, p.bins_per_da))


def codebook(p: Params) -> Tuple[np.ndarray, np.ndarray]:
    """(ID table [f, D/32], level table [Q, D/32]) as uint32."""
    f = num_bins(p)
    idt = np.zeros((f, p.words), dtype=np.uint32)
    lvt = np.zeros((p.n_levels, p.words), dtype=np.uint32)
    rc = _load().oracle_codebook(p.dim, f, p.n_levels, p.alpha, ctypes.c_uint64(p.seed),
                                 p.encoding, _p(idt), _p(lvt))
    if rc != 0:
        raise ValueError("invalid codebook parameters")
    return idt, lvt


def preprocess(offsets, mz, intensity, p: Params):
    """Raw CSR peaks -> (offsets int64, bin int32, level uint8) of unique bins."""
    off = _c(offsets, np.int64)
    mz = _c(mz, np.float64)
    it = _c(intensity, np.float64)
    n = off.shape[0] - 1
    cap = max(int(off[-1]), 1)
    o_off = np.zeros(n + 1, dtype=np.int64)
    o_bin = np.zeros(cap, dtype=np.int32)
    o_lv = np.zeros(cap, dtype=np.uint8)
    tot = _load().oracle_preprocess(n, _p(off), _p(mz), _p(it), p.mz_min, p.mz_max,
                                    p.bins_per_da, p.noise_frac, p.top_n, p.n_levels,
                                    _p(o_off), _p(o_bin), _p(o_lv))
    if tot < 0:
        raise MemoryError("oracle preprocess failed")
    return o_off, o_bin[:tot].copy(), o_lv[:tot].copy()


def encode(p: Params, idt, lvt, offsets, bins, levels) -> np.ndarray:
    """Eq. 1 + binarisation for every spectrum (or, with p.encoding == 2, the
    random-projection baseline): uint32 [n, D/32]."""
    off = _c(offsets, np.int64)
    b = _c(bins, np.int32)
    lv = _c(levels, np.uint8)
    idt = _c(idt, np.uint32)
    lvt = _c(lvt, np.uint32)
    n = off.shape[0] - 1
    if b.size and (b.min() < 0 or b.max() >= idt.shape[0]):
        raise ValueError("bin out of range")
    if lv.size and lv.max() >= lvt.shape[0]:
        raise ValueError("level out of range")
    out = np.zeros((n, p.words), dtype=np.uint32)
    if b.size == 0:
        b = np.zeros(1, dtype=np.int32)
        lv = np.zeros(1, dtype=np.uint8)
    if p.encoding == 2:
        _load().oracle_encode_lsh(p.dim, _p(idt), n, _p(off), _p(b), _p(lv), _p(out))
    else:
        _load().oracle_encode(p.dim, _p(idt), _p(lvt), n, _p(off), _p(b), _p(lv), _p(out))
    return out


def _windows(nq, kinds, values):
    k = np.broadcast_to(np.asarray(kinds, dtype=np.int32), (nq,)).copy()
    v = np.broadcast_to(np.asarray(values, dtype=np.float64), (nq,)).copy()
    return k, v


def search(p: Params, lib_hv, lib_pmz, lib_charge, q_hv, q_pmz, q_charge,
           kinds=0, values=500.0, charge_match=True):
    """Top-1 (library index, Hamming distance) per query; (-1, -1) if no candidate."""
    lib_hv = _c(lib_hv, np.uint32)
    q_hv = _c(q_hv, np.uint32)
    lp = _c(lib_pmz, np.float64)
    lc = _c(lib_charge, np.int8)
    qp = _c(q_pmz, np.float64)
    qc = _c(q_charge, np.int8)
    nq = qp.shape[0]
    k, v = _windows(nq, kinds, values)
    idx = np.zeros(nq, dtype=np.int64)
    dist = np.zeros(nq, dtype=np.int32)
    _load().oracle_search(p.dim, lp.shape[0], _p(lib_hv), _p(lp), _p(lc), nq, _p(q_hv), _p(qp),
                          _p(qc), _p(k), _p(v), int(bool(charge_match)), _p(idx), _p(dist))
    return idx, dist


def window_counts(lib_pmz, lib_charge, q_pmz, q_charge, kinds=0, values=500.0,
                  charge_match=True) -> np.ndarray:
    lp = _c(lib_pmz, np.float64)
    lc = _c(lib_charge, np.int8)
    qp = _c(q_pmz, np.float64)
    qc = _c(q_charge, np.int8)
    nq = qp.shape[0]
    k, v = _windows(nq, kinds, values)
    out = np.zeros(nq, dtype=np.int64)
    _load().oracle_window_counts(lp.shape[0], _p(lp), _p(lc), nq, _p(qp), _p(qc), _p(k), _p(v),
                                 int(bool(charge_match)), _p(out))
    return out


def window_distances(p: Params, lib_hv, lib_pmz, lib_charge, q_hv, q_pmz, q_charge,
                     kinds=0, values=500.0, charge_match=True):
    """All candidates with distances: (row_off [nq+1], idx, dist) in library order."""
    counts = window_counts(lib_pmz, lib_charge, q_pmz, q_charge, kinds, values, charge_match)
    row_off = np.zeros(counts.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=row_off[1:])
    tot = int(row_off[-1])
    idx = np.zeros(max(tot, 1), dtype=np.int64)
    dist = np.zeros(max(tot, 1), dtype=np.int32)
    lib_hv = _c(lib_hv, np.uint32)
    q_hv = _c(q_hv, np.uint32)
    lp = _c(lib_pmz, np.float64)
    lc = _c(lib_charge, np.int8)
    qp = _c(q_pmz, np.float64)
    qc = _c(q_charge, np.int8)
    nq = qp.shape[0]
    k, v = _windows(nq, kinds, values)
    _load().oracle_window_distances(p.dim, lp.shape[0], _p(lib_hv), _p(lp), _p(lc), nq, _p(q_hv),
                                    _p(qp), _p(qc), _p(k), _p(v), int(bool(charge_match)),
                                    _p(row_off), _p(idx), _p(dist))
    return row_off, idx[:tot], dist[:tot]


def encode_raw(p: Params, idt, lvt, raw) -> np.ndarray:
    """Preprocess then encode spectra given as an object with offsets/mz/intensity."""
    off, b, lv = preprocess(raw.offsets, raw.mz, raw.intensity, p)
    return encode(p, idt, lvt, off, b, lv)
