"""Python binding of libhyperoms (C ABI in include/hyperoms.h).

Argument marshalling only: every step of preprocessing, encoding and search
runs inside the native library (host C++ for preprocessing and codebook
generation, HIP kernels for everything on the device). PyTorch supplies
device memory and the current HIP stream. If the library is not built this
module raises at import; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhyperoms.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_2211_16422_amd.build` "
        "(hipcc, gfx950); there is no CPU fallback")

_lib = ctypes.CDLL(LIB_PATH)

HOMS_OK = 0
HOMS_E_INVALID = -1
HOMS_E_OOM = -2
HOMS_E_DEVICE = -3
HOMS_E_STATE = -4
HOMS_E_UNSUPPORTED = -5

TOL_DA = 0
TOL_PPM = 1

ENGINE_POPCOUNT = 0
ENGINE_MFMA_I8 = 1
ENGINE_MFMA_F8 = 2
ENGINE_MFMA_F4 = 3

# largest nq of homs_search_window_noalloc (HOMS_NOALLOC_MAX_QUERIES)
NOALLOC_MAX_QUERIES = 131072

ENCODING_ID_LEVEL = 0
ENCODING_RANDOM_ID = 1
ENCODING_LSH = 2


class HomsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class _Params(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("dim", ctypes.c_uint32),
                ("n_levels", ctypes.c_uint32), ("top_n", ctypes.c_uint32),
                ("mz_min", ctypes.c_double), ("mz_max", ctypes.c_double),
                ("bins_per_da", ctypes.c_double), ("noise_frac", ctypes.c_double),
                ("id_flips", ctypes.c_uint32), ("charge_match", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("encoding", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class _Window(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("value", ctypes.c_double)]


_P = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_st = ctypes.c_int32


def _sig(name, argtypes, restype=_st):
    f = getattr(_lib, name)
    f.argtypes = argtypes
    f.restype = restype
    return f


_sig("homs_params_default", [ctypes.POINTER(_Params)])
_sig("homs_num_bins", [ctypes.POINTER(_Params)], _i64)
_sig("homs_status_string", [_st], ctypes.c_char_p)
_sig("homs_last_error", [_P], ctypes.c_char_p)
_sig("homs_preprocess", [ctypes.POINTER(_Params), _i64, _P, _P, _P, _P, _P, _P, _P, _i32])
_sig("homs_create", [ctypes.POINTER(_Params), _i32, ctypes.POINTER(_P)])
_sig("homs_destroy", [_P], None)
_sig("homs_generate_codebook", [ctypes.POINTER(_Params), _P, _P])
_sig("homs_set_codebook", [_P, _P, _P])
_sig("homs_get_codebook", [_P, _P, _P])
_sig("homs_encode_queries", [_P, _i64, _P, _P, _P, _P, _P])
_sig("homs_encode_library", [_P, _i64, _P, _P, _P, _P, _P, _P])
_sig("homs_library_size", [_P, ctypes.POINTER(_i64)])
_sig("homs_library_export", [_P, _P, _P])
_sig("homs_library_order", [_P, _P, _P])
_sig("homs_window_bounds", [_P, _i64, _P, _P, ctypes.POINTER(_Window), _P, _P, _P])
_sig("homs_search_window", [_P, _i64, _P, _P, _P, ctypes.POINTER(_Window), _i32, _P, _P, _P])
_sig("homs_search_window_noalloc", [_P, _i64, _P, _P, _P, ctypes.POINTER(_Window), _i32, _P, _P,
                                    _P])
_sig("homs_preprocess_device", [_P, _i64, _P, _P, _P, _P, _P, _P, _P])
_sig("homs_cascade_search", [_P, _i64, _P, _P, _P, ctypes.POINTER(_Window),
                             ctypes.POINTER(_Window), _i32, _P, ctypes.c_double, _P, _P, _P, _P,
                             _P])
_sig("homs_debug_distances", [_P, _i64, _P, _P, _P, ctypes.POINTER(_Window), _P, _P, _P, _P])
_sig("homs_device_errors", [_P, ctypes.POINTER(ctypes.c_uint32), _P])


class _Profile(ctypes.Structure):
    _fields_ = [("search_ms", ctypes.c_double), ("encode_ms", ctypes.c_double),
                ("prep_ms", ctypes.c_double), ("search_launches", ctypes.c_int64),
                ("encode_launches", ctypes.c_int64), ("score_ms", ctypes.c_double),
                ("score_launches", ctypes.c_int64)]


_sig("homs_profile_enable", [_P, _i32])
_sig("homs_profile_read", [_P, ctypes.POINTER(_Profile)])


class _BatchedConfig(ctypes.Structure):
    _fields_ = [("narrow_max", ctypes.c_uint32), ("chunk_rows", ctypes.c_uint32),
                ("narrow_group", ctypes.c_uint32), ("grid", ctypes.c_uint32),
                ("bucket_da", ctypes.c_double), ("engine", ctypes.c_int32)]


_sig("homs_batched_config_get", [_P, ctypes.POINTER(_BatchedConfig)])
_sig("homs_batched_config_set", [_P, ctypes.POINTER(_BatchedConfig)])
_sig("homs_search_batched", [_P, _i64, _P, _P, _P, _P, _P, _P, _P, _i32, _P])
_sig("homs_autotune_batched", [_P, _i64, _P, _P, _P, _P, _P, _P, _P, _i32,
                               ctypes.POINTER(_BatchedConfig), ctypes.POINTER(ctypes.c_double),
                               _P])

EXPORTED = ["homs_params_default", "homs_num_bins", "homs_status_string", "homs_last_error",
            "homs_preprocess", "homs_create", "homs_destroy", "homs_generate_codebook", "homs_set_codebook",
            "homs_get_codebook", "homs_encode_queries", "homs_encode_library",
            "homs_library_size", "homs_library_export", "homs_library_order",
            "homs_window_bounds",
            "homs_search_window", "homs_search_window_noalloc", "homs_cascade_search", "homs_preprocess_device",
            "homs_debug_distances",
            "homs_device_errors",
            "homs_profile_enable", "homs_profile_read", "homs_batched_config_get",
            "homs_batched_config_set", "homs_search_batched", "homs_autotune_batched",
            "homs_model_create", "homs_model_destroy", "homs_model_set_weights",
            "homs_model_get_weights", "homs_model_embed", "homs_model_gradients",
            "homs_model_train_step", "homs_train_config_default", "homs_model_train",
            "homs_model_embed_library", "homs_model_library_embeddings", "homs_search_learned",
            "homs_measure_xor_popcount_rate", "homs_library_save", "homs_library_load",
            "homs_model_save", "homs_model_load", "homs_file_inspect"]

_sig("homs_model_create", [_P, _i32, _i32, _P, _P, _P, _P, ctypes.POINTER(_P)])
_sig("homs_model_destroy", [_P], None)
_sig("homs_model_set_weights", [_P, _P, _P, _P, _P])
_sig("homs_model_get_weights", [_P, _P, _P, _P, _P])
_sig("homs_model_embed", [_P, _i64, _P, _P, _P])
_sig("homs_model_gradients", [_P, _i32, _P, _P, ctypes.c_float, ctypes.POINTER(ctypes.c_float),
                              _P, _P, _P, _P, _P])
_sig("homs_model_train_step", [_P, _i32, _P, _P, ctypes.c_float, ctypes.c_float, _P, _P])


class _TrainConfig(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("epochs", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("lr", ctypes.c_float), ("tau", ctypes.c_float),
                ("reserved", ctypes.c_uint32), ("seed", ctypes.c_uint64)]


_sig("homs_train_config_default", [ctypes.POINTER(_TrainConfig)])
_sig("homs_model_train", [_P, _i64, _P, _P, ctypes.POINTER(_TrainConfig), _P,
                          ctypes.POINTER(_i64), _P])
_sig("homs_model_embed_library", [_P, _P])
_sig("homs_model_library_embeddings", [_P, _P, _P, _P])
_sig("homs_search_learned", [_P, _P, _i64, _P, _P, _P, ctypes.POINTER(_Window), _i32, _P, _P, _P,
                             _P, _P])

_sig("homs_measure_xor_popcount_rate", [_i32, ctypes.POINTER(ctypes.c_double)])

FILE_LIBRARY = 1
FILE_MODEL = 2


class _FileInfo(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_uint32), ("version", ctypes.c_uint32),
                ("dim", ctypes.c_uint32), ("hidden", ctypes.c_int32), ("embed", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("n", ctypes.c_int64), ("step", ctypes.c_int64),
                ("codebook_hash", ctypes.c_uint64), ("params", _Params)]


_sig("homs_library_save", [_P, ctypes.c_char_p])
_sig("homs_library_load", [_P, ctypes.c_char_p])
_sig("homs_model_save", [_P, ctypes.c_char_p])
_sig("homs_model_load", [_P, ctypes.c_char_p, ctypes.POINTER(_P)])
_sig("homs_file_inspect", [ctypes.c_char_p, ctypes.POINTER(_FileInfo)])


def file_info(path: str) -> dict:
    """homs_file_inspect: what a library or model file holds (host only; checks
    the size and the checksum)."""
    fi = _FileInfo()
    _check(_lib.homs_file_inspect(os.fsencode(path), ctypes.byref(fi)))
    out = {"kind": fi.kind, "version": fi.version, "dim": fi.dim, "hidden": fi.hidden,
           "embed": fi.embed, "n": fi.n, "step": fi.step, "codebook_hash": fi.codebook_hash}
    if fi.kind == FILE_LIBRARY:
        p = fi.params
        out["params"] = {"dim": p.dim, "n_levels": p.n_levels, "top_n": p.top_n,
                         "mz_min": p.mz_min, "mz_max": p.mz_max, "bins_per_da": p.bins_per_da,
                         "noise_frac": p.noise_frac, "id_flips": p.id_flips,
                         "charge_match": p.charge_match, "seed": p.seed,
                         "encoding": p.encoding}
    return out


def measure_xor_popcount_rate(device: int = 0) -> float:
    """homs_measure_xor_popcount_rate: sustained xor+popcount lane-ops/s."""
    r = ctypes.c_double(0.0)
    _check(_lib.homs_measure_xor_popcount_rate(device, ctypes.byref(r)))
    return r.value


@dataclass(frozen=True)
class Params:
    """homs_params (Table 1; Section 4.2 defaults)."""

    dim: int = 8192
    n_levels: int = 16
    top_n: int = 50
    mz_min: float = 101.0
    mz_max: float = 1500.0
    bins_per_da: float = 20.0
    noise_frac: float = 0.01
    id_flips: int = 0
    charge_match: bool = True
    seed: int = 0
    encoding: int = 0  # ENCODING_*

    def _c(self) -> _Params:
        p = _Params()
        _lib.homs_params_default(ctypes.byref(p))
        p.dim, p.n_levels, p.top_n = self.dim, self.n_levels, self.top_n
        p.mz_min, p.mz_max = self.mz_min, self.mz_max
        p.bins_per_da, p.noise_frac = self.bins_per_da, self.noise_frac
        p.id_flips, p.charge_match, p.seed = self.id_flips, int(self.charge_match), self.seed
        p.encoding = self.encoding
        return p

    @property
    def words(self) -> int:
        return self.dim // 32


def last_error(ctx=None) -> str:
    m = _lib.homs_last_error(ctx)
    return m.decode() if m else ""


def _check(status: int, ctx=None):
    if status != HOMS_OK:
        raise HomsError(status, last_error(ctx) or _lib.homs_status_string(status).decode())


def num_bins(p: Params) -> int:
    c = p._c()
    return int(_lib.homs_num_bins(ctypes.byref(c)))


def generate_codebook(p: Params) -> Tuple[np.ndarray, np.ndarray]:
    """homs_generate_codebook: (ID table [f, D/32], level table [Q, D/32]) on the host."""
    f = num_bins(p)
    idt = np.zeros((f, p.words), dtype=np.uint32)
    lvt = np.zeros((p.n_levels, p.words), dtype=np.uint32)
    c = p._c()
    _check(_lib.homs_generate_codebook(ctypes.byref(c), _np_ptr(idt), _np_ptr(lvt)))
    return idt, lvt


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def preprocess(p: Params, offsets, mz, intensity, n_threads: int = 0
               ) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """homs_preprocess: raw CSR peaks (host) -> (offsets, bin, level) (host)."""
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    mz = np.ascontiguousarray(mz, dtype=np.float64)
    it = np.ascontiguousarray(intensity, dtype=np.float64)
    n = off.shape[0] - 1
    cap = max(int(off[-1]), 1)
    o_off = np.zeros(n + 1, dtype=np.int64)
    o_bin = np.empty(cap, dtype=np.int32)
    o_lv = np.empty(cap, dtype=np.uint8)
    tot = _i64(0)
    c = p._c()
    _check(_lib.homs_preprocess(ctypes.byref(c), n, _np_ptr(off), _np_ptr(mz), _np_ptr(it),
                                _np_ptr(o_off), _np_ptr(o_bin), _np_ptr(o_lv),
                                ctypes.byref(tot), n_threads))
    t = tot.value
    return o_off, o_bin[:t], o_lv[:t]


def _stream(dev) -> int:
    import torch
    return torch.cuda.current_stream(dev).cuda_stream


def _dptr(t, dtype, name: str, device) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, context is on {device}")
    return t.data_ptr()


class Context:
    """A homs_ctx: codebook, device-resident sorted library, workspace."""

    def __init__(self, params: Params, device: int = 0):
        import torch
        self.params = params
        self.device = torch.device("cuda", device)
        self.words = params.dim // 32
        self.n_bins = num_bins(params)
        h = _P()
        c = params._c()
        _check(_lib.homs_create(ctypes.byref(c), device, ctypes.byref(h)))
        self._h = h

    # --- lifetime
    def close(self):
        if getattr(self, "_h", None):
            _lib.homs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _ck(self, status):
        _check(status, self._h)

    # --- codebook
    def get_codebook(self) -> Tuple[np.ndarray, np.ndarray]:
        idt = np.zeros((self.n_bins, self.words), dtype=np.uint32)
        lvt = np.zeros((self.params.n_levels, self.words), dtype=np.uint32)
        self._ck(_lib.homs_get_codebook(self._h, _np_ptr(idt), _np_ptr(lvt)))
        return idt, lvt

    def set_codebook(self, id_table: Optional[np.ndarray] = None,
                     level_table: Optional[np.ndarray] = None):
        a = b = None
        if id_table is not None:
            a = np.ascontiguousarray(id_table, dtype=np.uint32)
            if a.shape != (self.n_bins, self.words):
                raise ValueError("id table shape")
        if level_table is not None:
            b = np.ascontiguousarray(level_table, dtype=np.uint32)
            if b.shape != (self.params.n_levels, self.words):
                raise ValueError("level table shape")
        self._ck(_lib.homs_set_codebook(self._h, _np_ptr(a) if a is not None else None,
                                        _np_ptr(b) if b is not None else None))

    # --- encoding
    def encode_queries(self, offsets, bins, levels, out=None):
        """homs_encode_queries on device CSR tensors -> uint32 [n, D/32] (int32 view)."""
        import torch
        n = offsets.shape[0] - 1
        if out is None:
            out = torch.empty((n, self.words), dtype=torch.int32, device=self.device)
        self._ck(_lib.homs_encode_queries(
            self._h, n, _dptr(offsets, torch.int64, "offsets", self.device),
            _dptr(bins, torch.int32, "bins", self.device),
            _dptr(levels, torch.uint8, "levels", self.device),
            _dptr(out, torch.int32, "out", self.device), _stream(self.device)))
        return out

    def encode_library(self, offsets, bins, levels, pmz, charge):
        import torch
        n = offsets.shape[0] - 1
        self._ck(_lib.homs_encode_library(
            self._h, n, _dptr(offsets, torch.int64, "offsets", self.device),
            _dptr(bins, torch.int32, "bins", self.device),
            _dptr(levels, torch.uint8, "levels", self.device),
            _dptr(pmz, torch.float64, "pmz", self.device),
            _dptr(charge, torch.int8, "charge", self.device), _stream(self.device)))

    def library_size(self) -> int:
        n = _i64(0)
        self._ck(_lib.homs_library_size(self._h, ctypes.byref(n)))
        return n.value

    def library_export(self):
        import torch
        out = torch.empty((self.library_size(), self.words), dtype=torch.int32,
                          device=self.device)
        self._ck(_lib.homs_library_export(self._h, _dptr(out, torch.int32, "out", self.device),
                                          _stream(self.device)))
        return out

    def library_save(self, path: str):
        """homs_library_save: the encoded library to a file."""
        self._ck(_lib.homs_library_save(self._h, os.fsencode(path)))

    def library_load(self, path: str):
        """homs_library_load: the library of a file written with these parameters."""
        self._ck(_lib.homs_library_load(self._h, os.fsencode(path)))

    def library_order(self):
        """homs_library_order: library index of each sorted row (uint32 as int32)."""
        import torch
        out = torch.empty(max(self.library_size(), 1), dtype=torch.int32, device=self.device)
        self._ck(_lib.homs_library_order(self._h, _dptr(out, torch.int32, "out", self.device),
                                         _stream(self.device)))
        return out[:self.library_size()]

    # --- search
    @staticmethod
    def _win(kind: int, value: float) -> _Window:
        w = _Window()
        w.kind, w.reserved, w.value = kind, 0, value
        return w

    def window_bounds(self, pmz, charge, kind=TOL_DA, value=500.0):
        import torch
        nq = pmz.shape[0]
        lo = torch.empty(nq, dtype=torch.int64, device=self.device)
        hi = torch.empty(nq, dtype=torch.int64, device=self.device)
        w = self._win(kind, value)
        self._ck(_lib.homs_window_bounds(
            self._h, nq, _dptr(pmz, torch.float64, "pmz", self.device),
            _dptr(charge, torch.int8, "charge", self.device), ctypes.byref(w),
            _dptr(lo, torch.int64, "lo", self.device), _dptr(hi, torch.int64, "hi", self.device),
            _stream(self.device)))
        return lo, hi

    def search_window(self, q_hv, pmz, charge, kind=TOL_DA, value=500.0,
                      engine=ENGINE_POPCOUNT, out_idx=None, out_dist=None):
        """homs_search_window -> (library index int64, Hamming distance int32)."""
        import torch
        nq = pmz.shape[0]
        if q_hv.shape != (nq, self.words):
            raise ValueError("q_hv must be [nq, D/32]")
        if out_idx is None:
            out_idx = torch.empty(nq, dtype=torch.int64, device=self.device)
        if out_dist is None:
            out_dist = torch.empty(nq, dtype=torch.int32, device=self.device)
        w = self._win(kind, value)
        self._ck(_lib.homs_search_window(
            self._h, nq, _dptr(q_hv, torch.int32, "q_hv", self.device),
            _dptr(pmz, torch.float64, "pmz", self.device),
            _dptr(charge, torch.int8, "charge", self.device), ctypes.byref(w), engine,
            _dptr(out_idx, torch.int64, "out_idx", self.device),
            _dptr(out_dist, torch.int32, "out_dist", self.device), _stream(self.device)))
        return out_idx, out_dist

    def search_window_noalloc(self, q_hv, pmz, charge, out_idx, out_dist, kind=TOL_DA,
                              value=500.0, engine=ENGINE_POPCOUNT):
        """homs_search_window_noalloc: homs_search_window with its scratch in the
        library's static device array (no allocation; nq <= NOALLOC_MAX_QUERIES);
        the caller passes the outputs."""
        import torch
        nq = pmz.shape[0]
        if q_hv.shape != (nq, self.words):
            raise ValueError("q_hv must be [nq, D/32]")
        w = self._win(kind, value)
        self._ck(_lib.homs_search_window_noalloc(
            self._h, nq, _dptr(q_hv, torch.int32, "q_hv", self.device),
            _dptr(pmz, torch.float64, "pmz", self.device),
            _dptr(charge, torch.int8, "charge", self.device), ctypes.byref(w), engine,
            _dptr(out_idx, torch.int64, "out_idx", self.device),
            _dptr(out_dist, torch.int32, "out_dist", self.device), _stream(self.device)))
        return out_idx, out_dist

    def preprocess_device(self, offsets, mz, intensity, check=True):
        """homs_preprocess_device: raw peaks (device CSR: int64 offsets, float64 m/z and
        intensities) -> device CSR (offsets int64, bins int32, levels uint8).

        With `check` (the default) the context's device error flags are read (and
        cleared) after the call, and a spectrum that would keep more than 2,048 peaks
        (possible only with top_n above 2,048; flag bit 1; it gets no entries) raises
        HomsError(HOMS_E_INVALID)."""
        import torch
        n = offsets.shape[0] - 1
        raw = int(offsets[-1].item()) if n > 0 else 0
        cap = max(1, min(raw, n * int(self.params.top_n)))
        out_off = torch.empty(n + 1, dtype=torch.int64, device=self.device)
        out_bin = torch.empty(cap, dtype=torch.int32, device=self.device)
        out_lv = torch.empty(cap, dtype=torch.uint8, device=self.device)
        self._ck(_lib.homs_preprocess_device(
            self._h, n, _dptr(offsets, torch.int64, "offsets", self.device),
            _dptr(mz, torch.float64, "mz", self.device),
            _dptr(intensity, torch.float64, "intensity", self.device),
            _dptr(out_off, torch.int64, "out_offsets", self.device),
            _dptr(out_bin, torch.int32, "out_bin", self.device),
            _dptr(out_lv, torch.uint8, "out_level", self.device), _stream(self.device)))
        total = int(out_off[-1].item())
        if check:
            flags = self.device_errors()
            if flags & 2:
                raise HomsError(HOMS_E_INVALID,
                                "homs_preprocess_device: a spectrum keeps more than 2048 peaks "
                                f"(device error flags {flags:#x}); it was given no entries")
            if flags:
                raise HomsError(HOMS_E_INVALID, f"device error flags {flags:#x}")
        return out_off, out_bin[:total], out_lv[:total]

    def cascade_search(self, q_hv, pmz, charge, lib_decoy, narrow=(TOL_PPM, 20.0),
                       wide=(TOL_DA, 500.0), engine=ENGINE_MFMA_F4, fdr_level=0.01):
        """homs_cascade_search -> (library index int64, distance int32, stage int8,
        q-value float64); lib_decoy: uint8 per library index (1 = decoy)."""
        import torch
        nq = pmz.shape[0]
        if q_hv.shape != (nq, self.words):
            raise ValueError("q_hv must be [nq, D/32]")
        out_idx = torch.empty(nq, dtype=torch.int64, device=self.device)
        out_dist = torch.empty(nq, dtype=torch.int32, device=self.device)
        out_stage = torch.empty(nq, dtype=torch.int8, device=self.device)
        out_q = torch.empty(nq, dtype=torch.float64, device=self.device)
        wn = self._win(*narrow)
        ww = self._win(*wide)
        self._ck(_lib.homs_cascade_search(
            self._h, nq, _dptr(q_hv, torch.int32, "q_hv", self.device),
            _dptr(pmz, torch.float64, "pmz", self.device),
            _dptr(charge, torch.int8, "charge", self.device), ctypes.byref(wn), ctypes.byref(ww),
            engine, _dptr(lib_decoy, torch.uint8, "lib_decoy", self.device), float(fdr_level),
            _dptr(out_idx, torch.int64, "out_idx", self.device),
            _dptr(out_dist, torch.int32, "out_dist", self.device),
            _dptr(out_stage, torch.int8, "out_stage", self.device),
            _dptr(out_q, torch.float64, "out_q", self.device), _stream(self.device)))
        return out_idx, out_dist, out_stage, out_q

    def debug_distances(self, q_hv, pmz, charge, kind=TOL_DA, value=500.0):
        """All candidates with distances: (row_off, lib index, dist) in sorted order."""
        import torch
        lo, hi = self.window_bounds(pmz, charge, kind, value)
        cnt = (hi - lo)
        row_off = torch.zeros(pmz.shape[0] + 1, dtype=torch.int64, device=self.device)
        torch.cumsum(cnt, 0, out=row_off[1:])
        tot = int(row_off[-1].item())
        idx = torch.empty(max(tot, 1), dtype=torch.int64, device=self.device)
        dist = torch.empty(max(tot, 1), dtype=torch.int32, device=self.device)
        w = self._win(kind, value)
        self._ck(_lib.homs_debug_distances(
            self._h, pmz.shape[0], _dptr(q_hv, torch.int32, "q_hv", self.device),
            _dptr(pmz, torch.float64, "pmz", self.device),
            _dptr(charge, torch.int8, "charge", self.device), ctypes.byref(w),
            _dptr(row_off, torch.int64, "row_off", self.device),
            _dptr(idx, torch.int64, "idx", self.device),
            _dptr(dist, torch.int32, "dist", self.device), _stream(self.device)))
        return row_off, idx[:tot], dist[:tot]

    # --- batched (mixed-window) search
    def batched_config(self) -> dict:
        c = _BatchedConfig()
        self._ck(_lib.homs_batched_config_get(self._h, ctypes.byref(c)))
        return {f: getattr(c, f) for f, _ in _BatchedConfig._fields_}

    def set_batched_config(self, **kw):
        cfg = self.batched_config()
        cfg.update(kw)
        c = _BatchedConfig(**cfg)
        self._ck(_lib.homs_batched_config_set(self._h, ctypes.byref(c)))

    def _batched_args(self, q_hv, pmz, charge, kinds, values, out_idx, out_dist):
        import torch
        nq = pmz.shape[0]
        if q_hv.shape != (nq, self.words):
            raise ValueError("q_hv must be [nq, D/32]")
        if out_idx is None:
            out_idx = torch.empty(nq, dtype=torch.int64, device=self.device)
        if out_dist is None:
            out_dist = torch.empty(nq, dtype=torch.int32, device=self.device)
        args = (nq, _dptr(q_hv, torch.int32, "q_hv", self.device),
                _dptr(pmz, torch.float64, "pmz", self.device),
                _dptr(charge, torch.int8, "charge", self.device),
                _dptr(kinds, torch.int8, "kinds", self.device),
                _dptr(values, torch.float64, "values", self.device),
                _dptr(out_idx, torch.int64, "out_idx", self.device),
                _dptr(out_dist, torch.int32, "out_dist", self.device))
        return args, out_idx, out_dist

    def search_batched(self, q_hv, pmz, charge, kinds, values, use_graph=True, out_idx=None,
                       out_dist=None):
        """homs_search_batched: per-query windows (kinds: 0 Da / 1 ppm) in one launch."""
        args, out_idx, out_dist = self._batched_args(q_hv, pmz, charge, kinds, values, out_idx,
                                                     out_dist)
        self._ck(_lib.homs_search_batched(self._h, *args, int(bool(use_graph)),
                                          _stream(self.device)))
        return out_idx, out_dist

    def autotune_batched(self, q_hv, pmz, charge, kinds, values, reps=2, out_idx=None,
                         out_dist=None):
        """homs_autotune_batched -> (best config dict, ms per batch)."""
        args, out_idx, out_dist = self._batched_args(q_hv, pmz, charge, kinds, values, out_idx,
                                                     out_dist)
        best = _BatchedConfig()
        ms = ctypes.c_double(0.0)
        self._ck(_lib.homs_autotune_batched(self._h, *args, reps, ctypes.byref(best),
                                            ctypes.byref(ms), _stream(self.device)))
        return {f: getattr(best, f) for f, _ in _BatchedConfig._fields_}, ms.value

    def profile_enable(self, on: bool = True):
        self._ck(_lib.homs_profile_enable(self._h, int(on)))

    def profile_read(self) -> dict:
        p = _Profile()
        self._ck(_lib.homs_profile_read(self._h, ctypes.byref(p)))
        return {"search_ms": p.search_ms, "encode_ms": p.encode_ms, "prep_ms": p.prep_ms,
                "search_launches": p.search_launches, "encode_launches": p.encode_launches,
                "score_ms": p.score_ms, "score_launches": p.score_launches}

    def device_errors(self) -> int:
        f = ctypes.c_uint32(0)
        self._ck(_lib.homs_device_errors(self._h, ctypes.byref(f), _stream(self.device)))
        return f.value


def to_device_csr(off, bins, levels, device):
    """Host CSR (numpy) -> device tensors for the encode entry points."""
    import torch
    return (torch.from_numpy(np.ascontiguousarray(off, dtype=np.int64)).to(device),
            torch.from_numpy(np.ascontiguousarray(bins, dtype=np.int32)).to(device),
            torch.from_numpy(np.ascontiguousarray(levels, dtype=np.uint8)).to(device))


WEIGHT_NAMES = ("W1", "b1", "W2", "b2")


def sketch_weights(dim: int, hidden: int, embed: int, seed: int = 0,
                   center: Optional[np.ndarray] = None) -> dict:
    """Weights under which the network needs no training: it computes a
    signed block-sum sketch (CountSketch) of the bipolar hypervector. The D
    components are dealt at random into `embed` blocks of D / embed, each
    component with a random sign, z_j = sum over block j of s_d x_d; hidden
    units 2j and 2j + 1 carry ReLU(z_j) and ReLU(-z_j) and W2 takes their
    difference, so z is the sketch exactly (integers of magnitude <= D /
    embed, exact in bfloat16). The shortlist score is the cosine of the two
    sketches: a training-free shortlist at the same embedding width.

    center (optional, [dim]): a vector subtracted from x before the sketch
    (through the hidden biases, b1 = -+ the sketch of center), typically the
    mean bipolar hypervector of the library: spectrum hypervectors share a
    large common part, and without it the cosines of all pairs crowd near 1."""
    if hidden < 2 * embed or dim % embed:
        raise ValueError("needs hidden >= 2 * embed and embed dividing dim")
    rng = np.random.default_rng(seed)
    comp = rng.permutation(dim).reshape(embed, dim // embed)
    sign = rng.choice(np.array([-1.0, 1.0], np.float32), size=(embed, dim // embed))
    W1 = np.zeros((hidden, dim), np.float32)
    W2 = np.zeros((embed, hidden), np.float32)
    rows = np.arange(embed)
    W1[2 * rows[:, None], comp] = sign
    W1[2 * rows[:, None] + 1, comp] = -sign
    W2[rows, 2 * rows] = 1.0
    W2[rows, 2 * rows + 1] = -1.0
    b1 = np.zeros(hidden, np.float32)
    if center is not None:
        c = np.asarray(center, np.float64)
        if c.shape != (dim,):
            raise ValueError("center must have dim components")
        m = (sign.astype(np.float64) * c[comp]).sum(axis=1)
        b1[2 * rows] = -m
        b1[2 * rows + 1] = m
    return {"W1": W1, "b1": b1, "W2": W2, "b2": np.zeros(embed, np.float32)}


class Model:
    """A homs_model (learned shortlist) on a context's device.

    weights: dict of float32 host arrays W1 [hidden, D], b1 [hidden],
    W2 [embed, hidden], b2 [embed] (the initial weights are the caller's)."""

    def __init__(self, ctx: Context, weights: dict):
        self.ctx = ctx
        self.hidden, self.dim = weights["W1"].shape
        self.embed_dim = weights["W2"].shape[0]
        if self.dim != ctx.params.dim:
            raise ValueError("W1 must be [hidden, D]")
        w = self._host(weights)
        h = _P()
        ctx._ck(_lib.homs_model_create(ctx._h, self.hidden, self.embed_dim,
                                       *[_np_ptr(w[k]) for k in WEIGHT_NAMES], ctypes.byref(h)))
        self._h = h

    @classmethod
    def load(cls, ctx: "Context", path: str) -> "Model":
        """homs_model_load: a model (weights, Adam state) from a model file."""
        h = _P()
        ctx._ck(_lib.homs_model_load(ctx._h, os.fsencode(path), ctypes.byref(h)))
        m = cls.__new__(cls)
        m.ctx, m._h = ctx, h
        info = file_info(path)
        m.hidden, m.dim, m.embed_dim = info["hidden"], info["dim"], info["embed"]
        return m

    def save(self, path: str):
        """homs_model_save: weights, Adam moments and step count to a file."""
        self.ctx._ck(_lib.homs_model_save(self._h, os.fsencode(path)))

    def _host(self, weights):
        shapes = {"W1": (self.hidden, self.dim), "b1": (self.hidden,),
                  "W2": (self.embed_dim, self.hidden), "b2": (self.embed_dim,)}
        out = {}
        for k in WEIGHT_NAMES:
            a = np.ascontiguousarray(weights[k], dtype=np.float32)
            if a.shape != shapes[k]:
                raise ValueError(f"{k} must have shape {shapes[k]}")
            out[k] = a
        return out

    def close(self):
        if getattr(self, "_h", None):
            _lib.homs_model_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_weights(self, weights: dict):
        w = self._host(weights)
        self.ctx._ck(_lib.homs_model_set_weights(self._h, *[_np_ptr(w[k]) for k in WEIGHT_NAMES]))

    def get_weights(self) -> dict:
        w = {"W1": np.zeros((self.hidden, self.dim), np.float32),
             "b1": np.zeros(self.hidden, np.float32),
             "W2": np.zeros((self.embed_dim, self.hidden), np.float32),
             "b2": np.zeros(self.embed_dim, np.float32)}
        self.ctx._ck(_lib.homs_model_get_weights(self._h, *[_np_ptr(w[k]) for k in WEIGHT_NAMES]))
        return w

    def embed(self, hv, out=None):
        """homs_model_embed -> float32 [n, embed] unit embeddings."""
        import torch
        dev = self.ctx.device
        n = hv.shape[0]
        if out is None:
            out = torch.empty((n, self.embed_dim), dtype=torch.float32, device=dev)
        self.ctx._ck(_lib.homs_model_embed(self._h, n, _dptr(hv, torch.int32, "hv", dev),
                                           _dptr(out, torch.float32, "out", dev), _stream(dev)))
        return out

    def gradients(self, q_hv, r_hv, tau: float):
        """homs_model_gradients -> (loss, {W1, b1, W2, b2} gradients) without an update."""
        import torch
        dev = self.ctx.device
        g = {"W1": np.zeros((self.hidden, self.dim), np.float32),
             "b1": np.zeros(self.hidden, np.float32),
             "W2": np.zeros((self.embed_dim, self.hidden), np.float32),
             "b2": np.zeros(self.embed_dim, np.float32)}
        loss = ctypes.c_float(0.0)
        self.ctx._ck(_lib.homs_model_gradients(
            self._h, q_hv.shape[0], _dptr(q_hv, torch.int32, "q_hv", dev),
            _dptr(r_hv, torch.int32, "r_hv", dev), tau, ctypes.byref(loss),
            *[_np_ptr(g[k]) for k in WEIGHT_NAMES], _stream(dev)))
        return loss.value, g

    def train_step(self, q_hv, r_hv, tau: float, lr: float, loss_out=None):
        """homs_model_train_step; returns the device float32 [1] loss tensor."""
        import torch
        dev = self.ctx.device
        if loss_out is None:
            loss_out = torch.empty(1, dtype=torch.float32, device=dev)
        self.ctx._ck(_lib.homs_model_train_step(
            self._h, q_hv.shape[0], _dptr(q_hv, torch.int32, "q_hv", dev),
            _dptr(r_hv, torch.int32, "r_hv", dev), tau, lr,
            _dptr(loss_out, torch.float32, "loss", dev), _stream(dev)))
        return loss_out

    def train(self, q_hv, target_idx, epochs: int = 2, batch: int = 1024, lr: float = 3e-5,
              tau: float = 0.02, seed: int = 0, losses: bool = False):
        """homs_model_train on (query row, library index of its exact top-1) pairs.
        Returns the number of steps (and the device float32 losses per step)."""
        import torch
        dev = self.ctx.device
        n = q_hv.shape[0]
        if target_idx.shape != (n,):
            raise ValueError("target_idx must be [n]")
        cfg = _TrainConfig()
        _lib.homs_train_config_default(ctypes.byref(cfg))
        cfg.epochs, cfg.batch, cfg.lr, cfg.tau, cfg.seed = epochs, batch, lr, tau, seed
        out = (torch.empty(max(1, epochs * (n // batch)), dtype=torch.float32, device=dev)
               if losses else None)
        steps = _i64(0)
        self.ctx._ck(_lib.homs_model_train(
            self._h, n, _dptr(q_hv, torch.int32, "q_hv", dev) if n else None,
            _dptr(target_idx, torch.int64, "target_idx", dev) if n else None,
            ctypes.byref(cfg), _dptr(out, torch.float32, "losses", dev) if losses else None,
            ctypes.byref(steps), _stream(dev)))
        return (steps.value, out[:steps.value]) if losses else steps.value

    def embed_library(self):
        self.ctx._ck(_lib.homs_model_embed_library(self._h, _stream(self.ctx.device)))

    def library_embeddings(self):
        """homs_model_library_embeddings -> (E4M3 codes uint8 [n, E], bf16 bits
        int16 [n, E]) of the library's scoring embeddings, sorted library order."""
        import torch
        c = self.ctx
        n = c.library_size()
        codes = torch.empty((n, self.embed_dim), dtype=torch.uint8, device=c.device)
        bf = torch.empty((n, self.embed_dim), dtype=torch.int16, device=c.device)
        c._ck(_lib.homs_model_library_embeddings(
            self._h, _dptr(codes, torch.uint8, "codes", c.device),
            _dptr(bf, torch.int16, "bf16", c.device), _stream(c.device)))
        return codes, bf

    def search(self, q_hv, pmz, charge, k: int, kind=TOL_DA, value=500.0, shortlist=False):
        """homs_search_learned -> (idx int64, dist int32, fallback uint8[, shortlist int64 [nq, k]])."""
        import torch
        c = self.ctx
        dev = c.device
        nq = pmz.shape[0]
        if q_hv.shape != (nq, c.words):
            raise ValueError("q_hv must be [nq, D/32]")
        idx = torch.empty(nq, dtype=torch.int64, device=dev)
        dist = torch.empty(nq, dtype=torch.int32, device=dev)
        fb = torch.empty(nq, dtype=torch.uint8, device=dev)
        sl = torch.empty((nq, k), dtype=torch.int64, device=dev) if shortlist else None
        w = c._win(kind, value)
        c._ck(_lib.homs_search_learned(
            c._h, self._h, nq, _dptr(q_hv, torch.int32, "q_hv", dev),
            _dptr(pmz, torch.float64, "pmz", dev), _dptr(charge, torch.int8, "charge", dev),
            ctypes.byref(w), k, _dptr(idx, torch.int64, "idx", dev),
            _dptr(dist, torch.int32, "dist", dev), _dptr(fb, torch.uint8, "fallback", dev),
            _dptr(sl, torch.int64, "shortlist", dev) if shortlist else None, _stream(dev)))
        return (idx, dist, fb, sl) if shortlist else (idx, dist, fb)
