"""Host-side checks of libhyperoms that need no GPU: every symbol declared in
include/hyperoms.h is exported, host preprocessing and codebook generation
match the oracle bit for bit, and invalid arguments are rejected."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
from conftest import ROOT, gpu_available
from synth import WORKLOADS, make_workload


@pytest.fixture(scope="module")
def h():
    lib = os.path.join(ROOT, "paper_2211_16422_amd", "libhyperoms.so")
    if not os.path.exists(lib):
        from paper_2211_16422_amd.build import build
        build()
    import paper_2211_16422_amd.hyperoms as mod
    return mod


def test_exports_every_declared_symbol(h):
    text = open(os.path.join(ROOT, "include", "hyperoms.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    declared = set(re.findall(r"\b(homs_[a-z_0-9]+)\s*\(", text))
    assert len(declared) >= 15
    lib = ctypes.CDLL(h.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(h.EXPORTED)


@pytest.mark.parametrize("dim,bpd", [(2048, 20.0), (8192, 20.0), (1024, 25.0)])
def test_codebook_matches_oracle(h, dim, bpd):
    a = h.generate_codebook(h.Params(dim=dim, bins_per_da=bpd, seed=11))
    b = oracle.codebook(oracle.Params(dim=dim, bins_per_da=bpd, seed=11))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


@pytest.mark.parametrize("encoding", [1, 2])
def test_baseline_codebooks_match_oracle(h, encoding):
    """Random position rows of the Section 4.2 baselines, generated on the
    host by the library and by the oracle from the same stream."""
    a = h.generate_codebook(h.Params(dim=1024, seed=3, encoding=encoding))
    b = oracle.codebook(oracle.Params(dim=1024, seed=3, encoding=encoding))
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_preprocess_matches_oracle(h):
    g = make_workload(WORKLOADS["tiny"], n_ref=3000, n_query=500, seed=2)
    for raw in (g.library, g.queries):
        for kw in ({}, {"bins_per_da": 25.0, "top_n": 20, "n_levels": 8}):
            a = h.preprocess(h.Params(dim=2048, **kw), raw.offsets, raw.mz, raw.intensity)
            b = oracle.preprocess(raw.offsets, raw.mz, raw.intensity,
                                  oracle.Params(dim=2048, **kw))
            for x, y in zip(a, b):
                assert np.array_equal(x, y)


def test_preprocess_edge_inputs(h):
    p = h.Params(dim=512)
    off = np.array([0, 0, 3], dtype=np.int64)
    mz = np.array([101.0, 101.0, 1499.9999])
    it = np.array([4.0, 4.0, 0.0])
    a = h.preprocess(p, off, mz, it)
    b = oracle.preprocess(off, mz, it, oracle.Params(dim=512))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    # all-zero intensities: level 0 everywhere
    a = h.preprocess(p, np.array([0, 2]), np.array([200.0, 300.0]), np.array([0.0, 0.0]))
    assert a[2].tolist() == [0, 0]
    empty = h.preprocess(p, np.array([0]), np.zeros(0), np.zeros(0))
    assert empty[0].tolist() == [0] and empty[1].size == 0


def test_invalid_arguments(h):
    with pytest.raises(h.HomsError) as e:
        h.preprocess(h.Params(dim=1000), np.array([0, 1]), np.array([200.0]), np.array([1.0]))
    assert e.value.status == h.HOMS_E_INVALID
    with pytest.raises(h.HomsError):
        h.preprocess(h.Params(), np.array([0, 1]), np.array([np.nan]), np.array([1.0]))
    with pytest.raises(h.HomsError):
        h.preprocess(h.Params(), np.array([0, 1]), np.array([200.0]), np.array([-1.0]))
    with pytest.raises(h.HomsError):
        h.preprocess(h.Params(), np.array([1, 1]), np.array([200.0]), np.array([1.0]))
    with pytest.raises(h.HomsError):
        h.preprocess(h.Params(n_levels=1), np.array([0, 1]), np.array([200.0]), np.array([1.0]))
    assert h.num_bins(h.Params(mz_min=5.0, mz_max=1.0)) == -1
    assert h.num_bins(h.Params()) == 27980


@pytest.mark.skipif(gpu_available(), reason="checks the no-device error path")
def test_create_without_device_fails_cleanly(h):
    with pytest.raises(h.HomsError) as e:
        h.Context(h.Params(dim=512))
    assert e.value.status in (h.HOMS_E_DEVICE, h.HOMS_E_INVALID)


def test_noalloc_limit_matches_header(h):
    text = open(os.path.join(ROOT, "include", "hyperoms.h")).read()
    m = re.search(r"#define\s+HOMS_NOALLOC_MAX_QUERIES\s+(\d+)", text)
    assert m and int(m.group(1)) == h.NOALLOC_MAX_QUERIES


def test_sketch_weights_centre(h):
    """The centred training-free sketch network computes the sketch of x - c
    (through its hidden biases), checked with the float64 MLP oracle; without
    a centre its biases are zero and it computes the sketch of x."""
    from oracle import mlp
    rng = np.random.default_rng(0)
    D, H, E = 2048, 256, 64
    c = rng.uniform(-1, 1, D)
    X = 1.0 - 2.0 * rng.integers(0, 2, (5, D))
    f64 = lambda w: {k: v.astype(np.float64) for k, v in w.items()}  # noqa: E731
    plain = h.sketch_weights(D, H, E, seed=3)
    assert not plain["b1"].any() and not plain["b2"].any()
    z_c = mlp.forward(f64(h.sketch_weights(D, H, E, seed=3, center=c)), X)["z"]
    z_shift = mlp.forward(f64(plain), X - c)["z"]
    assert np.abs(z_c - z_shift).max() < 1e-5
    # the sketch itself: integer block sums of +-x
    z = mlp.forward(f64(plain), X)["z"]
    assert np.array_equal(z, np.round(z)) and np.abs(z).max() <= D // E
