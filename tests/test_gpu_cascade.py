"""Cascade search with target-decoy FDR (Sections 2.1, 3.4, 4.1) through the
C ABI against the oracle: every query's stage of identification, match,
distance and q-value must be identical (q-values are exact: integer counts
and one IEEE double division each)."""
import math

import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]

import oracle  # noqa: E402
from oracle import fdr  # noqa: E402
from synth import WORKLOADS, make_workload  # noqa: E402

NARROW = (1, 20.0)  # +-20 ppm
WIDE = (0, 500.0)   # +-500 Da


def _h():
    import paper_2211_16422_amd.hyperoms as h
    return h


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


class Setup:
    """Library (references, then as many decoys) and queries (half of them
    with a precursor mass shift) encoded by both sides from raw spectra."""

    def __init__(self, dim, n_ref, n_query, seed):
        h = _h()
        self.g = make_workload(WORKLOADS["tiny"], n_ref=n_ref, n_query=n_query, seed=seed)
        self.op = oracle.Params(dim=dim)
        hp = h.Params(dim=dim)
        idt, lvt = oracle.codebook(self.op)
        lib, q = self.g.library, self.g.queries
        self.o_lib = oracle.encode_raw(self.op, idt, lvt, lib)
        self.o_q = oracle.encode_raw(self.op, idt, lvt, q)
        self.decoy = np.arange(lib.n) >= n_ref
        self.ctx = h.Context(hp)
        lo, lb, ll = h.preprocess(hp, lib.offsets, lib.mz, lib.intensity)
        qo, qb, ql = h.preprocess(hp, q.offsets, q.mz, q.intensity)
        self.ctx.encode_library(*h.to_device_csr(lo, lb, ll, "cuda:0"), _dev(lib.pmz),
                                _dev(lib.charge))
        self.q_hv = self.ctx.encode_queries(*h.to_device_csr(qo, qb, ql, "cuda:0"))
        self.q_pmz = _dev(q.pmz)
        self.q_ch = _dev(q.charge)

    def gpu(self, decoy, engine, level):
        i, d, st, qv = self.ctx.cascade_search(self.q_hv, self.q_pmz, self.q_ch,
                                               _dev(decoy.astype(np.uint8)), NARROW, WIDE,
                                               engine, level)
        return i.cpu().numpy(), d.cpu().numpy(), st.cpu().numpy(), qv.cpu().numpy()

    def oracle(self, decoy, level):
        g = self.g
        return fdr.cascade(self.op, self.o_lib, g.library.pmz, g.library.charge, decoy,
                           self.o_q, g.queries.pmz, g.queries.charge, NARROW, WIDE, level)


@pytest.fixture(scope="module")
def small():
    s = Setup(2048, 1500, 400, 5)
    yield s
    s.ctx.close()


def _same(got, want):
    for a, b in zip(got, want):
        assert a.shape == b.shape
    gi, gd, gs, gq = got
    wi, wd, ws, wq = want
    assert np.array_equal(gs, ws)
    assert np.array_equal(gi, wi)
    assert np.array_equal(gd, wd)
    assert np.array_equal(np.isinf(gq), np.isinf(wq))
    fin = ~np.isinf(wq)
    assert np.array_equal(gq[fin], wq[fin])  # bit-identical doubles


@pytest.mark.parametrize("engine", [0, 2, 3])  # popcount, fp8, fp4
@pytest.mark.parametrize("level", [0.01, 0.05])
def test_cascade_matches_oracle(small, engine, level):
    want = small.oracle(small.decoy, level)
    got = small.gpu(small.decoy, engine, level)
    _same(got, want)
    # the workload exercises both stages and the rejections
    stage = want[2]
    assert np.any(stage == 1) and np.any(stage == 2)


@pytest.mark.parametrize("level", [0.0, 1.0])
def test_cascade_extreme_levels(small, level):
    _same(small.gpu(small.decoy, 3, level), small.oracle(small.decoy, level))


def test_cascade_without_or_only_decoys(small):
    none = np.zeros_like(small.decoy)
    got = small.gpu(none, 3, 0.01)
    _same(got, small.oracle(none, 0.01))
    # without decoys every PSM has FDR 0: every query with a narrow candidate
    # is identified in stage 1
    assert np.all((got[2] == 1) | (got[2] == 2) | (got[0] < 0))
    every = np.ones_like(small.decoy)
    got = small.gpu(every, 3, 0.01)
    _same(got, small.oracle(every, 0.01))
    assert np.all(got[2] == 0)
    assert np.all(np.isinf(got[3]))


def test_cascade_full_dimension_ragged():
    s = Setup(8192, 900, 301, 9)
    try:
        for engine in (0, 3):
            _same(s.gpu(s.decoy, engine, 0.01), s.oracle(s.decoy, 0.01))
    finally:
        s.ctx.close()


def test_cascade_arguments(small):
    h = _h()
    dec = _dev(small.decoy.astype(np.uint8))
    with pytest.raises(h.HomsError):
        small.ctx.cascade_search(small.q_hv, small.q_pmz, small.q_ch, dec, fdr_level=1.5)
    with pytest.raises(h.HomsError):
        small.ctx.cascade_search(small.q_hv, small.q_pmz, small.q_ch, dec, fdr_level=math.nan)
    with pytest.raises(h.HomsError):
        small.ctx.cascade_search(small.q_hv, small.q_pmz, small.q_ch, dec, narrow=(0, -1.0))
    with pytest.raises(h.HomsError):
        small.ctx.cascade_search(small.q_hv, small.q_pmz, small.q_ch, dec, engine=9)
    # no queries: nothing to do
    i, d, st, qv = small.ctx.cascade_search(small.q_hv[:0], small.q_pmz[:0], small.q_ch[:0], dec)
    assert i.numel() == 0 and st.numel() == 0
