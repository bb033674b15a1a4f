"""Parity of the HIP path (through the C ABI) with the oracle on the small
workload: every encoded bit, every candidate window, every in-window
distance and every top-1 (index, distance) must be identical."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]

import oracle  # noqa: E402
from synth import WORKLOADS, make_workload, subset  # noqa: E402


def _h():
    import paper_2211_16422_amd.hyperoms as h
    return h


def _dev(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.to("cuda:0")


def _np_u32(t):
    return t.cpu().numpy().view(np.uint32)


class Setup:
    """Tiny workload encoded by both sides, each from the raw spectra."""

    def __init__(self, dim=2048, n_ref=2000, n_query=200, seed=0, kind=0, value=500.0):
        h = _h()
        self.g = make_workload(WORKLOADS["tiny"], n_ref=n_ref, n_query=n_query, seed=seed)
        self.op = oracle.Params(dim=dim)
        self.hp = h.Params(dim=dim)
        idt, lvt = oracle.codebook(self.op)
        lib, q = self.g.library, self.g.queries
        self.o_lib = oracle.encode_raw(self.op, idt, lvt, lib)
        self.o_q = oracle.encode_raw(self.op, idt, lvt, q)
        self.ctx = h.Context(self.hp)
        lo, lb, ll = h.preprocess(self.hp, lib.offsets, lib.mz, lib.intensity)
        qo, qb, ql = h.preprocess(self.hp, q.offsets, q.mz, q.intensity)
        self.lib_csr = h.to_device_csr(lo, lb, ll, "cuda:0")
        self.q_csr = h.to_device_csr(qo, qb, ql, "cuda:0")
        self.ctx.encode_library(*self.lib_csr, _dev(lib.pmz), _dev(lib.charge))
        self.q_hv = self.ctx.encode_queries(*self.q_csr)
        self.q_pmz = _dev(q.pmz)
        self.q_ch = _dev(q.charge)


@pytest.fixture(scope="module")
def tiny():
    s = Setup()
    yield s
    s.ctx.close()


def test_codebook_matches_oracle(tiny):
    idt, lvt = tiny.ctx.get_codebook()
    o_id, o_lv = oracle.codebook(tiny.op)
    assert np.array_equal(idt, o_id) and np.array_equal(lvt, o_lv)


def test_encode_every_bit(tiny):
    import torch
    torch.cuda.synchronize()
    assert np.array_equal(_np_u32(tiny.q_hv), tiny.o_q)
    lib = _np_u32(tiny.ctx.library_export())
    assert np.array_equal(lib, tiny.o_lib)
    assert tiny.ctx.device_errors() == 0


def test_window_counts(tiny):
    lo, hi = tiny.ctx.window_bounds(tiny.q_pmz, tiny.q_ch)
    cnt = (hi - lo).cpu().numpy()
    g = tiny.g
    want = oracle.window_counts(g.library.pmz, g.library.charge, g.queries.pmz, g.queries.charge)
    assert np.array_equal(cnt, want)


def test_every_distance(tiny):
    g = tiny.g
    row, idx, dist = tiny.ctx.debug_distances(tiny.q_hv, tiny.q_pmz, tiny.q_ch)
    row, idx, dist = row.cpu().numpy(), idx.cpu().numpy(), dist.cpu().numpy()
    o_row, o_idx, o_dist = oracle.window_distances(tiny.op, tiny.o_lib, g.library.pmz,
                                                   g.library.charge, tiny.o_q, g.queries.pmz,
                                                   g.queries.charge)
    assert np.array_equal(row, o_row)
    for q in range(g.queries.n):
        a, b = row[q], row[q + 1]
        order = np.argsort(idx[a:b], kind="stable")
        assert np.array_equal(idx[a:b][order], o_idx[a:b])
        assert np.array_equal(dist[a:b][order], o_dist[a:b])


ENGINES = [0, 1, 2, 3]  # popcount, MFMA int8, MFMA fp8, MFMA fp4


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("kind,value", [(0, 500.0), (1, 20.0), (0, 0.0), (0, 5.0)])
def test_top1(tiny, kind, value, engine):
    g = tiny.g
    idx, dist = tiny.ctx.search_window(tiny.q_hv, tiny.q_pmz, tiny.q_ch, kind=kind, value=value,
                                      engine=engine)
    o_idx, o_dist = oracle.search(tiny.op, tiny.o_lib, g.library.pmz, g.library.charge,
                                  tiny.o_q, g.queries.pmz, g.queries.charge, kind, value)
    assert np.array_equal(idx.cpu().numpy(), o_idx)
    assert np.array_equal(dist.cpu().numpy(), o_dist)


@pytest.mark.parametrize("dim,n_ref,n_query", [(8192, 1500, 333), (512, 700, 1000),
                                              (1536, 3000, 257), (16384, 1100, 301),
                                              (32768, 500, 130)])
def test_top1_other_dims_ragged(dim, n_ref, n_query):
    """D = 8192 (Section 4.2) and other supported D, up to the higher-capacity
    vectors of Section 4.3 (16,384) and the largest D the ABI accepts, with query
    counts that leave ragged tiles and library sizes that leave ragged row
    blocks; every engine must agree with the oracle."""
    s = Setup(dim=dim, n_ref=n_ref, n_query=n_query, seed=3)
    g = s.g
    try:
        assert np.array_equal(_np_u32(s.q_hv), s.o_q)
        o_idx, o_dist = oracle.search(s.op, s.o_lib, g.library.pmz, g.library.charge, s.o_q,
                                      g.queries.pmz, g.queries.charge)
        for engine in ENGINES:
            idx, dist = s.ctx.search_window(s.q_hv, s.q_pmz, s.q_ch, engine=engine)
            assert np.array_equal(idx.cpu().numpy(), o_idx), engine
            assert np.array_equal(dist.cpu().numpy(), o_dist), engine
    finally:
        s.ctx.close()


@pytest.mark.parametrize("dim", [8192, 2048])
def test_top1_full_size_paths(dim):
    """The one-shot matrix-core kernels on the paths they take at full size.
    42,000 library spectra fill more than ten absolute 4,096-row chunks (both
    charge segments cross several), and 1,400 queries of charges 2 and 3 make
    at least six 256-query tiles, so the work map covers more than one patch
    of 4 tiles x 8 chunks; +-500 Da windows start and end inside 256-row
    blocks. Every engine is compared with the oracle element by element
    (Section 3.4: best match over each query's whole window), for the open
    window and a narrow 20 ppm one."""
    s = Setup(dim=dim, n_ref=21_000, n_query=1_400, seed=7)
    g = s.g
    try:
        assert g.library.n >= 40_000 and g.queries.n >= 1_300
        assert set(np.unique(g.queries.charge)) == {2, 3}
        lo, hi = s.ctx.window_bounds(s.q_pmz, s.q_ch)
        lo, hi = lo.cpu().numpy(), hi.cpu().numpy()
        assert np.array_equal(hi - lo, oracle.window_counts(g.library.pmz, g.library.charge,
                                                             g.queries.pmz, g.queries.charge))
        # window edges fall inside 256-row blocks, except where a window is
        # clipped at its charge segment's first or last row (queries within
        # 500 Da of the precursor range's ends: 41% of the lower edges and 51%
        # of the upper ones with this seed)
        n2 = int(np.sum(g.library.charge == 2))
        starts, ends = np.array([0, n2]), np.array([n2, g.library.n])
        free_lo, free_hi = ~np.isin(lo, starts), ~np.isin(hi, ends)
        assert free_lo.mean() > 0.4 and free_hi.mean() > 0.4
        assert np.mean(lo[free_lo] % 256 != 0) > 0.95 and np.mean(hi[free_hi] % 256 != 0) > 0.95
        for kind, value in ((0, 500.0), (1, 20.0)):
            o_idx, o_dist = oracle.search(s.op, s.o_lib, g.library.pmz, g.library.charge, s.o_q,
                                          g.queries.pmz, g.queries.charge, kind, value)
            for engine in ENGINES:
                idx, dist = s.ctx.search_window(s.q_hv, s.q_pmz, s.q_ch, kind=kind, value=value,
                                                engine=engine)
                assert np.array_equal(idx.cpu().numpy(), o_idx), (kind, engine)
                assert np.array_equal(dist.cpu().numpy(), o_dist), (kind, engine)
    finally:
        s.ctx.close()


def test_exact_copies_and_duplicates(tiny):
    """Queries that copy library spectra: distance 0; a decoy shares its
    reference's pmz and charge, and exact duplicates go to the lowest index."""
    h = _h()
    g = tiny.g
    rows = np.array([0, 5, 1999, 2000, 2500, 3999])
    q = subset(g.library, rows)
    qo, qb, ql = h.preprocess(tiny.hp, q.offsets, q.mz, q.intensity)
    qhv = tiny.ctx.encode_queries(*h.to_device_csr(qo, qb, ql, "cuda:0"))
    o_q = tiny.o_lib[rows]
    for engine in ENGINES[1:]:
        i2, d2 = tiny.ctx.search_window(qhv, _dev(q.pmz), _dev(q.charge), engine=engine)
        assert np.all(d2.cpu().numpy() == 0)
    idx, dist = tiny.ctx.search_window(qhv, _dev(q.pmz), _dev(q.charge))
    o_idx, o_dist = oracle.search(tiny.op, tiny.o_lib, g.library.pmz, g.library.charge, o_q,
                                  q.pmz, q.charge)
    assert np.array_equal(idx.cpu().numpy(), o_idx)
    assert np.all(dist.cpu().numpy() == 0)


def test_edge_cases(tiny):
    """Empty windows (-1, -1): NaN precursor, a charge absent from the
    library, a precursor far outside the library range; nq = 0."""
    import torch
    qhv = tiny.q_hv[:4].contiguous()
    pmz = _dev(np.array([np.nan, 900.0, 5000.0, 900.0]))
    ch = _dev(np.array([2, 9, 2, 3], dtype=np.int8))
    for engine in ENGINES:
        idx, dist = tiny.ctx.search_window(qhv, pmz, ch, engine=engine)
        idx, dist = idx.cpu().numpy(), dist.cpu().numpy()
        assert idx[:3].tolist() == [-1, -1, -1] and dist[:3].tolist() == [-1, -1, -1]
        assert idx[3] >= 0
    e_idx, e_dist = tiny.ctx.search_window(qhv[:0], pmz[:0], ch[:0])
    assert e_idx.numel() == 0 and e_dist.numel() == 0
    torch.cuda.synchronize()


@pytest.mark.parametrize("distinct", [1, 2])
def test_custom_codebook_ties(distinct):
    """Codebooks whose position vectors take only `distinct` values and whose
    level vectors are all equal make many library vectors identical (with
    one value, every non-empty spectrum encodes to the same vector by the
    majority rule), so exact distance ties are everywhere on the device; the
    lowest library index must win each of them."""
    h = _h()
    D = 2048
    hp = h.Params(dim=D)
    op = oracle.Params(dim=D)
    rng = np.random.default_rng(1)
    f = h.num_bins(hp)
    base = rng.integers(0, 2**32, size=(distinct, D // 32), dtype=np.uint32)
    idt = base[(np.arange(f) * distinct) // f].copy()
    lvt = np.repeat(rng.integers(0, 2**32, size=(1, D // 32), dtype=np.uint32), 16, axis=0)
    g = make_workload(WORKLOADS["tiny"], n_ref=400, n_query=64, seed=5)
    with h.Context(hp) as ctx:
        ctx.set_codebook(idt, lvt)
        lo, lb, ll = h.preprocess(hp, g.library.offsets, g.library.mz, g.library.intensity)
        qo, qb, ql = h.preprocess(hp, g.queries.offsets, g.queries.mz, g.queries.intensity)
        ctx.encode_library(*h.to_device_csr(lo, lb, ll, "cuda:0"), _dev(g.library.pmz),
                           _dev(g.library.charge))
        qhv = ctx.encode_queries(*h.to_device_csr(qo, qb, ql, "cuda:0"))
        o_lib = oracle.encode(op, idt, lvt, lo, lb, ll)
        o_q = oracle.encode(op, idt, lvt, qo, qb, ql)
        assert np.array_equal(_np_u32(qhv), o_q)
        o_idx, o_dist = oracle.search(op, o_lib, g.library.pmz, g.library.charge, o_q,
                                      g.queries.pmz, g.queries.charge)
        # the codebook makes many library vectors identical: ties are real
        assert len(np.unique(o_lib, axis=0)) < len(o_lib)
        for engine in ENGINES:
            idx, dist = ctx.search_window(qhv, _dev(g.queries.pmz), _dev(g.queries.charge),
                                          engine=engine)
            assert np.array_equal(idx.cpu().numpy(), o_idx), engine
            assert np.array_equal(dist.cpu().numpy(), o_dist), engine


def test_encode_range_error_flag():
    """A bin outside [0, f) is skipped and raises the device error flag."""
    import torch
    h = _h()
    hp = h.Params(dim=512)
    with h.Context(hp) as ctx:
        off = torch.tensor([0, 2], dtype=torch.int64, device="cuda:0")
        b = torch.tensor([3, 10**7], dtype=torch.int32, device="cuda:0")
        lv = torch.tensor([1, 1], dtype=torch.uint8, device="cuda:0")
        ctx.encode_queries(off, b, lv)
        assert ctx.device_errors() & 1
        assert ctx.device_errors() == 0
        with pytest.raises(h.HomsError):
            ctx.encode_library(off, b, lv, torch.zeros(1, dtype=torch.float64, device="cuda:0"),
                               torch.zeros(1, dtype=torch.int8, device="cuda:0"))
