"""Parity of the batched persistent search (mixed narrow ppm / open Da
windows, charges 2-4) with the oracle, eager and through hipGraph replays,
across configurations and after autotuning."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]

import oracle  # noqa: E402
from synth import WORKLOADS, make_workload  # noqa: E402


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


class Mixed:
    """A mixed-window workload encoded by both sides from the raw spectra."""

    def __init__(self, dim=2048, n_ref=1500, n_query=600, seed=4):
        import paper_2211_16422_amd.hyperoms as h
        self.h = h
        self.g = make_workload(WORKLOADS["batched"], n_ref=n_ref, n_query=n_query, seed=seed)
        self.op = oracle.Params(dim=dim)
        self.hp = h.Params(dim=dim)
        idt, lvt = oracle.codebook(self.op)
        lib = self.g.library
        self.o_lib = oracle.encode_raw(self.op, idt, lvt, lib)
        self.idt, self.lvt = idt, lvt
        self.ctx = h.Context(self.hp)
        lo, lb, ll = h.preprocess(self.hp, lib.offsets, lib.mz, lib.intensity)
        self.ctx.encode_library(*h.to_device_csr(lo, lb, ll, "cuda:0"), _dev(lib.pmz),
                                _dev(lib.charge))

    def queries(self, raw, kinds, values):
        h = self.h
        qo, qb, ql = h.preprocess(self.hp, raw.offsets, raw.mz, raw.intensity)
        q_hv = self.ctx.encode_queries(*h.to_device_csr(qo, qb, ql, "cuda:0"))
        o_q = oracle.encode_raw(self.op, self.idt, self.lvt, raw)
        o_idx, o_dist = oracle.search(self.op, self.o_lib, self.g.library.pmz,
                                      self.g.library.charge, o_q, raw.pmz, raw.charge, kinds,
                                      values)
        return q_hv, o_idx, o_dist


@pytest.fixture(scope="module")
def mixed():
    m = Mixed()
    yield m
    m.ctx.close()


def _check(idx, dist, o_idx, o_dist):
    assert np.array_equal(idx.cpu().numpy(), o_idx)
    assert np.array_equal(dist.cpu().numpy(), o_dist)


def test_mixed_windows_have_both_classes(mixed):
    g = mixed.g
    cnt = oracle.window_counts(g.library.pmz, g.library.charge, g.queries.pmz, g.queries.charge,
                               g.tol_kind, g.tol_value)
    narrow = cnt[g.tol_kind == 1]
    wide = cnt[g.tol_kind == 0]
    assert narrow.max() < 64 and wide.min() > 64 and set(np.unique(g.queries.charge)) == {2, 3, 4}


ENGINES = [0, 2, 3]  # wide tiles by popcount, by fp8 or fp4 matrix cores


@pytest.mark.parametrize("engine", ENGINES)
@pytest.mark.parametrize("use_graph", [False, True])
def test_batched_matches_oracle(mixed, use_graph, engine):
    g = mixed.g
    before = mixed.ctx.batched_config()
    try:
        mixed.ctx.set_batched_config(engine=engine)
        q_hv, o_idx, o_dist = mixed.queries(g.queries, g.tol_kind, g.tol_value)
        idx, dist = mixed.ctx.search_batched(q_hv, _dev(g.queries.pmz), _dev(g.queries.charge),
                                             _dev(g.tol_kind), _dev(g.tol_value),
                                             use_graph=use_graph)
        _check(idx, dist, o_idx, o_dist)
    finally:
        mixed.ctx.set_batched_config(**before)


@pytest.mark.parametrize("cfg", [
    dict(narrow_max=0),                      # everything tiled
    dict(narrow_max=1 << 30),                # everything per query
    dict(chunk_rows=64, grid=3),             # many small items, few workgroups
    dict(grid=1, narrow_group=4),            # one persistent workgroup drains the queue
    dict(bucket_da=1e-3, chunk_rows=100000),
])
@pytest.mark.parametrize("engine", ENGINES)
def test_batched_configurations(mixed, cfg, engine):
    g = mixed.g
    before = mixed.ctx.batched_config()
    try:
        mixed.ctx.set_batched_config(engine=engine, **cfg)
        q_hv, o_idx, o_dist = mixed.queries(g.queries, g.tol_kind, g.tol_value)
        idx, dist = mixed.ctx.search_batched(q_hv, _dev(g.queries.pmz), _dev(g.queries.charge),
                                             _dev(g.tol_kind), _dev(g.tol_value),
                                             use_graph=False)
        _check(idx, dist, o_idx, o_dist)
    finally:
        mixed.ctx.set_batched_config(**before)


def test_graph_replays_with_new_batches(mixed):
    """One captured graph replayed on three different batches written into the
    same buffers, with eager work in between; every replay is checked."""
    import torch
    import paper_2211_16422_amd.hyperoms as h
    g = mixed.g
    n = g.queries.n
    bufs = None
    for rep, seed in enumerate([11, 12, 13]):
        other = make_workload(WORKLOADS["batched"], n_ref=1500, n_query=n, seed=4)
        # same library (seed 4), fresh queries drawn from the generator's query stream
        rng = np.random.default_rng(seed)
        from synth.spectra import make_queries, make_references
        refs = make_references(1500, np.random.default_rng(
            np.random.SeedSequence(4).spawn(5)[0]), charges=(2, 3, 4))
        raw = make_queries(refs, n, rng)
        kinds = (rng.random(n) < 0.7).astype(np.int8)
        values = np.where(kinds == 1, 20.0, 500.0)
        assert np.array_equal(other.library.pmz[:1500], refs.pmz)
        q_hv, o_idx, o_dist = mixed.queries(raw, kinds, values)
        if bufs is None:
            bufs = dict(q_hv=q_hv.clone(), pmz=_dev(raw.pmz), ch=_dev(raw.charge),
                        k=_dev(kinds), v=_dev(values),
                        idx=torch.empty(n, dtype=torch.int64, device="cuda:0"),
                        dist=torch.empty(n, dtype=torch.int32, device="cuda:0"))
        else:
            bufs["q_hv"].copy_(q_hv)
            bufs["pmz"].copy_(_dev(raw.pmz))
            bufs["ch"].copy_(_dev(raw.charge))
            bufs["k"].copy_(_dev(kinds))
            bufs["v"].copy_(_dev(values))
        torch.cuda.synchronize()
        # eager work on the same stream between replays
        e_idx, e_dist = mixed.ctx.search_window(bufs["q_hv"], bufs["pmz"], bufs["ch"],
                                                engine=h.ENGINE_POPCOUNT)
        mixed.ctx.search_batched(bufs["q_hv"], bufs["pmz"], bufs["ch"], bufs["k"], bufs["v"],
                                 use_graph=True, out_idx=bufs["idx"], out_dist=bufs["dist"])
        torch.cuda.synchronize()
        _check(bufs["idx"], bufs["dist"], o_idx, o_dist)
        assert e_idx.numel() == n


def test_autotune_keeps_results(mixed):
    g = mixed.g
    q_hv, o_idx, o_dist = mixed.queries(g.queries, g.tol_kind, g.tol_value)
    args = (q_hv, _dev(g.queries.pmz), _dev(g.queries.charge), _dev(g.tol_kind),
            _dev(g.tol_value))
    best, ms = mixed.ctx.autotune_batched(*args, reps=1)
    assert ms > 0 and best == mixed.ctx.batched_config()
    idx, dist = mixed.ctx.search_batched(*args, use_graph=True)
    _check(idx, dist, o_idx, o_dist)


def test_batched_empty_and_degenerate(mixed):
    import torch
    g = mixed.g
    q_hv, _, _ = mixed.queries(g.queries, g.tol_kind, g.tol_value)
    k = _dev(np.zeros(4, dtype=np.int8))
    v = _dev(np.array([500.0, 500.0, 0.0, 500.0]))
    pmz = _dev(np.array([np.nan, 5000.0, 777.0, 900.0]))
    ch = _dev(np.array([2, 2, 3, 9], dtype=np.int8))
    idx, dist = mixed.ctx.search_batched(q_hv[:4].contiguous(), pmz, ch, k, v, use_graph=False)
    assert idx.cpu().tolist() == [-1, -1, -1, -1] and dist.cpu().tolist() == [-1, -1, -1, -1]
    e_idx, _ = mixed.ctx.search_batched(q_hv[:0], pmz[:0], ch[:0], k[:0], v[:0])
    assert e_idx.numel() == 0
    torch.cuda.synchronize()
