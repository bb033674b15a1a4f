"""homs_search_window_noalloc (scratch in the library's static device array,
no allocation) against homs_search_window on the same inputs: identical
indices and distances, on two calls in a row, the second with fewer queries
(the array keeps the first call's contents), for every engine; and the query
limit refused with HOMS_E_INVALID before anything runs."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]

from synth import WORKLOADS, make_workload  # noqa: E402


def _h():
    import paper_2211_16422_amd.hyperoms as h
    return h


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.fixture(scope="module")
def setup():
    h = _h()
    g = make_workload(WORKLOADS["tiny"], n_ref=3000, n_query=1500, seed=23)
    ctx = h.Context(h.Params(dim=2048))
    lib, q = g.library, g.queries
    hp = ctx.params
    lo, lb, ll = h.preprocess(hp, lib.offsets, lib.mz, lib.intensity)
    qo, qb, ql = h.preprocess(hp, q.offsets, q.mz, q.intensity)
    ctx.encode_library(*h.to_device_csr(lo, lb, ll, "cuda:0"), _dev(lib.pmz), _dev(lib.charge))
    q_hv = ctx.encode_queries(*h.to_device_csr(qo, qb, ql, "cuda:0"))
    yield ctx, q_hv, _dev(q.pmz), _dev(q.charge)
    ctx.close()


@pytest.mark.parametrize("engine", ["ENGINE_POPCOUNT", "ENGINE_MFMA_I8", "ENGINE_MFMA_F8",
                                    "ENGINE_MFMA_F4"])
def test_noalloc_equals_search_window(setup, engine):
    import torch
    h = _h()
    ctx, q_hv, q_pmz, q_ch = setup
    eng = getattr(h, engine)
    # call 1: every query, +-500 Da; call 2: a shuffled subset of 417, 20 ppm
    # and then +-500 Da again, so a window of the first call's size follows
    # the smaller one in the same array
    sub = torch.from_numpy(np.random.default_rng(4).permutation(q_pmz.shape[0])[:417]).to("cuda:0")
    cases = [(q_hv, q_pmz, q_ch, h.TOL_DA, 500.0),
             (q_hv[sub].contiguous(), q_pmz[sub].contiguous(), q_ch[sub].contiguous(),
              h.TOL_PPM, 20.0),
             (q_hv[sub].contiguous(), q_pmz[sub].contiguous(), q_ch[sub].contiguous(),
              h.TOL_DA, 500.0)]
    for hv, pmz, ch, kind, value in cases:
        n = pmz.shape[0]
        want_idx, want_dist = ctx.search_window(hv, pmz, ch, kind, value, eng)
        # outputs start as garbage so that nothing is left over by chance
        got_idx = torch.full((n,), 12345, dtype=torch.int64, device="cuda:0")
        got_dist = torch.full((n,), 777, dtype=torch.int32, device="cuda:0")
        ctx.search_window_noalloc(hv, pmz, ch, got_idx, got_dist, kind, value, eng)
        torch.cuda.synchronize()
        assert np.array_equal(got_idx.cpu().numpy(), want_idx.cpu().numpy()), (engine, n, kind)
        assert np.array_equal(got_dist.cpu().numpy(), want_dist.cpu().numpy()), (engine, n, kind)
        assert (want_idx.cpu().numpy() >= 0).mean() > 0.5


def test_noalloc_limit_refused(setup):
    import torch
    h = _h()
    ctx, q_hv, q_pmz, q_ch = setup
    n = h.NOALLOC_MAX_QUERIES + 1
    hv = torch.zeros((n, ctx.words), dtype=torch.int32, device="cuda:0")
    pmz = torch.full((n,), 700.0, dtype=torch.float64, device="cuda:0")
    ch = torch.full((n,), 2, dtype=torch.int8, device="cuda:0")
    idx = torch.empty(n, dtype=torch.int64, device="cuda:0")
    dist = torch.empty(n, dtype=torch.int32, device="cuda:0")
    with pytest.raises(h.HomsError) as e:
        ctx.search_window_noalloc(hv, pmz, ch, idx, dist)
    assert e.value.status == h.HOMS_E_INVALID
    assert "at most" in str(e.value)
    # the context still works afterwards
    a, b = ctx.search_window(q_hv[:64].contiguous(), q_pmz[:64].contiguous(),
                             q_ch[:64].contiguous())
    c = torch.empty_like(a)
    d = torch.empty_like(b)
    ctx.search_window_noalloc(q_hv[:64].contiguous(), q_pmz[:64].contiguous(),
                              q_ch[:64].contiguous(), c, d)
    torch.cuda.synchronize()
    assert torch.equal(a, c) and torch.equal(b, d)
