"""The encoding baselines of Section 4.2 (random position vectors; random-
projection LSH) on the GPU through the C ABI against the oracle: every
encoded bit of library and queries, and the top-1 search over them."""
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


@pytest.mark.parametrize("encoding", [1, 2])
@pytest.mark.parametrize("dim", [2048, 8192])
def test_baseline_encoding_and_search(encoding, dim):
    import paper_2211_16422_amd.hyperoms as h
    g = make_workload(WORKLOADS["tiny"], n_ref=1200, n_query=301, seed=12)
    op = oracle.Params(dim=dim, encoding=encoding)
    hp = h.Params(dim=dim, encoding=encoding)
    idt, lvt = oracle.codebook(op)
    lib, q = g.library, g.queries
    o_lib = oracle.encode_raw(op, idt, lvt, lib)
    o_q = oracle.encode_raw(op, idt, lvt, q)
    ctx = h.Context(hp)
    try:
        gi, gl = ctx.get_codebook()
        assert np.array_equal(gi, idt) and np.array_equal(gl, lvt)
        ctx.encode_library(*h.to_device_csr(*h.preprocess(hp, lib.offsets, lib.mz,
                                                          lib.intensity), "cuda:0"),
                           _dev(lib.pmz), _dev(lib.charge))
        q_hv = ctx.encode_queries(*h.to_device_csr(*h.preprocess(hp, q.offsets, q.mz,
                                                                 q.intensity), "cuda:0"))
        assert np.array_equal(q_hv.cpu().numpy().view(np.uint32), o_q)
        assert np.array_equal(ctx.library_export().cpu().numpy().view(np.uint32), o_lib)
        assert ctx.device_errors() == 0
        o_idx, o_dist = oracle.search(op, o_lib, lib.pmz, lib.charge, o_q, q.pmz, q.charge)
        for engine in (h.ENGINE_POPCOUNT, h.ENGINE_MFMA_F4):
            idx, dist = ctx.search_window(q_hv, _dev(q.pmz), _dev(q.charge), engine=engine)
            assert np.array_equal(idx.cpu().numpy(), o_idx)
            assert np.array_equal(dist.cpu().numpy(), o_dist)
    finally:
        ctx.close()


def test_lsh_encoding_of_hand_spectra():
    """Closed forms through the device: one peak gives its random row; two
    peaks of equal level give the OR of their rows (ties -> 1)."""
    import paper_2211_16422_amd.hyperoms as h
    hp = h.Params(dim=2048, encoding=2)
    ctx = h.Context(hp)
    try:
        idt, _ = ctx.get_codebook()
        off = np.array([0, 1, 3], dtype=np.int64)
        bins = np.array([17, 40, 41], dtype=np.int32)
        lv = np.array([9, 5, 5], dtype=np.uint8)
        hv = ctx.encode_queries(*h.to_device_csr(off, bins, lv, "cuda:0")).cpu().numpy()
        hv = hv.view(np.uint32)
        assert np.array_equal(hv[0], idt[17])
        assert np.array_equal(hv[1], idt[40] | idt[41])
    finally:
        ctx.close()


@pytest.mark.parametrize("encoding", [0, 2])
def test_encode_every_size_class(encoding):
    """The encode kernels run one launch per peak-count class (below 64, 64 to
    255, 256 and more, with the widest counters from 65,536 peaks for the
    paper's encoding): spectra of 0 to 70,000 entries (bins drawn with
    repeats, each entry a peak) must encode bit for bit like the oracle."""
    import paper_2211_16422_amd.hyperoms as h
    D = 2048
    hp = h.Params(dim=D, encoding=encoding)
    op = oracle.Params(dim=D, encoding=encoding)
    sizes = [0, 1, 2, 63, 64, 65, 255, 256, 257, 1000, 65535, 65536, 70000, 5, 300]
    rng = np.random.default_rng(3)
    ctx = h.Context(hp)
    try:
        idt, lvt = ctx.get_codebook()
        off = np.zeros(len(sizes) + 1, dtype=np.int64)
        off[1:] = np.cumsum(sizes)
        bins = rng.integers(0, idt.shape[0], int(off[-1])).astype(np.int32)
        lv = rng.integers(0, 16, int(off[-1])).astype(np.uint8)
        got = ctx.encode_queries(*h.to_device_csr(off, bins, lv, "cuda:0"))
        want = oracle.encode(op, idt, lvt, off, bins, lv)
        assert np.array_equal(got.cpu().numpy().view(np.uint32), want)
        assert ctx.device_errors() == 0
    finally:
        ctx.close()
