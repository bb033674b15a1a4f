"""Library and model files on the GPU (Sections 3.2-3.3: encoded reference
hypervectors are kept and reused): a library saved and loaded into a fresh
context gives the same rows, the same order and search results identical to
the freshly encoded one; files of other parameters or another codebook, or
damaged files, are refused and leave the context's library as it was; a saved
and loaded model carries its weights and its optimiser state."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]

from synth import WORKLOADS, make_workload  # noqa: E402
from test_persist_cpu import checksum  # noqa: E402


def _h():
    import paper_2211_16422_amd.hyperoms as h
    return h


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.fixture(scope="module")
def encoded():
    h = _h()
    g = make_workload(WORKLOADS["tiny"], n_ref=3000, n_query=300, seed=4)
    hp = h.Params(dim=2048)
    ctx = h.Context(hp)
    lib, q = g.library, g.queries
    ctx.encode_library(*h.to_device_csr(*h.preprocess(hp, lib.offsets, lib.mz, lib.intensity),
                                        "cuda:0"), _dev(lib.pmz), _dev(lib.charge))
    q_hv = ctx.encode_queries(*h.to_device_csr(*h.preprocess(hp, q.offsets, q.mz, q.intensity),
                                               "cuda:0"))
    yield h, hp, g, ctx, q_hv
    ctx.close()


def test_library_round_trip(encoded, tmp_path):
    h, hp, g, ctx, q_hv = encoded
    path = str(tmp_path / "lib.homs")
    ctx.library_save(path)
    info = h.file_info(path)
    idt, lvt = h.generate_codebook(hp)
    assert info["n"] == g.library.n and info["dim"] == 2048
    assert info["codebook_hash"] == checksum(idt.tobytes() + lvt.tobytes())
    q_pmz, q_ch = _dev(g.queries.pmz), _dev(g.queries.charge)
    with h.Context(hp) as c2:
        c2.library_load(path)
        assert c2.library_size() == g.library.n
        assert np.array_equal(c2.library_export().cpu().numpy(),
                              ctx.library_export().cpu().numpy())
        assert np.array_equal(c2.library_order().cpu().numpy(),
                              ctx.library_order().cpu().numpy())
        for kind, value in ((0, 500.0), (1, 20.0)):
            for engine in (h.ENGINE_POPCOUNT, h.ENGINE_MFMA_F4):
                a = ctx.search_window(q_hv, q_pmz, q_ch, kind, value, engine)
                b = c2.search_window(q_hv, q_pmz, q_ch, kind, value, engine)
                assert all(np.array_equal(x.cpu().numpy(), y.cpu().numpy())
                           for x, y in zip(a, b)), (kind, engine)


def test_foreign_or_damaged_library_is_refused(encoded, tmp_path):
    h, hp, g, ctx, q_hv = encoded
    path = str(tmp_path / "lib.homs")
    ctx.library_save(path)
    q_pmz, q_ch = _dev(g.queries.pmz), _dev(g.queries.charge)
    want = [t.cpu().numpy() for t in ctx.search_window(q_hv, q_pmz, q_ch)]
    with h.Context(h.Params(dim=2048, seed=1)) as other:
        with pytest.raises(h.HomsError) as e:
            other.library_load(path)
        assert e.value.status == h.HOMS_E_INVALID
    with h.Context(hp) as custom:
        idt, lvt = custom.get_codebook()
        idt[5, 0] ^= 1
        custom.set_codebook(idt, None)
        with pytest.raises(h.HomsError):
            custom.library_load(path)
    data = bytearray(open(path, "rb").read())
    data[-100] ^= 0x01
    bad = str(tmp_path / "bad.homs")
    open(bad, "wb").write(bytes(data))
    with pytest.raises(h.HomsError):
        ctx.library_load(bad)
    got = [t.cpu().numpy() for t in ctx.search_window(q_hv, q_pmz, q_ch)]
    assert all(np.array_equal(a, b) for a, b in zip(got, want))


def test_model_round_trip(encoded, tmp_path):
    import torch
    h, hp, g, ctx, q_hv = encoded
    rng = np.random.default_rng(3)
    D, H, E = 2048, 128, 64
    w = {"W1": (rng.uniform(-1, 1, (H, D)) / np.sqrt(D)).astype(np.float32),
         "b1": np.zeros(H, np.float32),
         "W2": (rng.uniform(-1, 1, (E, H)) / np.sqrt(H)).astype(np.float32),
         "b2": np.zeros(E, np.float32)}
    m = h.Model(ctx, w)
    qa, qb = q_hv[:64].contiguous(), q_hv[64:128].contiguous()
    for _ in range(3):
        m.train_step(qa, qb, 0.05, 1e-3)
    path = str(tmp_path / "m.homs")
    m.save(path)
    info = h.file_info(path)
    assert (info["hidden"], info["embed"], info["step"]) == (H, E, 3)
    m2 = h.Model.load(ctx, path)
    w1, w2 = m.get_weights(), m2.get_weights()
    assert all(np.array_equal(w1[k], w2[k]) for k in w1)
    # the optimiser state came along: one more identical step stays identical
    m.train_step(qa, qb, 0.05, 1e-3)
    m2.train_step(qa, qb, 0.05, 1e-3)
    torch.cuda.synchronize()
    w1, w2 = m.get_weights(), m2.get_weights()
    assert all(np.array_equal(w1[k].view(np.uint32), w2[k].view(np.uint32)) for k in w1)
    e1 = m.embed(q_hv[:50].contiguous()).cpu().numpy()
    e2 = m2.embed(q_hv[:50].contiguous()).cpu().numpy()
    assert np.array_equal(e1, e2)
    m.close()
    m2.close()
