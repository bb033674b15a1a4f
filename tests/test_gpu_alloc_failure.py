"""Device-allocation failures (the HOMS_TEST_FAIL_ALLOC hook of dev_malloc):
a sequence of calls that allocates device memory at every step (context,
library encode, search workspace, model, library embeddings, shortlist
search, training step, library load) is run with its n-th allocation
failing, for n = 1, 2, ... until a run needs fewer than n allocations. Each
failure must surface as HOMS_E_OOM from the call that allocated, leave
every object closable, and leave the process able to run the whole
sequence again with results identical to an undisturbed run."""
import os

import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]

from synth import WORKLOADS, make_workload  # noqa: E402

HOOK = "HOMS_TEST_FAIL_ALLOC"


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.fixture(scope="module")
def data():
    import paper_2211_16422_amd.hyperoms as h
    g = make_workload(WORKLOADS["tiny"], n_ref=1500, n_query=300, seed=31)
    hp = h.Params(dim=2048)
    lib, q = g.library, g.queries
    rng = np.random.default_rng(5)
    D, H, E = 2048, 256, 64
    w = {"W1": (rng.uniform(-1, 1, (H, D)) / np.sqrt(D)).astype(np.float32),
         "b1": np.zeros(H, np.float32),
         "W2": (rng.uniform(-1, 1, (E, H)) / np.sqrt(H)).astype(np.float32),
         "b2": np.zeros(E, np.float32)}
    return {"hp": hp, "lib_csr": h.preprocess(hp, lib.offsets, lib.mz, lib.intensity),
            "q_csr": h.preprocess(hp, q.offsets, q.mz, q.intensity),
            "lib_pmz": lib.pmz, "lib_ch": lib.charge, "q_pmz": q.pmz, "q_ch": q.charge,
            "weights": w}


def _sequence(d, path):
    """Every allocating call in turn; returns the results, closes everything."""
    import torch
    import paper_2211_16422_amd.hyperoms as h
    out = {}
    ctx = model = ctx2 = None
    try:
        ctx = h.Context(d["hp"])
        ctx.encode_library(*h.to_device_csr(*d["lib_csr"], "cuda:0"), _dev(d["lib_pmz"]),
                           _dev(d["lib_ch"]))
        q_hv = ctx.encode_queries(*h.to_device_csr(*d["q_csr"], "cuda:0"))
        q_pmz, q_ch = _dev(d["q_pmz"]), _dev(d["q_ch"])
        idx, dist = ctx.search_window(q_hv, q_pmz, q_ch, h.TOL_DA, 500.0, h.ENGINE_MFMA_F4)
        out["window"] = (idx.cpu().numpy(), dist.cpu().numpy())
        model = h.Model(ctx, d["weights"])
        model.embed_library()
        li, ld, fb = model.search(q_hv, q_pmz, q_ch, 16)
        out["learned"] = (li.cpu().numpy(), ld.cpu().numpy(), fb.cpu().numpy())
        model.train_step(q_hv[:64].contiguous(), q_hv[64:128].contiguous(), 0.05, 1e-3)
        out["weights"] = {k: v.copy() for k, v in model.get_weights().items()}
        ctx.library_save(path)
        ctx2 = h.Context(d["hp"])
        ctx2.library_load(path)
        i2, d2 = ctx2.search_window(q_hv, q_pmz, q_ch, h.TOL_DA, 500.0, h.ENGINE_POPCOUNT)
        out["loaded"] = (i2.cpu().numpy(), d2.cpu().numpy())
        torch.cuda.synchronize()
        return out
    finally:
        for o in (model, ctx2, ctx):
            if o is not None:
                o.close()


def _same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        if k == "weights":
            for n in a[k]:
                assert np.array_equal(a[k][n], b[k][n]), n
        else:
            for x, y in zip(a[k], b[k]):
                assert np.array_equal(x, y), k


def test_every_allocation_failure_is_reported(data, tmp_path):
    import paper_2211_16422_amd.hyperoms as h
    os.environ.pop(HOOK, None)
    path = str(tmp_path / "lib.homs")
    ref = _sequence(data, path)
    failed = 0
    try:
        for n in range(1, 200):
            os.environ[HOOK] = f"{n}:{n}"  # a new value re-arms the count
            try:
                res = _sequence(data, path)
            except h.HomsError as e:
                assert e.status == h.HOMS_E_OOM, (n, e.status, str(e))
                failed += 1
                os.environ.pop(HOOK, None)
                _same(_sequence(data, path), ref)  # nothing left broken
                continue
            # fewer than n allocations: every one has failed once
            _same(res, ref)
            break
        else:
            pytest.fail("the sequence kept allocating")
    finally:
        os.environ.pop(HOOK, None)
    assert failed >= 10, failed  # context, library, workspace, model, embeddings, ...


def test_context_usable_after_a_failed_allocation(data, tmp_path):
    """A library load whose first device allocation fails reports HOMS_E_OOM
    and keeps the context's library: the same context searches with it, and
    the load then succeeds."""
    import paper_2211_16422_amd.hyperoms as h
    os.environ.pop(HOOK, None)
    path = str(tmp_path / "lib.homs")
    ref = _sequence(data, path)["window"]
    ctx = h.Context(data["hp"])
    try:
        ctx.encode_library(*h.to_device_csr(*data["lib_csr"], "cuda:0"), _dev(data["lib_pmz"]),
                           _dev(data["lib_ch"]))
        q_hv = ctx.encode_queries(*h.to_device_csr(*data["q_csr"], "cuda:0"))
        q_pmz, q_ch = _dev(data["q_pmz"]), _dev(data["q_ch"])
        ctx.library_save(path)
        os.environ[HOOK] = "1:load"
        try:
            with pytest.raises(h.HomsError) as e:
                ctx.library_load(path)
        finally:
            os.environ.pop(HOOK, None)
        assert e.value.status == h.HOMS_E_OOM
        for load in (False, True):
            if load:
                ctx.library_load(path)
            idx, dist = ctx.search_window(q_hv, q_pmz, q_ch, h.TOL_DA, 500.0, h.ENGINE_MFMA_F4)
            assert np.array_equal(idx.cpu().numpy(), ref[0]), load
            assert np.array_equal(dist.cpu().numpy(), ref[1]), load
    finally:
        ctx.close()
