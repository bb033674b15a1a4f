"""The library order of Section 3.4's candidate filter, produced by the
library's own radix sort: rows by (charge, precursor m/z, library index), so
that every candidate set is one run of rows. Checked element by element
against numpy's stable lexsort, with many exact ties (rounded precursors,
decoys sharing their reference's precursor), -0.0 beside +0.0 (equal, so
ordered by library index), NaN precursors of different payloads (all after
+inf, by library index), signed charges, and sizes around the sort's
4,096-element tiles."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]


def _encode_without_peaks(ctx, pmz, charge):
    import torch
    n = pmz.shape[0]
    dev = ctx.device
    off = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    bins = torch.zeros(1, dtype=torch.int32, device=dev)
    lv = torch.zeros(1, dtype=torch.uint8, device=dev)
    ctx.encode_library(off, bins, lv, torch.from_numpy(pmz).to(dev),
                       torch.from_numpy(charge).to(dev))


@pytest.mark.parametrize("charge_match", [True, False])
@pytest.mark.parametrize("n", [1, 255, 4096, 4097, 70_001, 300_000])
def test_library_order(n, charge_match):
    import paper_2211_16422_amd.hyperoms as h
    rng = np.random.default_rng(n)
    pmz = np.round(rng.uniform(-50.0, 1500.0, n), 1)  # about 15,500 distinct values
    pmz[rng.random(n) < 0.001] = np.nan
    pmz[3::97] = 0.0
    pmz[7::89] = -0.0
    nan2 = np.array([0x7FF4000000000001, 0xFFF8000000000000], np.uint64).view(np.float64)
    pmz[11::131] = nan2[0]
    pmz[13::127] = nan2[1]
    charge = rng.integers(-3, 6, n).astype(np.int8)
    idx = np.arange(n)
    with h.Context(h.Params(dim=512, charge_match=charge_match)) as ctx:
        _encode_without_peaks(ctx, pmz, charge)
        order = ctx.library_order().cpu().numpy().view(np.uint32)
    want = np.lexsort((idx, pmz, charge)) if charge_match else np.lexsort((idx, pmz))
    assert np.array_equal(order.astype(np.int64), want)


def test_library_order_of_a_workload():
    """References then decoys: every decoy shares its reference's precursor
    and charge, so each pair is an exact tie resolved by library index."""
    import paper_2211_16422_amd.hyperoms as h
    from synth import WORKLOADS, make_workload
    g = make_workload(WORKLOADS["tiny"], n_ref=9000, n_query=1, seed=5)
    lib = g.library
    with h.Context(h.Params(dim=512)) as ctx:
        _encode_without_peaks(ctx, lib.pmz, lib.charge)
        order = ctx.library_order().cpu().numpy().view(np.uint32)
    want = np.lexsort((np.arange(lib.n), lib.pmz, lib.charge))
    assert np.array_equal(order.astype(np.int64), want)
