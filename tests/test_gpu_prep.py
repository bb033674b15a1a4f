"""Device preprocessing (Section 3.2, Table 1) through the C ABI against the
oracle's: every spectrum's unique bins and levels must be identical, on the
synthetic workload and on hand-built edge cases (range boundaries, the noise
floor, intensity and m/z ties in the top-N, colliding bins, empty spectra,
spectra larger than LDS holds, and the one case that is refused); encoding from the device output equals the oracle's
encoding of the raw spectra."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not gpu_available(), reason="needs an MI355X GPU")]

import oracle  # noqa: E402
from synth import WORKLOADS, make_workload  # noqa: E402


def _h():
    import paper_2211_16422_amd.hyperoms as h
    return h


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.fixture(scope="module")
def ctx():
    h = _h()
    c = h.Context(h.Params(dim=2048))
    yield c
    c.close()


def _device(ctx, off, mz, inten, check=True):
    o, b, l = ctx.preprocess_device(_dev(np.asarray(off, dtype=np.int64)),
                                    _dev(np.asarray(mz, dtype=np.float64)),
                                    _dev(np.asarray(inten, dtype=np.float64)), check=check)
    return o.cpu().numpy(), b.cpu().numpy(), l.cpu().numpy()


def _same(got, want):
    assert np.array_equal(got[0], want[0])
    assert np.array_equal(got[1], want[1])
    assert np.array_equal(got[2], want[2])


def test_workload_spectra_match_oracle(ctx):
    g = make_workload(WORKLOADS["tiny"], n_ref=1500, n_query=700, seed=4)
    op = oracle.Params(dim=2048)
    for s in (g.library, g.queries):
        want = oracle.preprocess(s.offsets, s.mz, s.intensity, op)
        got = _device(ctx, s.offsets, s.mz, s.intensity)
        _same(got, want)
    assert ctx.device_errors() == 0


def _pack(spectra):
    off = np.zeros(len(spectra) + 1, dtype=np.int64)
    off[1:] = np.cumsum([len(m) for m, _ in spectra])
    mz = np.concatenate([np.asarray(m, dtype=np.float64) for m, _ in spectra] or [np.zeros(0)])
    inten = np.concatenate([np.asarray(i, dtype=np.float64) for _, i in spectra] or
                           [np.zeros(0)])
    return off, mz, inten


def test_edge_cases_match_oracle(ctx):
    rng = np.random.default_rng(2)
    spectra = [
        ([], []),                                              # empty
        ([50.0, 1500.0, 2000.0], [1.0, 2.0, 3.0]),             # nothing in range
        ([101.0, 1499.999999, 1500.0], [1.0, 1.0, 9.0]),       # range edges
        ([200.0, 300.0, 400.0], [100.0, 1.0, 0.99]),           # noise floor: 1.0 kept, 0.99 not
        ([500.0] * 5 + [501.0] * 3, [2.0] * 8),                # equal m/z and intensity ties
        ([600.0, 600.01, 600.02, 600.049], [4.0, 9.0, 1.0, 16.0]),  # one bin, summed in m/z order
        (list(rng.uniform(101, 1500, 60)), [5.0] * 60),        # 60 tied intensities, top 50
        ([700.0], [0.0]),                                      # a single zero-intensity peak
        (list(rng.uniform(101, 1500, 2048)), list(rng.lognormal(0, 1, 2048))),  # at the limit
    ]
    off, mz, inten = _pack(spectra)
    want = oracle.preprocess(off, mz, inten, oracle.Params(dim=2048))
    _same(_device(ctx, off, mz, inten), want)
    assert ctx.device_errors() == 0


def test_large_spectra_match_oracle(ctx):
    """Spectra with more raw peaks than the workgroup kernel holds in LDS
    (2,048): the top-N candidates are gathered by a radix select over
    (intensity desc, m/z asc, position asc) keys. Cases: kept peaks under the
    LDS size (most below the noise floor), many kept peaks with distinct
    intensities, ties of intensity across the top_n boundary (broken by m/z,
    then by position, including equal m/z), and one spectrum of 40,000 peaks;
    every one must equal the oracle."""
    rng = np.random.default_rng(3)
    n = 5000
    floor_heavy = (list(rng.uniform(101, 1500, n)),
                   [100.0] * 100 + list(rng.uniform(0.0, 0.5, n - 100)))   # 100 kept of 5000
    distinct = (list(rng.uniform(101, 1500, n)), list(rng.lognormal(0, 1, n)))
    tie_i = (list(rng.uniform(101, 1500, n)), [7.0] * 30 + [3.0] * 40 + [1.0] * (n - 70))
    mz_dup = [float(x) for x in np.round(rng.uniform(101, 1500, n), 1)]   # many equal m/z
    tie_mz = (mz_dup, [7.0] * 20 + [5.0] * 60 + [1.0] * (n - 80))
    same = ([800.0] * 3000, [2.0] * 3000)                                 # one m/z, one intensity
    out_of_range = (list(rng.uniform(1500, 2000, 2500)) + [300.0, 301.0], [1.0] * 2502)
    huge = (list(rng.uniform(101, 1500, 40000)), list(rng.lognormal(0, 1, 40000)))
    small = (list(rng.uniform(101, 1500, 30)), list(rng.lognormal(0, 1, 30)))
    spectra = [small, floor_heavy, distinct, tie_i, tie_mz, small, same, out_of_range, huge]
    off, mz, inten = _pack(spectra)
    want = oracle.preprocess(off, mz, inten, oracle.Params(dim=2048))
    _same(_device(ctx, off, mz, inten), want)
    assert ctx.device_errors() == 0


def test_too_many_kept_peaks_are_flagged():
    """With top_n above the LDS size (3,000), a spectrum keeping more than
    2,048 peaks cannot be processed: it gets no entries, device error bit 1
    is set and the binding raises; the spectra around it are unaffected, and
    a large spectrum keeping fewer peaks still matches the oracle."""
    h = _h()
    c = h.Context(h.Params(dim=2048, top_n=3000))
    try:
        rng = np.random.default_rng(4)
        small = (list(rng.uniform(101, 1500, 30)), list(rng.lognormal(0, 1, 30)))
        big = (list(rng.uniform(101, 1500, 2600)), list(rng.uniform(1.0, 2.0, 2600)))
        few = (list(rng.uniform(101, 1500, 2600)),
               [50.0] * 1000 + list(rng.uniform(0.0, 0.4, 1600)))          # 1,000 kept
        off, mz, inten = _pack([small, big, small])
        with pytest.raises(h.HomsError) as e:  # the binding reads the flag and raises
            _device(c, off, mz, inten)
        assert e.value.status == h.HOMS_E_INVALID and "2048" in str(e.value)
        o, b, l = _device(c, off, mz, inten, check=False)
        assert c.device_errors() & 2
        assert o[2] - o[1] == 0  # the oversized spectrum gets no entries
        want = oracle.preprocess(*_pack([small]), oracle.Params(dim=2048, top_n=3000))
        assert np.array_equal(b[o[0]:o[1]], want[1]) and np.array_equal(b[o[2]:o[3]], want[1])
        assert np.array_equal(l[o[0]:o[1]], want[2])
        off, mz, inten = _pack([small, few])
        want = oracle.preprocess(off, mz, inten, oracle.Params(dim=2048, top_n=3000))
        _same(_device(c, off, mz, inten), want)
        assert c.device_errors() == 0
        # no spectra at all
        o, b, l = _device(c, [0], [], [])
        assert list(o) == [0] and b.size == 0
    finally:
        c.close()


def test_encode_from_raw_on_device(ctx):
    """Raw peaks in device memory -> device preprocessing -> encoding equals the
    oracle's preprocessing and encoding of the same raw spectra."""
    g = make_workload(WORKLOADS["tiny"], n_ref=300, n_query=257, seed=8)
    q = g.queries
    o, b, l = ctx.preprocess_device(_dev(q.offsets), _dev(q.mz), _dev(q.intensity))
    hv = ctx.encode_queries(o, b, l).cpu().numpy().view(np.uint32)
    op = oracle.Params(dim=2048)
    idt, lvt = oracle.codebook(op)
    assert np.array_equal(hv, oracle.encode_raw(op, idt, lvt, q))


def test_two_pass_path_when_staging_is_too_large():
    """With top_n = 2,048 the staging area of 220,000 spectra (2,048 entries
    of 5 bytes each) would exceed its 2 GB budget, so the device takes the
    two-pass path (count, scan, write); its results must be identical too."""
    h = _h()
    c = h.Context(h.Params(dim=2048, top_n=2048))
    try:
        rng = np.random.default_rng(9)
        n = 220000
        counts = rng.integers(0, 5, n)
        off = np.zeros(n + 1, dtype=np.int64)
        off[1:] = np.cumsum(counts)
        mz = rng.uniform(90.0, 1510.0, int(off[-1]))
        inten = rng.uniform(0.0, 100.0, int(off[-1]))
        want = oracle.preprocess(off, mz, inten, oracle.Params(dim=2048, top_n=2048))
        got = _device(c, off, mz, inten)
        _same(got, want)
        assert c.device_errors() == 0
    finally:
        c.close()
