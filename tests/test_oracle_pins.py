"""Pins of the oracle against facts fixed by the paper or by mathematics.

Each test checks the oracle against something other than itself: published
RNG outputs, closed forms of the codebook construction (Sections 3.3.1 and
3.3.2), closed forms of the majority rule (Section 3.3, Eq. 1 and its
binarisation), hand-derived preprocessing results (Section 3.2; Table 1),
identities of the Hamming distance (Section 3.4), brute force on tiny inputs
and planted recovery. None of these needs a GPU.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
from synth import WORKLOADS, make_workload


def bits_of(hv_row: np.ndarray, D: int) -> np.ndarray:
    """Unpack a packed row into its D bits (bit d = word d//32, bit d%32)."""
    return np.unpackbits(hv_row.view(np.uint8), bitorder="little")[:D]


def popcount_rows(x: np.ndarray) -> np.ndarray:
    return np.bitwise_count(x).sum(axis=-1)


# ---------------------------------------------------------------- SplitMix64

def test_splitmix64_published_outputs(golden_dir):
    rows = []
    with open(os.path.join(golden_dir, "splitmix64.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                s, i, v = line.split()
                rows.append((int(s), int(i), int(v)))
    for seed in {r[0] for r in rows}:
        want = [(i, v) for s, i, v in rows if s == seed]
        got = oracle.splitmix64(seed, max(i for i, _ in want) + 1)
        for i, v in want:
            assert int(got[i]) == v, (seed, i)


# ------------------------------------------------------------------ codebook

@pytest.mark.parametrize("D,f,Q,alpha", [(256, 128, 16, 128), (2048, 300, 16, 1024),
                                         (512, 50, 8, 100)])
def test_codebook_closed_forms(D, f, Q, alpha):
    """H(F_i, F_j) = |k_i - k_j| with k_i = floor(alpha*i/(f-1)); likewise for
    levels with m_j = floor((D/2) j/(Q-1)) (Sections 3.3.1 and 3.3.2). The
    scaled-down (D=256, f=128) case is the one of Fig. 3(b)."""
    p = oracle.Params(dim=D, n_levels=Q, mz_min=0.0, mz_max=f / 20.0, bins_per_da=20.0,
                      id_flips=alpha, seed=7)
    assert oracle.num_bins(p) == f
    idt, lvt = oracle.codebook(p)
    k = (alpha * np.arange(f, dtype=np.int64)) // (f - 1)
    H = popcount_rows(idt[:, None, :] ^ idt[None, :, :])
    assert np.array_equal(H, np.abs(k[:, None] - k[None, :]))
    assert H[0, f - 1] == alpha
    m = ((D // 2) * np.arange(Q, dtype=np.int64)) // (Q - 1)
    HL = popcount_rows(lvt[:, None, :] ^ lvt[None, :, :])
    assert np.array_equal(HL, np.abs(m[:, None] - m[None, :]))
    assert HL[0, Q - 1] == D // 2
    # similarity to F_0 never increases along the bins (Section 3.3.1)
    assert np.all(np.diff(H[0]) >= 0)
    # the flipped sets are nested: F_i agrees with F_0 wherever F_{f-1} does
    outside = ~(idt[0] ^ idt[f - 1])
    assert np.all(((idt ^ idt[0]) & outside) == 0)


def test_codebook_base_vector_is_rng_bits():
    """F_0 is the first D/64 SplitMix64 outputs, bit d from output d//64."""
    D = 512
    p = oracle.Params(dim=D, mz_min=0.0, mz_max=1.0, bins_per_da=20.0, seed=12345)
    idt, _ = oracle.codebook(p)
    words = oracle.splitmix64(12345, D // 64)
    want = np.concatenate([[(int(w) >> b) & 1 for b in range(64)] for w in words])
    assert np.array_equal(bits_of(idt[0], D), want.astype(np.uint8))


def test_codebook_full_size_endpoints():
    """Table 1 bins (0.05 Da over [101, 1500]) give f = 27,980; alpha = D/2
    (Section 4.2) puts F_0 and F_{f-1} exactly D/2 apart."""
    p = oracle.Params(dim=2048)
    assert oracle.num_bins(p) == 27980
    assert oracle.num_bins(oracle.Params(dim=2048, bins_per_da=25.0)) == 34975
    idt, lvt = oracle.codebook(p)
    assert popcount_rows(idt[0] ^ idt[-1]) == 1024
    i = np.array([0, 1, 7, 13999, 20000, 27979])
    k = (1024 * i) // 27979
    H = popcount_rows(idt[i][:, None] ^ idt[i][None, :])
    assert np.array_equal(H, np.abs(k[:, None] - k[None, :]))


# -------------------------------------------------------------------- encode

def _encode_peaks(D, idt, lvt, peaks):
    off = np.array([0, len(peaks)], dtype=np.int64)
    b = np.array([p[0] for p in peaks], dtype=np.int32)
    lv = np.array([p[1] for p in peaks], dtype=np.uint8)
    return oracle.encode(oracle.Params(dim=D), idt, lvt, off, b, lv)[0]


@pytest.fixture(scope="module")
def small_tables():
    rng = np.random.default_rng(3)
    D = 256
    idt = rng.integers(0, 2**32, size=(40, D // 32), dtype=np.uint32)
    lvt = rng.integers(0, 2**32, size=(16, D // 32), dtype=np.uint32)
    return D, idt, lvt


def test_encode_single_peak_is_bound_vector(small_tables):
    """Majority of one vector is that vector: I = F_i (*) L_j, i.e. XOR."""
    D, idt, lvt = small_tables
    for b, l in [(0, 0), (5, 3), (39, 15)]:
        assert np.array_equal(_encode_peaks(D, idt, lvt, [(b, l)]), idt[b] ^ lvt[l])


def test_encode_closed_forms_2_3_4(small_tables):
    """Binarisation maps a zero sum to -1 (bit 1): two peaks give the OR of
    their bits, three the bitwise majority, four 'at least two of four'."""
    D, idt, lvt = small_tables
    v = [idt[b] ^ lvt[l] for b, l in [(1, 2), (7, 9), (11, 0), (30, 15)]]
    assert np.array_equal(_encode_peaks(D, idt, lvt, [(1, 2), (7, 9)]), v[0] | v[1])
    maj = (v[0] & v[1]) | (v[0] & v[2]) | (v[1] & v[2])
    assert np.array_equal(_encode_peaks(D, idt, lvt, [(1, 2), (7, 9), (11, 0)]), maj)
    two_of_four = np.zeros_like(v[0])
    for a, b in itertools.combinations(range(4), 2):
        two_of_four |= v[a] & v[b]
    got = _encode_peaks(D, idt, lvt, [(1, 2), (7, 9), (11, 0), (30, 15)])
    assert np.array_equal(got, two_of_four)


def test_encode_tie_rules(small_tables):
    """{v, v, w} -> v and {v, not v} -> all ones (zero sums become -1)."""
    D, idt, lvt = small_tables
    idt = idt.copy()
    v = idt[2] ^ lvt[4]
    idt[3] = v ^ lvt[6]            # peak (3, 6) binds to v as well
    idt[4] = ~v ^ lvt[1]           # peak (4, 1) binds to the complement of v
    w = idt[9] ^ lvt[0]
    assert np.array_equal(_encode_peaks(D, idt, lvt, [(2, 4), (3, 6), (9, 0)]), v)
    assert not np.array_equal(v, w)
    ones = np.full(D // 32, 0xFFFFFFFF, dtype=np.uint32)
    assert np.array_equal(_encode_peaks(D, idt, lvt, [(2, 4), (4, 1)]), ones)
    assert np.array_equal(_encode_peaks(D, idt, lvt, []), ones)


def test_encode_peak_order_and_bipolar_sum(small_tables):
    """Eq. 1 is a sum, so peak order does not matter; the sign of the bipolar
    sum computed with a matrix product gives the same bits."""
    D, idt, lvt = small_tables
    rng = np.random.default_rng(11)
    for n in [5, 6, 17, 40]:
        bins = rng.choice(40, size=n, replace=False)
        lv = rng.integers(0, 16, size=n)
        peaks = list(zip(bins.tolist(), lv.tolist()))
        a = _encode_peaks(D, idt, lvt, peaks)
        rng.shuffle(peaks)
        assert np.array_equal(a, _encode_peaks(D, idt, lvt, peaks))
        X = np.stack([1 - 2 * bits_of(idt[b] ^ lvt[l], D).astype(np.int64) for b, l in peaks])
        I = np.ones(n, dtype=np.int64) @ X
        want = np.packbits((I <= 0).astype(np.uint8), bitorder="little").view(np.uint32)
        assert np.array_equal(a, want)


# ---------------------------------------------------------------- preprocess

def _pre(spectra, **kw):
    p = oracle.Params(**kw)
    off = [0]
    mz, it = [], []
    for s in spectra:
        mz += [x[0] for x in s]
        it += [x[1] for x in s]
        off.append(len(mz))
    o, b, l = oracle.preprocess(np.array(off), np.array(mz, dtype=np.float64),
                                np.array(it, dtype=np.float64), p)
    return [list(zip(b[o[i]:o[i + 1]].tolist(), l[o[i]:o[i + 1]].tolist()))
            for i in range(len(spectra))]


def test_preprocess_hand_case():
    """Table 1 range [101, 1500) with 0.05 Da bins, the 1% noise rule, sqrt
    scaling, summing of colliding peaks and 16 levels (Section 3.2):
      100.99 and 1500.0 are outside the range; 800.0 (0.48 < 1% of 49) is
      noise; 101.0 and 101.04 share bin 0 -> sqrt16 + sqrt9 = 7; 1499.99 is
      bin 27979 -> 7; 700.0 is bin 11980 -> sqrt(0.5) = 0.7071...;
      levels: 7/7 -> 16 -> clamped to 15; 0.7071/7 * 16 = 1.616 -> 1."""
    got = _pre([[(100.99, 100.0), (101.0, 16.0), (101.04, 9.0), (1499.99, 49.0),
                 (1500.0, 1000.0), (700.0, 0.5), (800.0, 0.48)]])
    assert got == [[(0, 15), (11980, 1), (27979, 15)]]


def test_preprocess_top_n_ties_and_levels():
    """top_n keeps the most intense peaks, ties to the lower m/z; half of the
    largest value lands exactly on level 8 of 16."""
    got = _pre([[(300.0, 5.0), (200.0, 5.0), (400.0, 5.0)]], top_n=2)
    assert got == [[(1980, 15), (3980, 15)]]
    got = _pre([[(200.0, 16.0), (300.0, 4.0)]])
    assert got == [[(1980, 15), (3980, 8)]]
    # no noise rule: a bin at 1/32 of the largest value falls to level 0
    got = _pre([[(200.0, 1024.0), (300.0, 1.0)]], noise_frac=0.0)
    assert got == [[(1980, 15), (3980, 0)]]


def test_preprocess_empty_and_out_of_range():
    got = _pre([[], [(50.0, 3.0), (2000.0, 4.0)], [(101.0, 2.0)]])
    assert got == [[], [], [(0, 15)]]


def test_preprocess_bin_width_004():
    """Large-scale setting of Table 1: 0.04 Da bins (25 bins per Da)."""
    got = _pre([[(101.0, 1.0), (101.039, 1.0), (101.041, 1.0), (1499.999, 1.0)]],
               bins_per_da=25.0)
    # 101.039 -> 0.975 -> bin 0, summed with 101.0 -> 2; 101.041 -> bin 1
    # -> 1; 1499.999 -> 34974.975 -> bin 34974 -> 1; levels 16 -> 15, 8, 8
    assert got == [[(0, 15), (1, 8), (34974, 8)]]


def test_preprocess_invariants_on_workload():
    g = make_workload(WORKLOADS["tiny"], n_ref=300, n_query=50)
    p = oracle.Params(dim=2048)
    for raw in (g.library, g.queries):
        off, b, lv = oracle.preprocess(raw.offsets, raw.mz, raw.intensity, p)
        for i in range(raw.n):
            bb, ll = b[off[i]:off[i + 1]], lv[off[i]:off[i + 1]]
            assert len(bb) <= p.top_n
            assert np.all(np.diff(bb) > 0)
            assert np.all((bb >= 0) & (bb < 27980)) and np.all(ll < 16)
            if len(bb):
                assert ll.max() == 15


# ------------------------------------------------------------ distance/search

def _rand_hv(rng, n, D):
    return rng.integers(0, 2**32, size=(n, D // 32), dtype=np.uint32)


def test_hamming_identities():
    """H(x,x)=0, symmetry, H(x, not x)=D, triangle inequality and
    H = (D - <x, y>)/2 for the bipolar forms (Section 3.4)."""
    rng = np.random.default_rng(5)
    D = 512
    X = _rand_hv(rng, 24, D)
    X[3] = ~X[2]
    p = oracle.Params(dim=D)
    z = np.zeros(24)
    c = np.full(24, 2, dtype=np.int8)
    off, idx, dist = oracle.window_distances(p, X, z, c, X, z, c, values=1.0)
    assert np.array_equal(np.diff(off), np.full(24, 24))
    H = dist.reshape(24, 24)
    assert np.array_equal(idx.reshape(24, 24), np.tile(np.arange(24), (24, 1)))
    assert np.all(np.diag(H) == 0)
    assert np.array_equal(H, H.T)
    assert H[2, 3] == D
    assert np.all(H[:, :, None] <= H[:, None, :] + H.T[None, :, :])
    B = np.stack([1 - 2 * bits_of(x, D).astype(np.int64) for x in X])
    assert np.array_equal(H, (D - B @ B.T) // 2)
    assert np.array_equal(H, np.bitwise_count(X[:, None] ^ X[None, :]).sum(-1))


def test_search_brute_force_tiny():
    """Top-1 against a pure-Python brute force: same charge, |dm| <= tol,
    smallest distance, lowest index on ties; (-1, -1) if no candidate."""
    rng = np.random.default_rng(9)
    D = 128
    nl, nq = 60, 40
    lib = _rand_hv(rng, nl, D)
    lib[10] = lib[11]  # exact duplicates: the lower index must win
    lib[25] = lib[11]
    q = _rand_hv(rng, nq, D)
    q[0] = lib[11]
    lp = rng.uniform(400, 420, nl)
    lc = rng.integers(2, 4, nl).astype(np.int8)
    qp = rng.uniform(395, 425, nq)
    qc = rng.integers(2, 4, nq).astype(np.int8)
    qp[0], qc[0] = lp[11], lc[11]
    lp[10], lc[10] = lp[11], lc[11]
    lp[25], lc[25] = lp[11], lc[11]
    qp[1] = 1000.0  # no candidate
    kinds = rng.integers(0, 2, nq)
    vals = np.where(kinds == 0, 3.0, 5000.0)
    idx, dist = oracle.search(oracle.Params(dim=D), lib, lp, lc, q, qp, qc, kinds, vals)
    for i in range(nq):
        tol = vals[i] if kinds[i] == 0 else (qp[i] * vals[i]) / 1e6
        best = (-1, -1)
        for r in range(nl):
            if lc[r] != qc[i] or not (qp[i] - tol <= lp[r] <= qp[i] + tol):
                continue
            h = sum(bin(int(a) ^ int(b)).count("1") for a, b in zip(q[i], lib[r]))
            if best[0] < 0 or h < best[1]:
                best = (r, h)
        assert (idx[i], dist[i]) == best, i
    assert (idx[0], dist[0]) == (10, 0)
    assert (idx[1], dist[1]) == (-1, -1)


def test_window_boundaries():
    """Candidates satisfy pmz_q - tol <= pmz_r <= pmz_q + tol with the same
    charge (Section 3.4); ppm tolerance is pmz_q * ppm / 1e6."""
    lp = np.array([400.0, 1400.0, np.nextafter(1400.0, 2000.0), 900.0, 900.0])
    lc = np.array([2, 2, 2, 3, 2], dtype=np.int8)
    qp = np.array([900.0, 900.0, 1000.0])
    qc = np.array([2, 2, 2], dtype=np.int8)
    kinds = np.array([0, 1, 1])
    vals = np.array([500.0, 20.0, 20.0])
    cnt = oracle.window_counts(lp, lc, qp, qc, kinds, vals)
    # q0 (+-500 Da): 400 and 1400 exactly on the edges, next-after 1400 out,
    # charge-3 excluded, 900 in -> 3; q1 (20 ppm of 900 = 0.018 Da): 900 only
    assert cnt.tolist() == [3, 1, 0]
    cnt = oracle.window_counts(lp, lc, qp, qc, kinds, vals, charge_match=False)
    assert cnt.tolist() == [4, 2, 0]


def test_planted_recovery():
    """Random 2048-bit codewords are >= ~900 bits apart; a query made from a
    codeword with t = 100 flipped bits is closer to it than to any other one
    (triangle inequality), so top-1 must return its source."""
    rng = np.random.default_rng(21)
    D, nl, nq, t = 2048, 500, 200, 100
    lib = _rand_hv(rng, nl, D)
    Hmin = min(int(np.bitwise_count(lib[i] ^ lib[j]).sum())
               for i in range(50) for j in range(i + 1, nl))
    assert Hmin > 2 * t
    src = rng.integers(0, nl, nq)
    q = lib[src].copy()
    for i in range(nq):
        for d in rng.choice(D, size=t, replace=False):
            q[i, d // 32] ^= np.uint32(1 << (d % 32))
    z = np.zeros(nl)
    c = np.full(nl, 2, dtype=np.int8)
    idx, dist = oracle.search(oracle.Params(dim=D), lib, z, c, q, np.zeros(nq),
                              np.full(nq, 2, dtype=np.int8))
    assert np.array_equal(idx, src)
    assert np.all(dist == t)


def test_spectrum_level_exact_copies():
    """Queries that are exact copies of library spectra encode identically, so
    they sit at distance 0 from their source (or a lower-index duplicate)."""
    g = make_workload(WORKLOADS["tiny"], n_ref=200, n_query=10)
    p = oracle.Params(dim=2048)
    idt, lvt = oracle.codebook(p)
    lib_hv = oracle.encode_raw(p, idt, lvt, g.library)
    rows = np.array([3, 77, 150, 199, 250])
    from synth import subset
    q = subset(g.library, rows)
    q_hv = oracle.encode_raw(p, idt, lvt, q)
    idx, dist = oracle.search(p, lib_hv, g.library.pmz, g.library.charge, q_hv, q.pmz, q.charge)
    assert np.all(dist == 0)
    assert np.all(idx <= rows)
    assert np.array_equal(lib_hv[idx], q_hv)
