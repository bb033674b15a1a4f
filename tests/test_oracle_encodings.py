"""Pins of the oracle's encoding baselines of Section 4.2 (Fig. 4(c)): ID-level
encoding with independent random position vectors, and random-projection LSH
of the spectrum vector. Checked against the SplitMix64 stream (itself pinned
to published outputs), closed forms of the weighted sign, and a reduction to
the Eq. 1 majority of the main encoding. None of these needs a GPU."""
import numpy as np
import pytest

import oracle


def _params(D, f, Q=16, encoding=0, seed=5):
    return oracle.Params(dim=D, n_levels=Q, mz_min=0.0, mz_max=f / 20.0, bins_per_da=20.0,
                         seed=seed, encoding=encoding)


@pytest.mark.parametrize("encoding", [1, 2])
def test_random_position_rows_continue_the_stream(encoding):
    """The level table is the main encoding's; position row i is the next D/64
    outputs of the stream after the main generator's draws (F_0 bits, the
    F order, L_0 bits, the L order: 2 D/64 + 2 (D - 1) outputs)."""
    D, f = 256, 40
    idt0, lvt0 = oracle.codebook(_params(D, f))
    idt, lvt = oracle.codebook(_params(D, f, encoding=encoding))
    assert np.array_equal(lvt, lvt0)
    used = 2 * (D // 64) + 2 * (D - 1)
    out = oracle.splitmix64(5, used + f * (D // 64))
    for i in range(f):
        words = out[used + i * (D // 64): used + (i + 1) * (D // 64)]
        assert np.array_equal(idt[i].view(np.uint64), words)
    # independent rows: pairwise distances near D/2 (none near 0)
    H = np.bitwise_count(idt[:, None, :] ^ idt[None, :, :]).sum(axis=-1)
    off = H[~np.eye(f, dtype=bool)]
    assert off.min() > D // 4 and off.max() < 3 * D // 4


def _lsh(D, table, peaks):
    """Encode one spectrum given as [(row, level)] with the LSH oracle."""
    p = oracle.Params(dim=D, encoding=2)
    off = np.array([0, len(peaks)], dtype=np.int64)
    bins = np.array([r for r, _ in peaks], dtype=np.int32)
    lv = np.array([l for _, l in peaks], dtype=np.uint8)
    lvt = np.zeros((16, D // 32), dtype=np.uint32)
    return oracle.encode(p, table, lvt, off, bins, lv)[0]


def test_lsh_closed_forms():
    rng = np.random.default_rng(1)
    D = 128
    T = rng.integers(0, 2 ** 32, size=(6, D // 32), dtype=np.uint64).astype(np.uint32)
    # one peak: its row
    assert np.array_equal(_lsh(D, T, [(2, 7)]), T[2])
    # a heavier peak decides every component (weights 5 vs 1)
    assert np.array_equal(_lsh(D, T, [(0, 4), (1, 0)]), T[0])
    # equal weights: agreeing components keep their bit, the others tie -> 1
    assert np.array_equal(_lsh(D, T, [(0, 3), (1, 3)]), T[0] | T[1])
    # three equal weights: bitwise majority
    maj = (T[0] & T[1]) | (T[0] & T[2]) | (T[1] & T[2])
    assert np.array_equal(_lsh(D, T, [(0, 9), (1, 9), (2, 9)]), maj)
    # weights 2 + 2 against 3: the pair wins where it agrees, else the single row
    got = _lsh(D, T, [(0, 1), (1, 1), (2, 2)])
    want = (T[0] & T[1]) | ((T[0] ^ T[1]) & T[2])
    assert np.array_equal(got, want)
    # order of the peaks does not matter; no peaks: every bit is a tie -> 1
    assert np.array_equal(_lsh(D, T, [(4, 2), (3, 5), (5, 1)]),
                          _lsh(D, T, [(5, 1), (4, 2), (3, 5)]))
    assert np.all(_lsh(D, T, []) == 0xFFFFFFFF)


def test_lsh_with_equal_weights_is_the_eq1_majority():
    """With one level for every peak the weights are equal, and with all-zero
    level vectors Eq. 1 binds each position vector with nothing, so both
    encodings are the same majority with the same tie rule."""
    rng = np.random.default_rng(4)
    D, f = 256, 30
    T = rng.integers(0, 2 ** 32, size=(f, D // 32), dtype=np.uint64).astype(np.uint32)
    zero_lv = np.zeros((16, D // 32), dtype=np.uint32)
    n = 40
    counts = rng.integers(0, 12, n)
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum(counts)
    bins = np.concatenate([rng.choice(f, c, replace=False) for c in counts]).astype(np.int32)
    lv = np.full(bins.shape[0], 6, dtype=np.uint8)
    lsh = oracle.encode(oracle.Params(dim=D, encoding=2), T, zero_lv, off, bins, lv)
    eq1 = oracle.encode(oracle.Params(dim=D), T, zero_lv, off, bins, lv)
    assert np.array_equal(lsh, eq1)
