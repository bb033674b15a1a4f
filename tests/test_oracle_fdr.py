"""Pins of the FDR and cascade oracle (Sections 2.1, 3.4 and 4.1).

The q-value function is checked on a hand-worked example, on ties, against an
independent formulation (the target-decoy filter run at every achievable FDR
level, taking for each PSM the smallest level that accepts it), on special
cases and on its monotonicity. The cascade is checked on planted data whose
stage of identification is known by construction. None of these needs a GPU.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import fdr


def test_q_values_hand_example():
    # distances 1..6, decoys at 3, 5, 6: cumulative (targets, decoys) at each
    # threshold: (1,0) (2,0) (2,1) (3,1) (3,2) (3,3) -> FDR 0, 0, 1/2, 1/3, 2/3, 1
    dist = np.array([1, 2, 3, 4, 5, 6])
    decoy = np.array([0, 0, 1, 0, 1, 1], dtype=bool)
    q = fdr.q_values(dist, decoy)
    assert list(q) == [0.0, 0.0, 1 / 3, 1 / 3, 2 / 3, 1.0]
    assert list(fdr.identified(dist, decoy, 0.34)) == [True, True, False, True, False, False]


def test_q_values_ties_share_a_threshold():
    # two PSMs at distance 5 (one decoy) are accepted or rejected together
    dist = np.array([5, 5, 2, 9])
    decoy = np.array([0, 1, 0, 0], dtype=bool)
    q = fdr.q_values(dist, decoy)
    assert q[2] == 0.0
    assert q[0] == q[1] == 1 / 3  # min(FDR(5) = 1/2, FDR(9) = 1/3)
    assert q[3] == 1 / 3


def test_q_values_special_cases():
    assert fdr.q_values(np.array([], dtype=np.int64), np.array([], dtype=bool)).size == 0
    # no decoys: every PSM at FDR 0
    assert np.all(fdr.q_values(np.array([7, 3, 9]), np.zeros(3, dtype=bool)) == 0.0)
    # only decoys: no threshold has a target, never accepted
    q = fdr.q_values(np.array([7, 3, 9]), np.ones(3, dtype=bool))
    assert np.all(np.isinf(q))
    assert not np.any(fdr.identified(np.array([7, 3, 9]), np.ones(3, dtype=bool), 1.0))
    # a decoy best match ahead of the targets: FDR undefined at its threshold
    q = fdr.q_values(np.array([1, 2, 3]), np.array([1, 0, 0], dtype=bool))
    assert list(q) == [0.5, 0.5, 0.5]


def _q_by_filtering(dist, decoy):
    """Independent formulation: the target-decoy filter at level a accepts
    every PSM up to the largest threshold whose FDR is <= a; a PSM's q-value
    is the smallest achievable level at which it is accepted."""
    levels = sorted({d for d in dist})
    fdrs = []
    for t in levels:
        tg = sum(1 for d, y in zip(dist, decoy) if d <= t and not y)
        dc = sum(1 for d, y in zip(dist, decoy) if d <= t and y)
        fdrs.append(dc / tg if tg else math.inf)
    out = []
    for d in dist:
        best = math.inf
        for a in sorted(set(f for f in fdrs if f != math.inf)):
            ok = [t for t, f in zip(levels, fdrs) if f <= a]
            if ok and d <= max(ok):
                best = a
                break
        out.append(best)
    return np.array(out)


@pytest.mark.parametrize("seed", range(6))
def test_q_values_match_the_filter_formulation(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    dist = rng.integers(0, 12, n)
    decoy = rng.random(n) < rng.uniform(0.1, 0.7)
    assert np.array_equal(fdr.q_values(dist, decoy), _q_by_filtering(dist, decoy))


def test_q_values_monotone_in_distance():
    rng = np.random.default_rng(5)
    dist = rng.integers(0, 200, 300)
    decoy = rng.random(300) < 0.3
    q = fdr.q_values(dist, decoy)
    order = np.argsort(dist, kind="stable")
    assert np.all(np.diff(q[order]) >= 0)


# ------------------------------------------------------------------ cascade

def _flip(row, rng, t, D):
    out = row.copy()
    for d in rng.choice(D, size=t, replace=False):
        out[d // 32] ^= np.uint32(1 << (d % 32))
    return out


@pytest.fixture(scope="module")
def planted():
    """400 random codewords (200 targets, then 200 decoys) 2.5 Da apart, charge 2."""
    rng = np.random.default_rng(11)
    D, nl = 2048, 400
    lib = rng.integers(0, 2 ** 32, size=(nl, D // 32), dtype=np.uint64).astype(np.uint32)
    pmz = 400.0 + 2.5 * np.arange(nl)
    charge = np.full(nl, 2, dtype=np.int8)
    decoy = np.arange(nl) >= 200
    return D, lib, pmz, charge, decoy, rng


def test_cascade_planted_stages(planted):
    """Group A copies targets (100 bits flipped) at their own precursor m/z:
    found by the narrow stage. Group B copies other targets 101.25 Da away
    from any library precursor: nothing in the narrow window, found by the
    open stage. Every PSM is a target at distance 100, so q = 0."""
    D, lib, pmz, charge, decoy, rng = planted
    t = 100
    a_src = np.arange(0, 60, 2)
    b_src = np.arange(1, 61, 2)
    q_hv = np.stack([_flip(lib[i], rng, t, D) for i in np.concatenate([a_src, b_src])])
    q_pmz = np.concatenate([pmz[a_src], pmz[b_src] + 101.25])
    q_ch = np.full(q_pmz.shape[0], 2, dtype=np.int8)
    idx, dist, stage, qv = fdr.cascade(oracle.Params(dim=D), lib, pmz, charge, decoy, q_hv,
                                       q_pmz, q_ch, narrow=(1, 20.0), wide=(0, 500.0))
    assert np.array_equal(idx, np.concatenate([a_src, b_src]))
    assert np.all(dist == t)
    assert list(stage) == [1] * 30 + [2] * 30
    assert np.all(qv == 0.0)


def test_cascade_decoy_hits_raise_the_fdr(planted):
    """Three queries copy decoys at the same distance as 30 target copies: the
    FDR at that threshold is 3/30. At 1% nothing is identified in either
    stage (the open stage sees the same matches); at 10% the 30 target
    matches are identified by the narrow stage, the decoy matches never: they
    go on to the open stage alone, where no threshold has a target (q = inf)."""
    D, lib, pmz, charge, decoy, rng = planted
    t = 100
    src = np.concatenate([np.arange(100, 130), np.array([250, 300, 350])])
    q_hv = np.stack([_flip(lib[i], rng, t, D) for i in src])
    q_pmz = pmz[src]
    q_ch = np.full(src.shape[0], 2, dtype=np.int8)
    p = oracle.Params(dim=D)
    idx, dist, stage, qv = fdr.cascade(p, lib, pmz, charge, decoy, q_hv, q_pmz, q_ch,
                                       narrow=(1, 20.0), wide=(0, 500.0), level=0.01)
    assert np.array_equal(idx, src)
    assert np.all(stage == 0)
    assert np.all(qv == 0.1)
    idx, dist, stage, qv = fdr.cascade(p, lib, pmz, charge, decoy, q_hv, q_pmz, q_ch,
                                       narrow=(1, 20.0), wide=(0, 500.0), level=0.1)
    assert list(stage) == [1] * 30 + [0] * 3
    assert np.all(qv[:30] == 0.1)
    assert np.all(np.isinf(qv[30:]))
