"""Pins of the learned-shortlist oracle: analytic gradients against central
finite differences in float64, closed forms of the loss and of the unit
embedding, the Adam update against its first-step closed form, and the
shortlist search against brute force."""
import numpy as np
import pytest

from oracle import mlp


def _small(seed=0, D=64, H=16, E=8, B=5):
    rng = np.random.default_rng(seed)
    p = mlp.init_params(D, H, E, rng)
    p["b1"] = rng.normal(0, 0.1, H)
    p["b2"] = rng.normal(0, 0.1, E)
    Xq = np.where(rng.random((B, D)) < 0.5, 1.0, -1.0)
    Xr = np.where(rng.random((B, D)) < 0.5, 1.0, -1.0)
    return p, Xq, Xr


def test_gradients_match_finite_differences():
    p, Xq, Xr = _small()
    tau = 0.1
    loss, g = mlp.loss_and_grads(p, Xq, Xr, tau)
    rng = np.random.default_rng(1)
    h = 1e-6
    for name in ("W1", "b1", "W2", "b2"):
        flat = p[name].reshape(-1)
        for j in rng.choice(flat.size, size=min(25, flat.size), replace=False):
            old = flat[j]
            flat[j] = old + h
            lp, _ = mlp.loss_and_grads(p, Xq, Xr, tau)
            flat[j] = old - h
            lm, _ = mlp.loss_and_grads(p, Xq, Xr, tau)
            flat[j] = old
            fd = (lp - lm) / (2 * h)
            an = g[name].reshape(-1)[j]
            assert abs(fd - an) <= 1e-6 + 1e-5 * abs(fd), (name, j, fd, an)


def test_loss_closed_forms():
    """Equal embeddings everywhere: every logit is 1/tau, so the loss is
    log(B); orthonormal query/reference pairs: loss = log(1 + (B-1) e^(-1/tau))."""
    B, tau = 6, 0.2
    E = np.tile(np.eye(8)[:1], (B, 1))
    loss, dq, dr = mlp.info_nce(E, E, tau)
    assert abs(loss - np.log(B)) < 1e-12
    E = np.eye(8)[:B]
    loss, _, _ = mlp.info_nce(E, E, tau)
    assert abs(loss - np.log(1 + (B - 1) * np.exp(-1 / tau))) < 1e-12


def test_embedding_is_unit_and_bipolar_unpacking():
    p, Xq, _ = _small(D=128)
    e = mlp.embed(p, Xq)
    assert np.allclose((e * e).sum(axis=1), 1.0, atol=1e-9)
    hv = np.array([[0x00000001, 0x80000000, 0, 0]], dtype=np.uint32)
    x = mlp.bipolar(hv, 128)
    assert x[0, 0] == -1 and x[0, 1] == 1 and x[0, 63] == -1 and x[0, 62] == 1
    assert (x == 1).sum() == 126


def test_adam_first_step_closed_form():
    """After one step from zero state, m_hat = g and v_hat = g^2, so each
    weight moves by -lr * g / (|g| + eps)."""
    p, Xq, Xr = _small(seed=3)
    loss, g = mlp.loss_and_grads(p, Xq, Xr, 0.1)
    before = {k: v.copy() for k, v in p.items()}
    mlp.adam(p, g, {}, lr=1e-2)
    for k in p:
        want = before[k] - 1e-2 * g[k] / (np.abs(g[k]) + 1e-8)
        assert np.allclose(p[k], want, rtol=0, atol=1e-12)


def test_training_lowers_the_loss():
    p, Xq, Xr = _small(seed=4, D=64, H=32, E=8, B=16)
    st = {}
    first, _ = mlp.loss_and_grads(p, Xq, Xr, 0.1)
    for _ in range(60):
        _, g = mlp.loss_and_grads(p, Xq, Xr, 0.1)
        mlp.adam(p, g, st, lr=3e-3)
    last, _ = mlp.loss_and_grads(p, Xq, Xr, 0.1)
    assert last < 0.5 * first


def test_shortlist_search_brute_force():
    rng = np.random.default_rng(6)
    D, nl, nq, k = 128, 80, 12, 5
    lib = rng.integers(0, 2**32, size=(nl, D // 32), dtype=np.uint32)
    q = rng.integers(0, 2**32, size=(nq, D // 32), dtype=np.uint32)
    El = rng.normal(size=(nl, 4))
    Eq = rng.normal(size=(nq, 4))
    El[7] = El[3]  # a score tie: the lower index must be kept first
    lp = rng.uniform(400, 600, nl)
    lc = rng.integers(2, 4, nl).astype(np.int8)
    qp = rng.uniform(400, 600, nq)
    qc = rng.integers(2, 4, nq).astype(np.int8)
    idx, dist, lists = mlp.shortlist_search(El, Eq, lib, q, lp, lc, qp, qc, k, tol_da=50.0,
                                            dim=D)
    for i in range(nq):
        cand = [r for r in range(nl) if lc[r] == qc[i] and abs(lp[r] - qp[i]) <= 50.0]
        ranked = sorted(cand, key=lambda r: (-float(El[r] @ Eq[i]), r))[:k]
        assert list(lists[i]) == ranked
        if ranked:
            best = min(ranked, key=lambda r: (sum(bin(int(a) ^ int(b)).count("1")
                                                  for a, b in zip(lib[r], q[i])), r))
            assert idx[i] == best
        else:
            assert (idx[i], dist[i]) == (-1, -1)


def test_round_bf16_known_values():
    """bfloat16 keeps 8 significant bits: 1 + 2^-8 lies halfway between 1 and
    1 + 2^-7 and goes to the even one (1); 1 + 3 * 2^-9 is nearer 1 + 2^-7;
    exact bfloat16 values and signs pass through; 2^-133 is subnormal in
    float32 and exact in bfloat16."""
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -9, -(1 + 2.0 ** -7), 0.0, 3.0,
                  1 + 2.0 ** -8 + 2.0 ** -20, 2.0 ** -133, 65280.0, 65408.0])
    want = np.array([1.0, 1.0, 1 + 2.0 ** -7, -(1 + 2.0 ** -7), 0.0, 3.0, 1 + 2.0 ** -7,
                     2.0 ** -133, 65280.0, 65536.0])
    assert np.array_equal(mlp.round_bf16(x), want)


def test_round_hidden_forward_differs_only_by_bf16_rounding():
    """With rounding off the forward is unchanged; with it on, h is the
    nearest bfloat16 of the exact h (relative error at most half a unit in
    the last place, 2^-8 of the value)."""
    rng = np.random.default_rng(5)
    p = mlp.init_params(256, 64, 32, rng)
    X = 1.0 - 2.0 * rng.integers(0, 2, (7, 256))
    a, b = mlp.forward(p, X), mlp.forward(p, X, round_hidden=True)
    assert np.allclose(a["a1"], b["a1"], rtol=0, atol=0)
    nz = a["h"] != 0
    rel = np.abs(b["h"][nz] - a["h"][nz]) / np.abs(a["h"][nz])
    assert rel.max() <= 2.0 ** -8 and (b["h"][~nz] == 0).all()
    assert not np.array_equal(a["h"], b["h"])


def test_round_e4m3_known_values():
    """E4M3 keeps 3 fraction bits: 1 + 1/16 lies halfway between 1 and 1.125
    and goes to the even one (1); 1 + 3/16 goes to 1.25; 3.3 = 1.65 * 2 is
    nearest 1.625 * 2; 17 is halfway between 16 and 18 (even: 16), 17.5 is
    nearer 18; 448 is the largest value and larger ones saturate; below 2^-6
    the spacing is 2^-9 (2^-10 is halfway between 0 and 2^-9: 0; 3 * 2^-10
    goes to 2^-8; 7.5 * 2^-9 goes to 8 * 2^-9 = 2^-6)."""
    x = np.array([1.0, 1 + 1 / 16, 1 + 3 / 16, 1.07, -3.3, 17.0, 17.5, 448.0, 500.0, -1e6,
                  2.0 ** -6, 2.0 ** -9, 2.0 ** -10, 3 * 2.0 ** -10, 7.5 * 2.0 ** -9, 0.0])
    want = np.array([1.0, 1.0, 1.25, 1.125, -3.25, 16.0, 18.0, 448.0, 448.0, -448.0,
                     2.0 ** -6, 2.0 ** -9, 0.0, 2.0 ** -8, 2.0 ** -6, 0.0])
    assert np.array_equal(mlp.round_e4m3(x), want)
    codes = mlp.e4m3_code(x)
    assert [int(c) for c in codes] == [0x38, 0x38, 0x3A, 0x39, 0xC5, 0x58, 0x59, 0x7E, 0x7E,
                                       0xFE, 0x08, 0x01, 0x00, 0x02, 0x08, 0x00]


def test_e4m3_codes_decode_to_their_values():
    """Every finite code decodes (from the format's definition) to a value
    that rounds back to the same code, and the values are strictly
    increasing in the code over the positive half."""
    c = np.arange(0x7F)
    e, m = c >> 3, c & 7
    val = np.where(e > 0, np.ldexp(1.0 + m / 8.0, e - 7), m * 2.0 ** -9)
    assert np.all(np.diff(val) > 0) and val[-1] == 448.0
    assert np.array_equal(mlp.e4m3_code(val), c.astype(np.uint8))
    assert np.array_equal(mlp.e4m3_code(-val[1:]), (c[1:] | 0x80).astype(np.uint8))
    assert np.array_equal(mlp.round_e4m3(val), val)
    # midpoints between neighbours go to the code with the even fraction
    mid = (val[1:] + val[:-1]) / 2
    want = np.where(c[:-1] % 2 == 0, c[:-1], c[1:])
    assert np.array_equal(mlp.e4m3_code(mid), want.astype(np.uint8))


def test_scoring_embeddings_relative_error():
    """Scaled by 16, a unit embedding's components lie in E4M3's range; the
    scoring value differs from e by at most 2^-4 of its magnitude in the
    normal range (half a unit in the last of 3 fraction bits) and by at most
    2^-10 / 16 absolutely below it."""
    rng = np.random.default_rng(2)
    e = rng.normal(size=(50, 256))
    e /= np.linalg.norm(e, axis=1, keepdims=True)
    s = mlp.scoring_embeddings(e)
    big = np.abs(16 * e) >= 2.0 ** -6
    assert np.all(np.abs(s - e)[big] <= 2.0 ** -4 * np.abs(e)[big])
    assert np.all(np.abs(s - e)[~big] <= 2.0 ** -10 / 16)
