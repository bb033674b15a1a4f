"""Learned-shortlist oracle — TEST INFRASTRUCTURE ONLY.

Float64 numpy definition of the small MLP that embeds hypervectors for the
learned shortlist (not in the paper; the paper's search is the exhaustive
Hamming top-1 of Section 3.4, which remains the reference answer):

    x  = bipolar form of the packed hypervector (bit 0 -> +1, bit 1 -> -1)
    a1 = W1 x + b1,   h = ReLU(a1)                      (D -> H)
    z  = W2 h + b2                                      (H -> E)
    e  = z / sqrt(z.z + eps)                            (unit embedding)
    score(q, r) = s_q . s_r,  s = E4M3(16 e) / 16       (scoring_embeddings)

Training loss for a batch of B (query, exact top-1 reference) pairs is
InfoNCE with in-batch negatives and temperature tau:

    S_ij = e_qi . e_rj / tau,   loss = mean_i [logsumexp_j S_ij - S_ii]

Adam (Kingma & Ba, 2015) updates the weights. The shortlist of a query is
the k candidates of its window (Section 3.4) with the largest scores, ties to
the lower library index; the answer is the exhaustive top-1 restricted to the
shortlist. Only tests, the smoke check and the benchmark's CPU baseline may
import this module; it imports nothing from the product package.
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np

EPS_NORM = 1e-12


def bipolar(hv: np.ndarray, dim: int) -> np.ndarray:
    """Packed uint32 rows [n, D/32] -> float64 +-1 [n, D]."""
    bits = np.unpackbits(np.ascontiguousarray(hv, dtype=np.uint32).view(np.uint8), axis=1,
                         bitorder="little")[:, :dim]
    return 1.0 - 2.0 * bits.astype(np.float64)


def init_params(dim: int, hidden: int, embed: int, rng: np.random.Generator
                ) -> Dict[str, np.ndarray]:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases (drawn by
    the caller's generator and handed to both sides)."""
    return {
        "W1": rng.uniform(-1, 1, (hidden, dim)) / np.sqrt(dim),
        "b1": np.zeros(hidden),
        "W2": rng.uniform(-1, 1, (embed, hidden)) / np.sqrt(hidden),
        "b2": np.zeros(embed),
    }


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Nearest bfloat16 value (ties to even) of each element, as float64: the
    value is first rounded to float32, then its 32-bit pattern is rounded to
    the upper 16 bits (finite inputs)."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(p: Dict[str, np.ndarray], X: np.ndarray, round_hidden: bool = False
            ) -> Dict[str, np.ndarray]:
    """round_hidden rounds h to bfloat16, the precision in which the hidden
    layer is handed to the second layer when the weights are stored in
    bfloat16 (pass bfloat16-rounded weights alongside)."""
    a1 = X @ p["W1"].T + p["b1"]
    h = np.maximum(a1, 0.0)
    if round_hidden:
        h = round_bf16(h)
    z = h @ p["W2"].T + p["b2"]
    s = np.sqrt((z * z).sum(axis=1, keepdims=True) + EPS_NORM)
    return {"X": X, "a1": a1, "h": h, "z": z, "s": s, "e": z / s}


def embed(p, X, round_hidden: bool = False):
    return forward(p, X, round_hidden)["e"]


# Scoring embeddings are stored in the 8-bit E4M3 format of the OCP 8-bit
# floating point specification (v1.0, 2023) after scaling by SCORE_SCALE, so
# that the components of a unit embedding sit in its normal range.
SCORE_SCALE = 16.0
E4M3_MAX = 448.0


def round_e4m3(x: np.ndarray) -> np.ndarray:
    """Nearest E4M3 value of each element (as float64), ties to even: 3
    fraction bits in each binade 2^e .. 2^(e+1) for e >= -6, multiples of 2^-9
    below 2^-6 (subnormals), magnitudes beyond 448 saturated to 448."""
    x = np.asarray(x, dtype=np.float64)
    a = np.minimum(np.abs(x), E4M3_MAX)
    _, ex = np.frexp(a)                        # a = f 2^ex with f in [0.5, 1)
    e = np.maximum(ex.astype(np.float64) - 1.0, -6.0)
    step = np.ldexp(1.0, (e - 3.0).astype(np.int64))
    r = np.minimum(np.round(a / step) * step, E4M3_MAX)  # np.round: ties to even
    return np.copysign(r, x)


def e4m3_code(x: np.ndarray) -> np.ndarray:
    """Byte of the E4M3 value nearest to each element: sign bit 7, biased
    exponent (bias 7) in bits 3-6, fraction in bits 0-2; exponent field 0 for
    the subnormals m 2^-9."""
    r = round_e4m3(x)
    a = np.abs(r)
    _, ex = np.frexp(a)
    normal = a >= 2.0 ** -6
    e = np.where(normal, ex - 1, -6)
    frac = np.where(normal, a / np.ldexp(1.0, e) - 1.0, a * 512.0)
    code = np.where(normal, ((e + 7) << 3) + np.round(frac * 8.0).astype(np.int64),
                    np.round(frac).astype(np.int64))
    return (code | np.where(np.signbit(r), 0x80, 0)).astype(np.uint8)


def scoring_embeddings(e: np.ndarray) -> np.ndarray:
    """Embeddings as the shortlist scores them: E4M3 of SCORE_SCALE e, scaled
    back (exact), so that score(q, r) = round_e4m3(16 e_q) . round_e4m3(16 e_r) / 256."""
    return round_e4m3(SCORE_SCALE * np.asarray(e, dtype=np.float64)) / SCORE_SCALE


def rounded_weights(p: Dict[str, np.ndarray]) -> Dict[str, np.ndarray]:
    """Weights as stored for bfloat16 matrix products (biases stay exact)."""
    return {"W1": round_bf16(p["W1"]), "b1": p["b1"], "W2": round_bf16(p["W2"]), "b2": p["b2"]}


def info_nce(Eq: np.ndarray, Er: np.ndarray, tau: float) -> Tuple[float, np.ndarray, np.ndarray]:
    """Loss and its gradients with respect to the query and reference embeddings."""
    B = Eq.shape[0]
    S = Eq @ Er.T / tau
    m = S.max(axis=1, keepdims=True)
    P = np.exp(S - m)
    Z = P.sum(axis=1, keepdims=True)
    loss = float(np.mean(np.log(Z[:, 0]) + m[:, 0] - np.diag(S)))
    dS = (P / Z - np.eye(B)) / B
    return loss, dS @ Er / tau, dS.T @ Eq / tau


def backward(p, c, dE) -> Dict[str, np.ndarray]:
    e, s = c["e"], c["s"]
    dz = (dE - e * (e * dE).sum(axis=1, keepdims=True)) / s
    g = {"W2": dz.T @ c["h"], "b2": dz.sum(axis=0)}
    dh = dz @ p["W2"]
    da1 = dh * (c["a1"] > 0.0)
    g["W1"] = da1.T @ c["X"]
    g["b1"] = da1.sum(axis=0)
    return g


def loss_and_grads(p, Xq: np.ndarray, Xr: np.ndarray, tau: float, round_hidden: bool = False):
    """Loss of a batch of pairs and the gradient of every parameter (the
    query and reference towers share the weights, so gradients add)."""
    cq, cr = forward(p, Xq, round_hidden), forward(p, Xr, round_hidden)
    loss, dEq, dEr = info_nce(cq["e"], cr["e"], tau)
    gq, gr = backward(p, cq, dEq), backward(p, cr, dEr)
    return loss, {k: gq[k] + gr[k] for k in gq}


def adam(p, g, state, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step in place; state holds m, v per parameter and the step t."""
    t = state.get("t", 0) + 1
    state["t"] = t
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = beta1 * m + (1 - beta1) * g[k]
        v[...] = beta2 * v + (1 - beta2) * g[k] * g[k]
        mh = m / (1 - beta1 ** t)
        vh = v / (1 - beta2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
    return p


def shortlist_search(E_lib, E_q, lib_hv, q_hv, lib_pmz, lib_charge, q_pmz, q_charge, k,
                     tol_da=500.0, dim=8192):
    """Top-k candidates by embedding score within each query's window (ties to
    the lower library index), then the exact Hamming top-1 over them.
    Returns (index, distance, shortlist) per query; (-1, -1) without candidates."""
    nq = E_q.shape[0]
    idx = np.full(nq, -1, dtype=np.int64)
    dist = np.full(nq, -1, dtype=np.int32)
    lists = []
    for i in range(nq):
        lo, hi = q_pmz[i] - tol_da, q_pmz[i] + tol_da
        cand = np.flatnonzero((lib_charge == q_charge[i]) & (lib_pmz >= lo) & (lib_pmz <= hi))
        if cand.size == 0:
            lists.append(cand)
            continue
        sc = E_lib[cand] @ E_q[i]
        order = np.lexsort((cand, -sc))[:k]
        short = cand[order]
        lists.append(short)
        h = np.bitwise_count(lib_hv[short] ^ q_hv[i]).sum(axis=1)
        j = np.lexsort((short, h))[0]
        idx[i], dist[i] = short[j], h[j]
    return idx, dist, lists
