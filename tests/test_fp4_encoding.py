"""The fp4 (e2m1) operand encoding of the matrix-core search, checked on the CPU.

The search contracts bit vectors on matrix cores: query bits become signed
magnitudes (-1)^b * beta_m and library bits select between two values u_m and
u_m + delta_m, where m = component mod 4 is the component's class. Since
delta_m * beta_m = -2 in every class, <x, y> = Q - 2 H with a constant Q per
query, and the kernel recovers the Hamming distance H of Section 3.4 as
(Q - <x, y>) / 2. These tests decode the nibbles the kernel writes by the
e2m1 definition (1 sign, 2 exponent bits with bias 1, 1 mantissa bit;
exponent 0 is subnormal) and check the identity exhaustively per class and on
random vectors, including the bound that keeps every partial sum exact in fp32.
"""
import numpy as np

# nibble patterns the kernel inserts (per class m = 0..3)
LIB_SEL = [0x1, 0x2, 0x4, 0x8]        # library bit stays at nibble bit m
LIB_BASE = [0xA, 0x8, 0x8, 0x2]       # value for a 0 bit
QUERY_MAG = [0x6, 0x4, 0x2, 0x2]      # query magnitude; its bit goes to the sign
Q_WEIGHTS = (10, 2, 2, 0)             # Q = -3D/4 + sum_m w_m |b|_m


def e2m1(n: int) -> float:
    sign = -1.0 if n & 8 else 1.0
    e, m = (n >> 1) & 3, n & 1
    mag = 0.5 * m if e == 0 else (1.0 + 0.5 * m) * 2.0 ** (e - 1)
    return sign * mag


def lib_value(m: int, bit: int) -> float:
    return e2m1((LIB_BASE[m] & ~LIB_SEL[m] & 0xF) | (LIB_SEL[m] if bit else 0))


def query_value(m: int, bit: int) -> float:
    return e2m1(QUERY_MAG[m] | (8 if bit else 0))


def test_e2m1_decoding_of_known_values():
    # the value table of the format
    assert [e2m1(n) for n in range(8)] == [0.0, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0]
    assert [e2m1(n | 8) for n in range(8)] == [-0.0, -0.5, -1.0, -1.5, -2.0, -3.0, -4.0, -6.0]


def test_every_class_has_the_same_cross_term():
    for m in range(4):
        delta = lib_value(m, 1) - lib_value(m, 0)
        beta = query_value(m, 0)
        assert query_value(m, 1) == -beta  # query side is symmetric
        assert delta * beta == -2.0
        # every product is an integer, so fp32 sums of them are exact
        for a in (0, 1):
            for b in (0, 1):
                p = lib_value(m, a) * query_value(m, b)
                assert p == int(p)


def _dot_and_q(x: np.ndarray, y: np.ndarray):
    cls = np.arange(x.size) % 4
    lib = np.array([[lib_value(m, 0), lib_value(m, 1)] for m in range(4)])
    qry = np.array([[query_value(m, 0), query_value(m, 1)] for m in range(4)])
    dot = float(np.sum(lib[cls, x] * qry[cls, y]))
    q = -3 * x.size // 4 + sum(w * int(y[cls == m].sum()) for m, w in enumerate(Q_WEIGHTS))
    return dot, q


def test_hamming_identity_on_random_vectors():
    rng = np.random.default_rng(7)
    for d in (512, 1536, 8192):
        for density in (0.5, 0.1, 0.9):
            x = (rng.random(d) < density).astype(np.int64)
            y = (rng.random(d) < 1 - density).astype(np.int64)
            dot, q = _dot_and_q(x, y)
            assert (q - dot) / 2 == int(np.sum(x != y))


def test_extreme_vectors_and_fp32_bound():
    for d in (512, 8192, 32768):
        for xv in (0, 1):
            for yv in (0, 1):
                x = np.full(d, xv, dtype=np.int64)
                y = np.full(d, yv, dtype=np.int64)
                dot, q = _dot_and_q(x, y)
                assert (q - dot) / 2 == (d if xv != yv else 0)
                # largest partial sum magnitude: 6 + 2 + 2 + 1 per 4 components
                assert abs(dot) <= 11 * d // 4 < 2 ** 24
