"""The fp4 (e2m1) operand encoding of the matrix-core search, checked on the CPU.

The search contracts bit vectors on matrix cores. On both sides a bit x of a
component of class m = component mod 4 selects between two e2m1 codes that
differ in bit m of the nibble alone, so the bit never moves in its word:
values u_m + 2 x s_m with (u, u + 2s) = (4, 6), (2, 4), (0, 2), (1, -1).
Every class has (2 s_m)^2 = 4, so <x, y> = 21D/4 + sum_m 2 u_m s_m (|a|_m +
|b|_m) + 4 a.b and 2H = K(a) + Q(b) - <x, y>, with a per-row constant
K(a) = 10|a|_0 + 6|a|_1 + 2|a|_2 and a per-query constant Q(b) = 21D/4 +
10|b|_0 + 6|b|_1 + 2|b|_2; the kernel recovers the Hamming distance H of
Section 3.4 as (Q - t) / 2 with t = <x, y> - K. These tests decode the
nibbles by the e2m1 definition (1 sign, 2 exponent bits with bias 1, 1
mantissa bit; exponent 0 is subnormal) and check the identity per class, on
random and extreme vectors, and the bound that keeps every partial sum exact
in fp32.
"""
import numpy as np

# nibble patterns the kernel inserts (per class m = 0..3), both operands
SEL = [0x1, 0x2, 0x4, 0x8]     # the bit stays at nibble bit m
BASE = [0x6, 0x4, 0x0, 0x2]    # code for a 0 bit: 4.0, 2.0, 0.0, 1.0
WEIGHTS = (10, 6, 2, 0)        # K and Q: sum_m w_m |x|_m (Q adds 21D/4)


def e2m1(n: int) -> float:
    sign = -1.0 if n & 8 else 1.0
    e, m = (n >> 1) & 3, n & 1
    mag = 0.5 * m if e == 0 else (1.0 + 0.5 * m) * 2.0 ** (e - 1)
    return sign * mag


def value(m: int, bit: int) -> float:
    return e2m1((BASE[m] & ~SEL[m] & 0xF) | (SEL[m] if bit else 0))


def test_e2m1_decoding_of_known_values():
    # the value table of the format
    assert [e2m1(n) for n in range(8)] == [0.0, 0.5, 1.0, 1.5, 2.0, 3.0, 4.0, 6.0]
    assert [e2m1(n | 8) for n in range(8)] == [-0.0, -0.5, -1.0, -1.5, -2.0, -3.0, -4.0, -6.0]


def test_every_class_has_the_same_cross_term():
    for m in range(4):
        assert BASE[m] & SEL[m] == 0  # the 0 code has the class bit clear
        u, step = value(m, 0), value(m, 1) - value(m, 0)
        assert step * step == 4.0  # the coefficient of a.b, the same in every class
        # the row and query constants: 2 + u * step per set bit of the class
        assert 2 + u * step == WEIGHTS[m]
        for a in (0, 1):
            for b in (0, 1):
                p = value(m, a) * value(m, b)
                assert p == int(p)  # every product is an integer


def _terms(x: np.ndarray, y: np.ndarray):
    cls = np.arange(x.size) % 4
    tab = np.array([[value(m, 0), value(m, 1)] for m in range(4)])
    dot = float(np.sum(tab[cls, x] * tab[cls, y]))
    k = sum(w * int(x[cls == m].sum()) for m, w in enumerate(WEIGHTS))
    q = 21 * x.size // 4 + sum(w * int(y[cls == m].sum()) for m, w in enumerate(WEIGHTS))
    return dot, k, q


def test_hamming_identity_on_random_vectors():
    rng = np.random.default_rng(7)
    for d in (512, 1536, 8192):
        for density in (0.5, 0.1, 0.9):
            x = (rng.random(d) < density).astype(np.int64)
            y = (rng.random(d) < 1 - density).astype(np.int64)
            dot, k, q = _terms(x, y)
            assert (q - (dot - k)) / 2 == int(np.sum(x != y))


def test_extreme_vectors_and_fp32_bound():
    for d in (512, 8192, 32768):
        for xv in (0, 1):
            for yv in (0, 1):
                x = np.full(d, xv, dtype=np.int64)
                y = np.full(d, yv, dtype=np.int64)
                dot, k, q = _terms(x, y)
                assert (q - (dot - k)) / 2 == (d if xv != yv else 0)
                # largest partial sum magnitude: 36 + 16 + 4 + 1 per 4 components
                assert abs(dot) <= 57 * d // 4 < 2 ** 24
                assert abs(dot - k) < 2 ** 24
