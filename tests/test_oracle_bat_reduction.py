"""Pins for oracle/bat.py (Sec. BAT, Alg. bat_deployment) and oracle/reduction.py
(Alg. montgomery_reduction, Alg. barrett)."""
import numpy as np
import pytest

from oracle import bat as B
from oracle import reduction as RD
from oracle.mat import modmatmul
from oracle.primes import prime_chain

Q0 = 268042241


def test_toeplitz_zero_fraction_matches_paper():
    # Sec. BAT: the sparse (2K-1) x K Toeplitz form of a K-chunk product holds
    # 12 zeros out of 4 x 7 entries (about 43%) for K = 4; BAT's dense block is K x K.
    K = 4
    X = np.zeros((2 * K - 1, K), dtype=int)
    for j in range(K):
        for i in range(K):
            X[i + j, j] = 1 + i          # any non-zero chunk values
    assert (X == 0).sum() == 12 and X.size == 28
    assert B.direct_scalar_bat(123456789 % Q0, Q0, 7, K).shape == (K, K)


@pytest.mark.parametrize("bp,k", [(7, 4), (8, 4), (4, 7)])
def test_direct_scalar_bat_identity(bp, k):
    q = Q0
    g = np.random.Generator(np.random.PCG64(bp * 10 + k))
    edges = [0, 1, q - 1, 2, 1 << 7, 1 << 14, 1 << 21, (1 << 27) + 5]
    for a in edges + [int(v) for v in g.integers(0, q, 20)]:
        Mx = B.direct_scalar_bat(a, q, bp, k)
        assert Mx.min() >= 0 and Mx.max() < (1 << bp)
        for b in edges + [int(v) for v in g.integers(0, q, 20)]:
            bc = B.chunk_decompose(b, bp, k)
            assert B.chunk_merge(bc, bp) == b
            psums = [sum(int(Mx[i, j]) * bc[j] for j in range(k)) for i in range(k)]
            assert all(p < k << (2 * bp) for p in psums)     # 2bp + log2 K bits
            assert B.chunk_merge(psums, bp) % q == a * b % q


def test_bat_modmatmul_equals_plain_modmatmul():
    g = np.random.Generator(np.random.PCG64(3))
    for q in prime_chain(2):
        for (H, V, W) in [(3, 5, 4), (1, 1, 1), (4, 8, 2)]:
            A = g.integers(0, q, (H, V))
            Bm = g.integers(0, q, (V, W))
            A[0, 0] = q - 1
            Bm[0, 0] = q - 1
            assert np.array_equal(B.bat_modmatmul(A, Bm, q), modmatmul(A, Bm, q))


def _mont_ref(z, q):
    return z * pow(1 << 32, -1, q) % q


def test_montgomery_edges_and_random():
    for q in prime_chain(4) + [17, 97, 7681]:
        edges = [0, 1, q - 1, (q - 1) ** 2, (q << 32) - 1, (1 << 45) - 1, q << 31]
        g = np.random.Generator(np.random.PCG64(q % 997))
        rnd = [int(v) for v in g.integers(0, 1 << 62, 2000) % (q << 32)]
        for z in edges + rnd:
            if z >= q << 32:
                continue
            b = RD.montgomery_reduce(z, q)
            assert 0 <= b < 2 * q
            assert b % q == _mont_ref(z, q)


def test_printed_montgomery_middle_sum_double_counts():
    # Reading G7: the algorithm as printed adds the full cross products into the
    # middle sum and then their high halves again; on random inputs that is
    # almost never floor(t*q / 2^32).  The oracle's reading takes the low halves.
    q = Q0
    g = np.random.Generator(np.random.PCG64(11))
    wrong = 0
    trials = 2000
    for t in g.integers(0, 1 << 32, trials):
        t = int(t)
        t_lo, t_hi = t & 0xFFFF, t >> 16
        q_lo, q_hi = q & 0xFFFF, q >> 16
        p_hi, p_lo = t_hi * q_hi, t_lo * q_lo
        p_mh, p_ml = t_hi * q_lo, t_lo * q_hi
        mid_lo = p_mh + p_ml + (p_lo >> 16)
        mid_hi = (p_mh >> 16) + (p_ml >> 16) + (mid_lo >> 16)
        wrong += (p_hi + mid_hi) != (t * q) >> 32
    assert wrong > trials * 0.9


def test_barrett_matches_modulo():
    for q in prime_chain(4) + [17, 97]:
        g = np.random.Generator(np.random.PCG64(q % 991))
        pairs = [(0, 0), (q - 1, q - 1), (1, q - 1), (q - 1, 1)]
        pairs += [(int(a), int(b)) for a, b in g.integers(0, q, (3000, 2))]
        for a, b in pairs:
            assert RD.barrett_mulmod(a, b, q) == a * b % q


def test_shoup_edges_and_random():
    from oracle.reduction import shoup_mulmod
    g = np.random.Generator(np.random.PCG64(21))
    for q in prime_chain(3) + [97, 257]:
        for a in (0, 1, q - 1, q, 2 * q - 1, (1 << 32) - 1):
            for w in (0, 1, 2, q - 1):
                assert shoup_mulmod(a, w, q) == a * w % q
        for a, w in zip(g.integers(0, 1 << 32, 500), g.integers(0, q, 500)):
            assert shoup_mulmod(int(a), int(w), q) == int(a) * int(w) % q


@pytest.mark.parametrize("bp,k", [(7, 4), (8, 4), (2, 3)])
def test_bat_lazy_reduce_is_congruent_and_bounded(bp, k):
    # the paper's byte form (bp = 8, a 64-bit partial sum), the 7-bit MFMA form, and a tiny case
    from oracle.reduction import bat_lazy_reduce
    g = np.random.Generator(np.random.PCG64(22))
    bound = (1 << (bp * k)) + k * ((1 << bp) - 1) ** 2 * ((1 << (bp * k)) - 1) // ((1 << bp) - 1)
    qs = [q for q in (prime_chain(2) + [97, 61, 7]) if q < 1 << (bp * k)]
    top = (1 << (2 * k * bp)) - 1
    for q in qs:
        for p in [0, 1, q, (1 << (bp * k)) - 1, 1 << (bp * k), top] + [int(v) for v in g.integers(0, top, 300, dtype=np.uint64)]:
            r = bat_lazy_reduce(p, q, bp, k)
            assert r % q == p % q and 0 <= r < bound


def test_bat_lazy_tiny_worked_example():
    # q = 7, bp = 2, k = 2: p = 0b1101_1011 = 219; low = 0b1011 = 11; c_2 = 0b01 = 1, c_3 = 0b11 = 3;
    # LC_0 = 2^4 mod 7 = 2 = [2, 0], LC_1 = 2^6 mod 7 = 1 = [1, 0];
    # T_0 = 1*2 + 3*1 = 5, T_1 = 0; r = 11 + 5 = 16 = 219 (mod 7)
    from oracle.reduction import bat_lazy_reduce, lazy_constants
    assert lazy_constants(7, 2, 2) == [[2, 0], [1, 0]]
    assert bat_lazy_reduce(219, 7, 2, 2) == 16
    assert 16 % 7 == 219 % 7


def test_bat_lazy_mulmod_matches_modulo():
    from oracle.reduction import bat_lazy_mulmod
    g = np.random.Generator(np.random.PCG64(23))
    for q in prime_chain(3):
        for a, w in [(0, 0), (q - 1, q - 1), (1, q - 1)] + list(zip(g.integers(0, q, 300), g.integers(0, q, 300))):
            assert bat_lazy_mulmod(int(a), int(w), q) == int(a) * int(w) % q
