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
