"""Pins for oracle/primes.py: primality, the prime chain, generators and psi."""
import numpy as np

import synthetic
from oracle import primes as P


def _trial(n):
    if n < 2:
        return False
    d = 2
    while d * d <= n:
        if n % d == 0:
            return False
        d += 1
    return True


def test_miller_rabin_matches_trial_division_small():
    for n in range(0, 20000):
        assert P.is_prime(n) == _trial(n), n


def test_miller_rabin_matches_trial_division_28bit():
    g = np.random.Generator(np.random.PCG64(7))
    for n in g.integers(1 << 27, 1 << 28, 300):
        n = int(n) | 1
        assert P.is_prime(n) == _trial(n), n
    # strong pseudoprimes to single bases must still be rejected
    for n in (2047, 3215031751, 25326001, 1373653):
        assert not P.is_prime(n)


def test_chain_two_independent_derivations_agree():
    # synthetic/ finds the chain by trial division, the oracle by Miller-Rabin
    assert P.prime_chain(48) == synthetic.primes(48)


def test_chain_properties():
    ch = P.prime_chain(48)
    assert ch[0] == 268042241          # 2045 * 2^17 + 1, largest such prime below 2^28
    assert len(set(ch)) == 48
    for q in ch:
        assert (1 << 27) < q < (1 << 28)
        assert q % (1 << 17) == 1
    assert ch == sorted(ch, reverse=True)


def test_wide_chain_two_derivations_agree():
    # 31-bit primes (the NTT's wide form): Miller-Rabin chain = trial-division chain
    ch = P.prime_chain(8, bits=31)
    assert ch == synthetic.wide_primes(8)
    for q in ch:
        assert (1 << 28) <= q < (1 << 31) and q % (1 << 17) == 1 and _trial(q)
    assert ch == sorted(ch, reverse=True)
    # and nothing skipped: every m * 2^17 + 1 between them that is not listed is composite
    for m in range(ch[-1] >> 17, (1 << 31) >> 17):
        q = (m << 17) + 1
        if q < (1 << 31):
            assert (q in ch) == _trial(q)


def test_smallest_generator_brute_force():
    for q in (17, 97, 193, 257, 7681, 12289):
        g = P.smallest_generator(q)
        # brute-force orders
        def order(x):
            k, y = 1, x
            while y != 1:
                y = y * x % q
                k += 1
            return k
        assert order(g) == q - 1
        assert all(order(h) < q - 1 for h in range(2, g))
    assert P.smallest_generator(268042241) == 3


def test_psi_is_primitive_2n_root():
    for q in P.prime_chain(6) + P.prime_chain(2, bits=31):
        for log_n in (4, 8, 12, 16):
            n = 1 << log_n
            s = P.psi(q, n)
            assert pow(s, n, q) == q - 1
            assert pow(s, 2 * n, q) == 1
            # order is exactly 2N: no smaller power-of-two order
            assert pow(s, n // 2, q) not in (1, q - 1) or n == 1
            # consistency across N: psi_N^2 = psi_{N/2}
            if log_n > 1:
                assert s * s % q == P.psi(q, n // 2)
