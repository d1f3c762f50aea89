"""Pins for the oracle's HE-Add and Rescale (reading G17).

Rescale is checked against plain integer arithmetic on the CRT value of each
coefficient, independent of the conversion formula the oracle uses: for one
dropped prime the result is exactly floor(C / q_drop); for two it is
floor(C / P) or one less (the fast conversion may add one P).
"""
from math import prod

import numpy as np
import pytest

from oracle import ckks as CK
from oracle.primes import prime_chain


def _crt(residues, primes):
    """Textbook CRT: the integer in [0, Q) with the given residues."""
    Q = prod(primes)
    x = 0
    for r, q in zip(residues, primes):
        h = Q // q
        x += int(r) * h * pow(h % q, -1, q)
    return x % Q


def _coeff(g, primes, n):
    return np.stack([g.integers(0, q, n) for q in primes]).astype(np.uint64)


CHAINS = {
    "decreasing": prime_chain(5),
    # the dropped prime is the largest, so its residues need reduction into the kept primes
    "largest_last": [prime_chain(5)[k] for k in (3, 1, 4, 2, 0)],
}


@pytest.mark.parametrize("chain", sorted(CHAINS))
def test_rescale_one_prime_is_floor_division(chain):
    primes = CHAINS[chain]
    n = 32
    g = np.random.Generator(np.random.PCG64(11))
    c = _coeff(g, primes, n)
    out = CK.ntt_rows(CK.rescale(CK.ntt_rows(c, primes), primes, 1), primes[:-1], inverse=True)
    ql = primes[-1]
    for k in range(n):
        C = _crt(c[:, k], primes)
        r = C // ql
        assert [int(v) for v in out[:, k]] == [r % q for q in primes[:-1]]


@pytest.mark.parametrize("chain", sorted(CHAINS))
def test_rescale_two_primes_is_floor_or_one_below(chain):
    primes = CHAINS[chain]
    n = 32
    g = np.random.Generator(np.random.PCG64(12))
    c = _coeff(g, primes, n)
    out = CK.ntt_rows(CK.rescale(CK.ntt_rows(c, primes), primes, 2), primes[:-2], inverse=True)
    P = primes[-1] * primes[-2]
    kept = primes[:-2]
    Qk = prod(kept)
    lows = 0
    for k in range(n):
        C = _crt(c[:, k], primes)
        got = _crt(out[:, k], kept)
        f = C // P
        assert got in (f % Qk, (f - 1) % Qk)
        lows += got != f % Qk
    assert lows < n       # the correction is occasional, not systematic


def test_rescale_of_multiple_is_exact_and_small_cases():
    primes = prime_chain(4)
    n = 16
    g = np.random.Generator(np.random.PCG64(13))
    m = _coeff(g, primes[:-1], n)
    # c = q_last * m (coefficients given by their residues mod every prime)
    M = [_crt(m[:, k], primes[:-1]) for k in range(n)]
    c = np.array([[(primes[-1] * v) % q for v in M] for q in primes], dtype=np.uint64)
    out = CK.rescale(CK.ntt_rows(c, primes), primes, 1)
    assert np.array_equal(out, CK.ntt_rows(m, primes[:-1]))
    # zero stays zero; L = 2 leaves one limb
    z = np.zeros((2, n), dtype=np.uint64)
    assert not CK.rescale(z, primes[:2], 1).any()
    with pytest.raises(ValueError):
        CK.rescale(z, primes[:2], 2)


def test_he_add_is_limbwise_integer_sum():
    primes = prime_chain(3)
    g = np.random.Generator(np.random.PCG64(14))
    a = np.stack([_coeff(g, primes, 8) for _ in range(2)])
    b = np.stack([_coeff(g, primes, 8) for _ in range(2)])
    s = CK.he_add(a, b, primes)
    for c in range(2):
        for i, q in enumerate(primes):
            assert [int(v) for v in s[c, i]] == [(int(x) + int(y)) % q for x, y in zip(a[c, i], b[c, i])]
    neg = np.stack([np.stack([(np.uint64(q) - a[c, i]) % np.uint64(q) for i, q in enumerate(primes)])
                    for c in range(2)])
    assert not CK.he_add(a, neg, primes).any()
