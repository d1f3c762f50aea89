"""Primes, generators and 2N-th roots of unity (oracle).

Test infrastructure: see ``oracle/__init__.py``.

Paper: Sec. II-A (ring R_Q = Z_Q[x]/(x^N+1), RNS bases q_i of ~28 bits,
Tab. Notation).  The paper does not fix the primes or the root; the readings
used here are the largest primes below 2^28 that are 1 mod 2^17 (below 2^31
for the NTT's wide form: ``prime_chain(count, bits=31)``) and psi from the
smallest generator.
"""


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin; bases {2, 7, 61} are exact for n < 4,759,123,141."""
    if n < 2:
        return False
    for p in (2, 3, 5, 7, 11, 13, 61):
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    assert n < 4_759_123_141
    for a in (2, 7, 61):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def prime_chain(count: int, bits: int = 28, two_adicity: int = 17):
    """The first ``count`` primes q < 2**bits with q = 1 (mod 2**two_adicity), largest first.

    q = 1 mod 2^17 makes every q usable for every N <= 2^16 (q = 1 mod 2N).
    """
    step = 1 << two_adicity
    m = ((1 << bits) - 2) // step
    out = []
    while len(out) < count and m > 0:
        q = m * step + 1
        if is_prime(q):
            out.append(q)
        m -= 1
    if len(out) < count:
        raise ValueError("not enough primes")
    return out


def factorize(n: int):
    """Distinct prime factors by trial division (n < 2^32 here)."""
    fs, p = [], 2
    while p * p <= n:
        if n % p == 0:
            fs.append(p)
            while n % p == 0:
                n //= p
        p += 1
    if n > 1:
        fs.append(n)
    return fs


def smallest_generator(q: int) -> int:
    """Smallest g that generates Z_q^* (g^((q-1)/f) != 1 for every prime f | q-1)."""
    fs = factorize(q - 1)
    g = 2
    while True:
        if all(pow(g, (q - 1) // f, q) != 1 for f in fs):
            return g
        g += 1


def psi(q: int, n: int) -> int:
    """Canonical primitive 2n-th root of unity mod q: psi = g^((q-1)/(2n)), g smallest generator.

    It satisfies psi^n = -1 (mod q), which is what makes the transform negacyclic
    (evaluation at the roots of x^n + 1).
    """
    if (q - 1) % (2 * n):
        raise ValueError("q != 1 mod 2n")
    g = smallest_generator(q)
    r = pow(g, (q - 1) // (2 * n), q)
    assert pow(r, n, q) == q - 1
    return r
