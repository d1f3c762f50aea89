"""Seeded synthetic inputs shared by the tests, the bench and the oracle timing.

This module draws random residues and lists the workload shapes; it holds none
of the transform arithmetic.  The prime list is found here by plain trial
division (independently of both the oracle and the library, which each check
primes their own way).

Workload shapes follow the paper's parameter sets (Tab. ntt_throughput_setup:
28-bit RNS primes, N up to 2^16) and the hot-path configurations:

  C1  N = 4096, one prime, batch 1                       (NTT, INTT, polymul)
  C2  N = 2^16 as 256 x 256, L = 24, 8 ct x 2 polys        (batched NTT / INTT)
  C3  N = 2^16, L = 24, dnum = 3, 8 special primes         (HE-Mult + relin)
  C4  64 ciphertexts, N in {2^13..2^16}, L in [4, 36]     (uneven batch)
  C5  Poisson arrivals of HE-Mult / Rotate requests        (request loop)

Residues are uniform in [0, q_i), drawn limb by limb in (ct, poly, limb) order
from numpy's PCG64 seeded generator; keys come from seed + 1000.
"""
import numpy as np

BITS = 28
TWO_ADICITY = 17


def _is_prime_trial(n: int) -> bool:
    if n < 2:
        return False
    if n % 2 == 0:
        return n == 2
    d = 3
    while d * d <= n:
        if n % d == 0:
            return False
        d += 2
    return True


_CHAIN = None


def primes(count: int):
    """Largest ``count`` primes q < 2^28 with q = 1 mod 2^17, largest first."""
    global _CHAIN
    if _CHAIN is None or len(_CHAIN) < count:
        step = 1 << TWO_ADICITY
        m = ((1 << BITS) - 2) // step
        out = []
        while len(out) < max(count, 48) and m > 0:
            q = m * step + 1
            if _is_prime_trial(q):
                out.append(q)
            m -= 1
        _CHAIN = out
    return list(_CHAIN[:count])


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def residues(gen: np.random.Generator, lead_shape, plist, n: int) -> np.ndarray:
    """uint32 array of shape lead_shape + [len(plist), n]; limb i uniform in [0, plist[i])."""
    lead_shape = tuple(lead_shape)
    out = np.empty(lead_shape + (len(plist), n), dtype=np.uint32)
    for idx in np.ndindex(*lead_shape) if lead_shape else [()]:
        for i, q in enumerate(plist):
            out[idx + (i,)] = gen.integers(0, q, n, dtype=np.uint32)
    return out


def ntt_batch(seed: int, log_n: int, L: int, batch: int):
    """[batch][L][N] residues over the first L chain primes."""
    p = primes(L)
    return p, residues(rng(seed), (batch,), p, 1 << log_n)


def ckks_params(L: int, dnum: int, ksp: int = None):
    alpha = -(-L // dnum)
    ksp = alpha if ksp is None else ksp
    p = primes(L + ksp)
    return p[:L], p[L:], alpha


def ckks_pair(seed: int, log_n: int, L: int, dnum: int, ksp: int = None, batch: int = 1):
    """Two ciphertext batches [batch][2][L][N] and a key [dnum][2][L+K][N], uniform residues."""
    qs, ps, _ = ckks_params(L, dnum, ksp)
    n = 1 << log_n
    g = rng(seed)
    a = residues(g, (batch, 2), qs, n)
    b = residues(g, (batch, 2), qs, n)
    key = residues(rng(seed + 1000), (dnum, 2), qs + ps, n)
    return qs, ps, a, b, key


def uneven_jobs(seed: int, count: int = 64):
    """Config C4 job list: (op, log_n, L), op 'he_mult' with p = 0.5 else 'ntt'."""
    g = rng(seed)
    jobs = []
    for _ in range(count):
        log_n = int(g.integers(13, 17))
        L = int(g.integers(4, 37))
        op = "he_mult" if g.random() < 0.5 else "ntt"
        jobs.append((op, log_n, L))
    return jobs
