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


_WIDE = None


def wide_primes(count: int):
    """Largest ``count`` primes q < 2^31 with q = 1 mod 2^17, largest first (the NTT's
    wide form: residues that do not fit four 7-bit chunks)."""
    global _WIDE
    if _WIDE is None or len(_WIDE) < count:
        step = 1 << TWO_ADICITY
        m = ((1 << 31) - 2) // step
        out = []
        while len(out) < max(count, 8) and m > 0:
            q = m * step + 1
            if _is_prime_trial(q):
                out.append(q)
            m -= 1
        _WIDE = out
    return list(_WIDE[:count])


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


def poisson_requests(seed: int, count: int, rate: float, log_ns=(14, 15, 16), L_range=(8, 36),
                     p_mult: float = 0.5, rot_steps=(1, 2, 4, 8, 16, 32, 64)):
    """Request-loop workload (C5): arrival times of a Poisson process with `rate`
    requests/s, op HE-Mult with probability p_mult else Rotate by a step from
    rot_steps, N drawn from log_ns, L uniform in L_range (inclusive)."""
    g = rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += float(g.exponential(1.0 / rate)) if rate > 0 else 0.0
        log_n = int(g.choice(log_ns))
        L = int(g.integers(L_range[0], L_range[1] + 1))
        op = "he_mult" if g.random() < p_mult else "rotate"
        steps = int(g.choice(rot_steps))
        out.append({"rid": i, "arrival": t, "op": op, "log_n": log_n, "L": L, "steps": steps})
    return out


def device_residues(seed: int, batch: int, plist, n: int):
    """int32 CUDA tensor [batch][len(plist)][n], limb i uniform in [0, plist[i]) from a
    seeded torch generator on the GPU (for inputs too large to draw on the host)."""
    import torch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed & 0x7FFFFFFF)
    out = torch.empty((batch, len(plist), n), dtype=torch.int32, device="cuda")
    for i, q in enumerate(plist):
        out[:, i, :] = torch.randint(0, q, (batch, n), generator=gen, device="cuda", dtype=torch.int64).to(torch.int32)
    return out


class DevicePool:
    """Seeded synthetic ciphertexts and keys generated on the GPU, per parameter set.

    For each (log_n, L) a few ciphertext pairs and one key per kind ('relin' or a
    rotation step) are drawn uniformly per limb in [0, q_i) with a seeded torch
    generator; requests reference them, so a long request stream does not hold
    one fresh key per request.
    """

    def __init__(self, seed: int, dnum: int = 3, variants: int = 2):
        self.seed, self.dnum, self.variants = seed, dnum, variants
        self.cts, self.keys = {}, {}

    def _uniform(self, shape, plist, n, salt):
        import torch
        gen = torch.Generator(device="cuda")
        gen.manual_seed((self.seed * 1000003 + salt) & 0x7FFFFFFF)
        rows = []
        for idx in np.ndindex(*shape):
            for q in plist:
                rows.append(torch.randint(0, q, (n,), generator=gen, device="cuda", dtype=torch.int64))
        return torch.stack(rows).to(torch.int32).reshape(tuple(shape) + (len(plist), n))

    def params(self, L):
        return ckks_params(L, self.dnum)

    def ciphertexts(self, log_n, L, variant):
        key = (log_n, L, variant % self.variants)
        if key not in self.cts:
            qs, _, _ = self.params(L)
            salt = (log_n * 64 + L) * 16 + key[2] * 2
            self.cts[key] = (self._uniform((2,), qs, 1 << log_n, salt),
                             self._uniform((2,), qs, 1 << log_n, salt + 1))
        return self.cts[key]

    def key(self, log_n, L, kind):
        k = (log_n, L, kind)
        if k not in self.keys:
            qs, ps, _ = self.params(L)
            kid = 0 if kind == "relin" else 1 + int(kind[1])
            self.keys[k] = self._uniform((self.dnum, 2), qs + ps, 1 << log_n, 100000 + (log_n * 64 + L) * 128 + kid)
        return self.keys[k]
