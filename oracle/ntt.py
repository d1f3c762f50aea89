"""Negacyclic NTT / INTT (oracle).

Test infrastructure: see ``oracle/__init__.py``.

Definition (Sec. II-A ring R_q = Z_q[x]/(x^N+1); App. "Radix-2 Cooley-Tukey NTT";
Sec. MAT "layout invariant 3-step negacyclic NTT", whose output is stated to be
directly in bit-reversed order): the forward transform evaluates a(x) at the N
roots of x^N + 1, which are psi^(odd), and stores them in bit-reversed order,

    ntt(a)[p] = a(psi^(2*brv_N(p) + 1)) = sum_n a_n psi^((2 brv_N(p)+1) n)  (mod q).

The paper does not spell the position map out; this reading (G2) is the standard
one produced by a Cooley-Tukey negacyclic butterfly network fed with bit-reversed
powers of psi, so the butterfly baseline and the 3-step form agree bit for bit.
"""
from functools import lru_cache

import numpy as np

U64 = np.uint64


def bitrev(i: int, bits: int) -> int:
    r = 0
    for _ in range(bits):
        r = (r << 1) | (i & 1)
        i >>= 1
    return r


@lru_cache(maxsize=32)
def bitrev_table(n: int) -> np.ndarray:
    bits = n.bit_length() - 1
    out = np.array([bitrev(i, bits) for i in range(n)], dtype=np.int64)
    out.setflags(write=False)
    return out


@lru_cache(maxsize=256)
def rev_powers(base: int, n: int, q: int) -> np.ndarray:
    """[base^brv_N(k) mod q for k < N] -- the butterfly twiddles of ``ntt_ct`` /
    ``intt_gs``.  Kept per (base, N, q) because every limb of a prime reuses it; the
    array is read-only."""
    out = _powers(base, n, q)[bitrev_table(n)]
    out.setflags(write=False)
    return out


def _powers(base: int, count: int, q: int) -> np.ndarray:
    out = np.empty(count, dtype=U64)
    x = 1
    for e in range(count):
        out[e] = x
        x = x * base % q
    return out


def ntt_def(a, q: int, psi: int) -> np.ndarray:
    """O(N^2) definition: out[p] = sum_n a_n psi^((2 brv(p)+1) n mod 2N) mod q.

    ``a`` is one polynomial (length N, residues in [0, q)).
    """
    a = np.asarray(a, dtype=U64)
    n = a.shape[-1]
    pw = _powers(psi, 2 * n, q)          # psi^e, e in [0, 2N)
    e_p = 2 * bitrev_table(n) + 1        # odd exponents, one per output position
    nn = np.arange(n, dtype=np.int64)
    out = np.empty(n, dtype=U64)
    for p0 in range(0, n, 256):
        rows = slice(p0, min(n, p0 + 256))
        expo = (e_p[rows, None] * nn[None, :]) % (2 * n)
        terms = (a[None, :] * pw[expo]) % U64(q)   # each term < q
        out[rows] = terms.sum(axis=1, dtype=U64) % U64(q)
    return out


def intt_def(ahat, q: int, psi: int) -> np.ndarray:
    """Inverse of ``ntt_def``: a_n = N^-1 sum_p ahat_p psi^(-(2 brv(p)+1) n) mod q."""
    ahat = np.asarray(ahat, dtype=U64)
    n = ahat.shape[-1]
    pw = _powers(pow(psi, -1, q), 2 * n, q)
    e_p = 2 * bitrev_table(n) + 1
    pp = np.arange(n)
    out = np.empty(n, dtype=U64)
    ninv = pow(n, -1, q)
    for n0 in range(0, n, 256):
        cols = np.arange(n0, min(n, n0 + 256))
        expo = (cols[:, None] * e_p[None, pp]) % (2 * n)
        terms = (ahat[None, :] * pw[expo]) % U64(q)
        s = terms.sum(axis=1, dtype=U64) % U64(q)
        out[cols] = (s * U64(ninv)) % U64(q)
    return out


def horner_eval(a, q: int, xs) -> np.ndarray:
    """Evaluate polynomial ``a`` (coefficients a_0..a_{N-1}) at each x in ``xs`` mod q by Horner's rule."""
    a = np.asarray(a, dtype=U64)
    xs = np.asarray(xs, dtype=U64)
    acc = np.zeros_like(xs)
    for coeff in a[::-1]:
        acc = (acc * xs + coeff) % U64(q)
    return acc


def ntt_ct(a, q: int, psi: int) -> np.ndarray:
    """Textbook iterative Cooley-Tukey negacyclic NTT (natural order in, bit-reversed out).

    Stage with m butterfly groups of half-width t: for group i the twiddle is
    psi^brv_N(m+i); (U, V) -> (U + V*w, U - V*w).  Works on the last axis of an
    array of any leading shape (a batch of limbs of one prime).  This is the bulk
    oracle for N > 4096; it is checked against ``ntt_def``.
    """
    x = np.array(a, dtype=U64, copy=True)
    n = x.shape[-1]
    lead = x.shape[:-1]
    psi_rev = rev_powers(psi, n, q)
    qq = U64(q)
    m, t = 1, n
    while m < n:
        t //= 2
        v = x.reshape(lead + (m, 2, t))
        w = psi_rev[m:2 * m].reshape((1,) * len(lead) + (m, 1))
        u = v[..., 0, :].copy()
        vw = (v[..., 1, :] * w) % qq
        v[..., 0, :] = (u + vw) % qq
        v[..., 1, :] = (u + qq - vw) % qq
        m *= 2
    return x


def intt_gs(ahat, q: int, psi: int) -> np.ndarray:
    """Textbook Gentleman-Sande inverse of ``ntt_ct`` (bit-reversed in, natural out), times N^-1."""
    x = np.array(ahat, dtype=U64, copy=True)
    n = x.shape[-1]
    lead = x.shape[:-1]
    ipsi_rev = rev_powers(pow(psi, -1, q), n, q)
    qq = U64(q)
    m, t = n // 2, 1
    while m >= 1:
        v = x.reshape(lead + (m, 2, t))
        w = ipsi_rev[m:2 * m].reshape((1,) * len(lead) + (m, 1))
        u = v[..., 0, :].copy()
        s = v[..., 1, :].copy()
        v[..., 0, :] = (u + s) % qq
        v[..., 1, :] = ((u + qq - s) % qq * w) % qq
        t *= 2
        m //= 2
    return (x * U64(pow(n, -1, q))) % qq


def ntt_limbs(x, primes, psis, inverse=False) -> np.ndarray:
    """Apply ``ntt_ct`` (or ``intt_gs``) limb by limb: x has shape [..., L, N]."""
    x = np.asarray(x, dtype=U64)
    out = np.empty_like(x)
    f = intt_gs if inverse else ntt_ct
    for i, (q, p) in enumerate(zip(primes, psis)):
        out[..., i, :] = f(x[..., i, :], q, p)
    return out
