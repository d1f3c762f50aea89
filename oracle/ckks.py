"""Hybrid key switching, HE-Mult, automorphism and rotation (oracle).

Test infrastructure: see ``oracle/__init__.py``.

The paper evaluates HE-Mult and Rotate with dnum-digit hybrid key switching
(Tab. perf_cmp, column "L, log2 q, Dnum"; Sec. Evaluation: BConv scales
polynomials up and down inside HE-Mult and Rotate; App. "Applying BAT to
preknown parameters": the evaluation-key inner product) but cites the key
switch rather than defining it.  The reading used here (G11, G13, G14):

  * digits: alpha = ceil(L / dnum); digit j holds limbs [j*alpha, min((j+1)*alpha, L));
    a digit with no limb is inactive and contributes zero;
  * ModUp(d): x = INTT(d); for each digit j and target t outside the digit,
    ext_j[t] = NTT_t(BConv_{D_j -> t}(x_{D_j})); for t inside the digit ext_j[t] = d[t];
  * inner product: acc_b[t] = sum_j ext_j[t] key_j.b[t], acc_a[t] likewise with key_j.a;
  * ModDown(acc): y = INTT_P(acc_P); z_i = NTT_{q_i}(BConv_{P -> q_i}(y));
    out_i = (acc_i - z_i) * P^-1 mod q_i;
  * HE-Mult (tensor product + relinearisation, no rescale):
    d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1; out = (d0 + ModDown(acc_b(d2)), d1 + ModDown(acc_a(d2)));
  * Rotate by r: g = 5^r mod 2N; c' = (sigma_g(c0), sigma_g(c1));
    out = (c0' + ModDown(acc_b(c1')), ModDown(acc_a(c1'))) with the key for g.

Ciphertexts and keys are in NTT form (bit-reversed evaluation order), limbs
ordered Q primes then P primes; key layout [dnum][2][L+K][N] with index 0 = b, 1 = a.
"""
from functools import lru_cache
from math import prod

import numpy as np

from .bconv import bconv_u64
from .ntt import bitrev, ntt_ct, intt_gs
from .primes import psi as _psi

U64 = np.uint64


@lru_cache(maxsize=None)
def psi_of(q: int, n: int) -> int:
    return _psi(q, n)


def ntt_rows(x, primes, inverse=False):
    x = np.asarray(x, dtype=U64)
    n = x.shape[-1]
    out = np.empty_like(x)
    for i, q in enumerate(primes):
        f = intt_gs if inverse else ntt_ct
        out[i] = f(x[i], q, psi_of(q, n))
    return out


def digits(L: int, dnum: int):
    alpha = -(-L // dnum)
    return [(j * alpha, min((j + 1) * alpha, L)) for j in range(dnum)], alpha


def modup(d, qs, ps, dnum):
    """[L][N] NTT form -> [dnum][L+K][N] NTT form."""
    d = np.asarray(d, dtype=U64)
    L, n = d.shape
    allp = list(qs) + list(ps)
    x = ntt_rows(d, qs, inverse=True)
    ext = np.zeros((dnum, len(allp), n), dtype=U64)
    ranges, _ = digits(L, dnum)
    for j, (lo, hi) in enumerate(ranges):
        if lo >= hi:
            continue
        src = list(qs[lo:hi])
        tgt = [t for t in range(len(allp)) if not lo <= t < hi]
        conv = bconv_u64(x[lo:hi], src, [allp[t] for t in tgt])
        ext[j, tgt] = ntt_rows(conv, [allp[t] for t in tgt])
        ext[j, lo:hi] = d[lo:hi]
    return ext


def inner_product(ext, key, primes):
    """acc[0] = sum_j ext_j * key_j.b, acc[1] = sum_j ext_j * key_j.a (mod each limb's prime)."""
    ext = np.asarray(ext, dtype=U64)
    key = np.asarray(key, dtype=U64)
    dnum, nl, n = ext.shape
    acc = np.zeros((2, nl, n), dtype=U64)
    for t, p in enumerate(primes):
        pp = U64(p)
        for j in range(dnum):
            for s in range(2):
                acc[s, t] = (acc[s, t] + ext[j, t] * key[j, s, t] % pp) % pp
    return acc


def moddown(acc, qs, ps):
    """[L+K][N] NTT form -> [L][N] NTT form, division by P = prod(ps)."""
    acc = np.asarray(acc, dtype=U64)
    L = len(qs)
    y = ntt_rows(acc[L:], ps, inverse=True)
    z = ntt_rows(bconv_u64(y, list(ps), list(qs)), qs)
    P = prod(ps)
    out = np.empty((L, acc.shape[1]), dtype=U64)
    for i, q in enumerate(qs):
        qq = U64(q)
        out[i] = ((acc[i] + qq - z[i]) % qq) * U64(pow(P % q, -1, q)) % qq
    return out


def he_add(a, b, qs):
    """HE-Add: limb-wise sum mod q_i of two polynomials or ciphertexts [..][L][N].

    The RNS isomorphism makes addition limb-wise (Sec. Background); the paper
    lists HE-Add among its four backbone operators (Sec. Evaluation, Tab.
    perf_cmp).  Valid in NTT and coefficient form alike.
    """
    a = np.asarray(a, dtype=U64)
    b = np.asarray(b, dtype=U64)
    out = np.empty_like(a)
    for i, q in enumerate(qs):
        out[..., i, :] = (a[..., i, :] + b[..., i, :]) % U64(q)
    return out


def rescale(c, qs, drop=1):
    """Rescale of one polynomial [L][N] (NTT form over qs) by the product P of its
    last `drop` primes -> [L - drop][N] over the first L - drop primes.

    The paper names Rescale as a backbone operator (Sec. Evaluation, Tab.
    perf_cmp) and drops two primes per level when a modulus needs more than
    32 bits (double rescaling, Sec. Evaluation "Security Parameter
    Selection"), but does not define it.  Reading G17: RNS rescaling is ModDown
    with the dropped primes in the role of P -- y = INTT_P(c_P);
    z_i = NTT_{q_i}(BConv_{P -> q_i}(y)); out_i = (c_i - z_i) P^-1 mod q_i -- with
    the fast (approximate) conversion and no rounding correction.  For drop = 1
    this is exactly floor(C / q_{L-1}) of each coefficient's CRT value C; for
    drop = 2 it is floor(C / P) or one less.
    """
    L = len(qs)
    if not 1 <= drop < L:
        raise ValueError("need 1 <= drop < L")
    return moddown(c, list(qs[:L - drop]), list(qs[L - drop:]))


def keyswitch(d, key, qs, ps, dnum):
    ext = modup(d, qs, ps, dnum)
    acc = inner_product(ext, key, list(qs) + list(ps))
    return moddown(acc[0], qs, ps), moddown(acc[1], qs, ps)


def tensor(a, b, qs):
    """d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1, limb-wise mod q_i (NTT form)."""
    a = np.asarray(a, dtype=U64)
    b = np.asarray(b, dtype=U64)
    d = np.empty((3,) + a.shape[1:], dtype=U64)
    for i, q in enumerate(qs):
        qq = U64(q)
        d[0, i] = a[0, i] * b[0, i] % qq
        d[1, i] = (a[0, i] * b[1, i] % qq + a[1, i] * b[0, i] % qq) % qq
        d[2, i] = a[1, i] * b[1, i] % qq
    return d


def he_mult(a, b, key, qs, ps, dnum):
    """One ciphertext pair [2][L][N] -> [2][L][N]."""
    d = tensor(a, b, qs)
    ks0, ks1 = keyswitch(d[2], key, qs, ps, dnum)
    out = np.empty((2,) + d.shape[1:], dtype=U64)
    for i, q in enumerate(qs):
        qq = U64(q)
        out[0, i] = (d[0, i] + ks0[i]) % qq
        out[1, i] = (d[1, i] + ks1[i]) % qq
    return out


def galois_element(r: int, n: int) -> int:
    """g = 5^r mod 2N (5 has order N/2 mod 2N, so r is taken mod N/2)."""
    return pow(5, r % (n // 2), 2 * n)


def automorphism_coeff(a, g: int, q: int) -> np.ndarray:
    """sigma_g(a)(x) = a(x^g) in coefficient form: x^i -> (-1)^floor(i g / N) x^(i g mod N)."""
    a = np.asarray(a, dtype=U64)
    n = a.shape[-1]
    out = np.zeros_like(a)
    for i in range(n):
        e = i * g % (2 * n)
        if e < n:
            out[..., e] = a[..., i]
        else:
            out[..., e - n] = (U64(q) - a[..., i]) % U64(q)
    return out


def automorphism_ntt(ahat, g: int) -> np.ndarray:
    """sigma_g in NTT form: slot p holds a(psi^(2 brv(p)+1)); sigma_g(a) there equals
    a(psi^((2 brv(p)+1) g)), which is slot brv(((2 brv(p)+1) g mod 2N - 1) / 2)."""
    ahat = np.asarray(ahat, dtype=U64)
    n = ahat.shape[-1]
    bits = n.bit_length() - 1
    idx = np.empty(n, dtype=np.int64)
    for p in range(n):
        e = (2 * bitrev(p, bits) + 1) * g % (2 * n)
        idx[p] = bitrev((e - 1) // 2, bits)
    return ahat[..., idx]


def rotate(ct, r: int, key, qs, ps, dnum):
    ct = np.asarray(ct, dtype=U64)
    n = ct.shape[-1]
    g = galois_element(r, n)
    c0 = automorphism_ntt(ct[0], g)
    c1 = automorphism_ntt(ct[1], g)
    ks0, ks1 = keyswitch(c1, key, qs, ps, dnum)
    out = np.empty_like(ct)
    for i, q in enumerate(qs):
        qq = U64(q)
        out[0, i] = (c0[i] + ks0[i]) % qq
        out[1, i] = ks1[i]
    return out
