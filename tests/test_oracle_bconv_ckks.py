"""Pins for oracle/bconv.py and oracle/ckks.py (App. BConv; hybrid key switching,
HE-Mult, automorphism, rotation as read in the oracle's module docstring)."""
from math import prod

import numpy as np
import pytest

from oracle import bconv as BC
from oracle import ckks as CK
from oracle.ntt import ntt_ct, intt_gs
from oracle.primes import prime_chain, psi as psi_of


def test_bconv_y_is_crt_lift_plus_small_multiple():
    src = prime_chain(5)
    Q = prod(src)
    g = np.random.Generator(np.random.PCG64(1))
    for _ in range(200):
        v = int(g.integers(0, 1 << 62)) * int(g.integers(0, 1 << 62)) * int(g.integers(0, 1 << 20)) % Q
        col = [v % q for q in src]
        y = BC.bconv_y(col, src)
        for q, a in zip(src, col):
            assert y % q == a
        assert 0 <= y < len(src) * Q
        assert (y - v) % Q == 0 and 0 <= (y - v) // Q < len(src)


def test_bconv_u64_equals_bigint():
    src = prime_chain(8)[:4]
    dst = prime_chain(8)[4:] + prime_chain(10)[8:]
    g = np.random.Generator(np.random.PCG64(2))
    a = np.stack([g.integers(0, q, 64) for q in src])
    a[:, 0] = 0
    a[:, 1] = [q - 1 for q in src]
    assert np.array_equal(BC.bconv_u64(a, src, dst), BC.bconv_bigint(a, src, dst))


def test_bconv_u64_equals_bigint_wide_primes():
    # primes in [2^30, 2^31): products of two residues stay below 2^62, so the uint64
    # form is still exact; the lift y is still a CRT lift plus a small multiple of Q
    import synthetic
    wp = synthetic.wide_primes(7)
    src, dst = wp[:3], wp[3:] + prime_chain(2)
    g = np.random.Generator(np.random.PCG64(3))
    a = np.stack([g.integers(0, q, 32) for q in src])
    a[:, 0] = [q - 1 for q in src]
    a[:, 1] = 0
    assert np.array_equal(BC.bconv_u64(a, src, dst), BC.bconv_bigint(a, src, dst))
    Q = prod(src)
    for n in range(a.shape[1]):
        col = [int(v) for v in a[:, n]]
        y = BC.bconv_y(col, src)
        assert all(y % q == c for q, c in zip(src, col)) and 0 <= y < len(src) * Q


def test_bconv_single_source_is_reduction():
    # |S| = 1: qhat = 1, so the conversion is plain reduction of a into each target
    src = [prime_chain(1)[0]]
    dst = prime_chain(4)[1:]
    a = np.array([[0, 1, 5, src[0] - 1]], dtype=np.uint64)
    out = BC.bconv_u64(a, src, dst)
    for j, p in enumerate(dst):
        assert list(out[j]) == [int(v) % p for v in a[0]]


def _ntt(x, primes):
    return CK.ntt_rows(x, primes)


def _intt(x, primes):
    return CK.ntt_rows(x, primes, inverse=True)


def test_moddown_of_p_times_m_is_m():
    n = 64
    qs = prime_chain(7)[:4]
    ps = prime_chain(7)[4:]
    P = prod(ps)
    g = np.random.Generator(np.random.PCG64(4))
    m = np.stack([g.integers(0, q, n) for q in qs]).astype(np.uint64)
    acc_coeff = np.zeros((7, n), dtype=np.uint64)
    for i, q in enumerate(qs):
        acc_coeff[i] = m[i] * np.uint64(P % q) % np.uint64(q)
    acc = _ntt(acc_coeff, qs + ps)
    out = CK.moddown(acc, qs, ps)
    assert np.array_equal(out, _ntt(m, qs))


def test_digits():
    assert CK.digits(24, 3) == ([(0, 8), (8, 16), (16, 24)], 8)
    assert CK.digits(4, 3) == ([(0, 2), (2, 4), (4, 4)], 2)
    assert CK.digits(7, 3) == ([(0, 3), (3, 6), (6, 7)], 3)


def test_automorphism_coeff_is_substitution():
    n, q = 16, prime_chain(1)[0]
    g = np.random.Generator(np.random.PCG64(8))
    a = g.integers(0, q, n)
    for gal in (3, 5, 25, 2 * n - 1):
        out = CK.automorphism_coeff(a, gal, q)
        # independent: a(x^g) as an integer polynomial of degree (n-1) g, folded by x^N = -1
        ref = [0] * n
        for i, c in enumerate(a):
            e = i * gal
            sign = -1 if (e // n) % 2 else 1
            ref[e % n] = (ref[e % n] + sign * int(c)) % q
        assert list(out) == ref


def test_automorphism_ntt_matches_coefficient_form_and_composes():
    n = 64
    q = prime_chain(1)[0]
    psi = psi_of(q, n)
    g = np.random.Generator(np.random.PCG64(9))
    a = g.integers(0, q, n).astype(np.uint64)
    ah = ntt_ct(a, q, psi)
    for r in (1, 2, 5, -1, 31):
        gal = CK.galois_element(r, n)
        assert gal % 2 == 1
        assert np.array_equal(CK.automorphism_ntt(ah, gal), ntt_ct(CK.automorphism_coeff(a, gal, q), q, psi))
    g1, g2 = CK.galois_element(3, n), CK.galois_element(7, n)
    comp = CK.automorphism_ntt(CK.automorphism_ntt(ah, g1), g2)
    assert np.array_equal(comp, CK.automorphism_ntt(ah, g1 * g2 % (2 * n)))
    assert CK.galois_element(n // 2, n) == 1


# ---- semantic pins with real RLWE keys: a mistake anywhere in ModUp / inner
# ---- product / ModDown (digit ranges, P factor, BConv constants, signs) turns
# ---- the small decryption error into a uniformly random element mod Q.

def _small(g, shape, bound):
    return g.integers(-bound, bound + 1, shape)


def _to_rns(v, primes):
    return np.stack([np.mod(v, q) for q in primes]).astype(np.uint64)


def _ksk(g, s_ntt, s_target_ntt, qs, ps, dnum, n):
    allp = qs + ps
    P = prod(ps)
    ranges, _ = CK.digits(len(qs), dnum)
    key = np.zeros((dnum, 2, len(allp), n), dtype=np.uint64)
    for j, (lo, hi) in enumerate(ranges):
        a = np.stack([g.integers(0, p, n) for p in allp]).astype(np.uint64)
        e = _ntt(_to_rns(_small(g, n, 3), allp), allp)
        for t, p in enumerate(allp):
            pp = np.uint64(p)
            b = (pp - a[t] * s_ntt[t] % pp + e[t]) % pp
            if lo <= t < hi:
                b = (b + np.uint64(P % p) * s_target_ntt[t] % pp) % pp
            key[j, 0, t] = b
            key[j, 1, t] = a[t]
    return key


def _centered_max(x_ntt, qs):
    coeff = _intt(x_ntt, qs)
    Q = prod(qs)
    worst = 0
    for col in range(coeff.shape[1]):
        # CRT reconstruction in Python integers
        v = 0
        for i, q in enumerate(qs):
            h = Q // q
            v += int(coeff[i, col]) * pow(h % q, -1, q) * h
        v %= Q
        if v > Q // 2:
            v -= Q
        worst = max(worst, abs(v))
    return worst


@pytest.mark.parametrize("L,dnum", [(6, 3), (5, 3), (4, 3), (4, 1), (6, 2)])
def test_keyswitch_semantics_with_real_keys(L, dnum):
    n = 64
    _, alpha = CK.digits(L, dnum)
    chain = prime_chain(L + alpha)
    qs, ps = chain[:L], chain[L:]
    allp = qs + ps
    g = np.random.Generator(np.random.PCG64(L * 10 + dnum))
    s = _small(g, n, 1)
    s_ntt = _ntt(_to_rns(s, allp), allp)
    s2_ntt = np.stack([s_ntt[t] * s_ntt[t] % np.uint64(p) for t, p in enumerate(allp)])
    key = _ksk(g, s_ntt, s2_ntt, qs, ps, dnum, n)
    d = np.stack([g.integers(0, q, n) for q in qs]).astype(np.uint64)
    ks0, ks1 = CK.keyswitch(d, key, qs, ps, dnum)
    diff = np.empty_like(ks0)
    for i, q in enumerate(qs):
        qq = np.uint64(q)
        diff[i] = (ks0[i] + ks1[i] * s_ntt[i] % qq + qq - d[i] * s2_ntt[i] % qq) % qq
    assert _centered_max(diff, qs) < 1 << 24          # versus Q ~ 2^(28 L)


@pytest.mark.parametrize("wide", [False, True])
def test_he_mult_and_rotate_decrypt_correctly(wide):
    # wide: primes in [2^30, 2^31) (the byte forms of the library); the oracle's
    # products of two residues stay below 2^62, so it is exact there too
    import synthetic
    n, L, dnum = 64, 6, 3
    _, alpha = CK.digits(L, dnum)
    chain = synthetic.wide_primes(L + alpha) if wide else prime_chain(L + alpha)
    qs, ps = chain[:L], chain[L:]
    allp = qs + ps
    g = np.random.Generator(np.random.PCG64(77))
    s = _small(g, n, 1)
    s_ntt = _ntt(_to_rns(s, allp), allp)
    s2_ntt = np.stack([s_ntt[t] * s_ntt[t] % np.uint64(p) for t, p in enumerate(allp)])
    relin = _ksk(g, s_ntt, s2_ntt, qs, ps, dnum, n)

    def enc():
        c1 = np.stack([g.integers(0, q, n) for q in qs]).astype(np.uint64)
        m = _ntt(_to_rns(_small(g, n, 1000), qs), qs)
        c0 = np.stack([(m[i] + np.uint64(q) - c1[i] * s_ntt[i] % np.uint64(q)) % np.uint64(q)
                       for i, q in enumerate(qs)])
        return np.stack([c0, c1]), m

    ca, ma = enc()
    cb, mb = enc()
    out = CK.he_mult(ca, cb, relin, qs, ps, dnum)
    diff = np.empty((L, n), dtype=np.uint64)
    for i, q in enumerate(qs):
        qq = np.uint64(q)
        dec = (out[0, i] + out[1, i] * s_ntt[i] % qq) % qq
        diff[i] = (dec + qq - ma[i] * mb[i] % qq) % qq
    assert _centered_max(diff, qs) < 1 << 24

    r = 3
    gal = CK.galois_element(r, n)
    srot_ntt = np.stack([CK.automorphism_ntt(s_ntt[t], gal) for t in range(len(allp))])
    rkey = _ksk(g, s_ntt, srot_ntt, qs, ps, dnum, n)
    rot = CK.rotate(ca, r, rkey, qs, ps, dnum)
    diff = np.empty((L, n), dtype=np.uint64)
    for i, q in enumerate(qs):
        qq = np.uint64(q)
        dec = (rot[0, i] + rot[1, i] * s_ntt[i] % qq) % qq
        diff[i] = (dec + qq - CK.automorphism_ntt(ma[i], gal)) % qq
    assert _centered_max(diff, qs) < 1 << 24
