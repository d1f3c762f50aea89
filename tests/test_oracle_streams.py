"""Pins of the chunked stream forms in oracle/streams.py (evaluation-key BAT and
the chunk-wise convolution product) against exact integer arithmetic and the
plain definitions of the key-switch inner product and the tensor product."""
import numpy as np
import pytest

from oracle import ckks as CK
from oracle import streams as S
from oracle.primes import prime_chain

U64 = np.uint64
EDGES32 = [0, 1, 2, 255, 256, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFF]


def test_conv_product_is_the_exact_product():
    g = np.random.default_rng(5)
    a = np.array(EDGES32 + list(g.integers(0, 1 << 32, 500, dtype=np.uint64)), dtype=U64)
    b = np.array(EDGES32[::-1] + list(g.integers(0, 1 << 32, 500, dtype=np.uint64)), dtype=U64)
    got = S.conv_product(a, b)
    assert [int(x) for x in got] == [int(x) * int(y) for x, y in zip(a, b)]


def test_chunk_conv_partial_sums():
    # seven partial sums, each at most 4 * 255^2 < 2^18; the outermost are single products
    a, b = np.array([0xFFFFFFFF, 0x01020304], dtype=U64), np.array([0xFFFFFFFF, 0x0A0B0C0D], dtype=U64)
    ps = S.chunk_conv(a, b)
    assert ps.shape == (7, 2)
    assert int(ps.max()) == 4 * 255 * 255 < 1 << 18
    assert int(ps[0, 1]) == 0x04 * 0x0D and int(ps[6, 1]) == 0x01 * 0x0A
    assert int(ps[3, 1]) == 0x04 * 0x0A + 0x03 * 0x0B + 0x02 * 0x0C + 0x01 * 0x0D


def test_evk_bat_expansion_identity():
    # sum_l 2^(8l) sum_i E[l][i] e_i == 2^32 k e (mod p), brute force in Python integers
    p = prime_chain(2)[1]
    g = np.random.default_rng(6)
    ks = [0, 1, p - 1] + [int(x) for x in g.integers(0, p, 40)]
    es = [0, 1, p - 1] + [int(x) for x in g.integers(0, p, 40)]
    E = S.evk_bat_expand(np.array(ks, dtype=U64), p)
    assert int(E.max()) <= 255
    for idx, k in enumerate(ks):
        for e in es:
            eb = [(e >> (8 * i)) & 0xFF for i in range(4)]
            v = sum((sum(int(E[idx, l, i]) * eb[i] for i in range(4))) << (8 * l) for l in range(4))
            assert v % p == (k * e << 32) % p
            assert v < p << 32


def test_redc_and_barrett_against_python():
    p = prime_chain(1)[0]
    g = np.random.default_rng(7)
    v = np.array([0, 1, (p << 32) - 1] + [int(x) for x in g.integers(0, p << 32, 300, dtype=np.uint64)], dtype=U64)
    rinv = pow(2, -32, p)
    assert [int(x) for x in S.redc(v, p)] == [int(x) * rinv % p for x in v]
    z = np.array([0, p - 1, p, p * p - 1] + [int(x) for x in g.integers(0, p * p, 300, dtype=np.uint64)], dtype=U64)
    assert [int(x) for x in S.barrett_reduce(z, p)] == [int(x) % p for x in z]


def _rand(g, qs, *lead, n=64):
    return np.stack([np.stack([g.integers(0, q, n) for q in qs], axis=-2) for _ in range(int(np.prod(lead)))]
                    ).reshape(*lead, len(qs), n).astype(U64)


@pytest.mark.parametrize("dnum", [1, 3, 4])
def test_evk_bat_inner_product_equals_definition(dnum):
    qs = prime_chain(5)
    g = np.random.default_rng(10 + dnum)
    ext = _rand(g, qs, dnum)
    key = _rand(g, qs, dnum, 2)
    ext[:, :, 0] = [q - 1 for q in qs]             # extreme residues in the first slot
    key[:, :, :, 0] = [q - 1 for q in qs]
    got = S.inner_product_evk_bat(ext, key, qs)
    assert np.array_equal(got, CK.inner_product(ext, key, qs))
    # brute force on a few slots
    for t, p in enumerate(qs):
        for n in (0, 7, 63):
            for s in range(2):
                assert int(got[s, t, n]) == sum(int(ext[j, t, n]) * int(key[j, s, t, n]) for j in range(dnum)) % p


def test_tensor_conv_equals_definition():
    qs = prime_chain(4)
    g = np.random.default_rng(21)
    a, b = _rand(g, qs, 2), _rand(g, qs, 2)
    a[:, :, 0] = b[:, :, 0] = [q - 1 for q in qs]
    assert np.array_equal(S.tensor_conv(a, b, qs), CK.tensor(a, b, qs))
