"""Pins for oracle/ntt.py, oracle/poly.py and oracle/mat.py.

The paper prints no numeric NTT example, so the oracle is pinned to what the
mathematics fixes: a hand-worked 4-point case, brute-force root sets and
Horner evaluation on small primes, closed forms (delta, constants, the
monomial x), the convolution theorem against an independently written
polynomial product, and inverse/round-trip identities.
"""
import numpy as np
import pytest

from oracle import ntt as T
from oracle import poly as PL
from oracle import mat as M
from oracle.primes import psi as psi_of, prime_chain

Q0 = 268042241


def _rev_str(i, bits):
    # bit reversal written independently of oracle.ntt.bitrev
    return int(format(i, "0%db" % bits)[::-1], 2) if bits else 0


def _polymul_mod_xn1(a, b, q):
    # independent negacyclic product: full integer product, then fold x^N = -1
    n = len(a)
    full = [0] * (2 * n)
    for i, ai in enumerate(a):
        for j, bj in enumerate(b):
            full[i + j] += int(ai) * int(bj)
    return [(full[k] - full[k + n]) % q for k in range(n)]


def test_hand_worked_n4_q17():
    # q = 17, N = 4: generator 3, psi = 3^(16/8) = 9 (9^4 = 16 = -1 mod 17).
    # Slots p = 0..3 evaluate at psi^(2 brv(p)+1) = psi^1, psi^5, psi^3, psi^7 = 9, 8, 15, 2.
    # a = 1 + 2x + 3x^2 + 4x^3:  a(9) = 3178 = 16, a(8) = 2257 = 13, a(15) = 14206 = 11, a(2) = 49 = 15.
    assert psi_of(17, 4) == 9
    out = T.ntt_def([1, 2, 3, 4], 17, 9)
    assert list(out) == [16, 13, 11, 15]
    assert list(T.ntt_ct([1, 2, 3, 4], 17, 9)) == [16, 13, 11, 15]
    assert list(T.intt_def(out, 17, 9)) == [1, 2, 3, 4]


@pytest.mark.parametrize("q,log_n", [(97, 4), (193, 5), (257, 6), (7681, 6), (Q0, 6)])
def test_brute_force_roots_and_positions(q, log_n):
    n = 1 << log_n
    psi = psi_of(q, n)
    x_p = T.ntt_def([0, 1] + [0] * (n - 2), q, psi)         # NTT of the monomial x
    if q < 100000:
        roots = {x for x in range(1, q) if pow(x, n, q) == q - 1}   # brute force
        assert len(roots) == n
        assert set(int(v) for v in x_p) == roots
    for p in range(n):
        assert pow(int(x_p[p]), n, q) == q - 1
        assert int(x_p[p]) == pow(psi, 2 * _rev_str(p, log_n) + 1, q)
    g = np.random.Generator(np.random.PCG64(log_n))
    for _ in range(3):
        a = g.integers(0, q, n)
        out = T.ntt_def(a, q, psi)
        for p in range(n):
            acc = 0
            for c in reversed(a):             # Horner in Python integers
                acc = (acc * int(x_p[p]) + int(c)) % q
            assert int(out[p]) == acc


@pytest.mark.parametrize("log_n", [4, 6, 8, 10])
def test_closed_forms(log_n):
    n = 1 << log_n
    q = Q0
    psi = psi_of(q, n)
    delta = [1] + [0] * (n - 1)
    assert all(v == 1 for v in T.ntt_def(delta, q, psi))
    assert all(v == 12345 for v in T.ntt_def([12345] + [0] * (n - 1), q, psi))
    g = np.random.Generator(np.random.PCG64(1))
    a = g.integers(0, q, n)
    b = g.integers(0, q, n)
    s = (a + b) % q
    assert np.array_equal(T.ntt_def(s, q, psi), (T.ntt_def(a, q, psi) + T.ntt_def(b, q, psi)) % q)


@pytest.mark.parametrize("log_n", [2, 3, 5, 7])
def test_convolution_theorem_vs_independent_product(log_n):
    n = 1 << log_n
    q = Q0
    psi = psi_of(q, n)
    g = np.random.Generator(np.random.PCG64(log_n + 10))
    a = g.integers(0, q, n)
    b = g.integers(0, q, n)
    ref = _polymul_mod_xn1(a, b, q)
    assert list(PL.negacyclic_mul(a, b, q)) == ref
    prod_hat = (T.ntt_def(a, q, psi) * T.ntt_def(b, q, psi)) % q
    assert list(T.intt_def(prod_hat, q, psi)) == ref
    # x^(N-1) * x = x^N = -1
    e = [0] * n
    e[n - 1] = 1
    x = [0, 1] + [0] * (n - 2)
    assert list(PL.negacyclic_mul(e, x, q)) == [q - 1] + [0] * (n - 1)


@pytest.mark.slow
def test_convolution_theorem_n4096():
    n, q = 4096, Q0
    psi = psi_of(q, n)
    g = np.random.Generator(np.random.PCG64(99))
    a = g.integers(0, q, n)
    b = g.integers(0, q, n)
    ref = PL.negacyclic_mul(a, b, q)
    got = T.intt_gs((T.ntt_ct(a, q, psi) * T.ntt_ct(b, q, psi)) % q, q, psi)
    assert np.array_equal(ref, got)
    assert np.array_equal(T.ntt_ct(a, q, psi), T.ntt_def(a, q, psi))


@pytest.mark.parametrize("log_n", [1, 2, 4, 6, 9, 11])
def test_fast_ntt_equals_definition(log_n):
    n = 1 << log_n
    for q in prime_chain(3):
        psi = psi_of(q, n)
        g = np.random.Generator(np.random.PCG64(q % 1000 + log_n))
        a = g.integers(0, q, (2, n))
        fast = T.ntt_ct(a, q, psi)
        for r in range(2):
            assert np.array_equal(fast[r], T.ntt_def(a[r], q, psi))
        assert np.array_equal(T.intt_gs(fast, q, psi), a)
        assert np.array_equal(T.intt_def(fast[0], q, psi), a[0])


def test_fast_ntt_n65536_horner_spot_check():
    n, q = 1 << 16, prime_chain(2)[1]
    psi = psi_of(q, n)
    g = np.random.Generator(np.random.PCG64(5))
    a = g.integers(0, q, n)
    out = T.ntt_ct(a, q, psi)
    pos = g.integers(0, n, 64)
    xs = [pow(psi, 2 * _rev_str(int(p), 16) + 1, q) for p in pos]
    assert np.array_equal(out[pos], T.horner_eval(a, q, xs))
    assert np.array_equal(T.intt_gs(out, q, psi), a)


@pytest.mark.parametrize("R,C", [(8, 8), (4, 16), (16, 4), (2, 32), (16, 16)])
def test_three_step_matches_definition(R, C):
    n = R * C
    q = Q0
    psi = psi_of(q, n)
    g = np.random.Generator(np.random.PCG64(R * 100 + C))
    a = g.integers(0, q, n)
    ref = T.ntt_def(a, q, psi)
    assert np.array_equal(M.three_step_ntt(a, q, psi, R, C), ref)
    assert np.array_equal(M.three_step_intt(ref, q, psi, R, C), a)


def test_three_step_twiddle_structure():
    # N^-1 is folded wholly into the inverse step-1 matrix, so the step-3 pair
    # multiplies to C*I and the step-1 pair to C^-1*I; the step-2 twiddles are
    # exact inverses element by element.
    q, R, C = Q0, 8, 16
    psi = psi_of(q, R * C)
    (tf1, t2, tf3), (itf1, it2, itf3) = M.twiddles(q, psi, R, C)
    eye_c = np.eye(C, dtype=np.uint64)
    eye_r = np.eye(R, dtype=np.uint64)
    assert np.array_equal(M.modmatmul(tf3, itf3, q), eye_c * np.uint64(C))
    assert np.array_equal(M.modmatmul(itf1, tf1, q), eye_r * np.uint64(pow(C, -1, q)))
    assert np.array_equal((t2 * it2) % q, np.ones((R, C), dtype=np.uint64))


@pytest.mark.parametrize("R,C1,C2", [(4, 4, 4), (8, 2, 4), (2, 8, 4), (4, 4, 8), (16, 2, 8), (2, 4, 32)])
def test_three_factor_matches_definition(R, C1, C2):
    n = R * C1 * C2
    q = Q0
    psi = psi_of(q, n)
    g = np.random.Generator(np.random.PCG64(R * 1000 + C1 * 10 + C2))
    a = g.integers(0, q, n)
    ref = T.ntt_def(a, q, psi)
    assert np.array_equal(M.three_factor_ntt(a, q, psi, R, C1, C2), ref)
    assert np.array_equal(M.three_factor_intt(ref, q, psi, R, C1, C2), a)


def test_three_factor_degenerate_and_structure():
    # C1 = 1 (or C2 = 1) is the two-factor form; the row factors invert to C1 * I and C2 * I
    q, R, C1, C2 = Q0, 4, 8, 4
    n = R * C1 * C2
    psi = psi_of(q, n)
    g = np.random.Generator(np.random.PCG64(77))
    a = g.integers(0, q, n)
    assert np.array_equal(M.three_factor_ntt(a, q, psi, R, 1, C1 * C2), M.three_step_ntt(a, q, psi, R, C1 * C2))
    assert np.array_equal(M.three_factor_ntt(a, q, psi, R, C1 * C2, 1), M.three_step_ntt(a, q, psi, R, C1 * C2))
    (tb, t3, tc), (itb, it3, itc) = M.row_twiddles(q, psi, R, C1, C2)
    assert np.array_equal(M.modmatmul(itb, tb, q), np.eye(C1, dtype=np.uint64) * np.uint64(C1))
    assert np.array_equal(M.modmatmul(tc, itc, q), np.eye(C2, dtype=np.uint64) * np.uint64(C2))
    assert np.array_equal((t3 * it3) % q, np.ones((C1, C2), dtype=np.uint64))


def test_golden_regression_fixture():
    import json
    import os
    from oracle import ckks as CK
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_regression.json")
    fx = json.load(open(path))
    for key, v in fx.items():
        if key.startswith("ntt_"):
            assert [int(x) for x in T.ntt_def(v["a"], v["q"], v["psi"])] == v["ntt"]
        else:
            assert [int(x) for x in CK.automorphism_ntt(np.array(v["ntt"], dtype=np.uint64), v["g"])] == v["rotated"]
