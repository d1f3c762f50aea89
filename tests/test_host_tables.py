"""CPU emulation of the BAT int8 GEMM steps with the library's own offline tables.

The tables come from libcross (host-only entry point cross_host_tables); the
GEMM, ChunkMerge and Montgomery steps are emulated here in numpy int64 exactly
as the kernels define them, and the result is compared with the oracle's NTT.
This checks the table layout, the BAT expansion and the 3-step reading
before any kernel runs.  Narrow primes (< 2^28): non-negative 7-bit chunks on
both sides.  Wide primes (2^28 <= q < 2^31): balanced signed 8-bit digits in
the table, the data's bytes fed as b - 128, and each accumulator started at the
row correction stored after the table bytes.
"""
import numpy as np
import pytest

from oracle.ntt import bitrev, ntt_ct, intt_gs
from oracle.primes import is_prime, prime_chain, psi as psi_of

WIDE = prime_chain(2, bits=31)


def _is_wide(q):
    return q >= 1 << 28


def _dense(tab, M, K):
    # fragment order: [K/64][M/32][K half][lane = m%32 + 32*kq][16 bytes], kq = (k%32)//16
    t = tab[:M * K].astype(np.int64).reshape(K // 64, M // 32, 2, 2, 32, 16)   # [s][b][h][kq][m%32][byte]
    return t.transpose(1, 4, 0, 2, 3, 5).reshape(M, K)


def _corr(tab, M, K):
    # wide tables: the M int32 row corrections after the table bytes
    assert tab.size == M * K + 4 * M
    return tab[M * K:].view(np.uint8).copy().view("<i4").astype(np.int64)


def _biased_bytes(X):
    # X: [inputs][cols] -> [(input, j)][cols]: byte j of each residue minus 128, the
    # signed int8 the wide kernels feed to the MFMA (x ^ 0x80808080)
    X = X.astype(np.int64)
    out = np.empty((X.shape[0] * 4, X.shape[1]), dtype=np.int64)
    for j in range(4):
        out[j::4] = ((X >> (8 * j)) & 0xFF) - 128
    return out


def _chunks_rows(X):
    # X: [inputs][cols] -> [(input, j)][cols]
    X = X.astype(np.int64)
    out = np.empty((X.shape[0] * 4, X.shape[1]), dtype=np.int64)
    for j in range(4):
        out[j::4] = (X >> (7 * j)) & 0x7F
    return out


def _gemm(tab, M, X, q):
    # one BAT step as the kernels compute it (square table, M = K = 4 * inputs)
    D = _dense(tab, M, M)
    if not _is_wide(q):
        assert tab.size == M * M and D.min() >= 0 and D.max() <= 127
        return D @ _chunks_rows(X)
    B = _biased_bytes(X)
    assert D.min() >= -128 and D.max() <= 127 and B.min() >= -128 and B.max() <= 127
    return _corr(tab, M, M)[:, None] + D @ B


def _merge_reduce(P, q, plain=False):
    # ChunkMerge (weights 2^(7i), wide 2^(8i)), then the tables' Montgomery factor
    # 2^32 divided out (plain tables: none)
    U = P.shape[0] // 4
    bits = 8 if _is_wide(q) else 7
    Z = sum(P[i::4].astype(object) << (bits * i) for i in range(4))
    assert int(np.max(np.abs(P))) < (1 << 31)
    if not _is_wide(q):
        assert int(np.min(P)) >= 0
    rinv = 1 if plain else pow(1 << 32, -1, q)
    return np.array((Z * rinv) % q, dtype=np.uint64).reshape(U, -1)


def _emulate(X, q, log_n, log_r, inverse, plain=False):
    # plain: the tables without the Montgomery factor (host tables 7-10, Barrett epilogue)
    from paper_2501_07047_amd import binding
    R, C = 1 << log_r, 1 << (log_n - log_r)
    rinv = pow(1 << 32, -1, q)
    tab = lambda w: binding.host_tables(q, log_n, log_r, w + 7 if plain else w)
    if not inverse:
        t1 = tab(0)
        t3 = tab(1)
        pairs = binding.host_tables(q, log_n, log_r, 4).reshape(R, C, 2)
        assert np.array_equal(pairs[..., 1].astype(np.uint64), (pairs[..., 0].astype(np.uint64) << 32) // q)
        tw = (pairs[..., 0].astype(object) * (1 << 32)) % q          # Montgomery form for the emulation
        A = X.reshape(R, C)
        Y = _merge_reduce(_gemm(t1, 4 * R, A, q), q, plain)         # [k][c]
        Y = np.array((Y.astype(object) * tw * rinv) % q, dtype=np.uint64)
        out = _merge_reduce(_gemm(t3, 4 * C, Y.T, q), q, plain)    # [c'][k]
        return out.T.reshape(-1)
    t3 = tab(3)
    t1 = tab(2)
    tw = (binding.host_tables(q, log_n, log_r, 5).reshape(C, R, 2)[..., 0].astype(object) * (1 << 32)) % q
    A = X.reshape(R, C)
    Y = _merge_reduce(_gemm(t3, 4 * C, A.T, q), q, plain)           # [c][k]
    Y = np.array((Y.astype(object) * tw * rinv) % q, dtype=np.uint64)
    out = _merge_reduce(_gemm(t1, 4 * R, Y.T, q), q, plain)        # [r][c]
    return out.reshape(-1)


@pytest.mark.parametrize("log_n,log_r", [(8, 4), (10, 5), (10, 4), (10, 6), (12, 6)])
def test_emulated_bat_ntt_matches_oracle(log_n, log_r):
    n = 1 << log_n
    for q, plain in [(p, False) for p in prime_chain(2) + WIDE] + [(prime_chain(1)[0], True)]:
        psi = psi_of(q, n)
        g = np.random.Generator(np.random.PCG64(log_n * 7 + log_r))
        a = g.integers(0, q, n).astype(np.uint64)
        a[0] = q - 1
        ref = ntt_ct(a, q, psi)
        assert np.array_equal(_emulate(a, q, log_n, log_r, False, plain), ref)
        assert np.array_equal(_emulate(ref, q, log_n, log_r, True, plain), a)
        assert np.array_equal(intt_gs(ref, q, psi), a)


def test_table_entries_are_7bit_chunks():
    from paper_2501_07047_amd import binding
    q = prime_chain(1)[0]
    for which in range(4):
        t = binding.host_tables(q, 12, 6, which)
        assert t.min() >= 0 and t.max() <= 127
    for which in (4, 5):
        t = binding.host_tables(q, 12, 6, which).reshape(-1, 2)
        assert int(t[:, 0].max()) < q


def test_wide_table_is_balanced_digit_bat():
    # DirectScalarBAT with bp = 8 on both sides and balanced signed digits, in closed
    # form: entry (m = 4k + i, 4r + j) of the forward step-1 table is digit i of the
    # representative of (TF1[k][r] * 2^32 * 2^(8j)) mod q in [-128 * 0x1010101,
    # 127 * 0x1010101] (the value itself unless it lies above that range)
    from paper_2501_07047_amd import binding
    lo, hi = -128 * 0x1010101, 127 * 0x1010101
    for q in WIDE:
        log_n, log_r = 10, 5
        R, C, n = 32, 32, 1024
        psi = psi_of(q, n)
        tab = binding.host_tables(q, log_n, log_r, 0)
        M = 4 * R
        D = _dense(tab, M, M)
        assert D.min() >= -128 and D.max() <= 127
        assert np.array_equal(_corr(tab, M, M), 128 * D.sum(axis=1))
        g = np.random.default_rng(3)
        for _ in range(300):
            r, k, j = int(g.integers(R)), int(g.integers(R)), int(g.integers(4))
            t = pow(psi, C * r * (2 * bitrev(k, log_r) + 1) % (2 * n), q)
            v = t * (1 << 32) * (1 << (8 * j)) % q
            val = sum(int(D[4 * k + i, 4 * r + j]) << (8 * i) for i in range(4))
            assert val == (v if v <= hi else v - q) and lo <= val <= hi


def test_wide_prime_limits():
    from paper_2501_07047_amd import binding
    q = WIDE[0]
    for which in (8, 9, 10, 11):        # no plain (Barrett) tables in the wide form
        with pytest.raises(binding.CrossError):
            binding.host_row_tables(q, 14, 5, 5, which)
    for which in (7, 8, 9, 10):         # nor plain step tables
        with pytest.raises(binding.CrossError):
            binding.host_tables(q, 12, 6, which)
    with pytest.raises(binding.CrossError) as e:     # the BAT-lazy fragment is 28-bit only
        binding.host_tables(q, 12, 6, 6)
    assert e.value.code == -4
    big = next(p for p in range((1 << 31) + 1, 1 << 32, 1 << 17) if is_prime(p))
    with pytest.raises(binding.CrossError) as e:     # at or above 2^31
        binding.host_tables(big, 12, 6, 0)
    assert e.value.code == -4


def test_bat_lazy_fragment_returns_each_lanes_chunk_products_in_lane():
    # Emulate v_mfma_i32_32x32x32_i8 with the library's BAT-lazy A operand: lane l
    # supplies A row l%32 / B column l%32 with K bytes 16*(l/32) .. +15, and holds
    # output rows 8*(v/4) + 4*(l/32) + v%4 of column l%32 in register v.  Lane l puts
    # the high chunks of its element t in B bytes 4t .. 4t+3 and must get
    # T_k = sum_j c_(4+j) LC[j][k] of that element back in registers 4t .. 4t+3.
    from oracle.reduction import bat_lazy_reduce, lazy_constants
    from paper_2501_07047_amd import binding
    g = np.random.Generator(np.random.PCG64(31))
    for q in prime_chain(3):
        frag = binding.host_tables(q, 16, 8, 6).astype(np.int64)
        assert frag.shape == (1024,)
        A = np.zeros((32, 32), dtype=np.int64)
        for l in range(64):
            A[l % 32, 16 * (l // 32):16 * (l // 32) + 16] = frag[16 * l:16 * l + 16]
        a = g.integers(0, q, (64, 4)).astype(np.int64)
        w = g.integers(0, q, (64, 4)).astype(np.int64)
        p = a * w
        hi = p >> 28
        Bm = np.zeros((32, 32), dtype=np.int64)
        for l in range(64):
            for t in range(4):
                for j in range(4):
                    Bm[16 * (l // 32) + 4 * t + j, l % 32] = (int(hi[l, t]) >> (7 * j)) & 0x7f
        C = A @ Bm
        LC = lazy_constants(q)
        for l in range(64):
            regs = [C[8 * (v // 4) + 4 * (l // 32) + v % 4, l % 32] for v in range(16)]
            for t in range(4):
                c = [(int(hi[l, t]) >> (7 * j)) & 0x7f for j in range(4)]
                T = [sum(c[j] * LC[j][k] for j in range(4)) for k in range(4)]
                assert regs[4 * t:4 * t + 4] == T
                lazy = (int(p[l, t]) & 0x0fffffff) + sum(T[k] << (7 * k) for k in range(4))
                assert lazy == bat_lazy_reduce(int(p[l, t]), q) and lazy % q == int(p[l, t]) % q


def _emulate3(X, q, log_n, log_r, log_c1, inverse, plain=False, t3_which=4):
    # three factors: the row-side step with the library's step-1 tables, then the
    # row transform with its row tables (cross_host_row_tables), in the kernels'
    # operand roles; Montgomery factors as in _emulate
    from paper_2501_07047_amd import binding
    R = 1 << log_r
    C1 = 1 << log_c1
    C = (1 << log_n) // R
    C2 = C // C1
    rinv = pow(1 << 32, -1, q)

    def mont(pairs):
        return (pairs[..., 0].astype(object) * (1 << 32)) % q

    def twist(Y, tw):
        return np.array((Y.astype(object) * tw * rinv) % q, dtype=np.uint64)

    # row tables 0-3, or their plain forms 8-11 (Barrett epilogue)
    rt = lambda w: binding.host_row_tables(q, log_n, log_r, log_c1, w + 8 if plain and w < 4 else w)
    mr = lambda P: _merge_reduce(P, q, plain)
    if not inverse:
        t1 = binding.host_tables(q, log_n, log_r, 7 if plain else 0)
        Y = twist(mr(_gemm(t1, 4 * R, X.reshape(R, C), q)), mont(rt(7).reshape(R, C, 2)))
        tb, tc = rt(0), rt(1)
        t3 = mont(rt(t3_which).reshape(C1, C2, 2))
        out = np.empty((R, C), dtype=np.uint64)
        for k in range(R):
            Z = twist(mr(_gemm(tb, 4 * C1, Y[k].reshape(C1, C2), q)), t3)               # [m][c2]
            out[k] = mr(_gemm(tc, 4 * C2, Z.T, q)).T.reshape(-1)                       # [m][c2']
        return out.reshape(-1)
    itc, itb = rt(2), rt(3)
    it3 = mont(rt(5).reshape(C2, C1, 2))         # [c2][m]
    it2 = mont(rt(6).reshape(R, C, 2))
    X = X.reshape(R, C1, C2)
    Y = np.empty((R, C), dtype=np.uint64)
    for k in range(R):
        Z = twist(mr(_gemm(itc, 4 * C2, X[k].T, q)), it3)                               # [c2][m]
        Yk = mr(_gemm(itb, 4 * C1, Z.T, q))                                             # [c1][c2]
        Y[k] = twist(Yk.reshape(-1), it2[k])
    t1 = binding.host_tables(q, log_n, log_r, 9 if plain else 2)
    return mr(_gemm(t1, 4 * R, Y, q)).reshape(-1)


@pytest.mark.parametrize("plain,wide", [(False, False), (True, False), (False, True)])
@pytest.mark.parametrize("log_n,log_r,log_c1", [(13, 5, 4), (14, 6, 4), (15, 5, 5), (16, 6, 5), (14, 4, 5)])
def test_emulated_three_factor_ntt_matches_oracle(log_n, log_r, log_c1, plain, wide):
    n = 1 << log_n
    q = WIDE[0] if wide else prime_chain(1)[0]
    psi = psi_of(q, n)
    g = np.random.Generator(np.random.PCG64(log_n * 11 + log_c1))
    a = g.integers(0, q, n).astype(np.uint64)
    a[0] = q - 1
    ref = ntt_ct(a, q, psi)
    assert np.array_equal(_emulate3(a, q, log_n, log_r, log_c1, False, plain), ref)
    assert np.array_equal(_emulate3(ref, q, log_n, log_r, log_c1, True, plain), a)


@pytest.mark.parametrize("log_n,log_r,log_c1", [(13, 5, 4), (16, 6, 5)])
def test_montgomery_form_t3_scales_the_forward_transform(log_n, log_r, log_c1):
    # the fused ModUp NTT + inner product runs the forward row transform with T3 * 2^32
    # (row table 12): its outputs are the NTT times 2^32 mod q, and the pairs keep the
    # Shoup quotient floor(w 2^32 / q) of the scaled twiddle
    from paper_2501_07047_amd import binding
    n = 1 << log_n
    q = prime_chain(1)[0]
    t3 = binding.host_row_tables(q, log_n, log_r, log_c1, 4).reshape(-1, 2).astype(object)
    t3m = binding.host_row_tables(q, log_n, log_r, log_c1, 12).reshape(-1, 2).astype(object)
    assert all(wm == (w << 32) % q for w, wm in zip(t3[:, 0], t3m[:, 0]))
    assert all(s == (wm << 32) // q for wm, s in zip(t3m[:, 0], t3m[:, 1]))
    g = np.random.Generator(np.random.PCG64(log_n))
    a = g.integers(0, q, n).astype(np.uint64)
    ref = ntt_ct(a, q, psi_of(q, n))
    got = _emulate3(a, q, log_n, log_r, log_c1, False, t3_which=12)
    assert np.array_equal(got, np.array([(int(v) << 32) % q for v in ref], dtype=np.uint64))


@pytest.mark.parametrize("wide", [False, True])
def test_equal_row_splits_share_one_table(wide):
    # C1 = C2: the row kernels stage one table for both sub-steps (forward TB and TC,
    # inverse ITC and ITB), so the library's two tables must be byte-identical
    from paper_2501_07047_amd import binding
    q = WIDE[0] if wide else prime_chain(1)[0]
    for log_n, log_r, log_c1 in ((13, 5, 4), (14, 4, 5), (16, 6, 5), (16, 4, 6)):
        rt = lambda w: binding.host_row_tables(q, log_n, log_r, log_c1, w)
        assert np.array_equal(rt(0), rt(1)) and np.array_equal(rt(2), rt(3))
        if not wide:
            assert np.array_equal(rt(8), rt(9)) and np.array_equal(rt(10), rt(11))


def test_row_split_limits():
    from paper_2501_07047_amd import binding
    q = prime_chain(1)[0]
    for bad in ((12, 4, 4), (16, 6, 3), (16, 3, 6), (16, 4, 7)):     # R*C < 8192, C1 < 16, R < 16, C1 > 64
        with pytest.raises(binding.CrossError):
            binding.host_row_tables(q, *bad, 0)
