"""CPU emulation of the BAT int8 GEMM steps with the library's own offline tables.

The tables come from libcross (host-only entry point cross_host_tables); the
GEMM, ChunkMerge and Montgomery steps are emulated here in numpy int64 exactly
as the kernels define them, and the result is compared with the oracle's NTT.
This checks the table layout, the BAT expansion and the 3-step reading
before any kernel runs.
"""
import numpy as np
import pytest

from oracle.ntt import ntt_ct, intt_gs
from oracle.primes import prime_chain, psi as psi_of


def _dense(tab, M, K):
    # fragment order: [K/64][M/32][K half][lane = m%32 + 32*kq][16 bytes], kq = (k%32)//16
    t = tab.astype(np.int64).reshape(K // 64, M // 32, 2, 2, 32, 16)   # [s][b][h][kq][m%32][byte]
    return t.transpose(1, 4, 0, 2, 3, 5).reshape(M, K)


def _chunks_rows(X):
    # X: [inputs][cols] -> [(input, j)][cols]
    X = X.astype(np.int64)
    out = np.empty((X.shape[0] * 4, X.shape[1]), dtype=np.int64)
    for j in range(4):
        out[j::4] = (X >> (7 * j)) & 0x7F
    return out


def _merge_reduce(P, q, plain=False):
    # ChunkMerge, then the tables' Montgomery factor 2^32 divided out (plain tables: none)
    U = P.shape[0] // 4
    Z = sum(P[i::4].astype(object) << (7 * i) for i in range(4))
    assert int(np.max(P)) < (1 << 31) and int(np.min(P)) >= 0
    rinv = 1 if plain else pow(1 << 32, -1, q)
    return np.array((Z * rinv) % q, dtype=np.uint64).reshape(U, -1)


def _emulate(X, q, log_n, log_r, inverse):
    from paper_2501_07047_amd import binding
    R, C = 1 << log_r, 1 << (log_n - log_r)
    rinv = pow(1 << 32, -1, q)
    if not inverse:
        t1 = _dense(binding.host_tables(q, log_n, log_r, 0), 4 * R, 4 * R)
        t3 = _dense(binding.host_tables(q, log_n, log_r, 1), 4 * C, 4 * C)
        pairs = binding.host_tables(q, log_n, log_r, 4).reshape(R, C, 2)
        assert np.array_equal(pairs[..., 1].astype(np.uint64), (pairs[..., 0].astype(np.uint64) << 32) // q)
        tw = (pairs[..., 0].astype(object) * (1 << 32)) % q          # Montgomery form for the emulation
        A = X.reshape(R, C)
        Y = _merge_reduce(t1 @ _chunks_rows(A), q)                 # [k][c]
        Y = np.array((Y.astype(object) * tw * rinv) % q, dtype=np.uint64)
        out = _merge_reduce(t3 @ _chunks_rows(Y.T), q)            # [c'][k]
        return out.T.reshape(-1)
    t3 = _dense(binding.host_tables(q, log_n, log_r, 3), 4 * C, 4 * C)
    t1 = _dense(binding.host_tables(q, log_n, log_r, 2), 4 * R, 4 * R)
    tw = (binding.host_tables(q, log_n, log_r, 5).reshape(C, R, 2)[..., 0].astype(object) * (1 << 32)) % q
    A = X.reshape(R, C)
    Y = _merge_reduce(t3 @ _chunks_rows(A.T), q)                   # [c][k]
    Y = np.array((Y.astype(object) * tw * rinv) % q, dtype=np.uint64)
    out = _merge_reduce(t1 @ _chunks_rows(Y.T), q)                # [r][c]
    return out.reshape(-1)


@pytest.mark.parametrize("log_n,log_r", [(8, 4), (10, 5), (10, 4), (10, 6), (12, 6)])
def test_emulated_bat_ntt_matches_oracle(log_n, log_r):
    n = 1 << log_n
    for q in prime_chain(2):
        psi = psi_of(q, n)
        g = np.random.Generator(np.random.PCG64(log_n * 7 + log_r))
        a = g.integers(0, q, n).astype(np.uint64)
        a[0] = q - 1
        ref = ntt_ct(a, q, psi)
        assert np.array_equal(_emulate(a, q, log_n, log_r, False), ref)
        assert np.array_equal(_emulate(ref, q, log_n, log_r, True), a)
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


def _emulate3(X, q, log_n, log_r, log_c1, inverse, plain=False):
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
        t1 = _dense(binding.host_tables(q, log_n, log_r, 0), 4 * R, 4 * R)
        Y = twist(_merge_reduce(t1 @ _chunks_rows(X.reshape(R, C)), q), mont(rt(7).reshape(R, C, 2)))
        tb, tc = _dense(rt(0), 4 * C1, 4 * C1), _dense(rt(1), 4 * C2, 4 * C2)
        t3 = mont(rt(4).reshape(C1, C2, 2))
        out = np.empty((R, C), dtype=np.uint64)
        for k in range(R):
            Z = twist(mr(tb @ _chunks_rows(Y[k].reshape(C1, C2))), t3)                   # [m][c2]
            out[k] = mr(tc @ _chunks_rows(Z.T)).T.reshape(-1)                           # [m][c2']
        return out.reshape(-1)
    itc, itb = _dense(rt(2), 4 * C2, 4 * C2), _dense(rt(3), 4 * C1, 4 * C1)
    it3 = mont(rt(5).reshape(C2, C1, 2))         # [c2][m]
    it2 = mont(rt(6).reshape(R, C, 2))
    X = X.reshape(R, C1, C2)
    Y = np.empty((R, C), dtype=np.uint64)
    for k in range(R):
        Z = twist(mr(itc @ _chunks_rows(X[k].T)), it3)                                   # [c2][m]
        Yk = mr(itb @ _chunks_rows(Z.T))                                                 # [c1][c2]
        Y[k] = twist(Yk.reshape(-1), it2[k])
    t1 = _dense(binding.host_tables(q, log_n, log_r, 2), 4 * R, 4 * R)
    return _merge_reduce(t1 @ _chunks_rows(Y), q).reshape(-1)


@pytest.mark.parametrize("plain", [False, True])
@pytest.mark.parametrize("log_n,log_r,log_c1", [(13, 5, 4), (14, 6, 4), (15, 5, 5), (16, 6, 5), (14, 4, 5)])
def test_emulated_three_factor_ntt_matches_oracle(log_n, log_r, log_c1, plain):
    n = 1 << log_n
    q = prime_chain(1)[0]
    psi = psi_of(q, n)
    g = np.random.Generator(np.random.PCG64(log_n * 11 + log_c1))
    a = g.integers(0, q, n).astype(np.uint64)
    a[0] = q - 1
    ref = ntt_ct(a, q, psi)
    assert np.array_equal(_emulate3(a, q, log_n, log_r, log_c1, False, plain), ref)
    assert np.array_equal(_emulate3(ref, q, log_n, log_r, log_c1, True, plain), a)


def test_row_split_limits():
    from paper_2501_07047_amd import binding
    q = prime_chain(1)[0]
    for bad in ((12, 4, 4), (16, 6, 3), (16, 3, 6), (16, 4, 7)):     # R*C < 8192, C1 < 16, R < 16, C1 > 64
        with pytest.raises(binding.CrossError):
            binding.host_row_tables(q, *bad, 0)
