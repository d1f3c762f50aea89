"""GPU parity of polymul, BConv, ModUp/ModDown, HE-Mult and Rotate against the oracle (bit-exact)."""
import numpy as np
import pytest

import synthetic
from oracle import ckks as CK
from oracle.bconv import bconv_u64
from oracle.poly import negacyclic_mul
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def _empty(shape):
    import torch
    return torch.empty(shape, dtype=torch.int32, device="cuda")


def test_config1_polymul_vs_schoolbook():
    from paper_2501_07047_amd import binding as B
    primes, a = synthetic.ntt_batch(1, 12, 1, 1)
    _, b = synthetic.ntt_batch(2, 12, 1, 1)
    out = _empty(a.shape)
    B.poly_mul(to_dev(a), to_dev(b), out, primes)
    ref = negacyclic_mul(a[0, 0], b[0, 0], primes[0])
    assert np.array_equal(to_host(out)[0, 0], ref)


@pytest.mark.parametrize("log_n,L,batch", [(6, 2, 2), (10, 3, 3)])
def test_polymul_small_and_aliasing(log_n, L, batch):
    from paper_2501_07047_amd import binding as B
    primes, a = synthetic.ntt_batch(3, log_n, L, batch)
    _, b = synthetic.ntt_batch(4, log_n, L, batch)
    da, db = to_dev(a), to_dev(b)
    B.poly_mul(da, db, db, primes)            # out aliases b
    got = to_host(db)
    for bi in range(batch):
        for i, q in enumerate(primes):
            assert np.array_equal(got[bi, i], negacyclic_mul(a[bi, i], b[bi, i], q))


@pytest.mark.parametrize("log_n,l,lp,batch", [(8, 3, 5, 2), (10, 8, 24, 1), (12, 12, 28, 1),
                                              (16, 12, 36, 1), (16, 16, 40, 1), (16, 24, 56, 1),
                                              (10, 32, 64, 2), (5, 1, 1, 1)])
def test_bconv_shapes(log_n, l, lp, batch):
    # includes the paper's BConv shapes (Tab. bc_skew_shape: 12->28, 12->36, 16->40, 24->56 at N=2^16)
    from paper_2501_07047_amd import binding as B
    allp = synthetic.primes(l + lp)
    src, dst = allp[:l], allp[l:]
    g = synthetic.rng(l * 100 + lp)
    x = synthetic.residues(g, (batch,), src, 1 << log_n)
    x[0, :, 0] = [q - 1 for q in src]
    x[0, :, 1] = 0
    out = _empty((batch, lp, 1 << log_n))
    B.bconv(to_dev(x), src, dst, out)
    got = to_host(out)
    for bi in range(batch):
        assert np.array_equal(got[bi], bconv_u64(x[bi], src, dst))


@pytest.mark.parametrize("log_n,l,lp,batch,mix", [(8, 3, 5, 2, "wide"), (12, 8, 24, 1, "wide"),
                                                  (16, 12, 36, 1, "narrow_src"), (10, 20, 40, 2, "wide"),
                                                  (10, 32, 8, 1, "wide_src"), (5, 1, 1, 1, "wide")])
def test_bconv_wide_primes(log_n, l, lp, batch, mix):
    # primes in [2^30, 2^31) take the byte form (b - 128 against balanced signed digits
    # with per-row corrections): one to four K blocks, wide / narrow sources and targets
    from paper_2501_07047_amd import binding as B
    wp = synthetic.wide_primes(l + lp)
    npr = synthetic.primes(l + lp)
    src = npr[:l] if mix == "narrow_src" else wp[:l]
    dst = npr[l:] if mix == "wide_src" else wp[l:]
    g = synthetic.rng(l * 100 + lp + 7)
    x = synthetic.residues(g, (batch,), src, 1 << log_n)
    x[0, :, 0] = [q - 1 for q in src]
    x[0, :, 1] = 0
    out = _empty((batch, lp, 1 << log_n))
    B.bconv(to_dev(x), src, dst, out)
    got = to_host(out)
    for bi in range(batch):
        assert np.array_equal(got[bi], bconv_u64(x[bi], src, dst)), "batch %d" % bi


def test_bconv_rejects_primes_from_2_31():
    from paper_2501_07047_amd import binding as B
    src = synthetic.wide_primes(2)
    x = synthetic.residues(synthetic.rng(1), (1,), src, 64)
    out = _empty((1, 1, 64))
    with pytest.raises(B.CrossError) as e:
        B.bconv(to_dev(x), src, [2147483659], out)     # a prime above 2^31
    assert e.value.code == -4                            # CROSS_ERANGE


def _ckks(log_n, L, dnum, K=None, seed=0, batch=1):
    return synthetic.ckks_pair(seed, log_n, L, dnum, K, batch)


@pytest.mark.parametrize("log_n,L,dnum,K", [(8, 6, 3, 2), (10, 4, 3, 2), (10, 5, 2, 3), (9, 3, 1, 3)])
def test_modup_moddown_small(log_n, L, dnum, K):
    from paper_2501_07047_amd import binding as B
    qs, ps, a, _, _ = _ckks(log_n, L, dnum, K, seed=log_n + L)
    d = a[:, 1]                                  # [batch][L][N]
    ext = _empty((1, dnum, L + K, 1 << log_n))
    B.keyswitch_modup(to_dev(d), ext, qs, ps, dnum)
    ref = CK.modup(d[0], qs, ps, dnum)
    got = to_host(ext)[0]
    assert np.array_equal(got, ref)
    out = _empty((1, L, 1 << log_n))
    B.keyswitch_moddown(to_dev(ref[:1]), out, qs, ps, dnum)
    assert np.array_equal(to_host(out)[0], CK.moddown(ref[0], qs, ps))


@pytest.mark.parametrize("log_n,L,dnum,K,batch", [(8, 6, 3, 2, 2), (10, 4, 3, 2, 1), (11, 7, 3, 3, 1),
                                                  (12, 5, 1, 5, 1), (6, 4, 2, 2, 2)])
def test_he_mult_small(log_n, L, dnum, K, batch):
    from paper_2501_07047_amd import binding as B
    qs, ps, a, b, key = _ckks(log_n, L, dnum, K, seed=log_n * 3 + L, batch=batch)
    out = _empty(a.shape)
    B.he_mult(to_dev(a), to_dev(b), to_dev(key), out, qs, ps, dnum)
    got = to_host(out)
    for bi in range(batch):
        assert np.array_equal(got[bi], CK.he_mult(a[bi], b[bi], key, qs, ps, dnum))


@pytest.mark.parametrize("log_n,L,dnum,K,steps", [(8, 6, 3, 2, 1), (10, 4, 3, 2, -3), (12, 7, 3, 3, 64)])
def test_rotate_small(log_n, L, dnum, K, steps):
    from paper_2501_07047_amd import binding as B
    qs, ps, a, _, key = _ckks(log_n, L, dnum, K, seed=log_n * 5 + L, batch=2)
    out = _empty(a.shape)
    B.rotate(to_dev(a), steps, to_dev(key), out, qs, ps, dnum)
    got = to_host(out)
    for bi in range(2):
        assert np.array_equal(got[bi], CK.rotate(a[bi], steps, key, qs, ps, dnum))


def test_config3_he_mult_full_size():
    # N = 2^16, L = 24, dnum = 3 (alpha = 8), K = 8 special primes: the benchmarked shape
    from paper_2501_07047_amd import binding as B
    qs, ps, a, b, key = _ckks(16, 24, 3, 8, seed=0, batch=1)
    out = _empty(a.shape)
    B.he_mult(to_dev(a), to_dev(b), to_dev(key), out, qs, ps, dnum=3)
    assert np.array_equal(to_host(out)[0], CK.he_mult(a[0], b[0], key, qs, ps, 3))


def test_rotate_n2_14():
    from paper_2501_07047_amd import binding as B
    qs, ps, a, _, key = _ckks(14, 8, 3, 3, seed=9, batch=1)
    out = _empty(a.shape)
    B.rotate(to_dev(a), 5, to_dev(key), out, qs, ps, 3)
    assert np.array_equal(to_host(out)[0], CK.rotate(a[0], 5, key, qs, ps, 3))


def test_ckks_argument_errors():
    from paper_2501_07047_amd import binding as B
    qs, ps, a, b, key = _ckks(8, 3, 3, 1, seed=1)
    da, db, dk = to_dev(a), to_dev(b), to_dev(key)
    with pytest.raises(B.CrossError):
        B.he_mult(da, db, dk, da, qs, ps, 3)                       # out aliases input
    with pytest.raises(B.CrossError):
        B.he_mult(da, db, dk, _empty(a.shape), qs, [qs[0]], 3)     # repeated prime
