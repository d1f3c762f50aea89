"""GPU parity at the sizes the benchmark times, against the oracle (bit-exact).

HE-Mult and Rotate at N = 2^16, L = 24, dnum = 3, K = 8 with a batch of eight
ciphertexts: the key-switch inner product takes four ciphertexts per thread, so
ciphertexts 0 and 3 sit in the first (full) group and 4 and 7 in the second;
the oracle checks those four.  HE-Mult and Rotate at L = 36, K = 12 (the largest
limb count of the request-loop and uneven-batch workloads).  The inner product
in both forms at batch 5 (a full group and a partial one) and batch 8.
"""
import numpy as np
import pytest

import synthetic
from oracle import ckks as CK
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

CHECKED = (0, 3, 4, 7)


def _empty(shape):
    import torch
    return torch.empty(shape, dtype=torch.int32, device="cuda")


def _with_edges(a, qs):
    # a few extreme residues in every limb of the first and last ciphertext
    for i, q in enumerate(qs):
        a[0, :, i, :4] = [0, 1, q - 1, q - 2]
        a[-1, :, i, -2:] = q - 1
    return a


def test_he_mult_batch8_n2_16_L24():
    # three calls on the same buffers: the first call on a shape allocates its
    # workspace and uploads its job lists, later calls reuse them, so every call
    # must give the first call's result (all eight ciphertexts), which the oracle checks
    from paper_2501_07047_amd import binding as B
    qs, ps, a, b, key = synthetic.ckks_pair(21, 16, 24, 3, 8, 8)
    _with_edges(a, qs)
    da, db, dk = to_dev(a), to_dev(b), to_dev(key)
    out = _empty(a.shape)
    calls = []
    for _ in range(3):
        out.fill_(0)
        B.he_mult(da, db, dk, out, qs, ps, 3)
        calls.append(to_host(out))
    for i in (1, 2):
        bad = [k for k in range(8) if not np.array_equal(calls[i][k], calls[0][k])]
        assert not bad, "call %d differs from the first on ciphertexts %s" % (i + 1, bad)
    for k in CHECKED:
        assert np.array_equal(calls[0][k], CK.he_mult(a[k], b[k], key, qs, ps, 3)), "ciphertext %d" % k


@pytest.mark.parametrize("batch", [3, 5])
def test_he_mult_odd_batch_n2_16_L24(batch):
    # batches that do not fill whole workgroups of the fused ModUp kernel: its blocks of
    # eight (row, ciphertext) pairs then straddle rows, and workgroups cross from one
    # target limb to the next (restaging the tables) in the middle of their range
    from paper_2501_07047_amd import binding as B
    qs, ps, a, b, key = synthetic.ckks_pair(23 + batch, 16, 24, 3, 8, batch)
    out = _empty(a.shape)
    B.he_mult(to_dev(a), to_dev(b), to_dev(key), out, qs, ps, 3)
    got = to_host(out)
    for k in (0, batch - 1):
        assert np.array_equal(got[k], CK.he_mult(a[k], b[k], key, qs, ps, 3)), "ciphertext %d" % k


def test_rotate_batch8_n2_16_L24():
    from paper_2501_07047_amd import binding as B
    qs, ps, a, _, key = synthetic.ckks_pair(22, 16, 24, 3, 8, 8)
    _with_edges(a, qs)
    out = _empty(a.shape)
    B.rotate(to_dev(a), 1, to_dev(key), out, qs, ps, 3)
    got = to_host(out)
    for k in CHECKED:
        assert np.array_equal(got[k], CK.rotate(a[k], 1, key, qs, ps, 3)), "ciphertext %d" % k


@pytest.mark.parametrize("op", ["he_mult", "rotate"])
def test_L36_K12_n2_16(op):
    # alpha = ceil(36 / 3) = 12 = K: 48 limbs per key-switch polynomial
    from paper_2501_07047_amd import binding as B
    qs, ps, a, b, key = synthetic.ckks_pair(23, 16, 36, 3, 12, 2)
    out = _empty(a.shape)
    if op == "he_mult":
        B.he_mult(to_dev(a), to_dev(b), to_dev(key), out, qs, ps, 3)
    else:
        B.rotate(to_dev(a), 64, to_dev(key), out, qs, ps, 3)
    got = to_host(out)
    for k in range(2):
        ref = CK.he_mult(a[k], b[k], key, qs, ps, 3) if op == "he_mult" else CK.rotate(a[k], 64, key, qs, ps, 3)
        assert np.array_equal(got[k], ref), "ciphertext %d" % k


def _ks_inputs(seed, log_n, LK, dnum, batch):
    p = synthetic.primes(LK)
    ext = synthetic.residues(synthetic.rng(seed), (batch, dnum), p, 1 << log_n)
    key = synthetic.residues(synthetic.rng(seed + 1000), (dnum, 2), p, 1 << log_n)
    for t, q in enumerate(p):
        ext[-1, :, t, :3] = [0, 1, q - 1]
        key[:, :, t, :2] = q - 1
    return p, ext, key


@pytest.mark.parametrize("log_n,batch", [(12, 5), (12, 8), (16, 8)])
@pytest.mark.parametrize("form", ["valu", "chunked"])
def test_inner_product_groups_of_four(form, log_n, batch):
    # L + K = 32 limbs, dnum = 3: batch 5 = one full group of four + one ciphertext,
    # batch 8 = two full groups
    from paper_2501_07047_amd import binding as Bd
    p, ext, key = _ks_inputs(40 + batch + log_n, log_n, 32, 3, batch)
    dkey = to_dev(key)
    if form == "chunked":
        dkey = Bd.evk_bat_prepare(dkey, p)
    out = _empty((batch, 2, 32, 1 << log_n))
    Bd.keyswitch_inner_product(to_dev(ext), dkey, out, p, form)
    got = to_host(out)
    for k in range(batch):
        assert np.array_equal(got[k], CK.inner_product(ext[k], key, p)), "ciphertext %d" % k


def test_partial_overlap_is_rejected():
    # out overlapping an input, or the key, by part of its range is an argument error
    import torch
    from paper_2501_07047_amd import binding as B
    qs, ps, a, b, key = synthetic.ckks_pair(3, 8, 3, 3, 1, 2)
    n_ct, n_key = a.size, key.size
    buf = torch.zeros(4 * n_ct + n_key, dtype=torch.int32, device="cuda")
    shape = a.shape
    da = buf[:n_ct].view(shape)
    da.copy_(to_dev(a))
    db = to_dev(b)
    dk = to_dev(key)
    half = n_ct // 2
    out_over_a = buf[half:half + n_ct].view(shape)            # shares the second half of a
    with pytest.raises(B.CrossError) as e:
        B.he_mult(da, db, dk, out_over_a, qs, ps, 3)
    assert e.value.code == -1
    with pytest.raises(B.CrossError) as e:
        B.rotate(da, 1, dk, out_over_a, qs, ps, 3)
    assert e.value.code == -1
    kb = buf[2 * n_ct:2 * n_ct + n_key].view(key.shape)
    kb.copy_(dk)
    out_over_key = buf[2 * n_ct - 16:3 * n_ct - 16].view(shape)  # last 16 words overlap the key
    with pytest.raises(B.CrossError) as e:
        B.he_mult(da, db, kb, out_over_key, qs, ps, 3)
    assert e.value.code == -1
    with pytest.raises(B.CrossError) as e:
        B.rotate(da, 1, kb, out_over_key, qs, ps, 3)
    assert e.value.code == -1
    # adjacent, non-overlapping buffers are accepted and match the oracle
    out_ok = buf[n_ct:2 * n_ct].view(shape)
    B.he_mult(da, db, dk, out_ok, qs, ps, 3)
    got = to_host(out_ok)
    for k in range(2):
        assert np.array_equal(got[k], CK.he_mult(a[k], b[k], key, qs, ps, 3))
    # BConv: out overlapping in
    src, dst = synthetic.primes(5)[:2], synthetic.primes(5)[2:]
    x = synthetic.residues(synthetic.rng(5), (1,), src, 256)
    bb = torch.zeros(2 * 256 + 3 * 256, dtype=torch.int32, device="cuda")
    bb[:512].copy_(to_dev(x).reshape(-1))
    with pytest.raises(B.CrossError) as e:
        B.bconv(bb[:512].view(1, 2, 256), src, dst, bb[256:256 + 768].view(1, 3, 256))
    assert e.value.code == -1


@pytest.mark.parametrize("log_n,L,K,batch", [(10, 5, 2, 2), (16, 24, 8, 1)])
def test_he_mult_on_butterfly_engine(log_n, L, K, batch):
    # the whole HE-Mult with its NTTs on the radix-2 butterfly kernels: same result
    from paper_2501_07047_amd import binding as B
    qs, ps, a, b, key = synthetic.ckks_pair(24 + log_n, log_n, L, 3, K, batch)
    out = _empty(a.shape)
    B.set_ntt_engine("butterfly")
    try:
        B.he_mult(to_dev(a), to_dev(b), to_dev(key), out, qs, ps, 3)
        got = to_host(out)
    finally:
        B.set_ntt_engine("mfma")
    for k in range(batch):
        assert np.array_equal(got[k], CK.he_mult(a[k], b[k], key, qs, ps, 3)), "ciphertext %d" % k


def test_modup_moddown_n2_16_L24():
    """The public ModUp and ModDown entry points at N = 2^16, L = 24, dnum = 3, K = 8, two
    polynomials (ModDown takes the fused-tail row kernel at this size)."""
    from paper_2501_07047_amd import binding as B
    qs, ps, a, _, _ = synthetic.ckks_pair(21, 16, 24, 3, 8, 1)
    d = a[0]                                     # two polynomials [2][L][N]
    d = _with_edges(d[None], qs)[0]
    ext = _empty((2, 3, 32, 1 << 16))
    B.keyswitch_modup(to_dev(d), ext, qs, ps, 3)
    got = to_host(ext)
    refs = [CK.modup(d[p], qs, ps, 3) for p in range(2)]
    for p in range(2):
        assert np.array_equal(got[p], refs[p]), "ModUp of polynomial %d" % p
    src = np.stack([refs[p][1] for p in range(2)])          # digit 1 extensions [2][L+K][N]
    out = _empty((2, 24, 1 << 16))
    B.keyswitch_moddown(to_dev(src), out, qs, ps, 3)
    got = to_host(out)
    for p in range(2):
        assert np.array_equal(got[p], CK.moddown(src[p], qs, ps)), "ModDown of polynomial %d" % p
