"""GPU parity of the key-switching streams in both forms (plain VALU and chunked:
evaluation-key BAT inner product, chunk-convolution tensor product) against the
oracle's plain definitions, bit-exact."""
import numpy as np
import pytest

import synthetic
from oracle import ckks as CK
from oracle import streams as S
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

FORMS = ["valu", "chunked"]


def _empty(shape):
    import torch
    return torch.empty(shape, dtype=torch.int32, device="cuda")


def _ks_inputs(seed, log_n, LK, dnum, B, edges=True):
    p = synthetic.primes(LK)
    g = synthetic.rng(seed)
    ext = synthetic.residues(g, (B, dnum), p, 1 << log_n)
    key = synthetic.residues(synthetic.rng(seed + 1000), (dnum, 2), p, 1 << log_n)
    if edges:
        for t, q in enumerate(p):
            ext[:, :, t, :3] = [0, 1, q - 1]
            key[:, :, t, :3] = [q - 1, q - 1, q - 1]
    return p, ext, key


def _oracle_ip(ext, key, p):
    return np.stack([CK.inner_product(ext[b], key, p) for b in range(ext.shape[0])])


def test_evk_bat_expansion_matches_oracle():
    from paper_2501_07047_amd import binding as B
    p, _, key = _ks_inputs(1, 6, 5, 3, 1)
    kb = to_host(B.evk_bat_prepare(to_dev(key), p))             # [dnum][2][LK][N][4] words
    for t, q in enumerate(p):
        E = S.evk_bat_expand(key[:, :, t, :], q)                # [dnum][2][N][l][i]
        words = sum(E[..., i].astype(np.uint64) << np.uint64(8 * i) for i in range(4))   # word l
        assert np.array_equal(kb[:, :, t, :, :].astype(np.uint64), words)


@pytest.mark.parametrize("log_n,LK,dnum,B", [(4, 3, 1, 1), (6, 5, 3, 2), (10, 9, 4, 3)])
@pytest.mark.parametrize("form", FORMS)
def test_inner_product_small(form, log_n, LK, dnum, B):
    from paper_2501_07047_amd import binding as Bd
    p, ext, key = _ks_inputs(10 + log_n, log_n, LK, dnum, B)
    dkey = to_dev(key)
    if form == "chunked":
        dkey = Bd.evk_bat_prepare(dkey, p)
    out = _empty((B, 2, LK, 1 << log_n))
    Bd.keyswitch_inner_product(to_dev(ext), dkey, out, p, form)
    assert np.array_equal(to_host(out), _oracle_ip(ext, key, p))


@pytest.mark.parametrize("form", FORMS)
def test_inner_product_full_size(form):
    # N = 2^16, L + K = 32 limbs, dnum = 3, two ciphertexts
    from paper_2501_07047_amd import binding as Bd
    p, ext, key = _ks_inputs(77, 16, 32, 3, 2)
    dkey = to_dev(key)
    if form == "chunked":
        dkey = Bd.evk_bat_prepare(dkey, p)
    out = _empty((2, 2, 32, 1 << 16))
    Bd.keyswitch_inner_product(to_dev(ext), dkey, out, p, form)
    assert np.array_equal(to_host(out), _oracle_ip(ext, key, p))


@pytest.mark.parametrize("log_n,L,B", [(4, 2, 1), (8, 3, 3), (16, 24, 2)])
@pytest.mark.parametrize("form", FORMS)
def test_tensor(form, log_n, L, B):
    from paper_2501_07047_amd import binding as Bd
    qs, _, a, b, _ = synthetic.ckks_pair(30 + log_n, log_n, L, 3, 1, B)
    for i, q in enumerate(qs):
        a[:, :, i, :2] = q - 1
        b[:, :, i, :2] = [q - 1, 0]
    out, d2 = _empty(a.shape), _empty((B, L, 1 << log_n))
    Bd.tensor(to_dev(a), to_dev(b), out, d2, qs, form)
    ref = np.stack([CK.tensor(a[k], b[k], qs) for k in range(B)])        # [B][3][L][N]
    assert np.array_equal(to_host(out), ref[:, :2])
    assert np.array_equal(to_host(d2), ref[:, 2])


def test_stream_argument_errors():
    from paper_2501_07047_amd import binding as Bd
    p, ext, key = _ks_inputs(3, 6, 3, 2, 1)
    dext, dkey = to_dev(ext), to_dev(key)
    with pytest.raises(Bd.CrossError) as e:            # out overlaps ext
        Bd.keyswitch_inner_product(dext, dkey, dext.view(-1)[:2 * 3 * 64].view(1, 2, 3, 64), p, "valu")
    assert e.value.code == -1
    with pytest.raises(Bd.CrossError) as e:            # 15 is not a prime
        Bd.evk_bat_prepare(dkey, [p[0], p[1], 15])
    assert e.value.code == -2
    qs, _, a, b, _ = synthetic.ckks_pair(4, 6, 2, 2, 1, 1)
    da, db = to_dev(a), to_dev(b)
    with pytest.raises(Bd.CrossError) as e:            # d2 overlaps out
        out = _empty(a.shape)
        Bd.tensor(da, db, out, out.view(-1)[:2 * 64].view(1, 2, 64), qs, "chunked")
    assert e.value.code == -1
