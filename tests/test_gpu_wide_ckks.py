"""GPU parity of the CKKS operators with wide primes (2^28 <= q < 2^31) against the oracle.

The NTT runs its byte form, BConv its byte form, and the VALU products (tensor,
key-switch inner product) keep their Barrett remainder in 64 bits; the fused row
kernels are narrow-only, so these shapes take the separate kernels.  Q and P both
wide, and narrow Q with wide P (larger special primes).  Batch 5 covers a full and
a partial group of the inner product's four-ciphertext threads.
"""
import numpy as np
import pytest

import synthetic
from oracle import ckks as CK
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def _empty(shape):
    import torch
    return torch.empty(shape, dtype=torch.int32, device="cuda")


def _params(L, K, form):
    wp = synthetic.wide_primes(L + K)
    if form == "wide":
        return wp[:L], wp[L:L + K]
    return synthetic.primes(L), wp[:K]              # narrow Q, wide P


def _inputs(seed, log_n, qs, ps, dnum, batch):
    g = synthetic.rng(seed)
    n = 1 << log_n
    a = synthetic.residues(g, (batch, 2), qs, n)
    b = synthetic.residues(g, (batch, 2), qs, n)
    key = synthetic.residues(synthetic.rng(seed + 1000), (dnum, 2), qs + ps, n)
    for i, q in enumerate(qs):                       # extreme residues
        a[0, :, i, :3] = [0, 1, q - 1]
        b[-1, :, i, -2:] = q - 1
    return a, b, key


@pytest.mark.parametrize("log_n,L,K,dnum,batch,form", [(10, 4, 2, 2, 5, "wide"), (12, 6, 3, 2, 2, "narrow_q"),
                                                       (16, 4, 2, 2, 1, "wide")])
def test_he_mult_wide_primes(log_n, L, K, dnum, batch, form):
    from paper_2501_07047_amd import binding as B
    qs, ps = _params(L, K, form)
    a, b, key = _inputs(log_n + L, log_n, qs, ps, dnum, batch)
    out = _empty(a.shape)
    B.he_mult(to_dev(a), to_dev(b), to_dev(key), out, qs, ps, dnum)
    got = to_host(out)
    for bi in range(batch):
        assert np.array_equal(got[bi], CK.he_mult(a[bi], b[bi], key, qs, ps, dnum)), "ciphertext %d" % bi


@pytest.mark.parametrize("log_n,L,K,dnum,steps,form", [(10, 4, 2, 2, 3, "wide"), (12, 5, 2, 3, -1, "narrow_q")])
def test_rotate_wide_primes(log_n, L, K, dnum, steps, form):
    from paper_2501_07047_amd import binding as B
    qs, ps = _params(L, K, form)
    a, _, key = _inputs(log_n * 7 + L, log_n, qs, ps, dnum, 2)
    out = _empty(a.shape)
    B.rotate(to_dev(a), steps, to_dev(key), out, qs, ps, dnum)
    got = to_host(out)
    for bi in range(2):
        assert np.array_equal(got[bi], CK.rotate(a[bi], steps, key, qs, ps, dnum)), "ciphertext %d" % bi


@pytest.mark.parametrize("log_n,L,drop", [(10, 5, 1), (12, 6, 2)])
def test_rescale_wide_primes(log_n, L, drop):
    from paper_2501_07047_amd import binding as B
    qs = synthetic.wide_primes(L)
    x = synthetic.residues(synthetic.rng(log_n + L), (3,), qs, 1 << log_n)
    out = _empty((3, L - drop, 1 << log_n))
    B.rescale(to_dev(x), out, qs, drop)
    got = to_host(out)
    for p in range(3):
        assert np.array_equal(got[p], CK.rescale(x[p], qs, drop)), "polynomial %d" % p
