"""GPU test of the allocation-free NTT (cross_ntt_noalloc) through the C ABI: its
output equals cross_ntt_forward / cross_ntt_inverse on the same input, on two calls
in a row (the second smaller), for both directions; oversize inputs and primes
without tables are rejected before anything is enqueued."""
import ctypes

import numpy as np
import pytest

import synthetic
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def _noalloc(B, d, primes, inverse, batch=None, L=None):
    ctx = B.context(d.device.index)
    arr = (ctypes.c_uint32 * len(primes))(*primes)
    nb, nl, n = d.shape
    st = B.lib().cross_ntt_noalloc(ctx, n.bit_length() - 1, arr, L or nl, batch or nb,
                                   ctypes.c_void_p(d.data_ptr()), int(inverse), B._stream(d))
    return st, ctx


@pytest.mark.parametrize("inverse", [False, True])
def test_noalloc_matches_ntt_entry_point_two_calls(inverse):
    import torch
    from paper_2501_07047_amd import binding as B
    ref_fn = B.ntt_inverse if inverse else B.ntt_forward
    # first call: the full headline shape (N = 2^16, 24 limbs, 16 polynomials = 96 MiB of
    # scratch); second call: a smaller one (N = 2^13, 5 limbs, 3 polynomials)
    for seed, log_n, L, batch in ((31, 16, 24, 16), (32, 13, 5, 3)):
        primes, x = synthetic.ntt_batch(seed, log_n, L, batch)
        ref = to_dev(x)
        ref_fn(ref, primes)                       # also builds the tables on the context
        d = to_dev(x)
        st, ctx = _noalloc(B, d, primes, inverse)
        assert st == 0, B.lib().cross_last_error(ctx)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(d), to_host(ref)), "shape %s" % ((log_n, L, batch),)


def test_noalloc_round_trip_and_small_sizes():
    import torch
    from paper_2501_07047_amd import binding as B
    for log_n, L, batch in ((12, 3, 2), (7, 2, 1), (16, 2, 1)):
        primes, x = synthetic.ntt_batch(40 + log_n, log_n, L, batch)
        B.ntt_forward(to_dev(x), primes)
        d = to_dev(x)
        st, ctx = _noalloc(B, d, primes, False)
        assert st == 0, B.lib().cross_last_error(ctx)
        st, ctx = _noalloc(B, d, primes, True)
        assert st == 0, B.lib().cross_last_error(ctx)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(d), x)


def test_noalloc_rejects_oversize_and_unknown_primes():
    import torch
    from paper_2501_07047_amd import binding as B
    primes, x = synthetic.ntt_batch(50, 16, 24, 1)
    d = to_dev(x)
    B.ntt_forward(to_dev(x), primes)
    # 24 limbs x 22 polynomials x 2^16 words = 132 MiB > 128 MiB: rejected on the host,
    # before any launch (the buffer itself is never touched)
    st, _ = _noalloc(B, d, primes, False, batch=22)
    assert st == -1
    # a prime far down the chain whose tables no other call builds at N = 2^9
    p11 = synthetic.primes(121)[120:]
    y = synthetic.residues(synthetic.rng(51), (1,), p11, 1 << 9)
    dy = to_dev(y)
    st, _ = _noalloc(B, dy, p11, False)
    assert st == -7
    torch.cuda.synchronize()
    assert np.array_equal(to_host(dy), y)         # nothing ran
    assert np.array_equal(to_host(d), x)
