"""GPU parity of HE-Add and Rescale (single and double) against the oracle (bit-exact)."""
import numpy as np
import pytest

import synthetic
from oracle import ckks as CK
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def _empty(shape):
    import torch
    return torch.empty(shape, dtype=torch.int32, device="cuda")


def _oracle_rescale(x, primes, drop):
    return np.stack([CK.rescale(x[p], primes, drop) for p in range(x.shape[0])])


# (log_n, L, drop, npoly): log_n = 5 and 7 run the limb transforms on the butterfly
# kernels, the rest on the BAT GEMMs; npoly = 3 is an odd ciphertext count
@pytest.mark.parametrize("log_n,L,drop,npoly", [(5, 3, 1, 1), (7, 4, 2, 2), (8, 4, 1, 3), (10, 5, 2, 2),
                                                (12, 6, 1, 2), (13, 9, 3, 1)])
def test_rescale_small(log_n, L, drop, npoly):
    from paper_2501_07047_amd import binding as B
    primes, x = synthetic.ntt_batch(100 + log_n, log_n, L, npoly)
    out = _empty((npoly, L - drop, 1 << log_n))
    B.rescale(to_dev(x), out, primes, drop)
    assert np.array_equal(to_host(out), _oracle_rescale(x, primes, drop))


def test_rescale_largest_prime_last():
    # the dropped prime is the largest of the chain: its coefficients must be reduced into the others
    from paper_2501_07047_amd import binding as B
    primes, x = synthetic.ntt_batch(7, 11, 5, 2)
    primes, x = primes[::-1], np.ascontiguousarray(x[:, ::-1])
    out = _empty((2, 4, 1 << 11))
    B.rescale(to_dev(x), out, primes, 1)
    assert np.array_equal(to_host(out), _oracle_rescale(x, primes, 1))


@pytest.mark.parametrize("drop", [1, 2])
def test_rescale_full_size(drop):
    # one ciphertext (two polynomials) at N = 2^16 with L = 24 limbs
    from paper_2501_07047_amd import binding as B
    primes, x = synthetic.ntt_batch(20 + drop, 16, 24, 2)
    out = _empty((1, 2, 24 - drop, 1 << 16))
    B.rescale(to_dev(x.reshape(1, 2, 24, -1)), out, primes, drop)
    assert np.array_equal(to_host(out).reshape(2, 24 - drop, -1), _oracle_rescale(x, primes, drop))


def test_rescale_twice_equals_oracle_twice():
    # a second rescale on the device output: the level chain of a multiplicative depth-2 circuit
    from paper_2501_07047_amd import binding as B
    primes, x = synthetic.ntt_batch(31, 12, 6, 2)
    o1 = _empty((2, 5, 1 << 12))
    o2 = _empty((2, 4, 1 << 12))
    B.rescale(to_dev(x), o1, primes, 1)
    B.rescale(o1, o2, primes[:5], 1)
    ref = _oracle_rescale(_oracle_rescale(x, primes, 1), primes[:5], 1)
    assert np.array_equal(to_host(o2), ref)


@pytest.mark.parametrize("log_n,L,npoly", [(4, 2, 3), (16, 24, 16)])
def test_he_add(log_n, L, npoly):
    from paper_2501_07047_amd import binding as B
    primes, a = synthetic.ntt_batch(40 + log_n, log_n, L, npoly)
    _, b = synthetic.ntt_batch(50 + log_n, log_n, L, npoly)
    ref = CK.he_add(a, b, primes)
    da, db = to_dev(a), to_dev(b)
    out = _empty(a.shape)
    B.he_add(da, db, out, primes)
    assert np.array_equal(to_host(out), ref)
    B.he_add(da, db, da, primes)             # out aliases a
    assert np.array_equal(to_host(da), ref)


def test_rescale_and_add_argument_errors():
    from paper_2501_07047_amd import binding as B
    primes, x = synthetic.ntt_batch(3, 8, 3, 2)
    dx = to_dev(x)
    with pytest.raises(B.CrossError) as e:
        B.rescale(dx, _empty((2, 0, 256)), primes, 3)       # drop must be below L
    assert e.value.code == -1
    with pytest.raises(B.CrossError) as e:
        B.rescale(dx, dx.view(-1)[:2 * 2 * 256].view(2, 2, 256), primes, 1)   # out overlaps in
    assert e.value.code == -1
    with pytest.raises(B.CrossError):
        B.rescale(dx, _empty((2, 2, 256)), [primes[0], primes[0], primes[2]], 1)   # repeated prime
    with pytest.raises(ValueError):
        B.rescale(dx, _empty((2, 2, 256)), primes[:2], 1)   # primes do not match L
    with pytest.raises(B.CrossError) as e:
        B.he_add(dx, dx, _empty(x.shape), [primes[0], primes[1], 15])   # 15 is not a prime
    assert e.value.code == -2
