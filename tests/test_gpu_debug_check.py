"""GPU tests of the debug mode (residue-range preconditions): with the check on,
valid inputs give the usual results; a residue at or above its prime is reported
as CROSS_EDOMAIN with its position, and nothing is computed."""
import numpy as np
import pytest

import synthetic
from oracle import ckks as CK
from oracle.ntt import ntt_ct
from oracle.primes import psi as psi_of
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture
def debug_on():
    from paper_2501_07047_amd import binding as B
    B.set_debug_check(True)
    try:
        yield B
    finally:
        B.set_debug_check(False)


def test_valid_inputs_pass_the_check(debug_on):
    B = debug_on
    primes, x = synthetic.ntt_batch(61, 12, 3, 2)
    for i, q in enumerate(primes):
        x[:, i, :2] = [0, q - 1]
    d = to_dev(x)
    B.ntt_forward(d, primes)
    got = to_host(d)
    for i, q in enumerate(primes):
        assert np.array_equal(got[:, i], ntt_ct(x[:, i].astype(np.uint64), q, psi_of(q, 1 << 12)))
    qs, ps, a, b, key = synthetic.ckks_pair(62, 10, 4, 2, 2, 1)
    import torch
    out = torch.empty(a.shape, dtype=torch.int32, device="cuda")
    B.he_mult(to_dev(a), to_dev(b), to_dev(key), out, qs, ps, 2)
    assert np.array_equal(to_host(out)[0], CK.he_mult(a[0], b[0], key, qs, ps, 2))


def test_out_of_range_residue_is_reported_and_nothing_runs(debug_on):
    import torch
    B = debug_on
    primes, x = synthetic.ntt_batch(63, 12, 3, 2)
    x[1, 2, 777] = primes[2]                   # q itself: polynomial 1, limb 2, coefficient 777
    d = to_dev(x)
    with pytest.raises(B.CrossError) as e:
        B.ntt_forward(d, primes)
    assert e.value.code == -8
    msg = str(e.value)
    assert "polynomial 1" in msg and "limb 2" in msg and "coefficient 777" in msg
    assert np.array_equal(to_host(d), x)       # the transform did not run
    # HE-Mult: a key residue out of range (limb 5 = the first special prime's limb of digit 0)
    qs, ps, a, b, key = synthetic.ckks_pair(64, 10, 4, 2, 2, 1)
    key[0, 1, 5, 3] = (qs + ps)[5] + 7
    out = torch.zeros(a.shape, dtype=torch.int32, device="cuda")
    with pytest.raises(B.CrossError) as e:
        B.he_mult(to_dev(a), to_dev(b), to_dev(key), out, qs, ps, 2)
    assert e.value.code == -8 and "relin_key" in str(e.value)
    assert not to_host(out).any()


def test_check_is_off_by_default():
    from paper_2501_07047_amd import binding as B
    primes, x = synthetic.ntt_batch(65, 10, 1, 1)
    x[0, 0, 0] = 0                              # a valid input; the check would pass anyway
    d = to_dev(x)
    B.ntt_forward(d, primes)                    # no synchronising check, no error
    B.ntt_inverse(d, primes)
    assert np.array_equal(to_host(d), x)
