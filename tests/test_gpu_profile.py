"""Kernel timing by dispatch-stamped events: per-family filter and report contents."""
import numpy as np
import pytest

import synthetic
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def test_profile_all_and_only_one_family():
    from paper_2501_07047_amd import binding as B
    primes, x = synthetic.ntt_batch(8, 13, 2, 2)
    d = to_dev(x)
    B.profile_report()
    try:
        B.profile_enable(True)
        B.ntt_forward(d, primes)
        B.ntt_inverse(d, primes)
        rep = B.profile_report()
        assert set(rep) == {"bat_gemm_left", "ntt_rows"}
        assert all(n == 2 and ms > 0 for n, ms in rep.values())
        B.profile_only("ntt_rows")
        for _ in range(3):
            B.ntt_forward(d, primes)
            B.ntt_inverse(d, primes)
        rep = B.profile_report()
        assert set(rep) == {"ntt_rows"} and rep["ntt_rows"][0] == 6 and rep["ntt_rows"][1] > 0
    finally:
        B.profile_enable(False)
        B.profile_only(None)
        B.profile_report()
    assert np.array_equal(to_host(d), x)
    # disabled: nothing recorded
    B.ntt_forward(d, primes)
    assert B.profile_report() == {}
