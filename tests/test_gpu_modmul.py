"""GPU parity of VecModMul under the four modular reductions (Barrett, Montgomery,
Shoup, BAT-lazy on MFMA) against the plain definition a * w mod q (bit-exact)."""
import numpy as np
import pytest

import synthetic
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu

METHODS = ["barrett", "montgomery", "shoup", "bat_lazy"]


def _empty(shape):
    import torch
    return torch.empty(shape, dtype=torch.int32, device="cuda")


def _ref(a, w, primes):
    out = np.empty_like(a)
    for i, q in enumerate(primes):
        out[:, i] = a[:, i].astype(np.uint64) * w[i].astype(np.uint64) % np.uint64(q)
    return out


@pytest.mark.parametrize("log_n,L,npoly", [(8, 3, 2), (12, 4, 3), (16, 24, 16)])
@pytest.mark.parametrize("method", METHODS)
def test_vec_modmul_matches_definition(method, log_n, L, npoly):
    from paper_2501_07047_amd import binding as B
    primes, a = synthetic.ntt_batch(60 + log_n, log_n, L, npoly)
    _, w = synthetic.ntt_batch(70 + log_n, log_n, L, 1)
    w = w[0]
    # edge residues in the first positions of every limb
    for i, q in enumerate(primes):
        a[0, i, :4] = [0, 1, q - 1, q - 1]
        w[i, :4] = [q - 1, q - 1, q - 1, 1]
    prep = B.vec_modmul_prepare(to_dev(w), primes, method)
    out = _empty(a.shape)
    B.vec_modmul(to_dev(a), prep, out, primes, method)
    assert np.array_equal(to_host(out), _ref(a, w, primes))


def test_prepared_forms_and_aliasing():
    from paper_2501_07047_amd import binding as B
    primes, w = synthetic.ntt_batch(81, 10, 3, 1)
    w = w[0]
    dw = to_dev(w)
    mont = to_host(B.vec_modmul_prepare(dw, primes, "montgomery")[0])
    sh = to_host(B.vec_modmul_prepare(dw, primes, "shoup"))
    for i, q in enumerate(primes):
        assert [int(v) for v in mont[i, :64]] == [(int(x) << 32) % q for x in w[i, :64]]
        assert np.array_equal(sh[0, i], w[i])
        assert [int(v) for v in sh[1, i, :64]] == [(int(x) << 32) // q for x in w[i, :64]]
    _, a = synthetic.ntt_batch(82, 10, 3, 2)
    da = to_dev(a)
    B.vec_modmul(da, B.vec_modmul_prepare(dw, primes, "bat_lazy"), da, primes, "bat_lazy")   # out aliases a
    assert np.array_equal(to_host(da), _ref(a, w, primes))


def test_vec_modmul_errors():
    from paper_2501_07047_amd import binding as B
    primes, w = synthetic.ntt_batch(83, 6, 2, 1)
    dw = to_dev(w[0])
    with pytest.raises(B.CrossError) as e:
        B.vec_modmul_prepare(dw, primes, "bat_lazy")            # N < 256: one prime per wave needed
    assert e.value.code == -7
    prep = B.vec_modmul_prepare(dw, primes, "barrett")
    _, a = synthetic.ntt_batch(84, 6, 2, 1)
    out = _empty(a.shape)
    B.vec_modmul(to_dev(a), prep, out, primes, "barrett")       # small N is fine for the VALU methods
    assert np.array_equal(to_host(out), _ref(a, w[0], primes))
    with pytest.raises(B.CrossError) as e:
        B.vec_modmul_prepare(dw, [primes[0], 15], "shoup")      # 15 is not prime
    assert e.value.code == -2
