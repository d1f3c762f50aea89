"""GPU parity of the NTT with wide primes (2^28 <= q < 2^31) against the oracle,
bit-exact: byte operands biased to b - 128, balanced signed-digit tables with
row corrections, signed ChunkMerge (32-bit at contraction depths up to 64, else
64-bit) and Montgomery step, in the two- and three-factor forms and the butterfly
path."""
import numpy as np
import pytest

import synthetic
from oracle.ntt import bitrev, horner_eval, intt_gs, ntt_ct
from oracle.primes import psi as psi_of
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def _oracle(x, primes, inverse=False):
    n = x.shape[-1]
    out = np.empty(x.shape, dtype=np.uint64)
    f = intt_gs if inverse else ntt_ct
    for i, q in enumerate(primes):
        out[:, i] = f(x[:, i].astype(np.uint64), q, psi_of(q, n))
    return out


def _inputs(seed, log_n, primes, batch):
    x = synthetic.residues(synthetic.rng(seed), (batch,), primes, 1 << log_n)
    # extremes of every byte: 0, 1, q - 1, and words whose bytes are all 0x7f / 0x80
    for i, q in enumerate(primes):
        x[0, i, :5] = [0, 1, q - 1, 0x7F7F7F7F % q, 0x80808080 % q]
    return x


def _roundtrip(B, x, primes):
    ref = _oracle(x, primes)
    d = to_dev(x)
    B.ntt_forward(d, primes)
    assert np.array_equal(to_host(d), ref)
    B.ntt_inverse(d, primes)
    assert np.array_equal(to_host(d), x)
    # the inverse of an arbitrary (not forward-produced) input as well
    y = _inputs(7, int(np.log2(x.shape[-1])), primes, 1)
    dy = to_dev(y)
    B.ntt_inverse(dy, primes)
    assert np.array_equal(to_host(dy), _oracle(y, primes, inverse=True))


# every row-kernel family: LDS tables (16 x 16, 32 x 16, 32 x 32, 64 x 32, 16 x 64) and
# global-memory tables (64 x 64); row-side steps of 32, 64 and 16 rows
@pytest.mark.parametrize("log_n,log_r,log_c1,L,batch", [(13, 5, 4, 2, 1), (14, 5, 5, 2, 2), (15, 6, 5, 1, 3),
                                                        (16, 6, 5, 2, 2), (16, 5, 6, 1, 1), (16, 4, 6, 1, 1),
                                                        (14, 4, 4, 2, 1), (16, 4, 6, 1, 2)])
def test_wide_three_factor_matches_oracle(log_n, log_r, log_c1, L, batch):
    from paper_2501_07047_amd import binding as B
    B.set_ntt_split3(log_n, log_r, log_c1)
    try:
        primes = synthetic.wide_primes(L)
        _roundtrip(B, _inputs(500 + log_n + log_c1, log_n, primes, batch), primes)
    finally:
        B.set_ntt_split3(log_n, 0, 0)


@pytest.mark.parametrize("log_n,L,batch", [(4, 2, 1), (7, 3, 2), (8, 1, 1), (10, 2, 3), (12, 3, 2), (13, 2, 1),
                                           (16, 1, 1)])
def test_wide_default_paths(log_n, L, batch):
    # butterfly below N = 2^8, two factors up to 2^12, three factors above
    from paper_2501_07047_amd import binding as B
    primes = synthetic.wide_primes(L)
    _roundtrip(B, _inputs(600 + log_n, log_n, primes, batch), primes)


@pytest.mark.parametrize("log_n,log_r", [(12, 4), (12, 8), (10, 5)])
def test_wide_two_factor_splits(log_n, log_r):
    from paper_2501_07047_amd import binding as B
    B.set_ntt_split(log_n, log_r)
    try:
        primes = synthetic.wide_primes(2)
        _roundtrip(B, _inputs(700 + log_r, log_n, primes, 2), primes)
    finally:
        B.set_ntt_split(log_n, log_n // 2)


@pytest.mark.parametrize("tile", [0, 1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_wide_every_tile_request(tile):
    # the wide form runs the staged 256 x 128, 128 x 64 and 64 x 64 tiles; other requests
    # fall back to the automatic choice and stay exact
    from paper_2501_07047_amd import binding as B
    B.set_gemm_tile(tile)
    try:
        primes = synthetic.wide_primes(2)
        for log_n in (12, 14):
            _roundtrip(B, _inputs(800 + tile, log_n, primes, 2), primes)
    finally:
        B.set_gemm_tile(0)


def test_wide_and_narrow_limbs_in_one_call():
    from paper_2501_07047_amd import binding as B
    for log_n in (12, 16):
        primes = [synthetic.wide_primes(2)[0], synthetic.primes(1)[0], synthetic.wide_primes(2)[1]]
        _roundtrip(B, _inputs(900 + log_n, log_n, primes, 2), primes)


def test_wide_butterfly_agrees_with_mfma():
    from paper_2501_07047_amd import binding as B
    primes = synthetic.wide_primes(2)
    for log_n in (12, 14):
        x = _inputs(950 + log_n, log_n, primes, 2)
        a, b = to_dev(x), to_dev(x)
        B.ntt_forward(a, primes)
        B.ntt_forward_butterfly(b, primes)
        assert np.array_equal(to_host(a), to_host(b))
        assert np.array_equal(to_host(b), _oracle(x, primes))
        B.ntt_inverse_butterfly(b, primes)
        assert np.array_equal(to_host(b), x)


def test_wide_full_size_spot_checks():
    # N = 2^16, 8 wide limbs x 16 polynomials (the benchmarked launch shape): Horner spot
    # checks of every limb, one limb in full, exact inverse
    from paper_2501_07047_amd import binding as B
    primes = synthetic.wide_primes(8)
    n = 1 << 16
    x = _inputs(3, 16, primes, 16)
    d = to_dev(x)
    B.ntt_forward(d, primes)
    got = to_host(d)
    g = np.random.Generator(np.random.PCG64(9))
    for i, q in enumerate(primes):
        psi = psi_of(q, n)
        for b in (0, 15):
            pos = g.integers(0, n, 6)
            xs = [pow(psi, 2 * bitrev(int(p), 16) + 1, q) for p in pos]
            assert np.array_equal(got[b, i, pos], horner_eval(x[b, i], q, xs))
    assert np.array_equal(got[:, 5], _oracle(x[:, 5:6], primes[5:6])[:, 0])
    B.ntt_inverse(d, primes)
    assert np.array_equal(to_host(d), x)


def test_wide_prime_errors():
    import torch
    from oracle.primes import is_prime
    from paper_2501_07047_amd import binding as B
    q = synthetic.wide_primes(1)[0]
    d = to_dev(np.zeros((1, 1, 1 << 13), dtype=np.uint32))
    B.set_ntt_reduction("barrett")                 # the wide form has a Montgomery epilogue only
    try:
        with pytest.raises(B.CrossError) as e:
            B.ntt_forward(d, [q])
        assert e.value.code == -7
    finally:
        B.set_ntt_reduction("montgomery")
    big = next(p for p in range((1 << 31) + 1, 1 << 32, 1 << 17) if is_prime(p))
    with pytest.raises(B.CrossError) as e:          # 2^31 and above
        B.ntt_forward(d, [big])
    assert e.value.code == -4
    a = torch.zeros((1, 1, 1 << 13), dtype=torch.int32, device="cuda")
    with pytest.raises(B.CrossError) as e:          # the other operations keep q < 2^28
        B.poly_mul(a, a.clone(), torch.empty_like(a), [q])
    assert e.value.code == -4
