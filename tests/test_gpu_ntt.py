"""GPU parity of the NTT entry points against the oracle (bit-exact)."""
import numpy as np
import pytest

import synthetic
from oracle.ntt import ntt_def, intt_def, ntt_ct, intt_gs, horner_eval, bitrev
from oracle.primes import psi as psi_of
from tests.gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


def _oracle_ntt(x, primes, inverse=False):
    n = x.shape[-1]
    out = np.empty(x.shape, dtype=np.uint64)
    f = intt_gs if inverse else ntt_ct
    for i, q in enumerate(primes):
        out[:, i] = f(x[:, i].astype(np.uint64), q, psi_of(q, n))
    return out


def test_config1_n4096_against_definition():
    from paper_2501_07047_amd import binding as B
    primes, x = synthetic.ntt_batch(0, 12, 1, 1)
    q = primes[0]
    psi = psi_of(q, 4096)
    d = to_dev(x)
    B.ntt_forward(d, primes)
    got = to_host(d)[0, 0]
    ref = ntt_def(x[0, 0], q, psi)
    assert np.array_equal(got, ref)
    B.ntt_inverse(d, primes)
    assert np.array_equal(to_host(d), x)
    dd = to_dev(ref[None, None])
    B.ntt_inverse(dd, primes)
    assert np.array_equal(to_host(dd)[0, 0], intt_def(ref, q, psi))


@pytest.mark.parametrize("log_n,L,batch", [(8, 1, 1), (9, 2, 3), (10, 3, 5), (11, 2, 2),
                                           (12, 4, 3), (13, 2, 2), (14, 3, 1), (15, 2, 3),
                                           (16, 2, 1)])
def test_sizes_and_ragged_batches(log_n, L, batch):
    from paper_2501_07047_amd import binding as B
    primes, x = synthetic.ntt_batch(log_n * 100 + L, log_n, L, batch)
    x[0, 0, :4] = [0, primes[0] - 1, 1, primes[0] - 2]
    ref = _oracle_ntt(x, primes)
    d = to_dev(x)
    B.ntt_forward(d, primes)
    assert np.array_equal(to_host(d), ref)
    B.ntt_inverse(d, primes)
    assert np.array_equal(to_host(d), x)


@pytest.mark.parametrize("log_n", [4, 5, 6, 7, 8, 12])
def test_butterfly_matches_oracle(log_n):
    from paper_2501_07047_amd import binding as B
    primes, x = synthetic.ntt_batch(log_n, log_n, 3, 2)
    ref = _oracle_ntt(x, primes)
    d = to_dev(x)
    B.ntt_forward_butterfly(d, primes)
    assert np.array_equal(to_host(d), ref)
    B.ntt_inverse_butterfly(d, primes)
    assert np.array_equal(to_host(d), x)
    # small sizes route cross_ntt_forward to the butterfly kernels as well
    d = to_dev(x)
    B.ntt_forward(d, primes)
    assert np.array_equal(to_host(d), ref)


@pytest.mark.parametrize("log_n,log_r", [(12, 4), (12, 8), (14, 5), (16, 7), (16, 9)])
def test_other_splits(log_n, log_r):
    from paper_2501_07047_amd import binding as B
    B.set_ntt_split(log_n, log_r)
    try:
        primes, x = synthetic.ntt_batch(log_r, log_n, 2, 2)
        ref = _oracle_ntt(x, primes)
        d = to_dev(x)
        B.ntt_forward(d, primes)
        assert np.array_equal(to_host(d), ref)
        B.ntt_inverse(d, primes)
        assert np.array_equal(to_host(d), x)
    finally:
        B.set_ntt_split(log_n, log_n // 2)


@pytest.mark.parametrize("split", ["default", "256x256"])
def test_config2_full_size_spot_checks(split):
    # N = 2^16, L = 24, 8 ciphertexts x 2 polys: in the library's default split (64 x 32 x 32,
    # the launch shape the bench's headline times) and as the two-factor 256 x 256 form
    from paper_2501_07047_amd import binding as B
    primes, x = synthetic.ntt_batch(2, 16, 24, 16)
    d = to_dev(x)
    if split == "256x256":
        B.set_ntt_split(16, 8)
    try:
        B.ntt_forward(d, primes)
        got = to_host(d)
        B.ntt_inverse(d, primes)
        assert np.array_equal(to_host(d), x)
    finally:
        B.set_ntt_split3(16, 0, 0)
    d = to_dev(got)
    bf = to_dev(x)
    B.ntt_forward_butterfly(bf, primes)
    assert np.array_equal(to_host(bf), got)            # two independent GPU paths agree
    g = np.random.Generator(np.random.PCG64(123))
    n = 1 << 16
    for limb in (0, 7, 23):
        q = primes[limb]
        psi = psi_of(q, n)
        for b in (0, 15):
            pos = g.integers(0, n, 16)
            xs = [pow(psi, 2 * bitrev(int(p), 16) + 1, q) for p in pos]
            assert np.array_equal(got[b, limb, pos], horner_eval(x[b, limb], q, xs))
    full = ntt_ct(x[:, 11].astype(np.uint64), primes[11], psi_of(primes[11], n))
    assert np.array_equal(got[:, 11], full)
    B.ntt_inverse(d, primes)
    assert np.array_equal(to_host(d), x)


def test_argument_errors():
    import torch
    from paper_2501_07047_amd import binding as B
    d = torch.zeros((1, 1, 4096), dtype=torch.int32, device="cuda")
    with pytest.raises(B.CrossError) as e:
        B.ntt_forward(d, [268042241 + 2])
    assert e.value.code in (-2, -3)
    with pytest.raises(B.CrossError) as e:
        B.ntt_forward(d, [7681])
    assert e.value.code == -3
    with pytest.raises(ValueError):
        B.ntt_forward(torch.zeros((1, 1, 1000), dtype=torch.int32, device="cuda"), [268042241])


def test_degenerate_arguments_are_rejected_before_any_launch():
    # empty batch, no limbs, N outside 2^4..2^16, more limbs than the limit, misaligned
    # and null data: every NTT entry point returns CROSS_EINVAL from its host checks and
    # leaves the buffer as it was
    import ctypes
    import torch
    from paper_2501_07047_amd import binding as B
    primes, x = synthetic.ntt_batch(77, 12, 2, 1)
    d = to_dev(x)
    lib, ctx, s = B.lib(), B.context(d.device.index), B._stream(d)
    arr = B._u32_array(primes * 33)                 # 66 entries: long enough for every L below
    ptr = ctypes.c_void_p(d.data_ptr())
    cases = [(12, 2, 0, ptr), (12, 0, 1, ptr), (3, 2, 1, ptr), (17, 2, 1, ptr), (12, 65, 1, ptr),
             (12, 2, 1, ctypes.c_void_p(d.data_ptr() + 4)), (12, 2, 1, None)]
    for fn in ("cross_ntt_forward", "cross_ntt_inverse", "cross_ntt_forward_butterfly",
               "cross_ntt_inverse_butterfly"):
        for log_n, L, batch, p in cases:
            st = getattr(lib, fn)(ctx, log_n, arr, L, batch, p, s)
            assert st == -1, (fn, log_n, L, batch)
            assert lib.cross_last_error(ctx)
    torch.cuda.synchronize()
    assert np.array_equal(to_host(d), x)


def test_degenerate_ckks_batches_are_rejected():
    # an empty batch is an argument error for BConv and HE-Mult as well
    import ctypes
    import torch
    from paper_2501_07047_amd import binding as B
    qs, ps = synthetic.primes(4)[:3], synthetic.primes(4)[3:]
    z = torch.zeros((1, 2, 3, 1 << 10), dtype=torch.int32, device="cuda")
    key = torch.zeros((3, 2, 4, 1 << 10), dtype=torch.int32, device="cuda")
    out = torch.full_like(z, 7)
    lib, ctx, s = B.lib(), B.context(0), B._stream(z)
    prm = B._params(qs, ps, 3, 1 << 10)
    st = lib.cross_he_mult(ctx, ctypes.byref(prm), ctypes.c_void_p(z.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                           ctypes.c_void_p(key.data_ptr()), ctypes.c_void_p(out.data_ptr()), 0, s)
    assert st == -1
    st = lib.cross_bconv(ctx, 10, B._u32_array(qs), 3, B._u32_array(ps), 1, ctypes.c_void_p(z.data_ptr()),
                         ctypes.c_void_p(out.data_ptr()), 0, s)
    assert st == -1
    torch.cuda.synchronize()
    assert bool((out == 7).all())


@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5, 6, 7, 8, 9])
def test_every_tile_shape_is_bit_exact(tile):
    from paper_2501_07047_amd import binding as B
    B.set_gemm_tile(tile)
    # (log_n, log_r or None for the default split, L, batch).  13 / 7 gives V = 64
    # columns per polynomial on the row side, so 3 polynomials leave a ragged
    # last column tile; 16 / 10 and 16 / 6 put a 1024-input contraction (the
    # 64-bit ChunkMerge) on either side.
    cases = ((16, 8, 2, 3), (12, None, 3, 2), (10, None, 2, 1), (14, None, 3, 1),
             (13, 7, 3, 1), (16, 10, 1, 1), (16, 6, 1, 1))
    try:
        for log_n, log_r, L, batch in cases:
            if log_r is not None:
                B.set_ntt_split(log_n, log_r)
            primes, x = synthetic.ntt_batch(tile * 10 + log_n, log_n, L, batch)
            ref = _oracle_ntt(x, primes)
            d = to_dev(x)
            B.ntt_forward(d, primes)
            assert np.array_equal(to_host(d), ref), (log_n, log_r, L, batch)
            B.ntt_inverse(d, primes)
            assert np.array_equal(to_host(d), x), (log_n, log_r, L, batch)
            if log_r is not None:
                B.set_ntt_split(log_n, log_n // 2)
    finally:
        B.set_gemm_tile(0)
        for log_n in (13, 16):
            B.set_ntt_split(log_n, log_n // 2)
            B.set_ntt_split3(log_n, 0, 0)


def test_autotune_picks_valid_split_caches_and_stays_exact(tmp_path):
    from paper_2501_07047_amd import binding as B
    cache = tmp_path / "tune.txt"
    try:
        for log_n in (12, 13):
            res = B.autotune(log_n, L=2, batch=2, cache_path=cache)
            if res["log_c1"]:       # three factors: row-side tile automatic
                assert log_n >= 13 and res["tile"] == 0 and 4 <= res["log_c1"] <= 5
            else:
                assert 4 <= res["log_r"] <= log_n - 4 and 1 <= res["tile"] <= 9
            assert res["us"] > 0
            assert B.get_ntt_split(log_n) == (res["log_r"], res["log_c1"])
            again = B.autotune(log_n, L=2, batch=2, cache_path=cache)
            # served from the cache file (microseconds are stored to 3 decimals)
            assert (again["log_r"], again["log_c1"], again["tile"]) == (res["log_r"], res["log_c1"], res["tile"])
            assert abs(again["us"] - res["us"]) < 1e-2
            primes, x = synthetic.ntt_batch(log_n, log_n, 3, 2)
            ref = _oracle_ntt(x, primes)
            d = to_dev(x)
            B.ntt_forward(d, primes)
            assert np.array_equal(to_host(d), ref)
        lines = cache.read_text().strip().splitlines()
        assert len(lines) == 2 and all(len(l.split()) == 9 for l in lines)
    finally:
        for log_n in (12, 13):
            B.set_ntt_split(log_n, log_n // 2)
            B.set_ntt_split3(log_n, 0, 0)


# every row-kernel shape C1 x C2 with C1, C2 in {16, 32, 64}: 64 x 64 reads its
# tables from global memory, the others stage them in LDS
@pytest.mark.parametrize("log_n,log_r,log_c1,L,batch", [(13, 5, 4, 2, 1), (14, 6, 4, 3, 2), (15, 5, 5, 2, 1),
                                                        (16, 6, 5, 3, 2), (16, 4, 6, 1, 1), (16, 8, 4, 2, 1),
                                                        (14, 5, 5, 2, 1), (14, 5, 4, 2, 1), (16, 5, 5, 1, 1),
                                                        (16, 5, 6, 1, 1), (14, 4, 6, 1, 2), (14, 4, 4, 1, 1)])
def test_three_factor_ntt_matches_oracle(log_n, log_r, log_c1, L, batch):
    from paper_2501_07047_amd import binding as B
    B.set_ntt_split3(log_n, log_r, log_c1)
    try:
        primes, x = synthetic.ntt_batch(200 + log_n + log_c1, log_n, L, batch)
        ref = _oracle_ntt(x, primes)
        d = to_dev(x)
        B.ntt_forward(d, primes)
        assert np.array_equal(to_host(d), ref)
        B.ntt_inverse(d, primes)
        assert np.array_equal(to_host(d), x)
    finally:
        B.set_ntt_split3(log_n, 0, 0)


def test_three_factor_full_size_spot_checks_and_ckks():
    # the benchmarked shape (N = 2^16, L = 24, 16 polynomials) with R x C1 x C2 = 64 x 32 x 32:
    # Horner spot checks of every limb, exact inverse, and HE-Mult through the same split
    from oracle import ckks as CK
    from oracle.ntt import horner_eval
    from oracle.primes import psi as psi_of
    from paper_2501_07047_amd import binding as B
    B.set_ntt_split3(16, 6, 5)
    try:
        primes, x = synthetic.ntt_batch(0, 16, 24, 16)
        d = to_dev(x)
        B.ntt_forward(d, primes)
        got = to_host(d)
        g = np.random.Generator(np.random.PCG64(5))
        n = 1 << 16
        for b in (0, 15):
            for i, q in enumerate(primes):
                psi = psi_of(q, n)
                for p in g.integers(0, n, 4):
                    e = (2 * int(bitrev_int(int(p), 16)) + 1)
                    assert int(got[b, i, p]) == int(horner_eval(x[b, i], q, [pow(psi, e, q)])[0])
        B.ntt_inverse(d, primes)
        assert np.array_equal(to_host(d), x)
        qs, ps, a, bb, key = synthetic.ckks_pair(3, 16, 24, 3, 8, 1)
        out = torch_empty(a.shape)
        B.he_mult(to_dev(a), to_dev(bb), to_dev(key), out, qs, ps, 3)
        assert np.array_equal(to_host(out)[0], CK.he_mult(a[0], bb[0], key, qs, ps, 3))
    finally:
        B.set_ntt_split3(16, 0, 0)


def bitrev_int(v, bits):
    r = 0
    for _ in range(bits):
        r = (r << 1) | (v & 1)
        v >>= 1
    return r


def torch_empty(shape):
    import torch
    return torch.empty(shape, dtype=torch.int32, device="cuda")


def test_three_factor_split_errors():
    from paper_2501_07047_amd import binding as B
    for bad in ((12, 4, 4), (16, 6, 3), (16, 3, 6)):
        with pytest.raises(B.CrossError):
            B.set_ntt_split3(*bad)


# Barrett epilogue (plain tables) in the row-side step and the row kernels, for every
# row-kernel family: one LDS table (16 x 16, 32 x 32, 64 x 64), two (64 x 32, 16 x 64)
@pytest.mark.parametrize("log_n,log_r,log_c1,L,batch", [(13, 5, 4, 2, 1), (16, 6, 5, 3, 2), (16, 5, 6, 1, 1),
                                                        (16, 4, 6, 1, 1)])
def test_three_factor_barrett_epilogue_matches_oracle(log_n, log_r, log_c1, L, batch):
    from paper_2501_07047_amd import binding as B
    B.set_ntt_split3(log_n, log_r, log_c1)
    B.set_ntt_reduction("barrett")
    try:
        primes, x = synthetic.ntt_batch(300 + log_n + log_c1, log_n, L, batch)
        x[0, :, 0] = [q - 1 for q in primes]
        ref = _oracle_ntt(x, primes)
        d = to_dev(x)
        B.ntt_forward(d, primes)
        assert np.array_equal(to_host(d), ref)
        B.ntt_inverse(d, primes)
        assert np.array_equal(to_host(d), x)
    finally:
        B.set_ntt_reduction("montgomery")
        B.set_ntt_split3(log_n, 0, 0)


@pytest.mark.parametrize("log_n,log_r,tile", [(8, 4, 0), (10, 5, 0), (12, 6, 0), (12, 4, 3), (12, 8, 5), (12, 6, 1)])
def test_two_factor_barrett_epilogue_matches_oracle(log_n, log_r, tile):
    # both step GEMMs with plain tables and the Barrett epilogue (tile requests outside
    # its staged tiles fall back to the automatic choice)
    from paper_2501_07047_amd import binding as B
    B.set_ntt_split(log_n, log_r)
    B.set_gemm_tile(tile)
    B.set_ntt_reduction("barrett")
    try:
        primes, x = synthetic.ntt_batch(320 + log_n + log_r, log_n, 3, 2)
        x[0, :, 0] = [q - 1 for q in primes]
        ref = _oracle_ntt(x, primes)
        d = to_dev(x)
        B.ntt_forward(d, primes)
        assert np.array_equal(to_host(d), ref)
        B.ntt_inverse(d, primes)
        assert np.array_equal(to_host(d), x)
    finally:
        B.set_ntt_reduction("montgomery")
        B.set_gemm_tile(0)
        B.set_ntt_split(log_n, log_n // 2)


def test_he_mult_with_barrett_ntt():
    # every NTT inside HE-Mult (three-factor at N = 2^14) with the Barrett epilogue
    from oracle import ckks as CK
    from paper_2501_07047_amd import binding as B
    B.set_ntt_reduction("barrett")
    try:
        qs, ps, a, bb, key = synthetic.ckks_pair(8, 14, 6, 3, 2, 1)
        out = torch_empty(a.shape)
        B.he_mult(to_dev(a), to_dev(bb), to_dev(key), out, qs, ps, 3)
        assert np.array_equal(to_host(out)[0], CK.he_mult(a[0], bb[0], key, qs, ps, 3))
    finally:
        B.set_ntt_reduction("montgomery")


def test_barrett_epilogue_rejects_small_primes():
    # 65537 = 2^16 + 1 is NTT-friendly for N = 2^13 but below the 2^21 the Barrett epilogue needs
    from paper_2501_07047_amd import binding as B
    B.set_ntt_split3(13, 5, 4)
    B.set_ntt_reduction("barrett")
    try:
        d = to_dev(np.zeros((1, 1, 1 << 13), dtype=np.uint32))
        with pytest.raises(B.CrossError) as e:
            B.ntt_forward(d, [65537])
        assert e.value.code == -7
    finally:
        B.set_ntt_reduction("montgomery")
        B.set_ntt_split3(13, 0, 0)
    with pytest.raises(KeyError):
        B.set_ntt_reduction("shoup")


@pytest.mark.parametrize("log_n,batch", [(13, 3), (16, 1)])
def test_max_limbs_three_factor(log_n, batch):
    # L = 64 limbs (the library's limit) through the default three-factor split; an odd
    # polynomial count at N = 2^13, spot limbs at N = 2^16
    from paper_2501_07047_amd import binding as B
    primes, x = synthetic.ntt_batch(400 + log_n, log_n, 64, batch)
    d = to_dev(x)
    B.ntt_forward(d, primes)
    got = to_host(d)
    limbs = range(64) if log_n == 13 else (0, 31, 63)
    for i in limbs:
        assert np.array_equal(got[:, i], _oracle_ntt(x[:, i:i + 1], primes[i:i + 1])[:, 0])
    B.ntt_inverse(d, primes)
    assert np.array_equal(to_host(d), x)
    with pytest.raises(B.CrossError):
        p65, x65 = synthetic.ntt_batch(1, 13, 65, 1)
        B.ntt_forward(to_dev(x65), p65)


def test_buffer_beyond_4gib():
    # N = 2^16, 24 limbs x 700 polynomials: a 4.4 GB buffer (and as much workspace), so
    # any 32-bit byte offset that is not relative to a nearby base would wrap; spot
    # polynomials at the start, middle and end against the oracle, exact round trip
    import torch
    from paper_2501_07047_amd import binding as B
    primes = synthetic.primes(24)
    batch, n = 700, 1 << 16
    assert batch * 24 * n * 4 > 1 << 32
    d = synthetic.device_residues(11, batch, primes, n)
    x = d.clone()
    B.ntt_forward(d, primes)
    for b in (0, 349, 699):
        for i in (0, 23):
            xi = x[b, i].cpu().numpy().view(np.uint32).astype(np.uint64)
            got = d[b, i].cpu().numpy().view(np.uint32)
            assert np.array_equal(got, ntt_ct(xi, primes[i], psi_of(primes[i], n)))
    B.ntt_inverse(d, primes)
    assert torch.equal(d, x)
    del d, x
    torch.cuda.empty_cache()
