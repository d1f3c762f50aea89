"""Host-side checks of the C ABI library: it loads, exports every symbol that
include/cross.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "cross.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cross_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    from paper_2501_07047_amd import binding
    assert sorted(binding.exported_symbols()) == _declared()


def test_library_exports_every_declared_symbol():
    from paper_2501_07047_amd import binding
    l = binding.lib()
    for name in _declared():
        assert hasattr(l, name), name


def test_root_matches_definition_and_validates():
    from paper_2501_07047_amd import binding
    from oracle.primes import psi, prime_chain
    for q in prime_chain(4):
        for log_n in (4, 12, 16):
            assert binding.root(q, log_n) == psi(q, 1 << log_n)
    with pytest.raises(binding.CrossError) as e:
        binding.root(268042241 + 2, 12)
    assert e.value.code in (-2, -3)
    for q in prime_chain(2, bits=31) + [2013265921]:     # wide primes (the NTT takes q < 2^31)
        assert binding.root(q, 12) == psi(q, 1 << 12)
    with pytest.raises(binding.CrossError) as e:
        binding.root(3221225473, 12)        # prime, 3 * 2^30 + 1 >= 2^31
    assert e.value.code == -4
    with pytest.raises(binding.CrossError) as e:
        binding.root(7681, 12)              # prime, 7681 - 1 = 2^9 * 15: no 2^13-th root
    assert e.value.code == -3


def test_null_context_is_rejected():
    from paper_2501_07047_amd import binding
    l = binding.lib()
    arr = (ctypes.c_uint32 * 1)(268042241)
    assert l.cross_ntt_forward(None, 12, arr, 1, 1, None, None) == -1
    assert l.cross_set_ntt_split(None, 16, 8) == -1
