"""Fast basis conversion (oracle), App. "Basis Conversion (BConv)".

Test infrastructure: see ``oracle/__init__.py``.

Conv_{B1->B2}(a)_j = sum_i [a_i * qhat_i^-1]_{q_i} * [qhat_i]_{p_j}  mod p_j,
with qhat_i = prod_{i' != i} q_{i'} over the source basis B1.  Step 1 is an
L x N VecModMul, step 2 an (N, L, L') MatModMul.  This is the *fast*
(approximate) conversion: the integer y = sum_i [a_i qhat_i^-1]_{q_i} qhat_i is
congruent to the CRT value of a modulo every source prime but may exceed it by
a multiple u*Q (0 <= u < |B1|); y, not the CRT value, is what is converted
(reading G9).
"""
from math import prod

import numpy as np

U64 = np.uint64


def bconv_bigint(a, src, dst) -> np.ndarray:
    """Python big-integer form: y = sum_i [a_i qhat_i^-1]_{q_i} qhat_i, out_j = y mod p_j.

    ``a`` has shape [len(src), N] (coefficient form); returns [len(dst), N].
    """
    a = np.asarray(a)
    Q = prod(src)
    qhat = [Q // q for q in src]
    qhat_inv = [pow(h % q, -1, q) for h, q in zip(qhat, src)]
    n = a.shape[1]
    out = np.zeros((len(dst), n), dtype=U64)
    for col in range(n):
        y = 0
        for i, q in enumerate(src):
            y += (int(a[i, col]) * qhat_inv[i] % q) * qhat[i]
        for j, p in enumerate(dst):
            out[j, col] = y % p
    return out


def bconv_y(a_col, src) -> int:
    """The integer y of one coefficient column (used by the range pins)."""
    Q = prod(src)
    y = 0
    for ai, q in zip(a_col, src):
        h = Q // q
        y += (int(ai) * pow(h % q, -1, q) % q) * h
    return y


def bconv_u64(a, src, dst) -> np.ndarray:
    """NumPy uint64 form of the same two steps, every product reduced before summing."""
    a = np.asarray(a, dtype=U64)
    Q = prod(src)
    out = np.zeros((len(dst), a.shape[1]), dtype=U64)
    b = []
    for i, q in enumerate(src):
        h = Q // q
        b.append((a[i] * U64(pow(h % q, -1, q))) % U64(q))       # step 1
    for j, p in enumerate(dst):
        acc = np.zeros(a.shape[1], dtype=U64)
        for i, q in enumerate(src):
            c = U64((Q // q) % p)
            acc = (acc + (b[i] % U64(p)) * c % U64(p)) % U64(p)   # step 2
        out[j] = acc
    return out
