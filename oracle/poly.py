"""Schoolbook negacyclic polynomial product (oracle).

Test infrastructure: see ``oracle/__init__.py``.

Paper Sec. II-A: elements of R_q = Z_q[x]/(x^N + 1); a product wraps x^N to -1.
"""
import numpy as np


def negacyclic_mul(a, b, q: int) -> np.ndarray:
    """c_k = sum_{i+j=k} a_i b_j - sum_{i+j=k+N} a_i b_j  (mod q), O(N^2)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    n = a.shape[0]
    qq = np.uint64(q)
    acc = np.zeros(2 * n, dtype=np.uint64)
    for i in range(n):
        acc[i:i + n] = (acc[i:i + n] + (a[i] * b) % qq) % qq
    return (acc[:n] + qq - acc[n:]) % qq
