"""Layout-invariant 3-step negacyclic NTT in matrix form (oracle model of Sec. MAT).

Test infrastructure: see ``oracle/__init__.py``.

Sec. "Applying MAT to 4-step NTT": the input is viewed as an R x C matrix
(row-major, n = r*C + c); step 1 is an R-point transform of every column
(a left matrix product with a twiddle matrix whose rows are permuted by the
bit reversal of R), step 2 an element-wise product with a twiddle matrix whose
rows are bit-reverse permuted, step 3 a C-point transform of every row (a right
product with a twiddle matrix whose columns are bit-reverse permuted).  The
explicit transpose of the classic 4-step NTT disappears because the second
product is taken with the data on the left, and the output lands directly in
bit-reversed order.

The printed formula leaves the negacyclic twist implicit (reading G3).  The
twist is folded into the step-1 and step-2 matrices as follows (derived in the
design notes from out[p] = sum_n a_n psi^((2 brv_N(p)+1) n), p = k*C + c',
brv_N(k*C + c') = brv_C(c')*R + brv_R(k)):

    TF1[k][r]  = psi^(C * r * (2 brv_R(k) + 1))
    T2[k][c]   = psi^(c * (2 brv_R(k) + 1))
    TF3[c][c'] = psi^(2R * c * brv_C(c'))
    out        = ((TF1 @ A) * T2) @ TF3        (all mod q)

Inverse (bit-reversed in, natural out), the same three steps undone in reverse:

    ITF3[c'][c] = psi^(-2R * brv_C(c') * c)
    IT2[k][c]   = psi^(-c * (2 brv_R(k) + 1))
    ITF1[r][k]  = N^-1 * psi^(-C * r * (2 brv_R(k) + 1))
    a           = ITF1 @ ((Ahat @ ITF3) * IT2)

These matrices are what the paper calls the offline-permuted twiddle factors.
"""
import numpy as np

from .ntt import bitrev_table

U64 = np.uint64


def _pow_matrix(psi: int, expo: np.ndarray, q: int, n2: int) -> np.ndarray:
    pw = np.empty(n2, dtype=U64)
    x = 1
    for e in range(n2):
        pw[e] = x
        x = x * psi % q
    return pw[np.mod(expo, n2)]


def twiddles(q: int, psi: int, R: int, C: int):
    """Forward (TF1, T2, TF3) and inverse (ITF1, IT2, ITF3) matrices, entries in [0, q)."""
    n = R * C
    n2 = 2 * n
    br = bitrev_table(R)
    bc = bitrev_table(C)
    r = np.arange(R, dtype=np.int64)
    c = np.arange(C, dtype=np.int64)
    odd = 2 * br + 1                                   # 2 brv_R(k) + 1, indexed by k
    tf1 = _pow_matrix(psi, C * odd[:, None] * r[None, :], q, n2)
    t2 = _pow_matrix(psi, odd[:, None] * c[None, :], q, n2)
    tf3 = _pow_matrix(psi, 2 * R * c[:, None] * bc[None, :], q, n2)
    ninv = pow(n, -1, q)
    itf3 = _pow_matrix(psi, -(2 * R) * bc[:, None] * c[None, :], q, n2)
    it2 = _pow_matrix(psi, -(odd[:, None] * c[None, :]), q, n2)
    itf1 = (_pow_matrix(psi, -(C * r[:, None] * odd[None, :]), q, n2) * U64(ninv)) % U64(q)
    return (tf1, t2, tf3), (itf1, it2, itf3)


def modmatmul(a: np.ndarray, b: np.ndarray, q: int) -> np.ndarray:
    """(a @ b) mod q for residue matrices, exact: every term is reduced before summing."""
    a = np.asarray(a, dtype=U64)
    b = np.asarray(b, dtype=U64)
    out = np.zeros((a.shape[0], b.shape[1]), dtype=U64)
    qq = U64(q)
    for k in range(a.shape[1]):
        out = (out + (a[:, k:k + 1] * b[k:k + 1, :]) % qq) % qq
    return out


def three_step_ntt(a, q: int, psi: int, R: int, C: int) -> np.ndarray:
    (tf1, t2, tf3), _ = twiddles(q, psi, R, C)
    A = np.asarray(a, dtype=U64).reshape(R, C)
    y = modmatmul(tf1, A, q)
    y = (y * t2) % U64(q)
    return modmatmul(y, tf3, q).reshape(-1)


def three_step_intt(ahat, q: int, psi: int, R: int, C: int) -> np.ndarray:
    _, (itf1, it2, itf3) = twiddles(q, psi, R, C)
    A = np.asarray(ahat, dtype=U64).reshape(R, C)
    y = modmatmul(A, itf3, q)
    y = (y * it2) % U64(q)
    return modmatmul(itf1, y, q).reshape(-1)


# ---- three factors: the C-point row transform of step 3 split once more ----------
#
# MAT extends to multi-dimensional tensors with one permutation per dimension
# (Sec. MAT).  Step 3 is a cyclic C-point DFT of every row with root
# w = psi^(2R) and bit-reversed output; with C = C1*C2, c = c1*C2 + c2 and
# output position c' = m*C2 + c2', brv_C(c') = brv_C2(c2')*C1 + brv_C1(m), so
#     w^(c * brv_C(c')) = w^(C2 c1 brv_C1(m)) * w^(c2 brv_C1(m)) * w^(C1 c2 brv_C2(c2'))
# (the cross term is a power of w^C = 1).  Each row, viewed as a C1 x C2 matrix
# (row-major, layout unchanged), is transformed by a left product over c1, an
# element-wise twiddle, and a right product over c2:
#
#     TB[m][c1]   = psi^(2R * C2 * c1 * brv_C1(m))
#     T3[m][c2]   = psi^(2R * c2 * brv_C1(m))
#     TC[c2][c2'] = psi^(2R * C1 * c2 * brv_C2(c2'))
#     row out     = ((TB @ Y_row) * T3) @ TC
#
# Inverse (no scaling: N^-1 stays in ITF1): ITC[c2'][c2] = TC^-1-conjugate
# psi^(-2R C1 c2 brv_C2(c2')), IT3 = psi^(-2R c2 brv_C1(m)),
# ITB[c1][m] = psi^(-2R C2 c1 brv_C1(m)); row = ITB @ ((Xrow @ ITC) * IT3), which is
# C times the forward input, absorbed by N^-1.

def row_twiddles(q: int, psi: int, R: int, C1: int, C2: int):
    """Forward (TB, T3, TC) and inverse (ITB, IT3, ITC) factors of the row transform."""
    n2 = 2 * R * C1 * C2
    b1 = bitrev_table(C1)
    b2 = bitrev_table(C2)
    c1 = np.arange(C1, dtype=np.int64)
    c2 = np.arange(C2, dtype=np.int64)
    tb = _pow_matrix(psi, 2 * R * C2 * b1[:, None] * c1[None, :], q, n2)
    t3 = _pow_matrix(psi, 2 * R * b1[:, None] * c2[None, :], q, n2)
    tc = _pow_matrix(psi, 2 * R * C1 * c2[:, None] * b2[None, :], q, n2)
    itb = _pow_matrix(psi, -(2 * R * C2) * c1[:, None] * b1[None, :], q, n2)
    it3 = _pow_matrix(psi, -(2 * R) * b1[:, None] * c2[None, :], q, n2)
    itc = _pow_matrix(psi, -(2 * R * C1) * b2[:, None] * c2[None, :], q, n2)
    return (tb, t3, tc), (itb, it3, itc)


def three_factor_ntt(a, q: int, psi: int, R: int, C1: int, C2: int) -> np.ndarray:
    C = C1 * C2
    (tf1, t2, _), _ = twiddles(q, psi, R, C)
    (tb, t3, tc), _ = row_twiddles(q, psi, R, C1, C2)
    y = (modmatmul(tf1, np.asarray(a, dtype=U64).reshape(R, C), q) * t2) % U64(q)
    out = np.empty((R, C1, C2), dtype=U64)
    for k in range(R):
        z = (modmatmul(tb, y[k].reshape(C1, C2), q) * t3) % U64(q)
        out[k] = modmatmul(z, tc, q)
    return out.reshape(-1)


def three_factor_intt(ahat, q: int, psi: int, R: int, C1: int, C2: int) -> np.ndarray:
    C = C1 * C2
    _, (itf1, it2, _) = twiddles(q, psi, R, C)
    _, (itb, it3, itc) = row_twiddles(q, psi, R, C1, C2)
    x = np.asarray(ahat, dtype=U64).reshape(R, C1, C2)
    y = np.empty((R, C), dtype=U64)
    for k in range(R):
        z = (modmatmul(x[k], itc, q) * it3) % U64(q)
        y[k] = modmatmul(itb, z, q).reshape(-1)
    y = (y * it2) % U64(q)
    return modmatmul(itf1, y, q).reshape(-1)
