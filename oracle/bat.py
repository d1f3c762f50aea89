"""Basis Aligned Transformation model (oracle), Sec. BAT and Alg. bat_deployment.

Test infrastructure: see ``oracle/__init__.py``.

A residue is cut into K chunks of bp bits (ChunkDecompose); a pre-known operand
a is expanded offline into a K x K block whose column j holds the chunks of
(a * 2^(bp*j) mod q) (DirectScalarBAT).  Then for every residue b

    a*b = sum_j (sum_i M[j][i] * b_i) * 2^(bp*j)   (mod q)     (Eqs. line2-line9,
                                                               reading 2^i as 2^(bp*i), G4)

and a (H x V) @ (V x W) modular product becomes a (K*H x K*V) @ (K*V x W)
low-precision product followed by ChunkMerge and one reduction mod q.
bp = 7 and K = 4 fit 28-bit residues into non-negative int8 chunks (reading G5).
"""
import numpy as np


def chunk_decompose(x: int, bp: int, k: int):
    return [(x >> (i * bp)) & ((1 << bp) - 1) for i in range(k)]


def chunk_merge(chunks, bp: int) -> int:
    return sum(int(c) << (i * bp) for i, c in enumerate(chunks))


def direct_scalar_bat(a: int, q: int, bp: int, k: int) -> np.ndarray:
    """K x K block: M[i][j] = chunk_i((a << (j*bp)) mod q)."""
    m = np.zeros((k, k), dtype=np.int64)
    for j in range(k):
        val = (a << (j * bp)) % q
        for i, ch in enumerate(chunk_decompose(val, bp, k)):
            m[i, j] = ch
    return m


def offline_compile_left(A, q: int, bp: int, k: int) -> np.ndarray:
    """(K*H) x (K*V) block expansion of a pre-known H x V residue matrix."""
    A = np.asarray(A)
    H, V = A.shape
    out = np.zeros((k * H, k * V), dtype=np.int64)
    for h in range(H):
        for v in range(V):
            out[h * k:(h + 1) * k, v * k:(v + 1) * k] = direct_scalar_bat(int(A[h, v]), q, bp, k)
    return out


def runtime_compile_right(B, bp: int, k: int) -> np.ndarray:
    """(K*V) x W stacking of the chunks of a runtime V x W residue matrix."""
    B = np.asarray(B, dtype=np.int64)
    V, W = B.shape
    out = np.zeros((k * V, W), dtype=np.int64)
    for i in range(k):
        out[i::k, :] = (B >> (i * bp)) & ((1 << bp) - 1)
    return out


def bat_modmatmul(A, B, q: int, bp: int = 7, k: int = 4) -> np.ndarray:
    """Main-FullMatMul of Alg. bat_deployment followed by the final reduction mod q."""
    ad = offline_compile_left(A, q, bp, k)
    bd = runtime_compile_right(B, bp, k)
    zchunk = np.array([[sum(int(ad[m, t]) * int(bd[t, w]) for t in range(ad.shape[1]))
                        for w in range(bd.shape[1])] for m in range(ad.shape[0])], dtype=object)
    H = ad.shape[0] // k
    out = np.zeros((H, bd.shape[1]), dtype=np.uint64)
    for h in range(H):
        for w in range(bd.shape[1]):
            z = chunk_merge([zchunk[h * k + i, w] for i in range(k)], bp)
            out[h, w] = z % q
    return out
