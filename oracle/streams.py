"""Chunked forms of the two key-switching vector streams (oracle).

Test infrastructure: see ``oracle/__init__.py``.

Evaluation-key BAT (App. "Applying BAT to Preknown Parameters", closing remark:
the paper keeps evaluation keys off its TPU matrix unit because the reduction is
only dnum x 4 bytes deep, and names fine-grained matrix engines as the place where
it could pay; reading G19).  The evaluation key is pre-known, so every key residue
k of limb prime p is expanded offline by DirectScalarBAT with bp = 8, K = 4 and the
Montgomery factor 2^32 folded in:

    E[l][i] = byte l of ((k * 2^32 * 2^(8 i)) mod p),        i, l < 4.

At run time the extended digit residue e is cut into its four bytes e_i and, with
j running over the dnum digits,

    y_l = sum_j sum_i E_j[l][i] * e_(j,i)          (each y_l < dnum * 4 * 255^2)
    V   = sum_l y_l 2^(8 l)  ==  2^32 * sum_j k_j e_j   (mod p),   V < p * 2^32,

and one Montgomery reduction (Alg. montgomery_reduction) returns sum_j k_j e_j mod p.

Chunk-wise product of two runtime residues (App. "Fall-back Algorithm for unknown
parameters", Fig. 1d_conv): both residues are cut into four bytes, the byte vectors
are convolved into seven partial sums psum_k = sum_(i+l=k) a_i b_l (each at most
18 bits), those are shifted by 8 k and accumulated into the exact 64-bit product,
and Barrett reduction (Alg. barrett) brings it below q.
"""
import numpy as np

from .ckks import U64

M32 = U64(0xFFFFFFFF)


def evk_bat_expand(k, p: int) -> np.ndarray:
    """E[..., l, i] = byte l of (k 2^(32 + 8 i) mod p) for every residue of k (any shape)."""
    k = np.asarray(k, dtype=U64)
    out = np.empty(k.shape + (4, 4), dtype=U64)
    for i in range(4):
        m = k * U64(pow(2, 32 + 8 * i, p)) % U64(p)         # < 2^56: exact in uint64
        for l in range(4):
            out[..., l, i] = (m >> U64(8 * l)) & U64(0xFF)
    return out


def redc(v, p: int) -> np.ndarray:
    """Montgomery reduction v 2^-32 mod p, v < p 2^32 (< 2^61 here), as t = (v mod 2^32)
    (-p^-1) mod 2^32, (v + t p) / 2^32 in [0, 2p), then one conditional subtraction."""
    v = np.asarray(v, dtype=U64)
    pneg = U64((-pow(p, -1, 1 << 32)) % (1 << 32))
    t = ((v & M32) * pneg) & M32                             # the uint64 wrap keeps the low word exact
    r = (v + t * U64(p)) >> U64(32)
    return np.where(r >= U64(p), r - U64(p), r)


def inner_product_evk_bat(ext, key, primes):
    """Key-switch inner product through the evaluation-key BAT: same result as
    ckks.inner_product (acc[s][t] = sum_j ext_j[t] key_j.s[t] mod p_t)."""
    ext = np.asarray(ext, dtype=U64)
    key = np.asarray(key, dtype=U64)
    dnum, nl, n = ext.shape
    acc = np.zeros((2, nl, n), dtype=U64)
    for t, p in enumerate(primes):
        e_bytes = [[(ext[j, t] >> U64(8 * i)) & U64(0xFF) for i in range(4)] for j in range(dnum)]
        for s in range(2):
            y = [np.zeros(n, dtype=U64) for _ in range(4)]
            for j in range(dnum):
                E = evk_bat_expand(key[j, s, t], p)
                for l in range(4):
                    for i in range(4):
                        y[l] += E[:, l, i] * e_bytes[j][i]
            v = sum((y[l] << U64(8 * l) for l in range(4)), np.zeros(n, dtype=U64))
            acc[s, t] = redc(v, p)
    return acc


def chunk_conv(a, b) -> np.ndarray:
    """The seven partial sums psum_k = sum_(i+l=k) a_i b_l of the byte chunks of a and b."""
    a = np.asarray(a, dtype=U64)
    b = np.asarray(b, dtype=U64)
    ac = [(a >> U64(8 * i)) & U64(0xFF) for i in range(4)]
    bc = [(b >> U64(8 * i)) & U64(0xFF) for i in range(4)]
    ps = np.zeros((7,) + a.shape, dtype=U64)
    for i in range(4):
        for l in range(4):
            ps[i + l] += ac[i] * bc[l]
    return ps


def conv_product(a, b) -> np.ndarray:
    """Exact product of two 32-bit residues from their shifted, accumulated partial sums."""
    ps = chunk_conv(a, b)
    return sum((ps[k] << U64(8 * k) for k in range(7)), np.zeros(ps.shape[1:], dtype=U64))


def barrett_reduce(z, q: int) -> np.ndarray:
    """Alg. barrett on every z < q^2, in exact integers: s = 2 ceil(log2 q),
    m = floor(2^s / q), t = (z m) >> s, z - t q, one conditional subtraction."""
    s = 2 * (q - 1).bit_length()
    m = (1 << s) // q

    def one(v):
        v = int(v)
        r = v - ((v * m) >> s) * q
        return r - q if r >= q else r

    z = np.asarray(z, dtype=U64)
    return np.array([one(v) for v in z.reshape(-1)], dtype=U64).reshape(z.shape)


def tensor_conv(a, b, qs):
    """HE-Mult tensor product with every runtime x runtime product taken as a
    chunk-wise convolution: same result as ckks.tensor."""
    a = np.asarray(a, dtype=U64)
    b = np.asarray(b, dtype=U64)
    d = np.empty((3,) + a.shape[1:], dtype=U64)
    for i, q in enumerate(qs):
        qq = U64(q)
        mul = lambda x, y: barrett_reduce(conv_product(x, y), q)
        d[0, i] = mul(a[0, i], b[0, i])
        d[1, i] = (mul(a[0, i], b[1, i]) + mul(a[1, i], b[0, i])) % qq
        d[2, i] = mul(a[1, i], b[1, i])
    return d
