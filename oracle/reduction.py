"""Modular reduction models (oracle).

Test infrastructure: see ``oracle/__init__.py``.

montgomery_reduce follows Alg. montgomery_reduction (64 -> 32 bits) with the
middle-product reading G7: the printed middle sum adds the full 32-bit cross
products and then their high halves again, which double counts; the quantity
the algorithm names (the upper 32 bits of t*q) is what is computed here, from
16-bit partial products as in the algorithm.  The result is z * 2^-32 mod q in
[0, 2q) provided z < q * 2^32 (a precondition the algorithm header omits).

barrett_mulmod follows Alg. barrett: s = 2*ceil(log2 q), m = floor(2^s / q),
t = (z*m) >> s, z -= t*q, one conditional subtraction (reading G8).

shoup_mulmod is Shoup's multiplication by a pre-known operand (the third
method of Sec. Evaluation "Impact of Modular Reduction Algorithm").

bat_lazy_reduce follows App. "BAT for Modular Reduction": the chunks of a
product above the low k chunks are multiplied by the chunk matrix of
LC_j = 2^(bp (k + j)) mod q and added back to the low part -- a lazy partial
reduction (congruent to the product, not below q).  The paper writes it with
bytes (bp = 8) for a 64-bit partial sum; the signed int8 MFMA path uses
bp = 7 (reading G5), i.e. k = 4 chunks of 7 bits for products below 2^56.
"""


def montgomery_reduce(z: int, q: int) -> int:
    assert 0 <= z < q << 32 and q < 1 << 32 and q % 2 == 1
    qinv = pow(q, -1, 1 << 32)
    z_lo, z_hi = z & 0xFFFFFFFF, z >> 32
    t = (z_lo * qinv) & 0xFFFFFFFF
    t_lo, t_hi = t & 0xFFFF, t >> 16
    q_lo, q_hi = q & 0xFFFF, q >> 16
    p_hi = t_hi * q_hi
    p_lo = t_lo * q_lo
    p_mh = t_hi * q_lo
    p_ml = t_lo * q_hi
    mid_lo = (p_mh & 0xFFFF) + (p_ml & 0xFFFF) + (p_lo >> 16)
    mid_hi = (p_mh >> 16) + (p_ml >> 16) + (mid_lo >> 16)
    t_final = p_hi + mid_hi                      # = floor(t*q / 2^32)
    b = z_hi + q - t_final
    assert 0 <= b < 2 * q
    return b


def barrett_mulmod(a: int, b: int, q: int) -> int:
    s = 2 * (q - 1).bit_length()
    m = (1 << s) // q
    z = a * b
    t = (z * m) >> s
    z -= t * q
    if z >= q:
        z -= q
    return z


def shoup_mulmod(a: int, w: int, q: int) -> int:
    """a * w mod q with w pre-known: w' = floor(w 2^32 / q), r = a w - floor(a w' / 2^32) q
    lies in [0, 2q) for a < 2^32 and w < q < 2^31; one conditional subtraction."""
    assert 0 <= a < 1 << 32 and 0 <= w < q < 1 << 31
    wp = (w << 32) // q
    r = a * w - ((a * wp) >> 32) * q
    assert 0 <= r < 2 * q
    return r - q if r >= q else r


def lazy_constants(q: int, bp: int = 7, k: int = 4):
    """LC[j][i] = chunk i (bp bits) of 2^(bp (k + j)) mod q, for j, i < k (needs q < 2^(bp k))."""
    assert q < 1 << (bp * k)
    mask = (1 << bp) - 1
    lc = [pow(2, bp * (k + j), q) for j in range(k)]
    return [[(lc[j] >> (bp * i)) & mask for i in range(k)] for j in range(k)]


def bat_lazy_reduce(p: int, q: int, bp: int = 7, k: int = 4) -> int:
    """Lazy partial reduction of p < 2^(2 k bp): r = low + sum_i T_i 2^(bp i) with
    T_i = sum_j c_(k+j) LC[j][i], c the bp-bit chunks of p, low its low k chunks.
    r is congruent to p mod q and r < 2^(bp k) + k (2^bp - 1)^2 (2^(bp k) - 1) / (2^bp - 1)."""
    assert 0 <= p < 1 << (2 * k * bp)
    mask = (1 << bp) - 1
    low = p & ((1 << (bp * k)) - 1)
    c = [(p >> (bp * (k + j))) & mask for j in range(k)]
    LC = lazy_constants(q, bp, k)
    T = [sum(c[j] * LC[j][i] for j in range(k)) for i in range(k)]
    return low + sum(T[i] << (bp * i) for i in range(k))


def bat_lazy_mulmod(a: int, w: int, q: int) -> int:
    """a * w mod q: 56-bit product, BAT lazy partial reduction (bp = 7, k = 4), final reduction."""
    return bat_lazy_reduce(a * w, q) % q
