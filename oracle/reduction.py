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
