"""Thin Python binding of libcross (argument marshalling only).

Every function takes torch tensors that live on a HIP device (any 4-byte
dtype; bit patterns are treated as uint32 residues), checks shapes, and calls
the C entry point of the same name in ``libcross.so`` with raw device
pointers and the current torch stream.  No arithmetic happens here: if the
shared library is missing, every call raises.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcross.so")

STATUS = {0: "CROSS_OK", -1: "CROSS_EINVAL", -2: "CROSS_ENOTPRIME", -3: "CROSS_ENOROOT",
          -4: "CROSS_ERANGE", -5: "CROSS_ENOMEM", -6: "CROSS_EDEVICE", -7: "CROSS_EUNSUPPORTED",
          -8: "CROSS_EDOMAIN"}


class CrossError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


_lib = None
_ctx = {}

c_u32 = ctypes.c_uint32
c_i32 = ctypes.c_int32
c_vp = ctypes.c_void_p
c_u32p = ctypes.POINTER(ctypes.c_uint32)

# name -> argtypes (restype is always int = cross_status unless noted)
SIGNATURES = {
    "cross_ctx_create": [ctypes.c_int, ctypes.POINTER(c_vp)],
    "cross_ctx_destroy": [c_vp],
    "cross_last_error": [c_vp],
    "cross_root": [c_u32, c_u32, c_u32p],
    "cross_set_ntt_split": [c_vp, c_u32, c_u32],
    "cross_set_gemm_tile": [c_vp, ctypes.c_int],
    "cross_set_ntt_split3": [c_vp, c_u32, c_u32, c_u32],
    "cross_set_ntt_reduction": [c_vp, ctypes.c_int],
    "cross_set_ntt_engine": [c_vp, ctypes.c_int],
    "cross_set_debug_check": [c_vp, ctypes.c_int],
    "cross_ntt_noalloc": [c_vp, c_u32, c_u32p, c_u32, c_u32, c_vp, ctypes.c_int, c_vp],
    "cross_get_ntt_split": [c_vp, c_u32, ctypes.POINTER(c_u32), ctypes.POINTER(c_u32)],
    "cross_host_row_tables": [c_u32, c_u32, c_u32, c_u32, c_u32, c_vp, ctypes.POINTER(ctypes.c_uint64)],
    "cross_autotune": [c_vp, c_u32, c_u32, c_u32, ctypes.c_char_p, ctypes.POINTER(c_u32), ctypes.POINTER(c_u32),
                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)],
    "cross_ntt_forward": [c_vp, c_u32, c_u32p, c_u32, c_u32, c_vp, c_vp],
    "cross_ntt_inverse": [c_vp, c_u32, c_u32p, c_u32, c_u32, c_vp, c_vp],
    "cross_ntt_forward_butterfly": [c_vp, c_u32, c_u32p, c_u32, c_u32, c_vp, c_vp],
    "cross_ntt_inverse_butterfly": [c_vp, c_u32, c_u32p, c_u32, c_u32, c_vp, c_vp],
    "cross_poly_mul": [c_vp, c_u32, c_u32p, c_u32, c_u32, c_vp, c_vp, c_vp, c_vp],
    "cross_bconv": [c_vp, c_u32, c_u32p, c_u32, c_u32p, c_u32, c_vp, c_vp, c_u32, c_vp],
    "cross_keyswitch_modup": [c_vp, c_vp, c_vp, c_vp, c_u32, c_vp],
    "cross_keyswitch_moddown": [c_vp, c_vp, c_vp, c_vp, c_u32, c_vp],
    "cross_he_mult": [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_u32, c_vp],
    "cross_rotate": [c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_u32, c_vp],
    "cross_he_add": [c_vp, c_u32, c_u32p, c_u32, c_u32, c_vp, c_vp, c_vp, c_vp],
    "cross_rescale": [c_vp, c_u32, c_u32p, c_u32, c_u32, c_u32, c_vp, c_vp, c_vp],
    "cross_vec_modmul_prepare": [c_vp, c_u32, c_u32p, c_u32, ctypes.c_int, c_vp, c_vp, c_vp],
    "cross_vec_modmul": [c_vp, c_u32, c_u32p, c_u32, c_u32, ctypes.c_int, c_vp, c_vp, c_vp, c_vp],
    "cross_evk_bat_prepare": [c_vp, c_u32, c_u32p, c_u32, c_u32, c_vp, c_vp, c_vp],
    "cross_keyswitch_inner_product": [c_vp, c_u32, c_u32p, c_u32, c_u32, c_u32, ctypes.c_int, c_vp, c_vp, c_vp,
                                      c_vp],
    "cross_tensor": [c_vp, c_u32, c_u32p, c_u32, c_u32, ctypes.c_int, c_vp, c_vp, c_vp, c_vp, c_vp],
    "cross_batch_create": [c_vp, c_vp, c_u32, ctypes.c_int, ctypes.POINTER(c_vp)],
    "cross_batch_workspace_bytes": [c_vp, c_vp, c_u32, ctypes.POINTER(ctypes.c_uint64)],
    "cross_batch_create_in": [c_vp, c_vp, c_u32, ctypes.c_int, c_vp, ctypes.c_uint64, c_vp, ctypes.POINTER(c_vp)],
    "cross_batch_run": [c_vp, c_vp],
    "cross_get_batch_tile": [c_vp, c_u32, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
    "cross_batch_info": [c_vp, ctypes.POINTER(c_u32), ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64)],
    "cross_batch_destroy": [c_vp],
    "cross_measure_peak": [c_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double)],
    "cross_profile_enable": [c_vp, ctypes.c_int],
    "cross_profile_only": [c_vp, ctypes.c_char_p],
    "cross_profile_report": [c_vp, ctypes.c_char_p, ctypes.c_uint64],
    "cross_host_tables": [c_u32, c_u32, c_u32, c_u32, c_vp, ctypes.POINTER(ctypes.c_uint64)],
}


def lib():
    """Load libcross.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libcross.so is not built (run __graft_entry__.build())")
        l = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            f = getattr(l, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        l.cross_ctx_destroy.restype = None
        l.cross_batch_destroy.restype = None
        l.cross_last_error.restype = ctypes.c_char_p
        _lib = l
    return _lib


def exported_symbols():
    return list(SIGNATURES)


def context(device=None):
    """Per-device library context, created on first use."""
    import torch
    dev = torch.cuda.current_device() if device is None else int(device)
    if dev not in _ctx:
        h = c_vp()
        st = lib().cross_ctx_create(dev, ctypes.byref(h))
        if st != 0:
            raise CrossError(st, "cross_ctx_create(%d)" % dev)
        _ctx[dev] = h
    return _ctx[dev]


def _check(st, ctx):
    if st != 0:
        raise CrossError(st, lib().cross_last_error(ctx).decode())


def _u32_array(values):
    vals = [int(v) for v in values]
    return (ctypes.c_uint32 * len(vals))(*vals)


def _dev_ptr(t, name):
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if t.element_size() != 4 or not t.is_contiguous():
        raise ValueError("%s must be a contiguous 4-byte tensor" % name)
    return c_vp(t.data_ptr())


def _stream(t):
    import torch
    return c_vp(torch.cuda.current_stream(t.device).cuda_stream)


def _log2(n):
    if n <= 0 or n & (n - 1):
        raise ValueError("N must be a power of two")
    return n.bit_length() - 1


def root(q, log_n):
    out = ctypes.c_uint32()
    st = lib().cross_root(q, log_n, ctypes.byref(out))
    if st != 0:
        raise CrossError(st, "cross_root(%d, %d)" % (q, log_n))
    return out.value


def set_ntt_split(log_n, log_r, device=None):
    ctx = context(device)
    _check(lib().cross_set_ntt_split(ctx, log_n, log_r), ctx)


def set_ntt_split3(log_n, log_r, log_c1, device=None):
    """Three-factor NTT split for size 2^log_n (log_c1 = 0: back to two factors)."""
    ctx = context(device)
    _check(lib().cross_set_ntt_split3(ctx, log_n, log_r, log_c1), ctx)


NTT_REDUCTION = {"montgomery": 0, "barrett": 1}


def set_ntt_reduction(method, device=None):
    """Epilogue reduction of every MFMA NTT step ("montgomery" or "barrett")."""
    ctx = context(device)
    _check(lib().cross_set_ntt_reduction(ctx, NTT_REDUCTION[method]), ctx)


def set_debug_check(enable=True, device=None):
    """Residue-range check of every input (CROSS_EDOMAIN on a residue not below its prime)."""
    ctx = context(device)
    _check(lib().cross_set_debug_check(ctx, int(bool(enable))), ctx)


NTT_ENGINE = {"mfma": 0, "butterfly": 1}


def set_ntt_engine(engine, device=None):
    """Engine of every NTT on the context ("mfma" or "butterfly"); the batch runtime keeps MFMA."""
    ctx = context(device)
    _check(lib().cross_set_ntt_engine(ctx, NTT_ENGINE[engine]), ctx)


def get_ntt_split(log_n, device=None):
    """(log_r, log_c1) used for 2^log_n transforms on this context (log_c1 = 0: two factors)."""
    ctx = context(device)
    r, c1 = c_u32(), c_u32()
    _check(lib().cross_get_ntt_split(ctx, log_n, ctypes.byref(r), ctypes.byref(c1)), ctx)
    return r.value, c1.value


def host_row_tables(q, log_n, log_r, log_c1, which):
    """Copy one three-factor row table into a numpy array (host only, no GPU)."""
    import numpy as np
    nbytes = ctypes.c_uint64(0)
    st = lib().cross_host_row_tables(q, log_n, log_r, log_c1, which, None, ctypes.byref(nbytes))
    if st != 0:
        raise CrossError(st, "cross_host_row_tables")
    buf = np.empty(nbytes.value, dtype=np.uint8)
    st = lib().cross_host_row_tables(q, log_n, log_r, log_c1, which, c_vp(buf.ctypes.data), ctypes.byref(nbytes))
    if st != 0:
        raise CrossError(st, "cross_host_row_tables")
    return buf.view(np.int8) if which < 4 or 8 <= which <= 11 else buf.view(np.uint32)


def set_gemm_tile(tile, device=None):
    """0 = auto, 1..9 = fixed workgroup tiles (see cross_set_gemm_tile)."""
    ctx = context(device)
    _check(lib().cross_set_gemm_tile(ctx, int(tile)), ctx)


def autotune(log_n, L=8, batch=8, cache_path=None, device=None):
    """Time the candidate factorings and tiles for 2^log_n transforms and keep the best
    on the context; returns {"log_r", "log_c1", "tile", "us"} (see cross_autotune)."""
    ctx = context(device)
    r, c1, t, us = c_u32(), c_u32(), ctypes.c_int(), ctypes.c_double()
    path = None if cache_path is None else str(cache_path).encode()
    _check(lib().cross_autotune(ctx, log_n, L, batch, path, ctypes.byref(r), ctypes.byref(c1), ctypes.byref(t),
                                ctypes.byref(us)), ctx)
    return {"log_r": r.value, "log_c1": c1.value, "tile": t.value, "us": us.value}


def _ntt(fn, data, primes):
    if data.dim() != 3:
        raise ValueError("data must be [batch][L][N]")
    batch, L, n = data.shape
    if L != len(primes):
        raise ValueError("len(primes) != L")
    ctx = context(data.device.index)
    _check(getattr(lib(), fn)(ctx, _log2(n), _u32_array(primes), L, batch,
                              _dev_ptr(data, "data"), _stream(data)), ctx)
    return data


def ntt_forward(data, primes):
    """In-place forward NTT of data[batch][L][N] (see cross_ntt_forward)."""
    return _ntt("cross_ntt_forward", data, primes)


def ntt_inverse(data, primes):
    return _ntt("cross_ntt_inverse", data, primes)


def ntt_noalloc(data, primes, inverse=False):
    """cross_ntt_noalloc: the NTT (or INTT) of `data` with no device allocation (scratch in
    the library's static device array; the tables must exist, e.g. from ntt_forward)."""
    batch, L, n = data.shape
    if L != len(primes):
        raise ValueError("data has %d limbs, %d primes given" % (L, len(primes)))
    ctx = context(data.device.index)
    _check(lib().cross_ntt_noalloc(ctx, _log2(n), _u32_array(primes), L, batch, _dev_ptr(data, "data"),
                                   int(bool(inverse)), _stream(data)), ctx)
    return data


def ntt_forward_butterfly(data, primes):
    return _ntt("cross_ntt_forward_butterfly", data, primes)


def ntt_inverse_butterfly(data, primes):
    return _ntt("cross_ntt_inverse_butterfly", data, primes)


def host_tables(q, log_n, log_r, which):
    """Copy one offline-compiled table into a numpy array (host only, no GPU)."""
    import numpy as np
    nbytes = ctypes.c_uint64(0)
    st = lib().cross_host_tables(q, log_n, log_r, which, None, ctypes.byref(nbytes))
    if st != 0:
        raise CrossError(st, "cross_host_tables")
    buf = np.empty(nbytes.value, dtype=np.uint8)
    st = lib().cross_host_tables(q, log_n, log_r, which, c_vp(buf.ctypes.data), ctypes.byref(nbytes))
    if st != 0:
        raise CrossError(st, "cross_host_tables")
    return buf.view(np.int8) if which < 4 or which >= 6 else buf.view(np.uint32)


def measure_peak(which, device=None):
    """which: "mfma_i8" -> TOP/s, "hbm_copy" -> GB/s (see cross_measure_peak)."""
    ctx = context(device)
    out = ctypes.c_double()
    _check(lib().cross_measure_peak(ctx, {"mfma_i8": 0, "hbm_copy": 1, "mfma_i8_32x32": 2}[which],
                                    ctypes.byref(out)), ctx)
    return out.value


def profile_enable(enable=True, device=None):
    ctx = context(device)
    _check(lib().cross_profile_enable(ctx, 1 if enable else 0), ctx)


def profile_only(family=None, device=None):
    """Time only the kernel family `family` (None: all families)."""
    ctx = context(device)
    _check(lib().cross_profile_only(ctx, (family or "").encode()), ctx)


def profile_report(device=None):
    """{kernel family: (launches, total_ms)} since the last report (synchronises)."""
    ctx = context(device)
    buf = ctypes.create_string_buffer(1 << 16)
    _check(lib().cross_profile_report(ctx, buf, len(buf)), ctx)
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out


class CkksParams(ctypes.Structure):
    """Mirror of cross_ckks_params."""
    _fields_ = [("log_n", c_u32), ("L", c_u32), ("K", c_u32), ("dnum", c_u32), ("primes", c_u32p)]


def _params(qs, ps, dnum, n):
    arr = _u32_array(list(qs) + list(ps))
    prm = CkksParams(_log2(n), len(qs), len(ps), dnum, ctypes.cast(arr, c_u32p))
    prm._keep = arr
    return prm


def _shape(t, shape, name):
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, tuple(shape), tuple(t.shape)))


def poly_mul(a, b, out, primes):
    """out = a * b in Z_q[x]/(x^N+1) limb-wise; all [batch][L][N] coefficient form."""
    batch, L, n = a.shape
    _shape(b, a.shape, "b")
    _shape(out, a.shape, "out")
    ctx = context(a.device.index)
    _check(lib().cross_poly_mul(ctx, _log2(n), _u32_array(primes), L, batch, _dev_ptr(a, "a"),
                                _dev_ptr(b, "b"), _dev_ptr(out, "out"), _stream(a)), ctx)
    return out


def bconv(inp, src_primes, dst_primes, out):
    """Fast basis conversion of inp [batch][l][N] into out [batch][lp][N] (coefficient form)."""
    batch, l, n = inp.shape
    _shape(out, (batch, len(dst_primes), n), "out")
    if l != len(src_primes):
        raise ValueError("inp limbs != len(src_primes)")
    ctx = context(inp.device.index)
    _check(lib().cross_bconv(ctx, _log2(n), _u32_array(src_primes), l, _u32_array(dst_primes),
                             len(dst_primes), _dev_ptr(inp, "inp"), _dev_ptr(out, "out"), batch,
                             _stream(inp)), ctx)
    return out


def keyswitch_modup(inp, out, qs, ps, dnum):
    """inp [batch][L][N] -> out [batch][dnum][L+K][N], NTT form."""
    batch, L, n = inp.shape
    _shape(out, (batch, dnum, L + len(ps), n), "out")
    prm = _params(qs, ps, dnum, n)
    ctx = context(inp.device.index)
    _check(lib().cross_keyswitch_modup(ctx, ctypes.byref(prm), _dev_ptr(inp, "inp"), _dev_ptr(out, "out"),
                                       batch, _stream(inp)), ctx)
    return out


def keyswitch_moddown(inp, out, qs, ps, dnum):
    """inp [batch][L+K][N] -> out [batch][L][N], NTT form."""
    batch, lk, n = inp.shape
    _shape(out, (batch, len(qs), n), "out")
    prm = _params(qs, ps, dnum, n)
    ctx = context(inp.device.index)
    _check(lib().cross_keyswitch_moddown(ctx, ctypes.byref(prm), _dev_ptr(inp, "inp"), _dev_ptr(out, "out"),
                                         batch, _stream(inp)), ctx)
    return out


def he_mult(a, b, key, out, qs, ps, dnum):
    """HE-Mult + relinearisation: a, b, out [batch][2][L][N]; key [dnum][2][L+K][N]."""
    batch, two, L, n = a.shape
    _shape(b, a.shape, "b")
    _shape(out, a.shape, "out")
    _shape(key, (dnum, 2, L + len(ps), n), "key")
    prm = _params(qs, ps, dnum, n)
    ctx = context(a.device.index)
    _check(lib().cross_he_mult(ctx, ctypes.byref(prm), _dev_ptr(a, "a"), _dev_ptr(b, "b"), _dev_ptr(key, "key"),
                               _dev_ptr(out, "out"), batch, _stream(a)), ctx)
    return out


def rotate(ct, steps, key, out, qs, ps, dnum):
    """Rotation by `steps` (Galois element 5^steps mod 2N): ct, out [batch][2][L][N]."""
    batch, two, L, n = ct.shape
    _shape(out, ct.shape, "out")
    _shape(key, (dnum, 2, L + len(ps), n), "key")
    prm = _params(qs, ps, dnum, n)
    ctx = context(ct.device.index)
    _check(lib().cross_rotate(ctx, ctypes.byref(prm), int(steps), _dev_ptr(ct, "ct"), _dev_ptr(key, "key"),
                              _dev_ptr(out, "out"), batch, _stream(ct)), ctx)
    return out


def he_add(a, b, out, primes):
    """HE-Add (limb-wise sum mod q_i): a, b, out [..][L][N] (polynomials or ciphertexts); may alias."""
    L, n = a.shape[-2:]
    _shape(b, a.shape, "b")
    _shape(out, a.shape, "out")
    if len(primes) != L:
        raise ValueError("len(primes) != L")
    npoly = a.numel() // (L * n)
    ctx = context(a.device.index)
    _check(lib().cross_he_add(ctx, _log2(n), _u32_array(primes), L, npoly, _dev_ptr(a, "a"), _dev_ptr(b, "b"),
                              _dev_ptr(out, "out"), _stream(a)), ctx)
    return out


def rescale(x, out, primes, drop=1):
    """Rescale by the product of the last `drop` primes: x [..][L][N] -> out [..][L-drop][N], NTT form."""
    L, n = x.shape[-2:]
    _shape(out, tuple(x.shape[:-2]) + (L - drop, n), "out")
    if len(primes) != L:
        raise ValueError("len(primes) != L")
    npoly = x.numel() // (L * n)
    ctx = context(x.device.index)
    _check(lib().cross_rescale(ctx, _log2(n), _u32_array(primes), L, int(drop), npoly, _dev_ptr(x, "x"),
                               _dev_ptr(out, "out"), _stream(x)), ctx)
    return out


MODRED = {"barrett": 0, "montgomery": 1, "shoup": 2, "bat_lazy": 3}


def vec_modmul_prepare(w, primes, method):
    """Prepared form of the pre-known operand w [L][N] for `method` (a MODRED key): a new
    device tensor of 2*L*N words."""
    import torch
    L, n = w.shape
    if len(primes) != L:
        raise ValueError("len(primes) != L")
    prep = torch.empty((2, L, n), dtype=torch.int32, device=w.device)
    ctx = context(w.device.index)
    _check(lib().cross_vec_modmul_prepare(ctx, _log2(n), _u32_array(primes), L, MODRED[method], _dev_ptr(w, "w"),
                                          _dev_ptr(prep, "w_prep"), _stream(w)), ctx)
    return prep


def vec_modmul(a, w_prep, out, primes, method):
    """out = a * w mod q limb-wise: a, out [..][L][N]; w_prep from vec_modmul_prepare (same method)."""
    L, n = a.shape[-2:]
    _shape(out, a.shape, "out")
    _shape(w_prep, (2, L, n), "w_prep")
    if len(primes) != L:
        raise ValueError("len(primes) != L")
    npoly = a.numel() // (L * n)
    ctx = context(a.device.index)
    _check(lib().cross_vec_modmul(ctx, _log2(n), _u32_array(primes), L, npoly, MODRED[method], _dev_ptr(a, "a"),
                                  _dev_ptr(w_prep, "w_prep"), _dev_ptr(out, "out"), _stream(a)), ctx)
    return out


STREAM_FORM = {"valu": 0, "chunked": 1}


def evk_bat_prepare(key, primes):
    """BAT-expanded evaluation key for the chunked inner product: key [dnum][2][LK][N] ->
    a new device tensor [dnum][2][LK][N][4] of words."""
    import torch
    dnum, two, LK, n = key.shape
    if two != 2 or len(primes) != LK:
        raise ValueError("key must be [dnum][2][LK][N] with LK primes")
    kb = torch.empty((dnum, 2, LK, n, 4), dtype=torch.int32, device=key.device)
    ctx = context(key.device.index)
    _check(lib().cross_evk_bat_prepare(ctx, _log2(n), _u32_array(primes), LK, dnum, _dev_ptr(key, "key"),
                                       _dev_ptr(kb, "key_bat"), _stream(key)), ctx)
    return kb


def keyswitch_inner_product(ext, key, out, primes, form="valu"):
    """out[b][s] = sum_j ext[b][j] key_j.s limb-wise: ext [B][dnum][LK][N], out [B][2][LK][N];
    key [dnum][2][LK][N] ("valu") or the evk_bat_prepare output ("chunked")."""
    B, dnum, LK, n = ext.shape
    _shape(out, (B, 2, LK, n), "out")
    _shape(key, (dnum, 2, LK, n) + ((4,) if form == "chunked" else ()), "key")
    if len(primes) != LK:
        raise ValueError("len(primes) != LK")
    ctx = context(ext.device.index)
    _check(lib().cross_keyswitch_inner_product(ctx, _log2(n), _u32_array(primes), LK, dnum, B, STREAM_FORM[form],
                                               _dev_ptr(ext, "ext"), _dev_ptr(key, "key"), _dev_ptr(out, "out"),
                                               _stream(ext)), ctx)
    return out


def tensor(a, b, out, d2, primes, form="valu"):
    """HE-Mult tensor product: a, b, out [B][2][L][N], d2 [B][L][N] (out = (a0 b0, a0 b1 + a1 b0),
    d2 = a1 b1 limb-wise)."""
    B, two, L, n = a.shape
    if two != 2:
        raise ValueError("a must be [B][2][L][N]")
    _shape(b, a.shape, "b")
    _shape(out, a.shape, "out")
    _shape(d2, (B, L, n), "d2")
    if len(primes) != L:
        raise ValueError("len(primes) != L")
    ctx = context(a.device.index)
    _check(lib().cross_tensor(ctx, _log2(n), _u32_array(primes), L, B, STREAM_FORM[form], _dev_ptr(a, "a"),
                              _dev_ptr(b, "b"), _dev_ptr(out, "out"), _dev_ptr(d2, "d2"), _stream(a)), ctx)
    return out, d2


OP_NTT_FORWARD, OP_NTT_INVERSE, OP_HE_MULT, OP_ROTATE = 1, 2, 3, 4


class Job(ctypes.Structure):
    """Mirror of cross_job."""
    _fields_ = [("op", c_u32), ("params", CkksParams), ("batch", c_u32), ("steps", c_i32),
                ("data", c_vp), ("ct_a", c_vp), ("ct_b", c_vp), ("key", c_vp), ("out", c_vp)]


def _ptr(t):
    return None if t is None else _dev_ptr(t, "buffer").value


def _marshal_jobs(jobs):
    """Job dicts -> (cross_job array, objects that must outlive it)."""
    arr = (Job * len(jobs))()
    keep = [arr]
    for i, j in enumerate(jobs):
        op = j["op"]
        if op in ("ntt_forward", "ntt_inverse"):
            d = j["data"]
            bt, L, n = d.shape
            prm = _params(j["primes"], [], 1, n)
            prm.K = 0
            arr[i] = Job(OP_NTT_FORWARD if op == "ntt_forward" else OP_NTT_INVERSE, prm, bt, 0,
                         _ptr(d), None, None, None, None)
        elif op == "he_mult":
            a = j["a"]
            prm = _params(j["qs"], j["ps"], j["dnum"], a.shape[-1])
            arr[i] = Job(OP_HE_MULT, prm, a.shape[0], 0, None, _ptr(a), _ptr(j["b"]), _ptr(j["key"]),
                         _ptr(j["out"]))
        elif op == "rotate":
            a = j["ct"]
            prm = _params(j["qs"], j["ps"], j["dnum"], a.shape[-1])
            arr[i] = Job(OP_ROTATE, prm, a.shape[0], int(j["steps"]), None, _ptr(a), None, _ptr(j["key"]),
                         _ptr(j["out"]))
        else:
            raise ValueError("unknown op %r" % op)
        keep.append(prm)
    return arr, keep


LIST_TILES = {0: "256x128", 1: "128x64", 2: "64x64"}


def get_batch_tile(log_n, inverse=False, device=None):
    """The batch runtime's work-list tile for size 2^log_n: (name, tuned)."""
    ctx = context(device)
    t, tuned = ctypes.c_int(), ctypes.c_int()
    _check(lib().cross_get_batch_tile(ctx, log_n, int(bool(inverse)), ctypes.byref(t), ctypes.byref(tuned)), ctx)
    return LIST_TILES[t.value], bool(tuned.value)


def batch_workspace_bytes(jobs, device=None):
    """Device bytes Batch(jobs, workspace=...) needs."""
    ctx = context(device)
    arr, keep = _marshal_jobs(jobs)
    n = ctypes.c_uint64(0)
    _check(lib().cross_batch_workspace_bytes(ctx, ctypes.cast(arr, c_vp), len(jobs), ctypes.byref(n)), ctx)
    return n.value


class Batch:
    """A planned batch of jobs (cross_batch).  Each job is a dict:
    {"op": "ntt_forward"|"ntt_inverse", "data": t[batch][L][N], "primes": [...]}
    {"op": "he_mult", "a", "b", "key", "out", "qs", "ps", "dnum"}
    {"op": "rotate", "ct", "key", "out", "qs", "ps", "dnum", "steps"}
    Tensors must stay alive while the batch exists.  With `workspace` (a device
    tensor of at least batch_workspace_bytes(jobs) bytes, 256-byte aligned) the
    batch allocates no device memory and closing it does not synchronise."""

    def __init__(self, jobs, use_graph=True, device=None, workspace=None, stream=None):
        self.handle = None
        self.ctx = context(device)
        arr, self._keep = _marshal_jobs(jobs)
        h = c_vp()
        if workspace is None:
            _check(lib().cross_batch_create(self.ctx, ctypes.cast(arr, c_vp), len(jobs), 1 if use_graph else 0,
                                            ctypes.byref(h)), self.ctx)
        else:
            import torch
            st = c_vp(torch.cuda.current_stream().cuda_stream) if stream is None else c_vp(stream)
            _check(lib().cross_batch_create_in(self.ctx, ctypes.cast(arr, c_vp), len(jobs), 1 if use_graph else 0,
                                               c_vp(workspace.data_ptr()),
                                               workspace.numel() * workspace.element_size(), st, ctypes.byref(h)),
                   self.ctx)
            self._keep.append(workspace)
        self.handle = h

    def run(self, stream=None):
        import torch
        s = c_vp(torch.cuda.current_stream().cuda_stream) if stream is None else c_vp(stream)
        _check(lib().cross_batch_run(self.handle, s), self.ctx)

    def info(self):
        n, ws, tiles = c_u32(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().cross_batch_info(self.handle, ctypes.byref(n), ctypes.byref(ws), ctypes.byref(tiles)), self.ctx)
        return {"launches": n.value, "workspace_bytes": ws.value, "gemm_tiles": tiles.value}

    def close(self):
        if getattr(self, "handle", None):
            lib().cross_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
