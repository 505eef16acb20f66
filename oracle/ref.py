"""ctypes marshalling for the C oracle (test infrastructure only).

Every function mirrors one entry point of ``pivco_ref.h``; the passage of the
paper each one follows is cited there.  Inputs and outputs are numpy arrays
or ``bytes``; errors raise ``OracleError`` carrying the C status code.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libpivco_ref.so")
_lib = None

OK, E_ARG, E_CAPACITY, E_CORRUPT, E_UNSUPPORTED = 0, -1, -2, -3, -4


class OracleError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: oracle status {code}")
        self.code = code


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from .build import build
            build()
        _lib = C.CDLL(_LIB_PATH)
        u8p, u16p, u64p = C.POINTER(C.c_uint8), C.POINTER(C.c_uint16), C.POINTER(C.c_uint64)
        u32p = C.POINTER(C.c_uint32)
        sig = {
            "pivco_ref_lengths": (C.c_int, [u64p, C.c_uint32, u8p]),
            "pivco_ref_codes": (C.c_int, [u8p, u16p]),
            "pivco_ref_p1q": (C.c_uint32, [C.c_uint64, C.c_uint64]),
            "pivco_ref_select_ans": (C.c_int, [C.c_uint32, C.c_uint64, C.c_uint64]),
            "pivco_ref_rans_encode": (C.c_int, [u8p, C.c_uint64, C.c_uint32, C.c_uint32, u8p,
                                                C.c_uint64, u64p]),
            "pivco_ref_rans_decode": (C.c_int, [u8p, C.c_uint64, C.c_uint64, C.c_uint32,
                                                C.c_uint32, u8p]),
            "pivco_ref_encode_bound": (C.c_uint64, [C.c_uint64, C.c_uint32, C.c_uint32]),
            "pivco_ref_encode": (C.c_int, [u8p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                           C.c_uint32, u8p, u8p, C.c_uint64, u64p]),
            "pivco_ref_encode_flat": (C.c_int, [u8p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                                C.c_uint32, u8p, u8p, C.c_uint64, u64p]),
            "pivco_ref_stream_info": (C.c_int, [u8p, C.c_uint64, u64p, u32p, u32p, u64p]),
            "pivco_ref_decode": (C.c_int, [u8p, C.c_uint64, u8p, C.c_uint64, u64p]),
            "pivco_ref_decode_merge": (C.c_int, [u8p, C.c_uint64, u8p, C.c_uint64, u64p]),
            "pivco_ref_decode_blocks": (C.c_int, [u8p, C.c_uint64, C.c_uint32, C.c_uint32, u8p,
                                                  C.c_uint64, u64p]),
            "pivco_ref_classical_encode": (C.c_int, [u8p, C.c_uint64, u8p, u8p, C.c_uint64, u64p]),
            "pivco_ref_classical_decode": (C.c_int, [u8p, C.c_uint64, u8p, u8p, C.c_uint64]),
            "pivco_ref_pivoted_to_classical": (C.c_int, [u8p, C.c_uint64, u8p, C.c_uint64, u64p]),
            "pivco_ref_block_info": (C.c_int, [u8p, C.c_uint64, C.c_uint32, u8p, u32p, u32p, u8p,
                                               u64p, u64p, u8p, u8p]),
            "pivco_ref_fse_norm": (C.c_int, [C.c_uint32, u16p]),
            "pivco_ref_fse_cost": (C.c_double, [C.c_uint32]),
            "pivco_ref_fse_select": (C.c_int, [C.c_uint64, C.c_uint64, C.c_uint32, u32p]),
            "pivco_ref_fse_encode": (C.c_int, [u8p, C.c_uint64, C.c_uint32, C.c_uint32, u8p, C.c_uint64,
                                               u64p]),
            "pivco_ref_fse_decode": (C.c_int, [u8p, C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32, u8p]),
            "pivco_ref_golomb_bound": (C.c_uint64, [C.c_uint64, C.c_uint32]),
            "pivco_ref_golomb_encode": (C.c_int, [u8p, C.c_uint64, C.c_uint32, u8p, C.c_uint64, u64p]),
            "pivco_ref_golomb_decode": (C.c_int, [u8p, C.c_uint64, u8p, C.c_uint64, u64p]),
            "pivco_ref_golomb_decode_merge": (C.c_int, [u8p, C.c_uint64, u8p, C.c_uint64, u64p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(_lib, name)
            f.restype = res
            f.argtypes = args
    return _lib


def _u8(a):
    a = np.ascontiguousarray(np.frombuffer(a, dtype=np.uint8) if isinstance(a, (bytes, bytearray))
                             else a, dtype=np.uint8)
    return a, a.ctypes.data_as(C.POINTER(C.c_uint8))


def _check(rc, what):
    if rc != 0:
        raise OracleError(rc, what)


def lengths(counts, max_len=11):
    """Optimal length-limited code lengths for 256 symbol counts."""
    c = np.ascontiguousarray(np.asarray(counts, dtype=np.uint64).reshape(256))
    out = np.zeros(256, dtype=np.uint8)
    _check(lib().pivco_ref_lengths(c.ctypes.data_as(C.POINTER(C.c_uint64)), max_len,
                                   out.ctypes.data_as(C.POINTER(C.c_uint8))), "lengths")
    return out


def codes(lens):
    ln, lp = _u8(np.asarray(lens, dtype=np.uint8).reshape(256))
    out = np.zeros(256, dtype=np.uint16)
    _check(lib().pivco_ref_codes(lp, out.ctypes.data_as(C.POINTER(C.c_uint16))), "codes")
    return out


def p1q(n_v, n_right):
    return int(lib().pivco_ref_p1q(n_v, n_right))


def select_ans(mode, n_v, n_right):
    return bool(lib().pivco_ref_select_ans(mode, n_v, n_right))


def rans_encode(bits_bytes, nbits, p1q_, chunk_log2=16):
    b, bp = _u8(bits_bytes)
    cap = ((nbits + (1 << chunk_log2) - 1) >> chunk_log2) * 136 + 2 * nbits + 16
    out = np.zeros(cap, dtype=np.uint8)
    ol = C.c_uint64(0)
    _check(lib().pivco_ref_rans_encode(bp, nbits, p1q_, chunk_log2,
                                       out.ctypes.data_as(C.POINTER(C.c_uint8)), cap,
                                       C.byref(ol)), "rans_encode")
    return out[:ol.value].tobytes()


def rans_decode(body, nbits, p1q_, chunk_log2=16):
    b, bp = _u8(body)
    out = np.zeros((nbits + 7) // 8 + 1, dtype=np.uint8)
    _check(lib().pivco_ref_rans_decode(bp, len(b), nbits, p1q_, chunk_log2,
                                       out.ctypes.data_as(C.POINTER(C.c_uint8))), "rans_decode")
    return out[:(nbits + 7) // 8].tobytes()


def encode_bound(n, block_size, ans_mode=0):
    return int(lib().pivco_ref_encode_bound(n, block_size, ans_mode))


def encode(data, block_size, max_len=11, ans_mode=0, chunk_log2=16, tree_len=None, flat=False):
    """Encode a uint8 array; returns the stream as a uint8 numpy array
    (v1, or v2 with flat-subtree trees when flat=True)."""
    d, dp = _u8(data)
    n = d.size
    cap = encode_bound(n, block_size, ans_mode) + 64
    out = np.zeros(cap, dtype=np.uint8)
    ol = C.c_uint64(0)
    tp = None
    if tree_len is not None:
        t, tp = _u8(np.asarray(tree_len, dtype=np.uint8).reshape(256))
    f = lib().pivco_ref_encode_flat if flat else lib().pivco_ref_encode
    _check(f(dp if n else None, n, block_size, max_len, ans_mode, chunk_log2,
             tp, out.ctypes.data_as(C.POINTER(C.c_uint8)), cap, C.byref(ol)), "encode")
    return out[:ol.value].copy()


def stream_info(stream):
    s, sp = _u8(stream)
    n = C.c_uint64(0); nb = C.c_uint32(0); bs = C.c_uint32(0); aw = C.c_uint64(0)
    _check(lib().pivco_ref_stream_info(sp, s.size, C.byref(n), C.byref(nb), C.byref(bs),
                                       C.byref(aw)), "stream_info")
    return {"n_total": n.value, "n_blocks": nb.value, "block_size": bs.value,
            "ans_words": aw.value}


def decode(stream, n=None, merge=False):
    """Decode a whole stream (decoder A by default, B with merge=True)."""
    s, sp = _u8(stream)
    if n is None:
        n = stream_info(s)["n_total"]
    out = np.zeros(max(n, 1), dtype=np.uint8)
    no = C.c_uint64(0)
    f = lib().pivco_ref_decode_merge if merge else lib().pivco_ref_decode
    _check(f(sp, s.size, out.ctypes.data_as(C.POINTER(C.c_uint8)), n, C.byref(no)), "decode")
    return out[:no.value]


def decode_blocks(stream, b0, b1):
    s, sp = _u8(stream)
    info = stream_info(s)
    cap = (b1 - b0) * info["block_size"]
    out = np.zeros(max(cap, 1), dtype=np.uint8)
    no = C.c_uint64(0)
    _check(lib().pivco_ref_decode_blocks(sp, s.size, b0, b1,
                                         out.ctypes.data_as(C.POINTER(C.c_uint8)), cap,
                                         C.byref(no)), "decode_blocks")
    return out[:no.value]


def classical_encode(data, lens):
    d, dp = _u8(data)
    l, lp = _u8(np.asarray(lens, dtype=np.uint8).reshape(256))
    cap = d.size * 2 + 8
    out = np.zeros(cap, dtype=np.uint8)
    nb = C.c_uint64(0)
    _check(lib().pivco_ref_classical_encode(dp, d.size, lp, out.ctypes.data_as(C.POINTER(C.c_uint8)),
                                            cap, C.byref(nb)), "classical_encode")
    return out[:(nb.value + 7) // 8].copy(), nb.value


def classical_decode(bits, nbits, lens, n):
    b, bp = _u8(bits)
    l, lp = _u8(np.asarray(lens, dtype=np.uint8).reshape(256))
    out = np.zeros(max(n, 1), dtype=np.uint8)
    _check(lib().pivco_ref_classical_decode(bp, nbits, lp, out.ctypes.data_as(C.POINTER(C.c_uint8)),
                                            n), "classical_decode")
    return out[:n]


def pivoted_to_classical(stream, cap):
    s, sp = _u8(stream)
    out = np.zeros(cap, dtype=np.uint8)
    nb = C.c_uint64(0)
    _check(lib().pivco_ref_pivoted_to_classical(sp, s.size, out.ctypes.data_as(C.POINTER(C.c_uint8)),
                                                cap, C.byref(nb)), "pivoted_to_classical")
    return out[:(nb.value + 7) // 8].copy(), nb.value


def block_info(stream, block):
    s, sp = _u8(stream)
    ln = np.zeros(256, dtype=np.uint8)
    mode = C.c_uint32(0); ni = C.c_uint32(0)
    depth = np.zeros(255, dtype=np.uint8); kind = np.zeros(255, dtype=np.uint8)
    flat = np.zeros(255, dtype=np.uint8)
    nv = np.zeros(255, dtype=np.uint64); nr = np.zeros(255, dtype=np.uint64)
    P8, P64 = C.POINTER(C.c_uint8), C.POINTER(C.c_uint64)
    _check(lib().pivco_ref_block_info(sp, s.size, block, ln.ctypes.data_as(P8), C.byref(mode),
                                      C.byref(ni), depth.ctypes.data_as(P8), nv.ctypes.data_as(P64),
                                      nr.ctypes.data_as(P64), kind.ctypes.data_as(P8),
                                      flat.ctypes.data_as(P8)),
           "block_info")
    k = ni.value
    return {"len": ln, "mode": mode.value, "n_internal": k, "depth": depth[:k].copy(),
            "n_v": nv[:k].copy(), "n_right": nr[:k].copy(), "kind": kind[:k].copy(),
            "flat": flat[:k].copy()}


def fse_norm(t):
    """Normalized counts (sum 2^11) of tANS table t (1..50)."""
    out = np.zeros(256, dtype=np.uint16)
    _check(lib().pivco_ref_fse_norm(t, out.ctypes.data_as(C.POINTER(C.c_uint16))), "fse_norm")
    return out


def fse_cost(t):
    return float(lib().pivco_ref_fse_cost(t))


def fse_select(n_v, n_right, depth):
    """(selected, marker) of the selective-tANS rule."""
    m = C.c_uint32(0)
    r = lib().pivco_ref_fse_select(n_v, n_right, depth, C.byref(m))
    return bool(r), m.value


def fse_encode(bits_bytes, nbits, marker, chunk_log2=16):
    b, bp = _u8(bits_bytes)
    cap = 8 * b.size + 256 * ((nbits >> chunk_log2) + 1) + 64
    out = np.zeros(cap, dtype=np.uint8)
    ol = C.c_uint64(0)
    _check(lib().pivco_ref_fse_encode(bp, nbits, marker, chunk_log2, out.ctypes.data_as(C.POINTER(C.c_uint8)),
                                      cap, C.byref(ol)), "fse_encode")
    return out[:ol.value].copy()


def fse_decode(body, nbits, marker, chunk_log2=16):
    b, bp = _u8(body)
    out = np.zeros((nbits + 7) // 8 + 1, dtype=np.uint8)
    _check(lib().pivco_ref_fse_decode(bp, b.size, nbits, marker, chunk_log2,
                                      out.ctypes.data_as(C.POINTER(C.c_uint8))), "fse_decode")
    return out[:(nbits + 7) // 8]


__all__ = ["OracleError", "lib", "lengths", "codes", "p1q", "select_ans", "rans_encode",
           "fse_norm", "fse_cost", "fse_select", "fse_encode", "fse_decode",
           "rans_decode", "encode_bound", "encode", "stream_info", "decode", "decode_blocks",
           "classical_encode", "classical_decode", "pivoted_to_classical", "block_info",
           "golomb_encode", "golomb_decode", "golomb_decode_merge",
           "OK", "E_ARG", "E_CAPACITY", "E_CORRUPT", "E_UNSUPPORTED"]


# --------------------------------------------------------------------------
# PivCo-Golomb (App. G)
# --------------------------------------------------------------------------

def golomb_encode(values, block_size):
    """Unary-coded values (uint8) in the pivoted list-of-bitmaps layout."""
    x, xp = _u8(values)
    cap = int(lib().pivco_ref_golomb_bound(x.size, block_size))
    out = np.zeros(max(cap, 1), dtype=np.uint8)
    olen = C.c_uint64(0)
    _check(lib().pivco_ref_golomb_encode(xp, x.size, block_size,
                                         out.ctypes.data_as(C.POINTER(C.c_uint8)), out.size,
                                         C.byref(olen)), "golomb_encode")
    return out[:olen.value].copy()


def _golomb_dec(stream, fn, n):
    s, sp = _u8(stream)
    if n is None:
        n = int.from_bytes(bytes(s[8:16]), "little") if s.size >= 16 else 0
    out = np.zeros(max(n, 1), dtype=np.uint8)
    got = C.c_uint64(0)
    _check(fn(sp, s.size, out.ctypes.data_as(C.POINTER(C.c_uint8)), n, C.byref(got)), "golomb_decode")
    return out[:got.value].copy()


def golomb_decode(stream, n=None):
    """Decoder A: each value's code read bit by bit (a cursor per bitmap)."""
    return _golomb_dec(stream, lib().pivco_ref_golomb_decode, n)


def golomb_decode_merge(stream, n=None):
    """Decoder B: bottom-up merge from the last bitmap (merge_vec_cst_plus1)."""
    return _golomb_dec(stream, lib().pivco_ref_golomb_decode_merge, n)
