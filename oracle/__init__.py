"""Plain CPU AES oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  It wraps ``aes_oracle.c`` (FIPS-197 Cipher,
InvCipher and KeyExpansion written out on a 4x4 byte state; NIST SP 800-38A
CBC and CTR with a 64-bit big-endian counter) through ctypes, and shares no
code with the GPU library.

Every entry point takes and returns plain ``bytes`` / numpy ``uint8`` arrays.
"""
import ctypes
import os
import threading

import numpy as np

from . import build as _build

OP_CBC_ENC = 0
OP_CBC_DEC = 1
OP_CTR = 2
OP_ECB_ENC = 3
OP_ECB_DEC = 4

# Request record of the batch driver (layout of oracle_req_t in aes_oracle.c).
REQ_DTYPE = np.dtype([("offset", "<u8"), ("length", "<u8"), ("key_idx", "<u4"),
                      ("op", "<u4"), ("iv", "u1", (16,))])

_lib = None
_lock = threading.Lock()


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        p = ctypes.c_void_p
        lib.oracle_sbox.argtypes = [p, p]
        lib.oracle_sbox.restype = None
        lib.oracle_expand_key.argtypes = [p, ctypes.c_uint32, p]
        lib.oracle_expand_key.restype = ctypes.c_int
        lib.oracle_ecb.argtypes = [p, ctypes.c_uint32, ctypes.c_int, p, p, ctypes.c_uint64]
        lib.oracle_ecb.restype = ctypes.c_int
        lib.oracle_mode.argtypes = [ctypes.c_uint32, p, ctypes.c_uint32, p, p, p,
                                    ctypes.c_uint64]
        lib.oracle_mode.restype = ctypes.c_int
        lib.oracle_batch.argtypes = [p, p, ctypes.c_uint64, p, ctypes.c_uint64, p, p,
                                     ctypes.c_uint32, ctypes.c_int]
        lib.oracle_batch.restype = ctypes.c_int
        _lib = lib
        return lib


def _u8(buf) -> np.ndarray:
    a = np.ascontiguousarray(np.frombuffer(bytes(buf), dtype=np.uint8)
                             if isinstance(buf, (bytes, bytearray, memoryview)) else buf,
                             dtype=np.uint8)
    return a


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class OracleError(RuntimeError):
    pass


def sbox():
    """Returns (S-box, inverse S-box) as two 256-entry uint8 arrays (FIPS-197 5.1.1)."""
    s = np.zeros(256, np.uint8)
    si = np.zeros(256, np.uint8)
    _load().oracle_sbox(_ptr(s), _ptr(si))
    return s, si


def expand_key(key, key_bits: int) -> np.ndarray:
    """FIPS-197 5.2 KeyExpansion; returns the (4*(Nr+1), 4) word array as bytes."""
    k = _u8(key)
    w = np.zeros(240, np.uint8)
    nr = _load().oracle_expand_key(_ptr(k), key_bits, _ptr(w))
    if nr < 0:
        raise OracleError(f"oracle_expand_key: {nr}")
    return w[: 16 * (nr + 1)].reshape(-1, 4).copy()


def ecb(key, key_bits: int, data, decrypt: bool = False) -> np.ndarray:
    """Block-by-block Cipher (or InvCipher) over whole 16-byte blocks."""
    k = _u8(key)
    d = _u8(data).copy()
    if d.size % 16:
        raise OracleError("ECB needs whole blocks")
    st = _load().oracle_ecb(_ptr(k), key_bits, int(decrypt), _ptr(d), _ptr(d), d.size // 16)
    if st != 0:
        raise OracleError(f"oracle_ecb: {st}")
    return d


def mode(op: int, key, key_bits: int, iv, data) -> np.ndarray:
    """One CBC-encrypt / CBC-decrypt / CTR / ECB-encrypt / ECB-decrypt request
    over a contiguous buffer (ECB takes no IV: iv may be None)."""
    k = _u8(key)
    v = _u8(np.zeros(16, np.uint8) if iv is None else iv)
    d = _u8(data)
    out = np.empty_like(d)
    st = _load().oracle_mode(op, _ptr(k), key_bits, _ptr(v), _ptr(d), _ptr(out), d.size)
    if st != 0:
        raise OracleError(f"oracle_mode: {st}")
    return out


def cbc_encrypt(key, key_bits, iv, data):
    return mode(OP_CBC_ENC, key, key_bits, iv, data)


def cbc_decrypt(key, key_bits, iv, data):
    return mode(OP_CBC_DEC, key, key_bits, iv, data)


def ctr(key, key_bits, t1, data):
    return mode(OP_CTR, key, key_bits, t1, data)


def batch(inp: np.ndarray, out: np.ndarray, reqs: np.ndarray, keys: np.ndarray,
          key_bits: np.ndarray, n_threads: int = 0) -> int:
    """Applies every request of ``reqs`` (REQ_DTYPE) from ``inp`` into ``out`` in place.

    ``keys`` is an (n_keys, 32) uint8 array (the first key_bits/8 bytes of a row
    are the key); ``key_bits`` an (n_keys,) uint32 array.  Bytes of ``out``
    outside every request are left as they are.  Returns the thread count used.
    """
    assert inp.dtype == np.uint8 and out.dtype == np.uint8 and inp.size == out.size
    assert inp.flags.c_contiguous and out.flags.c_contiguous
    reqs = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
    keys = np.ascontiguousarray(keys, dtype=np.uint8)
    key_bits = np.ascontiguousarray(key_bits, dtype=np.uint32)
    assert keys.ndim == 2 and keys.shape[1] == 32 and keys.shape[0] == key_bits.size
    st = _load().oracle_batch(_ptr(inp), _ptr(out), inp.size, _ptr(reqs), reqs.size,
                              _ptr(keys), _ptr(key_bits), key_bits.size, n_threads)
    if st < 0:
        raise OracleError(f"oracle_batch: {st}")
    return st
