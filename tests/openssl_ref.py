"""Independent AES from the system OpenSSL (libcrypto, EVP interface), via ctypes.

Used only by tests, as a black-box cross-check of the oracle.  OpenSSL's CTR
mode increments the whole 128-bit counter block, so it agrees with the 64-bit
counter of the oracle only while the low 64 bits do not wrap; callers keep to
that case.
"""
import ctypes
import ctypes.util

import numpy as np

_lib = None


def available() -> bool:
    try:
        _load()
        return True
    except OSError:
        return False


def _load():
    global _lib
    if _lib is not None:
        return _lib
    name = ctypes.util.find_library("crypto") or "libcrypto.so.3"
    lib = ctypes.CDLL(name)
    p = ctypes.c_void_p
    lib.EVP_CIPHER_CTX_new.restype = p
    lib.EVP_CIPHER_CTX_free.argtypes = [p]
    for nm in ("EVP_EncryptInit_ex", "EVP_DecryptInit_ex"):
        f = getattr(lib, nm)
        f.argtypes = [p, p, p, p, p]
        f.restype = ctypes.c_int
    for nm in ("EVP_EncryptUpdate", "EVP_DecryptUpdate"):
        f = getattr(lib, nm)
        f.argtypes = [p, p, ctypes.POINTER(ctypes.c_int), p, ctypes.c_int]
        f.restype = ctypes.c_int
    for nm in ("EVP_EncryptFinal_ex", "EVP_DecryptFinal_ex"):
        f = getattr(lib, nm)
        f.argtypes = [p, p, ctypes.POINTER(ctypes.c_int)]
        f.restype = ctypes.c_int
    lib.EVP_CIPHER_CTX_set_padding.argtypes = [p, ctypes.c_int]
    for bits in (128, 192, 256):
        for mode in ("ecb", "cbc", "ctr"):
            getattr(lib, f"EVP_aes_{bits}_{mode}").restype = p
    _lib = lib
    return lib


def _run(mode: str, bits: int, key, iv, data, decrypt: bool) -> np.ndarray:
    lib = _load()
    key = np.ascontiguousarray(np.frombuffer(bytes(key), np.uint8)[: bits // 8])
    data = np.ascontiguousarray(np.frombuffer(bytes(data), np.uint8))
    out = np.zeros(data.size + 32, np.uint8)
    ivb = None if iv is None else np.ascontiguousarray(np.frombuffer(bytes(iv), np.uint8))
    ctx = lib.EVP_CIPHER_CTX_new()
    try:
        cipher = getattr(lib, f"EVP_aes_{bits}_{mode}")()
        init = lib.EVP_DecryptInit_ex if decrypt else lib.EVP_EncryptInit_ex
        upd = lib.EVP_DecryptUpdate if decrypt else lib.EVP_EncryptUpdate
        fin = lib.EVP_DecryptFinal_ex if decrypt else lib.EVP_EncryptFinal_ex
        ok = init(ctx, cipher, None, key.ctypes.data,
                  None if ivb is None else ivb.ctypes.data)
        assert ok == 1
        lib.EVP_CIPHER_CTX_set_padding(ctx, 0)
        n1 = ctypes.c_int(0)
        n2 = ctypes.c_int(0)
        if data.size:
            ok = upd(ctx, out.ctypes.data, ctypes.byref(n1), data.ctypes.data, data.size)
            assert ok == 1
        ok = fin(ctx, out.ctypes.data + n1.value, ctypes.byref(n2))
        assert ok == 1
        return out[: n1.value + n2.value].copy()
    finally:
        lib.EVP_CIPHER_CTX_free(ctx)


def ecb(bits, key, data, decrypt=False):
    return _run("ecb", bits, key, None, data, decrypt)


def cbc(bits, key, iv, data, decrypt=False):
    return _run("cbc", bits, key, iv, data, decrypt)


def ctr(bits, key, iv, data):
    return _run("ctr", bits, key, iv, data, False)
