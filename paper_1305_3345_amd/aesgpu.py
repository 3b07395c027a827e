"""Thin ctypes binding of libaesgpu.so (the C ABI declared in include/aesgpu.h).

Argument marshalling only: every cipher step runs in the library's HIP
kernels.  Device buffers are torch tensors (their ``data_ptr()`` crosses the
boundary) or raw integer device addresses; streams are torch streams or raw
``hipStream_t`` integers (default: torch's current stream).  The library must
be built (``python -m paper_1305_3345_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

try:  # torch first: the library then binds to the HIP runtime torch has loaded
    import torch
except ImportError:  # host-only use (validation, planning) without torch
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaesgpu.so")

AES_OK = 0
AES_ERR_ARG = -1
AES_ERR_KEYSIZE = -2
AES_ERR_LENGTH = -3
AES_ERR_RANGE = -4
AES_ERR_OVERLAP = -5
AES_ERR_DEVICE = -6
AES_ERR_NOMEM = -7
AES_ERR_AGAIN = -8
AES_ERR_TIMEOUT = -9
AES_ERR_STATE = -10

AES_OP_CBC_ENC = 0
AES_OP_CBC_DEC = 1
AES_OP_CTR = 2
AES_OP_ECB_ENC = 3
AES_OP_ECB_DEC = 4
AES_DEVICE_NONE = -1
AES_NOALLOC_MAX_UNITS = 1 << 19
AES_CTR_TABLE = 0
AES_CTR_BITSLICE = 1
AES_DEC_TABLE = 0
AES_DEC_BITSLICE = 1

SCHED_DTYPE = np.dtype([("key_bits", "<u4"), ("nr", "<u4"), ("reserved0", "<u4", (2,)),
                        ("ek", "<u4", (60,)), ("dk", "<u4", (60,)), ("reserved1", "<u4", (4,))])
REQ_DTYPE = np.dtype([("offset", "<u8"), ("length", "<u8"), ("key_idx", "<u4"),
                      ("op", "<u4"), ("iv", "u1", (16,))])
UNIT_DTYPE = np.dtype([("offset", "<u8"), ("nbytes", "<u4"), ("meta", "<u4"),
                       ("w", "<u4", (4,))])
PLAN_INFO_DTYPE = np.dtype([("n_units_cbc_dec", "<u8"), ("n_units_ctr", "<u8"),
                            ("n_chains_cbc_enc", "<u8"), ("payload_bytes", "<u8"),
                            ("extent_bytes", "<u8"), ("tile_bytes", "<u4"),
                            ("reserved", "<u4")])
CONFIG_DTYPE = np.dtype([(k, "<u4") for k in (
    "tile_bytes", "ctr_nb", "ctr_wg", "dec_nb", "dec_wg", "chain_lanes", "chain_wg", "mixed_nb",
    "fuse", "grid", "ctr_variant", "chain_quad", "dec_variant")] + [("reserved", "<u4", (3,))])
assert CONFIG_DTYPE.itemsize == 64
assert SCHED_DTYPE.itemsize == 512 and REQ_DTYPE.itemsize == 40 and UNIT_DTYPE.itemsize == 32

_lib = None
_lock = threading.Lock()


class AesError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib().aes_strerror(status).decode()
        if status == AES_ERR_DEVICE:
            msg += f" (hipError {lib().aes_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{status}]")


def lib():
    """Loads libaesgpu.so once; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1305_3345_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        p = ctypes.c_void_p
        u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        sig = {
            "aes_strerror": (ctypes.c_char_p, [i32]),
            "aes_last_hip_error": (i32, []),
            "aes_expand_key": (i32, [p, u32, p]),
            "aes_ctx_create": (i32, [i32, ctypes.POINTER(p)]),
            "aes_ctx_destroy": (None, [p]),
            "aes_batch": (i32, [p, p, u32, p, p, u64, p, u64, p]),
            "aes_batch_noalloc": (i32, [p, p, u32, p, p, u64, p, u64, p]),
            "aes_cbc_encrypt_batch": (i32, [p, p, u32, p, p, u64, p, p, p, p, u64, p]),
            "aes_cbc_decrypt_batch": (i32, [p, p, u32, p, p, u64, p, p, p, p, u64, p]),
            "aes_ctr_batch": (i32, [p, p, u32, p, p, u64, p, p, p, p, u64, p]),
            "aes_ecb_encrypt_batch": (i32, [p, p, u32, p, p, u64, p, p, p, p, u64, p]),
            "aes_ecb_decrypt_batch": (i32, [p, p, u32, p, p, u64, p, p, p, p, u64, p]),
            "aes_plan_create": (i32, [p, p, u64, u32, u64, ctypes.POINTER(p)]),
            "aes_plan_launch": (i32, [p, p, p, p, p]),
            "aes_plan_info": (i32, [p, p]),
            "aes_plan_units": (i32, [p, p, u64, ctypes.POINTER(u64)]),
            "aes_plan_destroy": (None, [p]),
            "aes_ctx_get_config": (i32, [p, p]),
            "aes_ctx_set_config": (i32, [p, p]),
            "aes_tune": (i32, [p, p, u64, u32, u64, p, p, p, u32, p]),
            "aes_tune_key": (i32, [p, p, u64, u32, p, ctypes.c_size_t,
                                   ctypes.POINTER(ctypes.c_size_t)]),
            "aes_host_batch": (i32, [p, u32, p, p, u64, p, u64, u32]),
            "aes_request_launch": (i32, [p, p, u32, p, p, u64, p, p]),
            "aes_request_launches": (i32, [p, p, u32, p, p, u64, p, u64, p]),
            "aes_plan_graph": (i32, [p, p, p, p, ctypes.POINTER(p)]),
            "aes_requests_graph": (i32, [p, p, u32, p, p, u64, p, u64, ctypes.POINTER(p)]),
            "aes_graph_launch": (i32, [p, p]),
            "aes_graph_destroy": (None, [p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
        return L


def _check(status: int, where: str):
    if status != AES_OK:
        raise AesError(status, where)


def _ptr(x) -> int:
    """Device/host address of a tensor, numpy array or raw integer (0 for None)."""
    if x is None:
        return 0
    if isinstance(x, int):
        return x
    if torch is not None and isinstance(x, torch.Tensor):
        return x.data_ptr()
    if isinstance(x, np.ndarray):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def _nbytes(x) -> int:
    if torch is not None and isinstance(x, torch.Tensor):
        return x.numel() * x.element_size()
    if isinstance(x, np.ndarray):
        return x.nbytes
    raise TypeError("buffer size needed")


def _stream(stream) -> int:
    if stream is None:
        if torch is not None and torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
        return 0
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ----------------------------------------------------------------- key setup

def expand_key(key, key_bits: int) -> np.ndarray:
    """aes_expand_key: one schedule record (SCHED_DTYPE) for key_bits/8 key bytes."""
    k = np.ascontiguousarray(np.frombuffer(bytes(key), np.uint8) if not isinstance(key, np.ndarray)
                             else key, dtype=np.uint8)
    out = np.zeros(1, SCHED_DTYPE)
    _check(lib().aes_expand_key(k.ctypes.data, key_bits, out.ctypes.data), "aes_expand_key")
    return out[0]


def expand_keys(keys: np.ndarray, key_bits) -> np.ndarray:
    """Schedules for an (n, >=32) uint8 key array; key_bits per key or scalar."""
    kb = np.broadcast_to(np.asarray(key_bits, np.uint32), (keys.shape[0],))
    out = np.zeros(keys.shape[0], SCHED_DTYPE)
    for i in range(keys.shape[0]):
        out[i] = expand_key(np.ascontiguousarray(keys[i, : kb[i] // 8]), int(kb[i]))
    return out


def schedules_to_device(scheds: np.ndarray, device="cuda"):
    """Copies schedule records to a device uint8 tensor (512 bytes each)."""
    host = torch.from_numpy(np.ascontiguousarray(scheds).view(np.uint8).copy())
    return host.to(device)


# ------------------------------------------------------------------- context

class Context:
    """aes_ctx_create / aes_ctx_destroy.  device=AES_DEVICE_NONE gives a host-only context."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib().aes_ctx_create(device, ctypes.byref(h)), "aes_ctx_create")
        self.handle = h.value
        self.device = device

    def get_config(self) -> dict:
        """aes_ctx_get_config as a dict."""
        c = np.zeros(1, CONFIG_DTYPE)
        _check(lib().aes_ctx_get_config(self.handle, c.ctypes.data), "aes_ctx_get_config")
        return {k: int(c[0][k]) for k in CONFIG_DTYPE.names if k != "reserved"}

    def set_config(self, **kw):
        """aes_ctx_set_config with the given fields changed."""
        cur = self.get_config()
        cur.update(kw)
        c = np.zeros(1, CONFIG_DTYPE)
        for k, v in cur.items():
            c[0][k] = v
        _check(lib().aes_ctx_set_config(self.handle, c.ctypes.data), "aes_ctx_set_config")

    def close(self):
        if self.handle:
            lib().aes_ctx_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _sched_count(d_scheds, n_scheds):
    if n_scheds is not None:
        return n_scheds
    return _nbytes(d_scheds) // SCHED_DTYPE.itemsize


def batch(ctx: Context, d_scheds, d_in, d_out, reqs: np.ndarray, buf_bytes: int | None = None,
          n_scheds: int | None = None, stream=None):
    """aes_batch over a REQ_DTYPE request array."""
    reqs = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
    bb = _nbytes(d_in) if buf_bytes is None else buf_bytes
    _check(lib().aes_batch(ctx.handle, _ptr(d_scheds), _sched_count(d_scheds, n_scheds),
                           _ptr(d_in), _ptr(d_out), bb, reqs.ctypes.data, reqs.size,
                           _stream(stream)), "aes_batch")


def batch_noalloc(ctx: Context, d_scheds, d_in, d_out, reqs: np.ndarray,
                  buf_bytes: int | None = None, n_scheds: int | None = None, stream=None):
    """aes_batch_noalloc (aes_batch without any allocation) over a REQ_DTYPE
    request array."""
    reqs = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
    bb = _nbytes(d_in) if buf_bytes is None else buf_bytes
    _check(lib().aes_batch_noalloc(ctx.handle, _ptr(d_scheds), _sched_count(d_scheds, n_scheds),
                                   _ptr(d_in), _ptr(d_out), bb, reqs.ctypes.data, reqs.size,
                                   _stream(stream)), "aes_batch_noalloc")


def _single(name, ctx, d_scheds, d_in, d_out, offsets, lengths, key_idx, ivs, buf_bytes,
            n_scheds, stream):
    off = np.ascontiguousarray(offsets, dtype=np.uint64)
    ln = np.ascontiguousarray(lengths, dtype=np.uint64)
    ki = np.ascontiguousarray(key_idx, dtype=np.uint32)
    n = off.size
    iv = None if ivs is None else np.ascontiguousarray(ivs, dtype=np.uint8).reshape(-1)
    if ln.size != n or ki.size != n or (iv is not None and iv.size != 16 * n):
        raise ValueError("offsets, lengths, key_idx and ivs must describe the same requests")
    bb = _nbytes(d_in) if buf_bytes is None else buf_bytes
    _check(getattr(lib(), name)(ctx.handle, _ptr(d_scheds), _sched_count(d_scheds, n_scheds),
                                _ptr(d_in), _ptr(d_out), bb, off.ctypes.data, ln.ctypes.data,
                                ki.ctypes.data, None if iv is None else iv.ctypes.data, n,
                                _stream(stream)), name)


def cbc_encrypt_batch(ctx, d_scheds, d_in, d_out, offsets, lengths, key_idx, ivs,
                      buf_bytes=None, n_scheds=None, stream=None):
    _single("aes_cbc_encrypt_batch", ctx, d_scheds, d_in, d_out, offsets, lengths, key_idx, ivs,
            buf_bytes, n_scheds, stream)


def cbc_decrypt_batch(ctx, d_scheds, d_in, d_out, offsets, lengths, key_idx, ivs,
                      buf_bytes=None, n_scheds=None, stream=None):
    _single("aes_cbc_decrypt_batch", ctx, d_scheds, d_in, d_out, offsets, lengths, key_idx, ivs,
            buf_bytes, n_scheds, stream)


def ctr_batch(ctx, d_scheds, d_in, d_out, offsets, lengths, key_idx, ivs,
              buf_bytes=None, n_scheds=None, stream=None):
    _single("aes_ctr_batch", ctx, d_scheds, d_in, d_out, offsets, lengths, key_idx, ivs,
            buf_bytes, n_scheds, stream)


def ecb_encrypt_batch(ctx, d_scheds, d_in, d_out, offsets, lengths, key_idx, ivs=None,
                      buf_bytes=None, n_scheds=None, stream=None):
    """aes_ecb_encrypt_batch (ECB takes no IVs; ivs is ignored and may be None)."""
    _single("aes_ecb_encrypt_batch", ctx, d_scheds, d_in, d_out, offsets, lengths, key_idx, ivs,
            buf_bytes, n_scheds, stream)


def ecb_decrypt_batch(ctx, d_scheds, d_in, d_out, offsets, lengths, key_idx, ivs=None,
                      buf_bytes=None, n_scheds=None, stream=None):
    """aes_ecb_decrypt_batch (ECB takes no IVs; ivs is ignored and may be None)."""
    _single("aes_ecb_decrypt_batch", ctx, d_scheds, d_in, d_out, offsets, lengths, key_idx, ivs,
            buf_bytes, n_scheds, stream)


# --------------------------------------------------------------------- plans

class Plan:
    """aes_plan_create / launch / info / units / destroy."""

    def __init__(self, ctx: Context, reqs: np.ndarray, n_scheds: int, buf_bytes: int):
        reqs = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
        h = ctypes.c_void_p()
        _check(lib().aes_plan_create(ctx.handle, reqs.ctypes.data, reqs.size, n_scheds,
                                     buf_bytes, ctypes.byref(h)), "aes_plan_create")
        self.handle = h.value
        self.ctx = ctx  # keeps the context alive

    def launch(self, d_scheds, d_in, d_out, stream=None):
        _check(lib().aes_plan_launch(self.handle, _ptr(d_scheds), _ptr(d_in), _ptr(d_out),
                                     _stream(stream)), "aes_plan_launch")

    def info(self) -> dict:
        out = np.zeros(1, PLAN_INFO_DTYPE)
        _check(lib().aes_plan_info(self.handle, out.ctypes.data), "aes_plan_info")
        return {k: int(out[0][k]) for k in PLAN_INFO_DTYPE.names if k != "reserved"}

    def units(self) -> np.ndarray:
        n = ctypes.c_uint64()
        _check(lib().aes_plan_units(self.handle, None, 0, ctypes.byref(n)), "aes_plan_units")
        out = np.zeros(n.value, UNIT_DTYPE)
        _check(lib().aes_plan_units(self.handle, out.ctypes.data if n.value else None, n.value,
                                    ctypes.byref(n)), "aes_plan_units")
        return out

    def close(self):
        if self.handle:
            lib().aes_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune(ctx: Context, reqs: np.ndarray, d_scheds, d_in, d_out, iters: int = 5,
         buf_bytes: int | None = None, n_scheds: int | None = None) -> dict:
    """aes_tune: sets and returns the fastest launch configuration for reqs
    (from the file named by AESGPU_TUNE_CACHE when it holds this batch's
    signature)."""
    reqs = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
    best = np.zeros(1, CONFIG_DTYPE)
    bb = _nbytes(d_in) if buf_bytes is None else buf_bytes
    _check(lib().aes_tune(ctx.handle, reqs.ctypes.data, reqs.size,
                          _sched_count(d_scheds, n_scheds), bb, _ptr(d_scheds), _ptr(d_in),
                          _ptr(d_out), iters, best.ctypes.data), "aes_tune")
    return {k: int(best[0][k]) for k in CONFIG_DTYPE.names if k != "reserved"}


def host_batch(scheds: np.ndarray, inp: np.ndarray, out: np.ndarray, reqs: np.ndarray,
               n_threads: int = 0):
    """aes_host_batch: a batch on host threads with the CPU's AES instructions
    (host schedules from expand_keys, host numpy buffers; out may be inp)."""
    scheds = np.ascontiguousarray(scheds, dtype=SCHED_DTYPE)
    reqs = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
    if inp.dtype != np.uint8 or out.dtype != np.uint8 or inp.size != out.size:
        raise ValueError("inp and out must be uint8 arrays of one size")
    if not (inp.flags.c_contiguous and out.flags.c_contiguous and out.flags.writeable):
        raise ValueError("inp and out must be contiguous, out writeable")
    _check(lib().aes_host_batch(scheds.ctypes.data, scheds.size, inp.ctypes.data,
                                out.ctypes.data, inp.size, reqs.ctypes.data, reqs.size,
                                n_threads), "aes_host_batch")


def tune_key(ctx: Context, reqs: np.ndarray, n_scheds: int) -> str:
    """aes_tune_key: the tune cache's signature of a batch."""
    reqs = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
    n = ctypes.c_size_t(0)
    lib().aes_tune_key(ctx.handle, reqs.ctypes.data, reqs.size, n_scheds, None, 0,
                       ctypes.byref(n))
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(lib().aes_tune_key(ctx.handle, reqs.ctypes.data, reqs.size, n_scheds, buf,
                              n.value + 1, None), "aes_tune_key")
    return buf.value.decode()


def request_launch(ctx: Context, d_scheds, d_in, d_out, req, buf_bytes: int | None = None,
                   n_scheds: int | None = None, stream=None):
    """aes_request_launch for one REQ_DTYPE record."""
    r = np.ascontiguousarray(np.asarray(req, dtype=REQ_DTYPE).reshape(1))
    bb = _nbytes(d_in) if buf_bytes is None else buf_bytes
    _check(lib().aes_request_launch(ctx.handle, _ptr(d_scheds), _sched_count(d_scheds, n_scheds),
                                    _ptr(d_in), _ptr(d_out), bb, r.ctypes.data, _stream(stream)),
           "aes_request_launch")


def request_launches(ctx: Context, d_scheds, d_in, d_out, reqs: np.ndarray,
                     buf_bytes: int | None = None, n_scheds: int | None = None, stream=None):
    """aes_request_launches: one kernel launch per request, issued from C."""
    reqs = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
    bb = _nbytes(d_in) if buf_bytes is None else buf_bytes
    _check(lib().aes_request_launches(ctx.handle, _ptr(d_scheds), _sched_count(d_scheds, n_scheds),
                                      _ptr(d_in), _ptr(d_out), bb, reqs.ctypes.data, reqs.size,
                                      _stream(stream)), "aes_request_launches")


class Graph:
    """An instantiated HIP graph: aes_plan_graph / aes_requests_graph, launch, destroy."""

    def __init__(self, handle, keep=()):
        self.handle = handle
        self._keep = keep

    @classmethod
    def of_plan(cls, plan: Plan, d_scheds, d_in, d_out):
        h = ctypes.c_void_p()
        _check(lib().aes_plan_graph(plan.handle, _ptr(d_scheds), _ptr(d_in), _ptr(d_out),
                                    ctypes.byref(h)), "aes_plan_graph")
        return cls(h.value, (plan,))

    @classmethod
    def of_requests(cls, ctx: Context, d_scheds, d_in, d_out, reqs: np.ndarray,
                    buf_bytes: int | None = None, n_scheds: int | None = None):
        reqs = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
        h = ctypes.c_void_p()
        bb = _nbytes(d_in) if buf_bytes is None else buf_bytes
        _check(lib().aes_requests_graph(ctx.handle, _ptr(d_scheds),
                                        _sched_count(d_scheds, n_scheds), _ptr(d_in),
                                        _ptr(d_out), bb, reqs.ctypes.data, reqs.size,
                                        ctypes.byref(h)), "aes_requests_graph")
        return cls(h.value, (ctx,))

    def launch(self, stream=None):
        _check(lib().aes_graph_launch(self.handle, _stream(stream)), "aes_graph_launch")

    def close(self):
        if self.handle:
            lib().aes_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ serving


def host_route_crypt(sched, op: int, iv, src: np.ndarray, dst: np.ndarray = None) -> np.ndarray:
    """aes_host_route_crypt: one request on the host route (the CPU side of
    size-based dispatch) with a host schedule; dst defaults to a new array,
    and may be src itself (in place)."""
    L = lib()
    f = L.aes_host_route_crypt
    f.restype = ctypes.c_int
    f.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.c_uint64]
    sc = np.ascontiguousarray(np.asarray(sched, dtype=SCHED_DTYPE).reshape(1))
    src = np.ascontiguousarray(src, dtype=np.uint8)
    if dst is None:
        dst = np.empty_like(src)
    ivb = None if iv is None else np.ascontiguousarray(np.frombuffer(bytes(iv), np.uint8))
    _check(f(sc.ctypes.data, op, None if ivb is None else ivb.ctypes.data, src.ctypes.data,
             dst.ctypes.data, src.size), "aes_host_route_crypt")
    return dst


AES_SERVE_PERSISTENT = 0
AES_SERVE_PER_LAUNCH = 1
AES_XFER_COPY = 0
AES_XFER_DIRECT = 1

SERVER_CONFIG_DTYPE = np.dtype([("mode", "<u4"), ("ring_slots", "<u4"), ("key_slots", "<u4"),
                                ("n_workgroups", "<u4"), ("dec_workgroups", "<u4"),
                                ("n_streams", "<u4"), ("queue_units", "<u4"),
                                ("idle_timeout_ms", "<u4"), ("hbm_cap_bytes", "<u8"),
                                ("max_request_bytes", "<u8"), ("host_xfer", "<u4"),
                                ("reserved", "<u4", (7,))])
DONE_DTYPE = np.dtype([("ticket", "<u8"), ("status", "<i4"), ("units", "<u4"),
                       ("t_submit_ns", "<u8"), ("t_done_ns", "<u8"),
                       ("gpu_dispatch_ticks", "<u8"), ("gpu_done_ticks", "<u8")])
STATS_NAMES = ("submitted", "completed", "rejected_again", "fallbacks", "kernel_launches",
               "in_flight", "in_flight_bytes", "host_routed")
assert SERVER_CONFIG_DTYPE.itemsize == 80 and DONE_DTYPE.itemsize == 48

DONE_CB = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_servers = None


def _server_sig():
    L = lib()
    p = ctypes.c_void_p
    u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    for name, res, args in (
            ("aes_server_create", i32, [p, p, ctypes.POINTER(p)]),
            ("aes_server_set_key", i32, [p, u32, p]),
            ("aes_server_submit", i32, [p, u32, u32, p, p, p, u64, p, p, ctypes.POINTER(u64)]),
            ("aes_server_poll", i32, [p, p, u32, ctypes.POINTER(u32)]),
            ("aes_server_wait", i32, [p, u64, u64, p]),
            ("aes_server_replay", i32, [p, p, p, u64, p, p, p]),
            ("aes_server_stats", i32, [p, p]),
            ("aes_server_host_alloc", i32, [p, u64, ctypes.POINTER(p)]),
            ("aes_server_host_free", i32, [p, p]),
            ("aes_server_set_crossover", i32, [p, u32, u64]),
            ("aes_server_get_crossover", i32, [p, u32, ctypes.POINTER(u64)]),
            ("aes_server_calibrate", i32, [p, u32, p]),
            ("aes_server_destroy", i32, [p])):
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


class Server:
    """aes_server_*: persistent-kernel (mode 0) or per-request-launch (mode 1) serving.

    Keyword arguments set aes_server_config_t fields (0 = library default).
    Always close() a server (or use it as a context manager): a persistent
    kernel otherwise keeps running until its idle timeout.
    """

    def __init__(self, ctx: Context, **cfg):
        global _servers
        L = _server_sig()
        c = np.zeros(1, SERVER_CONFIG_DTYPE)
        for k, v in cfg.items():
            c[0][k] = v
        h = ctypes.c_void_p()
        _check(L.aes_server_create(ctx.handle, c.ctypes.data, ctypes.byref(h)),
               "aes_server_create")
        self.handle = h.value
        self.ctx = ctx
        self._cbs = {}
        self._host = {}  # host buffer address -> nbytes
        if _servers is None:
            import atexit
            import weakref
            _servers = weakref.WeakSet()
            atexit.register(lambda: [s.close() for s in list(_servers)])
        _servers.add(self)

    def set_key(self, slot: int, sched):
        s = np.ascontiguousarray(np.asarray(sched, dtype=SCHED_DTYPE).reshape(1))
        _check(lib().aes_server_set_key(self.handle, slot, s.ctypes.data), "aes_server_set_key")

    def submit(self, op: int, key_slot: int, iv, d_src, d_dst, length: int, callback=None):
        """Posts a request; returns its ticket.  Raises AesError (status
        AES_ERR_AGAIN when admission refuses).  callback(done_record) runs on
        the library's completion thread."""
        ivb = None if iv is None else np.ascontiguousarray(
            np.frombuffer(bytes(iv), np.uint8) if not isinstance(iv, np.ndarray) else iv,
            dtype=np.uint8)
        t = ctypes.c_uint64()
        cb = None
        if callback is not None:
            def _tramp(done_ptr, _user, _f=callback):
                rec = np.frombuffer(ctypes.string_at(done_ptr, DONE_DTYPE.itemsize),
                                    DONE_DTYPE)[0]
                _f(rec)
            cb = DONE_CB(_tramp)
        st = lib().aes_server_submit(self.handle, op, key_slot,
                                     None if ivb is None else ivb.ctypes.data, _ptr(d_src),
                                     _ptr(d_dst), length,
                                     ctypes.cast(cb, ctypes.c_void_p) if cb else None, None,
                                     ctypes.byref(t))
        _check(st, "aes_server_submit")
        if cb is not None:
            self._cbs[t.value] = cb  # keep the trampoline alive
        return t.value

    def wait(self, ticket: int, timeout_s: float = 30.0):
        out = np.zeros(1, DONE_DTYPE)
        _check(lib().aes_server_wait(self.handle, ticket, int(timeout_s * 1e9), out.ctypes.data),
               "aes_server_wait")
        return out[0]

    def poll(self, max_n: int = 1024) -> np.ndarray:
        out = np.zeros(max_n, DONE_DTYPE)
        n = ctypes.c_uint32()
        _check(lib().aes_server_poll(self.handle, out.ctypes.data, max_n, ctypes.byref(n)),
               "aes_server_poll")
        return out[: n.value]

    def replay(self, reqs: np.ndarray, arrival_s: np.ndarray, d_src_base, d_dst_base):
        reqs = np.ascontiguousarray(reqs, dtype=REQ_DTYPE)
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
        out = np.zeros(reqs.size, DONE_DTYPE)
        _check(lib().aes_server_replay(self.handle, reqs.ctypes.data, arr.ctypes.data, reqs.size,
                                       _ptr(d_src_base), _ptr(d_dst_base), out.ctypes.data),
               "aes_server_replay")
        return out

    def host_alloc(self, nbytes: int) -> np.ndarray:
        """Pinned host buffer mapped into the device (aes_server_host_alloc),
        as a uint8 numpy array over the library's memory.  Pass it (or
        slices of it) to submit/replay; it lives until host_free or close."""
        h = ctypes.c_void_p()
        _check(lib().aes_server_host_alloc(self.handle, nbytes, ctypes.byref(h)),
               "aes_server_host_alloc")
        self._host[h.value] = nbytes
        return np.ctypeslib.as_array((ctypes.c_uint8 * nbytes).from_address(h.value))

    def host_free(self, buf):
        addr = _ptr(buf)
        _check(lib().aes_server_host_free(self.handle, addr), "aes_server_host_free")
        self._host.pop(addr, None)

    def set_crossover(self, op: int, nbytes: int):
        """Size-based dispatch: requests of op shorter than nbytes whose
        payloads both lie in host buffers of this server run on the host
        route (0 = never; 2**64 - 1 = always)."""
        _check(lib().aes_server_set_crossover(self.handle, op, nbytes), "aes_server_set_crossover")

    def get_crossover(self, op: int) -> int:
        v = ctypes.c_uint64()
        _check(lib().aes_server_get_crossover(self.handle, op, ctypes.byref(v)),
               "aes_server_get_crossover")
        return v.value

    def calibrate(self, key_slot: int = 0) -> np.ndarray:
        """Measures and sets the five crossovers (aes_server_calibrate); returns them by op."""
        out = np.zeros(5, np.uint64)
        _check(lib().aes_server_calibrate(self.handle, key_slot, out.ctypes.data),
               "aes_server_calibrate")
        return out

    def stats(self) -> dict:
        out = np.zeros(len(STATS_NAMES), np.uint64)
        _check(lib().aes_server_stats(self.handle, out.ctypes.data), "aes_server_stats")
        return dict(zip(STATS_NAMES, (int(v) for v in out)))

    def close(self):
        if getattr(self, "handle", None):
            st = lib().aes_server_destroy(self.handle)
            self.handle = None
            self._cbs.clear()
            self._host.clear()
            _check(st, "aes_server_destroy")

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
