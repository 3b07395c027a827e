"""Seekable counter-based byte generator shared by the tests and the benchmark.

It holds none of the cipher's arithmetic.  Word i of stream (seed, stream) is
the SplitMix64 output function (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) applied to the counter

    x_i = seed * 2^32 + stream + (i + 1) * 0x9E3779B97F4A7C15   (mod 2^64)

with finaliser z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
z *= 0x94D049BB133111EB; z ^= z >> 31.  Bytes are the words in little-endian
order, so byte k of a stream is byte k % 8 of word k // 8 and any range can be
produced without producing what precedes it.  A numpy (host) and a torch
(device) version are given; both compute the same function.
"""
from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

# Stream ids used by every workload.
STREAM_KEYS = 1
STREAM_IVS = 2
STREAM_DATA = 3
STREAM_SIZES = 4
STREAM_OPS = 5
STREAM_KEYPICK = 6
STREAM_ARRIVALS = 7


def _base(seed: int, stream: int) -> int:
    return ((seed << 32) + stream) & MASK64


def words(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """Words start .. start+count-1 of a stream as uint64."""
    if count <= 0:
        return np.zeros(0, np.uint64)
    with np.errstate(over="ignore"):
        i = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
        z = np.uint64(_base(seed, stream)) + i * np.uint64(GAMMA)
        z ^= z >> np.uint64(30)
        z *= np.uint64(M1)
        z ^= z >> np.uint64(27)
        z *= np.uint64(M2)
        z ^= z >> np.uint64(31)
    return z


def bytes_(seed: int, stream: int, nbytes: int, offset: int = 0) -> np.ndarray:
    """nbytes bytes of a stream starting at byte ``offset``, as uint8."""
    if nbytes <= 0:
        return np.zeros(0, np.uint8)
    w0 = offset // 8
    w1 = (offset + nbytes + 7) // 8
    w = words(seed, stream, w0, w1 - w0)
    b = w.astype("<u8").view(np.uint8)
    s = offset - 8 * w0
    return b[s:s + nbytes].copy()


def uniform(seed: int, stream: int, count: int, start: int = 0) -> np.ndarray:
    """count uniform reals in [0, 1): u = (w >> 11) * 2^-53."""
    w = words(seed, stream, start, count)
    return (w >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def bytes_torch(seed: int, stream: int, nbytes: int, device, offset_words: int = 0,
                chunk_words: int = 1 << 24):
    """The same byte stream produced on a torch device (nbytes % 8 == 0).

    torch has no unsigned 64-bit arithmetic, so int64 is used: addition and
    multiplication wrap identically, and logical right shifts are arithmetic
    shifts with the sign-extended bits masked off.
    """
    import torch

    assert nbytes % 8 == 0
    n = nbytes // 8
    out = torch.empty(n, dtype=torch.int64, device=device)

    def s64(v):
        v &= MASK64
        return v - (1 << 64) if v >= 1 << 63 else v

    base = s64(_base(seed, stream))
    gamma = s64(GAMMA)
    m1 = s64(M1)
    m2 = s64(M2)

    def lsr(z, k):
        return (z >> k) & ((1 << (64 - k)) - 1)

    for c0 in range(0, n, chunk_words):
        c1 = min(n, c0 + chunk_words)
        i = torch.arange(offset_words + c0 + 1, offset_words + c1 + 1, dtype=torch.int64,
                         device=device)
        z = i * gamma + base
        z = z ^ lsr(z, 30)
        z = z * m1
        z = z ^ lsr(z, 27)
        z = z * m2
        z = z ^ lsr(z, 31)
        out[c0:c1] = z
    return out.view(torch.uint8)
