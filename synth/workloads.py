"""Seeded synthetic workloads: request lists, keys, IVs and payload bytes.

This module holds no cipher arithmetic.  It only draws numbers from the
SplitMix64 streams of ``synth.gen`` and lays them out as request records.
The same records feed the GPU library and the CPU oracle.

The paper (section 3.3) runs its AES service over per-page buffers (it names
encrypted filesystems and page-sized work) and sweeps the data size; it
prints no data.  Every workload here is therefore uniform random bytes with
the shapes below.

Request record (REQ_DTYPE): offset and length in bytes (the same offset in
the input and the output buffer), key index, op (0 CBC encrypt, 1 CBC
decrypt, 2 CTR) and a 16-byte IV (CBC) or initial counter block (CTR).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import gen

OP_CBC_ENC = 0
OP_CBC_DEC = 1
OP_CTR = 2
OP_NAMES = {OP_CBC_ENC: "cbc_enc", OP_CBC_DEC: "cbc_dec", OP_CTR: "ctr"}

PAGE = 4096

REQ_DTYPE = np.dtype([("offset", "<u8"), ("length", "<u8"), ("key_idx", "<u4"),
                      ("op", "<u4"), ("iv", "u1", (16,))])


@dataclass
class Workload:
    """A batch: requests over one buffer, with the keys they index."""
    name: str
    reqs: np.ndarray                 # REQ_DTYPE
    keys: np.ndarray                 # (n_keys, 32) uint8; first key_bits/8 bytes used
    key_bits: np.ndarray             # (n_keys,) uint32
    buf_bytes: int
    seed: int = 0
    labels: dict = field(default_factory=dict)

    def payload_bytes(self) -> int:
        return int(self.reqs["length"].sum())

    def data(self) -> np.ndarray:
        """The input buffer: uniform random bytes of stream 3."""
        return gen.bytes_(self.seed, gen.STREAM_DATA, self.buf_bytes)


def make_keys(seed: int, n: int, bits) -> tuple[np.ndarray, np.ndarray]:
    """n keys from stream 1 (32 bytes drawn per key) with the given sizes."""
    keys = gen.bytes_(seed, gen.STREAM_KEYS, 32 * n).reshape(n, 32)
    kb = np.broadcast_to(np.asarray(bits, dtype=np.uint32), (n,)).copy()
    return keys, kb


def pages(n_pages: int, op: int, key_bits: int, n_keys: int = 1, page: int = PAGE,
          seed: int = 0, ctr_low_zero: bool = True, name: str = "pages") -> Workload:
    """n_pages independent pages back to back; page p uses key p mod n_keys.

    CBC: a random 16-byte IV per page.  CTR: a random 8-byte nonce per page and
    a 64-bit counter starting at 0 (or random when ctr_low_zero is False).
    """
    keys, kb = make_keys(seed, n_keys, key_bits)
    reqs = np.zeros(n_pages, REQ_DTYPE)
    reqs["offset"] = np.arange(n_pages, dtype=np.uint64) * np.uint64(page)
    reqs["length"] = page
    reqs["key_idx"] = np.arange(n_pages, dtype=np.uint32) % np.uint32(n_keys)
    reqs["op"] = op
    ivs = gen.bytes_(seed, gen.STREAM_IVS, 16 * n_pages).reshape(n_pages, 16)
    if op == OP_CTR and ctr_low_zero:
        ivs[:, 8:] = 0
    reqs["iv"] = ivs
    return Workload(name, reqs, keys, kb, n_pages * page, seed)


def config1(seed: int = 0, n_pages: int = 256) -> tuple[Workload, Workload]:
    """AES-128-CBC encrypt then decrypt of 256 independent 4 KiB pages, one key,
    per-page random IVs.  Returns (encrypt workload, decrypt workload)."""
    enc = pages(n_pages, OP_CBC_ENC, 128, 1, seed=seed, name="cfg1_cbc_enc")
    dec = pages(n_pages, OP_CBC_DEC, 128, 1, seed=seed, name="cfg1_cbc_dec")
    return enc, dec


def config2(op: int, key_bits: int, seed: int = 0, n_pages: int = 65536) -> Workload:
    """65,536 pages of 4 KiB (256 MiB), 16 keys round-robin, CBC-decrypt or CTR
    (64-bit counter per page starting at 0, random nonce)."""
    return pages(n_pages, op, key_bits, 16, seed=seed,
                 name=f"cfg2_{OP_NAMES[op]}_{key_bits}")


def config3(seed: int = 0, n_reqs: int = 10000, max_pages: int = 256,
            n_pool: int = 64) -> Workload:
    """Uneven batch: sizes log-uniform from 4 KiB to max_pages*4 KiB in 4 KiB
    multiples (pages = round(max_pages^u)), op drawn as mode x direction
    50/50 each, a pool of n_pool keys each 128 or 256 bits (50/50), each
    request picking a pool key uniformly; requests packed back to back."""
    u = gen.uniform(seed, gen.STREAM_SIZES, n_reqs)
    npg = np.rint(np.power(float(max_pages), u)).astype(np.uint64)
    npg = np.clip(npg, 1, max_pages)
    lengths = npg * np.uint64(PAGE)
    offsets = np.zeros(n_reqs, np.uint64)
    if n_reqs > 1:
        offsets[1:] = np.cumsum(lengths)[:-1]
    ou = gen.uniform(seed, gen.STREAM_OPS, 2 * n_reqs).reshape(n_reqs, 2)
    is_ctr = ou[:, 0] >= 0.5
    is_dec = ou[:, 1] >= 0.5
    op = np.where(is_ctr, OP_CTR, np.where(is_dec, OP_CBC_DEC, OP_CBC_ENC)).astype(np.uint32)
    ku = gen.uniform(seed, gen.STREAM_KEYPICK, n_pool + n_reqs)
    pool_bits = np.where(ku[:n_pool] < 0.5, 128, 256).astype(np.uint32)
    keys, kb = make_keys(seed, n_pool, pool_bits)
    pick = np.minimum((ku[n_pool:] * n_pool).astype(np.uint32), n_pool - 1)
    reqs = np.zeros(n_reqs, REQ_DTYPE)
    reqs["offset"] = offsets
    reqs["length"] = lengths
    reqs["key_idx"] = pick
    reqs["op"] = op
    reqs["iv"] = gen.bytes_(seed, gen.STREAM_IVS, 16 * n_reqs).reshape(n_reqs, 16)
    wl = Workload("cfg3_mixed", reqs, keys, kb, int(lengths.sum()), seed)
    wl.labels["direction_dec"] = is_dec
    return wl


SERVE_SIZES = np.array([4, 8, 16, 32, 64], dtype=np.uint64) * 1024


@dataclass
class ServeTrace:
    """Serving requests: op, key slot, IV, size, source offset and arrival time."""
    reqs: np.ndarray          # REQ_DTYPE (offset into the staged payload buffer)
    arrivals_s: np.ndarray    # float64 seconds from the start
    keys: np.ndarray
    key_bits: np.ndarray
    buf_bytes: int
    rate: float


def config4(rate_per_s: float, n_reqs: int, seed: int = 0, n_slots: int = 256,
            start: int = 0) -> ServeTrace:
    """Poisson arrivals at rate_per_s; sizes uniform in {4,8,16,32,64} KiB;
    AES-128-CBC, encrypt/decrypt 50/50; keys from n_slots resident slots.
    ``start`` skips that many requests of the streams (warm-up vs measured)."""
    su = gen.uniform(seed, gen.STREAM_SIZES, n_reqs, start=start)
    sizes = SERVE_SIZES[np.minimum((su * 5).astype(np.int64), 4)]
    ou = gen.uniform(seed, gen.STREAM_OPS, n_reqs, start=start)
    op = np.where(ou < 0.5, OP_CBC_ENC, OP_CBC_DEC).astype(np.uint32)
    ku = gen.uniform(seed, gen.STREAM_KEYPICK, n_reqs, start=start)
    slot = np.minimum((ku * n_slots).astype(np.uint32), n_slots - 1)
    au = gen.uniform(seed, gen.STREAM_ARRIVALS, n_reqs, start=start)
    gaps = -np.log1p(-au) / float(rate_per_s)
    arrivals = np.cumsum(gaps)
    offsets = np.zeros(n_reqs, np.uint64)
    if n_reqs > 1:
        offsets[1:] = np.cumsum(sizes)[:-1]
    reqs = np.zeros(n_reqs, REQ_DTYPE)
    reqs["offset"] = offsets
    reqs["length"] = sizes
    reqs["key_idx"] = slot
    reqs["op"] = op
    reqs["iv"] = gen.bytes_(seed, gen.STREAM_IVS, 16 * n_reqs, offset=16 * start).reshape(
        n_reqs, 16)
    keys, kb = make_keys(seed, n_slots, 128)
    return ServeTrace(reqs, arrivals, keys, kb, int(sizes.sum()), rate_per_s)


def config5_ctr(seed: int = 0, total_bytes: int = 8 << 30, chunk: int = 16 << 20) -> Workload:
    """AES-256-CTR over total_bytes in chunk-sized requests of one continuous
    counter stream: chunk c starts at counter c * chunk / 16 with one nonce."""
    n = total_bytes // chunk
    keys, kb = make_keys(seed, 1, 256)
    nonce = gen.bytes_(seed, gen.STREAM_IVS, 8)
    reqs = np.zeros(n, REQ_DTYPE)
    reqs["offset"] = np.arange(n, dtype=np.uint64) * np.uint64(chunk)
    reqs["length"] = chunk
    reqs["key_idx"] = 0
    reqs["op"] = OP_CTR
    iv = np.zeros((n, 16), np.uint8)
    iv[:, :8] = nonce
    ctr0 = np.arange(n, dtype=np.uint64) * np.uint64(chunk // 16)
    iv[:, 8:] = ctr0.astype(">u8").view(np.uint8).reshape(n, 8)
    reqs["iv"] = iv
    return Workload("cfg5_ctr256", reqs, keys, kb, n * chunk, seed)


def config5_cbc(seed: int = 0, n_chains: int = 4096, chain: int = 1 << 20) -> Workload:
    """AES-256-CBC encrypt of n_chains independent chains of ``chain`` bytes."""
    keys, kb = make_keys(seed, 1, 256)
    reqs = np.zeros(n_chains, REQ_DTYPE)
    reqs["offset"] = np.arange(n_chains, dtype=np.uint64) * np.uint64(chain)
    reqs["length"] = chain
    reqs["key_idx"] = 0
    reqs["op"] = OP_CBC_ENC
    reqs["iv"] = gen.bytes_(seed, gen.STREAM_IVS, 16 * n_chains).reshape(n_chains, 16)
    return Workload("cfg5_cbcenc256", reqs, keys, kb, n_chains * chain, seed)


def sentinel(nbytes: int) -> np.ndarray:
    """Fill pattern for output buffers: bytes outside every request must keep it."""
    return (np.arange(nbytes, dtype=np.uint64) * np.uint64(151) + np.uint64(7)).astype(np.uint8)


def log_uniform_pages(u: np.ndarray, max_pages: int) -> np.ndarray:
    return np.clip(np.rint(np.power(float(max_pages), u)), 1, max_pages).astype(np.uint64)


def expected_config3_bytes(n_reqs: int = 10000, max_pages: int = 256) -> float:
    """Mean request size in bytes of the log-uniform size law (for reporting)."""
    return PAGE * (max_pages - 1) / math.log(max_pages)
