"""Pins of the CPU oracle against facts outside itself (no GPU needed).

* An independent implementation: the system OpenSSL (EVP ECB/CBC/CTR) on
  random keys of all three sizes, random blocks, IVs and lengths.
* Published properties of the Rijndael S-box (FIPS-197 5.1.1 and the design
  rationale): a permutation with S(0x00) = 0x63, no fixed points and no
  complemented fixed points, differential uniformity 4, nonlinearity 112.
* Mode identities of SP 800-38A: one-block CBC equals E(P xor IV), CBC
  decryption equals the block-parallel form D(C_j) xor C_(j-1), CTR is an
  involution and its keystream is E(T_1) || E(T_2) || ..., and the 64-bit
  counter wraps without touching the nonce half.
* ECB requests (ops 3 and 4) against OpenSSL's EVP ECB, block-position
  independence, whole-block lengths.
* Batch semantics: bytes outside every request keep their sentinel value and
  each request equals the same request run alone.
"""
import hashlib

import numpy as np
import pytest

import oracle
from synth import gen, workloads
from tests import openssl_ref

pytestmark = pytest.mark.skipif(not openssl_ref.available(), reason="libcrypto not found")

KEY_BITS = (128, 192, 256)


def rng(seed):
    return np.random.default_rng(seed)


# ----------------------------------------------------------------- S-box pins

def test_sbox_permutation_and_fixed_points():
    s, si = oracle.sbox()
    assert sorted(s.tolist()) == list(range(256))
    assert s[0] == 0x63
    assert all(si[s[x]] == x for x in range(256))
    assert all(s[x] != x for x in range(256)), "Rijndael S-box has no fixed points"
    assert all(s[x] != (x ^ 0xFF) for x in range(256)), "no complemented fixed points"


def test_sbox_differential_uniformity_and_nonlinearity():
    s, _ = oracle.sbox()
    s = s.astype(np.int64)
    x = np.arange(256)
    # difference distribution table: max over a != 0 of #{x : S(x) ^ S(x ^ a) = b}
    du = 0
    for a in range(1, 256):
        counts = np.bincount(s ^ s[x ^ a], minlength=256)
        du = max(du, counts.max())
    assert du == 4
    # nonlinearity = 128 - max |Walsh| / 2 over non-zero output masks
    parity = np.array([bin(v).count("1") & 1 for v in range(256)])
    sign = 1 - 2 * parity
    best = 0
    for b in range(1, 256):
        f = sign[s & b]
        # fast Walsh-Hadamard transform of (-1)^(b.S(x))
        w = f.astype(np.int64).copy()
        h = 1
        while h < 256:
            w = w.reshape(-1, 2, h)
            w = np.stack([w[:, 0] + w[:, 1], w[:, 0] - w[:, 1]], axis=1).reshape(-1)
            h *= 2
        best = max(best, int(np.abs(w).max()))
    assert 128 - best // 2 == 112


# --------------------------------------------------------- OpenSSL cross-check

@pytest.mark.parametrize("bits", KEY_BITS)
def test_ecb_matches_openssl(bits):
    r = rng(bits)
    for _ in range(8):
        key = r.integers(0, 256, 32, dtype=np.uint8)
        data = r.integers(0, 256, 16 * 37, dtype=np.uint8)
        ours = oracle.ecb(key[: bits // 8], bits, data)
        ref = openssl_ref.ecb(bits, key, data)
        assert np.array_equal(ours, ref)
        back = oracle.ecb(key[: bits // 8], bits, ours, decrypt=True)
        assert np.array_equal(back, data)
        assert np.array_equal(openssl_ref.ecb(bits, key, ours, decrypt=True), data)


@pytest.mark.parametrize("bits", KEY_BITS)
def test_ecb_mode_requests_match_openssl(bits):
    """The ECB request ops (3 = encrypt, 4 = decrypt) of the mode and batch
    entry points, against OpenSSL's EVP ECB (SP 800-38A 6.1)."""
    r = rng(50 + bits)
    for nblk in (0, 1, 3, 256, 1000):
        key = r.integers(0, 256, 32, dtype=np.uint8)
        data = r.integers(0, 256, 16 * nblk, dtype=np.uint8)
        enc = oracle.mode(oracle.OP_ECB_ENC, key[: bits // 8], bits, None, data)
        assert np.array_equal(enc, openssl_ref.ecb(bits, key, data))
        dec = oracle.mode(oracle.OP_ECB_DEC, key[: bits // 8], bits, None, enc)
        assert np.array_equal(dec, data)
        # each block on its own: moving a block moves its ciphertext
        if nblk >= 3:
            sw = data.reshape(-1, 16)[[2, 0, 1] + list(range(3, nblk))].reshape(-1)
            enc2 = oracle.mode(oracle.OP_ECB_ENC, key[: bits // 8], bits, None, sw)
            assert np.array_equal(enc2.reshape(-1, 16)[:3], enc.reshape(-1, 16)[[2, 0, 1]])
    with pytest.raises(oracle.OracleError):
        oracle.mode(oracle.OP_ECB_ENC, np.zeros(16, np.uint8), 128, None, np.zeros(20, np.uint8))


@pytest.mark.parametrize("bits", KEY_BITS)
def test_cbc_matches_openssl(bits):
    r = rng(100 + bits)
    for nblk in (0, 1, 2, 7, 64, 257):
        key = r.integers(0, 256, 32, dtype=np.uint8)
        iv = r.integers(0, 256, 16, dtype=np.uint8)
        data = r.integers(0, 256, 16 * nblk, dtype=np.uint8)
        enc = oracle.cbc_encrypt(key, bits, iv, data)
        assert np.array_equal(enc, openssl_ref.cbc(bits, key, iv, data))
        dec = oracle.cbc_decrypt(key, bits, iv, data)
        assert np.array_equal(dec, openssl_ref.cbc(bits, key, iv, data, decrypt=True))


@pytest.mark.parametrize("bits", KEY_BITS)
def test_ctr_matches_openssl_without_wrap(bits):
    r = rng(200 + bits)
    for n in (0, 1, 15, 16, 17, 100, 4096, 4096 + 5):
        key = r.integers(0, 256, 32, dtype=np.uint8)
        t1 = r.integers(0, 256, 16, dtype=np.uint8)
        t1[8] &= 0x7F  # low 64 bits far from 2^64: the 128-bit and 64-bit counters agree
        data = r.integers(0, 256, n, dtype=np.uint8)
        ours = oracle.ctr(key, bits, t1, data)
        assert np.array_equal(ours, openssl_ref.ctr(bits, key, t1, data))


# ------------------------------------------------------------- mode identities

@pytest.mark.parametrize("bits", KEY_BITS)
def test_one_block_cbc_is_cipher_of_p_xor_iv(bits):
    r = rng(300 + bits)
    key = r.integers(0, 256, 32, dtype=np.uint8)
    iv = r.integers(0, 256, 16, dtype=np.uint8)
    p = r.integers(0, 256, 16, dtype=np.uint8)
    assert np.array_equal(oracle.cbc_encrypt(key, bits, iv, p),
                          oracle.ecb(key[: bits // 8], bits, p ^ iv))


@pytest.mark.parametrize("bits", KEY_BITS)
def test_cbc_decrypt_equals_block_parallel_form(bits):
    r = rng(400 + bits)
    key = r.integers(0, 256, 32, dtype=np.uint8)
    iv = r.integers(0, 256, 16, dtype=np.uint8)
    c = r.integers(0, 256, 16 * 50, dtype=np.uint8)
    d = oracle.ecb(key[: bits // 8], bits, c, decrypt=True)
    prev = np.concatenate([iv, c[:-16]])
    assert np.array_equal(oracle.cbc_decrypt(key, bits, iv, c), d ^ prev)
    p = r.integers(0, 256, 16 * 50, dtype=np.uint8)
    assert np.array_equal(oracle.cbc_decrypt(key, bits, iv, oracle.cbc_encrypt(key, bits, iv, p)), p)


@pytest.mark.parametrize("bits", KEY_BITS)
def test_ctr_involution_and_keystream(bits):
    r = rng(500 + bits)
    key = r.integers(0, 256, 32, dtype=np.uint8)
    t1 = r.integers(0, 256, 16, dtype=np.uint8)
    p = r.integers(0, 256, 16 * 9 + 3, dtype=np.uint8)
    c = oracle.ctr(key, bits, t1, p)
    assert np.array_equal(oracle.ctr(key, bits, t1, c), p)
    ks = oracle.ctr(key, bits, t1, np.zeros(16 * 9 + 3, np.uint8))
    low = int.from_bytes(t1[8:].tobytes(), "big")
    blocks = []
    for j in range(10):
        t = t1.copy()
        t[8:] = np.frombuffer(((low + j) % (1 << 64)).to_bytes(8, "big"), np.uint8)
        blocks.append(t)
    want = oracle.ecb(key[: bits // 8], bits, np.concatenate(blocks))[: ks.size]
    assert np.array_equal(ks, want)


@pytest.mark.parametrize("bits", KEY_BITS)
def test_ctr_64bit_counter_wraps_without_carry_into_nonce(bits):
    # The counter is the low 64 bits, incremented mod 2^64 (the reading of SP
    # 800-38A B.1 with m = 64); the nonce half never changes.
    r = rng(600 + bits)
    key = r.integers(0, 256, 32, dtype=np.uint8)
    t1 = r.integers(0, 256, 16, dtype=np.uint8)
    t1[8:] = np.frombuffer(((1 << 64) - 2).to_bytes(8, "big"), np.uint8)
    ks = oracle.ctr(key, bits, t1, np.zeros(64, np.uint8))
    want = []
    for low in ((1 << 64) - 2, (1 << 64) - 1, 0, 1):
        t = t1.copy()
        t[8:] = np.frombuffer(low.to_bytes(8, "big"), np.uint8)
        want.append(oracle.ecb(key[: bits // 8], bits, t))
    assert np.array_equal(ks, np.concatenate(want))
    # and it differs from a 128-bit counter, which would carry into the nonce
    assert not np.array_equal(ks, openssl_ref.ctr(bits, key, t1, np.zeros(64, np.uint8)))


def test_key_expansion_prefix_and_sizes():
    r = rng(700)
    for bits, nr in ((128, 10), (192, 12), (256, 14)):
        key = r.integers(0, 256, bits // 8, dtype=np.uint8)
        w = oracle.expand_key(key, bits)
        assert w.shape == (4 * (nr + 1), 4)
        assert np.array_equal(w[: bits // 32].reshape(-1), key)
    with pytest.raises(oracle.OracleError):
        oracle.expand_key(np.zeros(16, np.uint8), 100)


def test_cbc_rejects_partial_blocks():
    with pytest.raises(oracle.OracleError):
        oracle.cbc_encrypt(np.zeros(16, np.uint8), 128, np.zeros(16, np.uint8),
                           np.zeros(17, np.uint8))


# --------------------------------------------------------------- batch driver

def _batch_expect_alone(wl, inp):
    out = workloads.sentinel(inp.size)
    for r in wl.reqs:
        o, n = int(r["offset"]), int(r["length"])
        kb = int(wl.key_bits[r["key_idx"]])
        out[o:o + n] = oracle.mode(int(r["op"]), wl.keys[r["key_idx"]][: kb // 8], kb,
                                   r["iv"], inp[o:o + n])
    return out


def test_batch_matches_requests_alone_and_keeps_sentinels():
    wl = workloads.config3(n_reqs=40, max_pages=4)
    wl.reqs["op"][::7] = oracle.OP_ECB_ENC
    wl.reqs["op"][3::7] = oracle.OP_ECB_DEC
    # open gaps between requests so that untouched bytes exist
    wl.reqs["offset"] = wl.reqs["offset"] + np.arange(wl.reqs.size, dtype=np.uint64) * 48
    wl.reqs["length"][::3] -= 16
    ctr = wl.reqs["op"] == workloads.OP_CTR
    wl.reqs["length"][ctr] -= 5  # CTR takes any length
    buf = int(wl.reqs["offset"][-1] + wl.reqs["length"][-1]) + 64
    inp = gen.bytes_(0, gen.STREAM_DATA, buf)
    want = _batch_expect_alone(wl, inp)
    for threads in (1, 3, 0):
        out = workloads.sentinel(buf)
        oracle.batch(inp, out, wl.reqs, wl.keys, wl.key_bits, n_threads=threads)
        assert np.array_equal(out, want)


def test_batch_validation_errors():
    wl = workloads.pages(4, workloads.OP_CBC_DEC, 128)
    inp = np.zeros(wl.buf_bytes, np.uint8)
    out = np.zeros_like(inp)
    bad = wl.reqs.copy()
    bad["length"][1] = 17
    with pytest.raises(oracle.OracleError):
        oracle.batch(inp, out, bad, wl.keys, wl.key_bits)
    bad = wl.reqs.copy()
    bad["offset"][3] = wl.buf_bytes
    with pytest.raises(oracle.OracleError):
        oracle.batch(inp, out, bad, wl.keys, wl.key_bits)
    bad = wl.reqs.copy()
    bad["key_idx"][0] = 7
    with pytest.raises(oracle.OracleError):
        oracle.batch(inp, out, bad, wl.keys, wl.key_bits)
    bad = wl.reqs.copy()
    bad["op"][2] = 5
    with pytest.raises(oracle.OracleError):
        oracle.batch(inp, out, bad, wl.keys, wl.key_bits)
    bad = wl.reqs.copy()
    bad["op"][2] = oracle.OP_ECB_DEC
    bad["length"][2] = 4008
    with pytest.raises(oracle.OracleError):
        oracle.batch(inp, out, bad, wl.keys, wl.key_bits)
    assert not out.any(), "nothing is written on a validation error"


# ------------------------------------------------------- regression digest

def test_golden_digests():
    """Digests written by tests/golden/make_golden.py (which calls only the
    oracle); a change here means the oracle's arithmetic changed."""
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_digests.json")
    with open(path) as f:
        golden = json.load(f)
    from tests.golden.make_golden import compute
    assert compute() == golden


# ------------------------------------------------------------- the generator

def test_generator_is_seekable_and_matches_torch():
    import torch
    a = gen.bytes_(0, 3, 1000)
    b = gen.bytes_(0, 3, 300, offset=700)
    assert np.array_equal(a[700:], b)
    t = gen.bytes_torch(0, 3, 1024, "cpu").numpy()
    assert np.array_equal(t[:1000], a)
    t2 = gen.bytes_torch(0, 3, 512, "cpu", offset_words=64).numpy()
    assert np.array_equal(t2, gen.bytes_(0, 3, 512, offset=512))
    u = gen.uniform(0, 4, 10000)
    assert 0.0 <= u.min() and u.max() < 1.0 and abs(u.mean() - 0.5) < 0.02


def test_config_shapes():
    wl = workloads.config2(workloads.OP_CTR, 256, n_pages=64)
    assert wl.buf_bytes == 64 * 4096 and (wl.reqs["iv"][:, 8:] == 0).all()
    assert (wl.reqs["key_idx"] == np.arange(64) % 16).all()
    c3 = workloads.config3()
    n = c3.reqs.size
    assert n == 10000
    pg = c3.reqs["length"] // 4096
    assert pg.min() == 1 and pg.max() == 256
    assert 0.2 < (c3.reqs["op"] == workloads.OP_CBC_ENC).mean() < 0.3
    assert set(np.unique(c3.key_bits).tolist()) == {128, 256}
    c5 = workloads.config5_ctr(total_bytes=64 << 20)
    assert c5.reqs.size == 4
    low = c5.reqs["iv"][:, 8:].copy().view(">u8").reshape(-1)
    assert (low == np.arange(4) * (16 << 20) // 16).all()
    tr = workloads.config4(1000.0, 500)
    assert set(np.unique(tr.reqs["length"]).tolist()) <= set((workloads.SERVE_SIZES).tolist())
    assert abs(tr.arrivals_s[-1] / 500 - 1e-3) < 3e-4
    hashlib.sha256(c3.reqs.tobytes()).hexdigest()
