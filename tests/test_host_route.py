"""The host route of size-based dispatch (aes_host_route_crypt, AES-NI on the
calling core) against the oracle, byte for byte, on the CPU.

Cases: every op and key size; lengths that exercise the eight-block groups
and the single-block remainder (1, 7, 8, 9, 17 and 256 blocks), CTR tails of
1..15 bytes, counters that wrap modulo 2^64 inside a request, in-place runs
of every op, zero length, and the argument errors."""
import os

import numpy as np
import pytest

import oracle
from synth import gen, workloads

OPS = (0, 1, 2, 3, 4)  # CBC-enc, CBC-dec, CTR, ECB-enc, ECB-dec


@pytest.fixture(scope="module")
def ag():
    from paper_1305_3345_amd import aesgpu
    if not os.path.exists(aesgpu.LIB_PATH):
        from paper_1305_3345_amd import build
        build.build()
    return aesgpu


def case(bits, seed):
    keys, kb = workloads.make_keys(seed, 1, bits)
    return keys[0][: bits // 8], int(kb[0])


@pytest.mark.parametrize("bits", [128, 192, 256])
@pytest.mark.parametrize("op", OPS)
def test_matches_oracle(ag, op, bits):
    key, kb = case(bits, bits + op)
    sched = ag.expand_key(key, kb)
    lengths = [16, 112, 128, 144, 272, 4096]
    if op == 2:
        lengths += [1, 15, 4096 + 7, 129]
    for i, n in enumerate(lengths):
        src = gen.bytes_(i, gen.STREAM_DATA, n)
        iv = gen.bytes_(i, gen.STREAM_IVS, 16)
        got = ag.host_route_crypt(sched, op, iv, src)
        want = oracle.mode(op, key, kb, iv, src)
        assert np.array_equal(got, want), f"op {op} bits {bits} length {n}"


def test_ctr_counter_wraps_in_low_half(ag):
    key, kb = case(128, 5)
    sched = ag.expand_key(key, kb)
    iv = gen.bytes_(5, gen.STREAM_IVS, 16).copy()
    iv[8:] = np.frombuffer(((1 << 64) - 3).to_bytes(8, "big"), np.uint8)
    src = gen.bytes_(5, gen.STREAM_DATA, 16 * 20 + 5)
    got = ag.host_route_crypt(sched, 2, iv, src)
    assert np.array_equal(got, oracle.mode(2, key, kb, iv, src))


@pytest.mark.parametrize("op", OPS)
def test_in_place(ag, op):
    key, kb = case(256, 40 + op)
    sched = ag.expand_key(key, kb)
    n = 16 * 37 + (3 if op == 2 else 0)
    src = gen.bytes_(9, gen.STREAM_DATA, n)
    iv = gen.bytes_(9, gen.STREAM_IVS, 16)
    buf = src.copy()
    ag.host_route_crypt(sched, op, iv, buf, buf)
    assert np.array_equal(buf, oracle.mode(op, key, kb, iv, src))


def test_ecb_without_iv_and_zero_length(ag):
    key, kb = case(128, 3)
    sched = ag.expand_key(key, kb)
    src = gen.bytes_(3, gen.STREAM_DATA, 64)
    assert np.array_equal(ag.host_route_crypt(sched, 3, None, src),
                          oracle.mode(3, key, kb, None, src))
    empty = np.zeros(0, np.uint8)
    assert ag.host_route_crypt(sched, 2, bytes(16), empty).size == 0


def test_errors(ag):
    key, kb = case(128, 1)
    sched = ag.expand_key(key, kb)
    src = np.zeros(64, np.uint8)
    with pytest.raises(ag.AesError) as e:
        ag.host_route_crypt(sched, 5, bytes(16), src)
    assert e.value.status == ag.AES_ERR_ARG
    with pytest.raises(ag.AesError) as e:
        ag.host_route_crypt(sched, 0, None, src)  # CBC needs an IV
    assert e.value.status == ag.AES_ERR_ARG
    with pytest.raises(ag.AesError) as e:
        ag.host_route_crypt(sched, 1, bytes(16), np.zeros(40, np.uint8))
    assert e.value.status == ag.AES_ERR_LENGTH
    bad = sched.copy()
    bad["nr"] = 12  # does not match 128-bit keys
    with pytest.raises(ag.AesError) as e:
        ag.host_route_crypt(bad, 2, bytes(16), src)
    assert e.value.status == ag.AES_ERR_KEYSIZE
    buf = np.zeros(128, np.uint8)
    with pytest.raises(ag.AesError) as e:  # partial overlap
        ag.host_route_crypt(sched, 2, bytes(16), buf[:64], buf[16:80])
    assert e.value.status == ag.AES_ERR_OVERLAP
