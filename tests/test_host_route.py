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


def mixed_host_workload(seed, n=300):
    """Every op, all key sizes, sizes 0..64 KiB (ragged CTR), gaps between
    requests, requests listed out of offset order."""
    r = np.random.default_rng(seed)
    reqs = np.zeros(n, workloads.REQ_DTYPE)
    reqs["op"] = r.integers(0, 5, n)
    blocks = r.integers(0, 4097, n)
    reqs["length"] = blocks * 16
    ctr = reqs["op"] == workloads.OP_CTR
    reqs["length"][ctr] = np.maximum(reqs["length"][ctr].astype(np.int64) - r.integers(0, 16, ctr.sum()), 0)
    reqs["offset"][1:] = np.cumsum((reqs["length"] + 15) // 16 * 16 + 48)[:-1]
    reqs["key_idx"] = r.integers(0, 6, n)
    reqs["iv"] = gen.bytes_(seed, gen.STREAM_IVS, 16 * n).reshape(n, 16)
    reqs["iv"][3, 8:] = np.frombuffer(((1 << 64) - 5).to_bytes(8, "big"), np.uint8)
    reqs["op"][3] = workloads.OP_CTR
    reqs = reqs[r.permutation(n)]
    keys, kb = workloads.make_keys(seed, 6, [128, 192, 256, 128, 256, 192])
    buf = int(reqs["offset"].max() + 65536 + 64)
    return workloads.Workload("host_batch", reqs, keys, kb, buf, seed)


def oracle_out(wl, inp, inplace=False):
    out = inp.copy() if inplace else workloads.sentinel(inp.size)
    oracle.batch(inp, out, wl.reqs, wl.keys, wl.key_bits, n_threads=0)
    return out


@pytest.mark.parametrize("n_threads", [1, 3, 0])
def test_host_batch_matches_oracle(ag, n_threads):
    """aes_host_batch on a mixed batch equals the oracle byte for byte,
    sentinels outside the requests untouched, for one, three and all threads."""
    wl = mixed_host_workload(5)
    inp = wl.data()
    out = workloads.sentinel(inp.size)
    ag.host_batch(ag.expand_keys(wl.keys, wl.key_bits), inp, out, wl.reqs, n_threads)
    want = oracle_out(wl, inp)
    assert np.array_equal(out, want)


def test_host_batch_in_place(ag):
    wl = mixed_host_workload(6)
    inp = wl.data()
    buf = inp.copy()
    ag.host_batch(ag.expand_keys(wl.keys, wl.key_bits), buf, buf, wl.reqs)
    assert np.array_equal(buf, oracle_out(wl, inp, inplace=True))


def test_host_batch_errors(ag):
    wl = mixed_host_workload(7, n=20)
    inp = wl.data()
    out = workloads.sentinel(inp.size)
    sch = ag.expand_keys(wl.keys, wl.key_bits)
    bad = wl.reqs.copy()
    bad["offset"][4] += 8  # misaligned: validation, nothing runs
    with pytest.raises(ag.AesError) as e:
        ag.host_batch(sch, inp, out, bad)
    assert e.value.status == ag.AES_ERR_RANGE
    assert np.array_equal(out, workloads.sentinel(inp.size))
    with pytest.raises(ag.AesError) as e:
        ag.host_batch(sch, inp, out, wl.reqs, n_threads=4096)
    assert e.value.status == ag.AES_ERR_ARG
    # A schedule whose round count does not match its key size: its requests
    # stay untouched, the others run, the call reports AES_ERR_KEYSIZE.
    sch2 = sch.copy()
    sch2["nr"][2] = 11
    ag.host_batch(sch, inp, out, wl.reqs)
    good = out.copy()
    out2 = workloads.sentinel(inp.size)
    with pytest.raises(ag.AesError) as e:
        ag.host_batch(sch2, inp, out2, wl.reqs)
    assert e.value.status == ag.AES_ERR_KEYSIZE
    for r in wl.reqs:
        a, b = int(r["offset"]), int(r["offset"] + r["length"])
        if r["key_idx"] == 2:
            assert np.array_equal(out2[a:b], workloads.sentinel(inp.size)[a:b])
        else:
            assert np.array_equal(out2[a:b], good[a:b])
