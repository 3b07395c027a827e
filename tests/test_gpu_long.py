"""GPU parity of the long-stream workloads: AES-256-CTR over 8 GiB in 512
chunks of 16 MiB forming one continuous counter stream, and AES-256-CBC
encryption of 4,096 chains of 1 MiB.

Both are checked against the oracle on every byte: the device buffers are
copied to the host 1 GiB at a time and the oracle's threaded batch runs the
requests of that piece (the chunks and chains do not cross 1 GiB
boundaries).  Two properties are checked besides, as extra checks that do
not replace the oracle: the chunked CTR batch equals the same stream cut
into 3 + 3 + 2 GiB requests (the counter continues across request
boundaries), and CBC decryption of the chains' output restores their
input."""
import os

import numpy as np
import pytest
import torch

import oracle
from synth import gen, workloads
from tests.gpu_util import ag, device_schedules, first_mismatch

pytestmark = pytest.mark.gpu

PIECE = 1 << 30


@pytest.fixture(scope="module")
def ctx():
    print("\n[gpu] context for long-stream tests", flush=True)
    c = ag().Context(0)
    yield c
    c.close()


def device_input(nbytes):
    return gen.bytes_torch(0, gen.STREAM_DATA, nbytes, torch.device("cuda:0"))


def check_against_oracle(wl, d_in, d_out, label):
    """Every request of wl against the oracle, one 1 GiB piece of the buffers
    at a time (requests must not cross a piece boundary)."""
    offs = wl.reqs["offset"].astype(np.uint64)
    ends = offs + wl.reqs["length"].astype(np.uint64)
    assert (offs // PIECE == (ends - 1) // PIECE).all()
    threads = len(os.sched_getaffinity(0))
    n_pieces = (wl.buf_bytes + PIECE - 1) // PIECE
    for p in range(n_pieces):
        lo, hi = p * PIECE, min(wl.buf_bytes, (p + 1) * PIECE)
        mine = wl.reqs[(offs >= lo) & (offs < hi)].copy()
        mine["offset"] -= np.uint64(lo)
        src = d_in[lo:hi].cpu().numpy()
        got = d_out[lo:hi].cpu().numpy()
        want = np.empty_like(src)
        oracle.batch(src, want, mine, wl.keys, wl.key_bits, n_threads=threads)
        msg = first_mismatch(got, want)
        assert msg is None, f"{label}, piece {p} (bytes {lo}..{hi}): {msg}"
        print(f"[gpu] {label}: piece {p + 1}/{n_pieces} ({mine.size} requests) equals the "
              f"oracle", flush=True)


def test_ctr_8gib_continuous_stream(ctx):
    print("[gpu] 8 GiB AES-256-CTR in 512 chunks", flush=True)
    a = ag()
    wl = workloads.config5_ctr()
    nbytes = wl.buf_bytes
    d_s = device_schedules(wl)
    d_in = device_input(nbytes)
    d_out = torch.empty_like(d_in)
    plan = a.Plan(ctx, wl.reqs, 1, nbytes)
    plan.launch(d_s, d_in, d_out)
    torch.cuda.synchronize()
    plan.close()
    check_against_oracle(wl, d_in, d_out, "8 GiB CTR stream")
    # the same stream cut differently (requests are limited to < 4 GiB):
    # 3 + 3 + 2 GiB with the counter continuing across them
    cuts = [0, 3 << 30, 6 << 30, nbytes]
    big = np.zeros(3, workloads.REQ_DTYPE)
    for i in range(3):
        big["offset"][i] = cuts[i]
        big["length"][i] = cuts[i + 1] - cuts[i]
        iv = wl.reqs["iv"][0].copy()
        iv[8:] = np.frombuffer((cuts[i] // 16).to_bytes(8, "big"), np.uint8)
        big["iv"][i] = iv
    big["op"] = workloads.OP_CTR
    d_big = torch.empty_like(d_in)
    plan = a.Plan(ctx, big, 1, nbytes)
    plan.launch(d_s, d_in, d_big)
    torch.cuda.synchronize()
    plan.close()
    assert torch.equal(d_big, d_out), "chunked batch differs from 3 + 3 + 2 GiB requests"


def test_cbc_encrypt_4096_chains_of_1mib(ctx):
    print("[gpu] 4,096 AES-256-CBC chains of 1 MiB", flush=True)
    a = ag()
    wl = workloads.config5_cbc()
    nbytes = wl.buf_bytes
    d_s = device_schedules(wl)
    d_in = device_input(nbytes)
    d_out = torch.empty_like(d_in)
    plan = a.Plan(ctx, wl.reqs, 1, nbytes)
    plan.launch(d_s, d_in, d_out)
    torch.cuda.synchronize()
    plan.close()
    check_against_oracle(wl, d_in, d_out, "4,096 CBC-encrypt chains")
    inv = wl.reqs.copy()
    inv["op"] = workloads.OP_CBC_DEC
    back = torch.empty_like(d_in)
    plan = a.Plan(ctx, inv, 1, nbytes)
    plan.launch(d_s, d_out, back)
    torch.cuda.synchronize()
    plan.close()
    assert torch.equal(back, d_in), "CBC decryption of the chains' output"
