"""GPU parity of the long-stream workloads: AES-256-CTR over 8 GiB in 512
chunks of 16 MiB forming one continuous counter stream, and AES-256-CBC
encryption of 4,096 chains of 1 MiB.

The oracle computes sampled spans (CTR keystream is seekable: the span at
byte a of a chunk uses counter ctr0 + a / 16) and whole sampled chains;
properties cover every byte: the chunked batch equals the same stream cut
into 3 + 3 + 2 GiB requests, CTR applied twice restores the input, and CBC
decryption of the chains' output restores their input."""
import numpy as np
import pytest
import torch

import oracle
from synth import gen, workloads
from tests.gpu_util import ag, device_schedules, first_mismatch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("\n[gpu] context for long-stream tests", flush=True)
    c = ag().Context(0)
    yield c
    c.close()


def device_input(nbytes):
    return gen.bytes_torch(0, gen.STREAM_DATA, nbytes, torch.device("cuda:0"))


def ctr_span_oracle(wl, r, a, n, src):
    """Oracle bytes a .. a+n of request r (a a multiple of 16)."""
    iv = r["iv"].copy()
    c = (int.from_bytes(iv[8:].tobytes(), "big") + a // 16) % (1 << 64)
    iv[8:] = np.frombuffer(c.to_bytes(8, "big"), np.uint8)
    kb = int(wl.key_bits[r["key_idx"]])
    return oracle.mode(workloads.OP_CTR, wl.keys[r["key_idx"]][: kb // 8], kb, iv, src)


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
    rng = np.random.default_rng(3)
    chunks = np.unique(np.concatenate([[0, wl.reqs.size - 1],
                                       rng.choice(wl.reqs.size, 30, replace=False)]))
    chunk = int(wl.reqs["length"][0])
    for ci in chunks:
        r = wl.reqs[ci]
        o = int(r["offset"])
        for start in (0, chunk - 65536, int(rng.integers(0, chunk // 16 - 4096)) * 16):
            n = 65536
            src = d_in[o + start:o + start + n].cpu().numpy()
            got = d_out[o + start:o + start + n].cpu().numpy()
            msg = first_mismatch(got, ctr_span_oracle(wl, r, start, n, src))
            assert msg is None, f"chunk {ci} at {start}: {msg}"
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
    del d_big
    # CTR twice restores the input
    back = torch.empty_like(d_in)
    plan = a.Plan(ctx, wl.reqs, 1, nbytes)
    plan.launch(d_s, d_out, back)
    torch.cuda.synchronize()
    plan.close()
    assert torch.equal(back, d_in), "CTR twice over 8 GiB"


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
    rng = np.random.default_rng(4)
    sample = np.unique(np.concatenate([[0, wl.reqs.size - 1],
                                       rng.choice(wl.reqs.size, 14, replace=False)]))
    kb = int(wl.key_bits[0])
    for ci in sample:
        r = wl.reqs[ci]
        o, n = int(r["offset"]), int(r["length"])
        want = oracle.mode(workloads.OP_CBC_ENC, wl.keys[0][: kb // 8], kb, r["iv"],
                           d_in[o:o + n].cpu().numpy())
        msg = first_mismatch(d_out[o:o + n].cpu().numpy(), want)
        assert msg is None, f"chain {ci}: {msg}"
    inv = wl.reqs.copy()
    inv["op"] = workloads.OP_CBC_DEC
    back = torch.empty_like(d_in)
    plan = a.Plan(ctx, inv, 1, nbytes)
    plan.launch(d_s, d_out, back)
    torch.cuda.synchronize()
    plan.close()
    assert torch.equal(back, d_in), "CBC decryption of the chains' output"
