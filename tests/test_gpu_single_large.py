"""GPU parity of large single-op calls (aes_cbc_decrypt_batch, aes_ctr_batch,
aes_ecb_*_batch with 20,000 requests), which the library plans in parallel
chunks straight into its staging buffer: byte for byte against the CPU
oracle (tolerance 0), bytes outside every request untouched.

Cases: requests of 0 to 3 pages (some zero-length, tiles crossing pages),
ragged CTR lengths and a counter wrap, callers' order that is not offset
order, in-place CBC decryption across tiles, every key size, two calls in a
row reusing the context's buffers, and the same call below the parallel
threshold for comparison."""
import numpy as np
import pytest

from synth import gen, workloads
from tests.gpu_util import ag, first_mismatch, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

N = 20000


@pytest.fixture(scope="module")
def ctx():
    print("\n[gpu] context for large single-call tests", flush=True)
    c = ag().Context(0)
    yield c
    c.close()


def large_workload(op, seed, n=N, ragged=False, shuffle=False):
    r = np.random.default_rng(seed)
    reqs = np.zeros(n, workloads.REQ_DTYPE)
    pages = r.choice([0, 1, 1, 1, 2, 3], n)
    reqs["length"] = pages * 4096
    if ragged:
        reqs["length"] = np.where(pages > 0, reqs["length"] - r.integers(0, 16, n), 0)
    reqs["offset"][1:] = np.cumsum((reqs["length"] + 15) // 16 * 16 + 32)[:-1]
    reqs["op"] = op
    reqs["key_idx"] = r.integers(0, 6, n)
    reqs["iv"] = gen.bytes_(seed, gen.STREAM_IVS, 16 * n).reshape(n, 16)
    if op == workloads.OP_CTR:
        reqs["iv"][7, 8:] = np.frombuffer(((1 << 64) - 2).to_bytes(8, "big"), np.uint8)
    if shuffle:
        reqs = reqs[r.permutation(n)]
    keys, kb = workloads.make_keys(seed, 6, [128, 192, 256, 128, 256, 192])
    buf = int(reqs["offset"].max() + 3 * 4096 + 64)
    return workloads.Workload("single_large", reqs, keys, kb, buf, seed)


def check(got, want, what):
    msg = first_mismatch(got, want)
    assert msg is None, f"{what}: {msg}"


@pytest.mark.parametrize("op,ragged,shuffle", [
    (workloads.OP_CTR, True, False), (workloads.OP_CTR, False, True),
    (workloads.OP_CBC_DEC, False, False), (workloads.OP_CBC_DEC, False, True)])
def test_large_single_call(ctx, op, ragged, shuffle):
    print(f"[gpu] single call of {N}: op={op} ragged={ragged} shuffle={shuffle}", flush=True)
    wl = large_workload(op, 11 + op + 2 * shuffle, ragged=ragged, shuffle=shuffle)
    inp = wl.data()
    want = run_oracle(wl, inp)
    check(run_gpu(ctx, wl, inp, form="single"), want, "first call")
    check(run_gpu(ctx, wl, inp, form="single"), want, "second call (reused buffers)")


@pytest.mark.parametrize("op", ["ecb_enc", "ecb_dec"])
def test_large_single_call_ecb(ctx, op):
    a = ag()
    print(f"[gpu] single call of {N}: {op}", flush=True)
    opnum = a.AES_OP_ECB_ENC if op == "ecb_enc" else a.AES_OP_ECB_DEC
    wl = large_workload(opnum, 21)
    inp = wl.data()
    check(run_gpu(ctx, wl, inp, form="single"), run_oracle(wl, inp), op)


def test_large_single_call_cbc_dec_in_place(ctx):
    print(f"[gpu] single call of {N}: CBC-dec in place", flush=True)
    wl = large_workload(workloads.OP_CBC_DEC, 31)
    inp = wl.data()
    check(run_gpu(ctx, wl, inp, form="single", inplace=True),
          run_oracle(wl, inp, inplace=True), "in place")


def test_parallel_and_serial_paths_agree(ctx):
    """The same requests as one call of 20,000 (parallel planning) and as
    calls of 2,000 (serial planning) produce the same bytes."""
    print("[gpu] parallel vs serial single-call planning", flush=True)
    import torch
    a = ag()
    wl = large_workload(workloads.OP_CTR, 41, ragged=True)
    inp = wl.data()
    whole = run_gpu(ctx, wl, inp, form="single")
    d_s = a.schedules_to_device(a.expand_keys(wl.keys, wl.key_bits))
    d_in = torch.from_numpy(inp.copy()).cuda()
    d_out = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
    r = wl.reqs
    for lo in range(0, N, 2000):
        s = r[lo:lo + 2000]
        a.ctr_batch(ctx, d_s, d_in, d_out, s["offset"], s["length"], s["key_idx"], s["iv"])
    torch.cuda.synchronize()
    check(d_out.cpu().numpy(), whole, "chunked calls vs one call")
