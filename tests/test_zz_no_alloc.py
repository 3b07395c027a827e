"""aes_batch_noalloc: aes_batch without any allocation (its unit table in a
fixed per-GPU device array, its planning in fixed host arrays).

Host tests (host-only context): the same validation errors as aes_batch, and
the unit limit.  GPU tests, through the C ABI: two calls in a row, the second
on a smaller input, each byte-identical to aes_batch on the same inputs and
to the oracle; in place (CBC decryption across tiles takes its predecessor
snapshots from the shared array); and a call of exactly the unit limit."""
import numpy as np
import pytest

from synth import workloads

FAKE = 1 << 40  # host-only context: device pointers are never dereferenced


@pytest.fixture(scope="module")
def a():
    from paper_1305_3345_amd import aesgpu
    aesgpu.lib()
    return aesgpu


@pytest.fixture()
def hctx(a):
    c = a.Context(a.AES_DEVICE_NONE)
    yield c
    c.close()


def _reqs(n=4, op=1, length=4096):
    r = np.zeros(n, workloads.REQ_DTYPE)
    r["offset"] = np.arange(n) * length
    r["length"] = length
    r["op"] = op
    return r


@pytest.mark.parametrize("case", ["cbc_len", "unaligned", "past_end", "key_idx", "overlap",
                                  "overlap_unsorted", "bad_op", "huge", "alias", "null", "ok",
                                  "empty"])
def test_noalloc_validates_like_batch(a, hctx, case):
    reqs = _reqs()
    d_in, d_out, buf = FAKE, FAKE + (1 << 30), 4 * 4096
    if case == "cbc_len":
        reqs["length"][2] = 4008
    elif case == "unaligned":
        reqs["offset"][1] += 8
    elif case == "past_end":
        reqs["length"][3] = 8192
    elif case == "key_idx":
        reqs["key_idx"][0] = 1
    elif case == "overlap":
        reqs["offset"][2] = 4096 + 16
        reqs["length"][2] = 1024
    elif case == "overlap_unsorted":
        reqs = reqs[[3, 0, 2, 1]].copy()
        reqs["offset"][0] = 4096 * 2 + 4096 - 16
        reqs["length"][0] = 32
        reqs["offset"][2] = 0
    elif case == "bad_op":
        reqs["op"][1] = 5
    elif case == "huge":
        reqs["length"][0] = 1 << 32
    elif case == "alias":
        d_out = d_in + 16
    elif case == "null":
        d_in = 0
    elif case == "empty":
        reqs["length"] = 0
    status = {}
    for name, fn in (("batch", a.batch), ("noalloc", a.batch_noalloc)):
        try:
            fn(hctx, FAKE + (2 << 30), d_in, d_out, reqs, buf_bytes=buf, n_scheds=1)
            status[name] = a.AES_OK
        except a.AesError as e:
            status[name] = e.status
    assert status["noalloc"] == status["batch"], status
    if case in ("ok",):
        assert status["noalloc"] == a.AES_ERR_DEVICE  # validated; nothing to launch on


def test_noalloc_unit_limit(a, hctx):
    """A batch of exactly AES_NOALLOC_MAX_UNITS units passes validation (then
    finds no device); one unit more is refused with AES_ERR_RANGE before any
    device work, for tiles and for chains alike."""
    m = a.AES_NOALLOC_MAX_UNITS
    buf = (m + 1) * 4096
    one = np.zeros(1, workloads.REQ_DTYPE)
    one["op"] = workloads.OP_CTR
    for length, want in ((m * 4096, a.AES_ERR_DEVICE), (m * 4096 + 1, a.AES_ERR_RANGE)):
        one["length"] = length
        with pytest.raises(a.AesError) as e:
            a.batch_noalloc(hctx, FAKE + (1 << 42), FAKE, FAKE, one, buf_bytes=buf, n_scheds=1)
        assert e.value.status == want, length
    # chains: one unit per request; m tiles of CBC decryption plus one chain
    two = np.zeros(2, workloads.REQ_DTYPE)
    two["op"] = [workloads.OP_CBC_DEC, workloads.OP_CBC_ENC]
    two["length"] = [m * 4096, 16]
    two["offset"] = [0, m * 4096]
    with pytest.raises(a.AesError) as e:
        a.batch_noalloc(hctx, FAKE + (1 << 42), FAKE, FAKE, two, buf_bytes=buf, n_scheds=1)
    assert e.value.status == a.AES_ERR_RANGE


def _all_ops(n, seed, max_pages):
    """A config-3 style mix with all five ops, ragged CTR lengths, gaps, and
    the request order shuffled (all drawn from the seeded streams)."""
    from synth import gen
    wl = workloads.config3(seed=seed, n_reqs=n, max_pages=max_pages)
    r = wl.reqs
    u = gen.uniform(seed, gen.STREAM_OPS, 3 * n).reshape(3, n)
    r["op"] = np.minimum((u[0] * 5).astype(np.uint32), 4)
    ctr = r["op"] == workloads.OP_CTR
    r["length"][ctr] -= (u[1][ctr] * 16).astype(np.uint64)
    r["offset"] += np.arange(n, dtype=np.uint64) * np.uint64(32)  # gaps between requests
    wl.buf_bytes = int(r["offset"][-1] + r["length"][-1] + 4096)
    wl.reqs = r[np.argsort(u[2], kind="stable")].copy()
    return wl


@pytest.mark.gpu
def test_noalloc_two_calls_match_batch(a):
    import torch

    import oracle
    from tests.gpu_util import device_schedules, first_mismatch
    print("\n[gpu] aes_batch_noalloc: two calls in a row, the second smaller", flush=True)
    ctx = a.Context(0)
    try:
        for k, (n, pages) in enumerate(((600, 64), (90, 8))):
            wl = _all_ops(n, seed=70 + k, max_pages=pages)
            inp = wl.data()
            d_s = device_schedules(wl)
            d_in = torch.from_numpy(inp).cuda()
            outs = {}
            for name, fn in (("noalloc", a.batch_noalloc), ("batch", a.batch)):
                d_out = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
                fn(ctx, d_s, d_in, d_out, wl.reqs)
                torch.cuda.synchronize()
                outs[name] = d_out.cpu().numpy()
            msg = first_mismatch(outs["noalloc"], outs["batch"])
            assert msg is None, f"call {k + 1} ({n} requests): noalloc vs aes_batch: {msg}"
            want = workloads.sentinel(inp.size)
            oracle.batch(inp, want, wl.reqs, wl.keys, wl.key_bits, n_threads=0)
            msg = first_mismatch(outs["noalloc"], want)
            assert msg is None, f"call {k + 1}: noalloc vs oracle: {msg}"
            print(f"[gpu] call {k + 1}: {n} requests, {wl.payload_bytes()} bytes equal",
                  flush=True)
    finally:
        ctx.close()


@pytest.mark.gpu
def test_noalloc_in_place_and_unit_limit(a):
    import torch

    from synth import gen
    from tests.gpu_util import device_schedules
    print("\n[gpu] aes_batch_noalloc: in place, then a call of exactly the unit limit",
          flush=True)
    ctx = a.Context(0)
    try:
        # In place: multi-tile CBC decryption (predecessor snapshots), CTR, chains.
        wl = _all_ops(200, seed=80, max_pages=32)
        inp = wl.data()
        d_s = device_schedules(wl)
        got = {}
        for name, fn in (("noalloc", a.batch_noalloc), ("batch", a.batch)):
            d = torch.from_numpy(inp.copy()).cuda()
            fn(ctx, d_s, d, d, wl.reqs)
            torch.cuda.synchronize()
            got[name] = d
        assert torch.equal(got["noalloc"], got["batch"]), "in place: noalloc vs aes_batch"
        del got
        # Exactly AES_NOALLOC_MAX_UNITS tiles (2 GiB of AES-256 CTR and CBC
        # decryption), compared with aes_batch on the device.
        m = a.AES_NOALLOC_MAX_UNITS
        wl2 = workloads.pages(m, workloads.OP_CTR, 256, n_keys=16)
        wl2.reqs["op"][1::2] = workloads.OP_CBC_DEC
        d_s2 = device_schedules(wl2)
        d_in = gen.bytes_torch(0, gen.STREAM_DATA, m * 4096, torch.device("cuda:0"))
        outs = []
        for fn in (a.batch_noalloc, a.batch):
            d_out = torch.empty_like(d_in)
            fn(ctx, d_s2, d_in, d_out, wl2.reqs)
            torch.cuda.synchronize()
            outs.append(d_out)
        assert torch.equal(outs[0], outs[1]), "unit limit: noalloc vs aes_batch"
        print(f"[gpu] {m} units (2 GiB) equal to aes_batch", flush=True)
    finally:
        ctx.close()
