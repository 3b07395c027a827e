"""GPU tests of serving with payloads in pinned host memory (buffers from
aes_server_host_alloc): every request's bytes must equal the oracle's
(tolerance 0) and bytes outside every request must keep their sentinel.

Transports: the persistent engine (its waves read and write the pinned pages
over the host link), the per-launch engine with copies through per-stream
HBM staging (AES_XFER_COPY), and the per-launch engine reading the pages
directly (AES_XFER_DIRECT).  Cases: host to host, host to device, device to
host, in place in host memory, requests above max_request_bytes (a normal
launch, always direct), trace replay from host bases, and the buffer errors
(range past a buffer's end, freeing while requests are in flight, freeing an
unknown pointer)."""
import numpy as np
import pytest
import torch

from synth import workloads
from tests.gpu_util import ag, first_mismatch
from tests.test_gpu_serving import make_trace, oracle_request, server, submit_retry, sync

pytestmark = pytest.mark.gpu

# (engine, host_xfer): persistent; per-launch with copies; per-launch direct
TRANSPORTS = [(0, 0), (1, 0), (1, 1)]


@pytest.fixture(scope="module")
def ctx():
    print("\n[gpu] context for host-payload serving tests", flush=True)
    c = ag().Context(0)
    yield c
    c.close()


def check_requests(wl, inp, out, what):
    for r in wl.reqs:
        o, n = int(r["offset"]), int(r["length"])
        msg = first_mismatch(out[o:o + n], oracle_request(wl, r, inp[o:o + n]))
        assert msg is None, f"{what}: request at {o} op {int(r['op'])}: {msg}"
    touched = np.zeros(inp.size, bool)
    for r in wl.reqs:
        touched[int(r["offset"]):int(r["offset"] + r["length"])] = True
    sent = workloads.sentinel(inp.size)
    assert np.array_equal(out[~touched], sent[~touched]), f"{what}: bytes outside requests"


def with_ecb(wl):
    """Turns every fifth whole-block request into ECB (encrypt or decrypt)."""
    whole = np.flatnonzero(wl.reqs["length"] % 16 == 0)[::5]
    a = ag()
    wl.reqs["op"][whole] = np.where(np.arange(whole.size) % 2 == 0, a.AES_OP_ECB_ENC,
                                    a.AES_OP_ECB_DEC)
    return wl


@pytest.mark.parametrize("engine,xfer", TRANSPORTS)
def test_host_to_host(ctx, engine, xfer):
    print(f"[gpu] host to host, engine={engine} xfer={xfer}", flush=True)
    wl = with_ecb(make_trace(150, seed=21))
    inp = wl.data()
    with server(ctx, wl, mode=engine, host_xfer=xfer) as s:
        h_in = s.host_alloc(inp.size)
        h_out = s.host_alloc(inp.size)
        h_in[:] = inp
        h_out[:] = workloads.sentinel(inp.size)
        base_in, base_out = h_in.ctypes.data, h_out.ctypes.data
        tickets = [submit_retry(s, r, base_in + int(r["offset"]), base_out + int(r["offset"]))
                   for r in wl.reqs]
        for t in tickets:
            assert s.wait(t)["status"] == 0
        out = h_out.copy()
        assert np.array_equal(h_in, inp), "input changed"
    check_requests(wl, inp, out, f"engine {engine} xfer {xfer}")


@pytest.mark.parametrize("engine,xfer", TRANSPORTS)
def test_mixed_placement(ctx, engine, xfer):
    """Host to device, device to host, and in place in host memory."""
    print(f"[gpu] host/device placement, engine={engine} xfer={xfer}", flush=True)
    wl = make_trace(60, seed=22)
    inp = wl.data()
    n = inp.size
    with server(ctx, wl, mode=engine, host_xfer=xfer) as s:
        h_in = s.host_alloc(n)
        h_out = s.host_alloc(n)
        h_in[:] = inp
        h_out[:] = workloads.sentinel(n)
        d_in = torch.from_numpy(inp).cuda()
        d_out = torch.from_numpy(workloads.sentinel(n)).cuda()
        sync()
        forms = {"host->device": (h_in.ctypes.data, d_out.data_ptr()),
                 "device->host": (d_in.data_ptr(), h_out.ctypes.data)}
        got = {}
        for form, (src, dst) in forms.items():
            tickets = [submit_retry(s, r, src + int(r["offset"]), dst + int(r["offset"]))
                       for r in wl.reqs]
            for t in tickets:
                assert s.wait(t)["status"] == 0
        got["host->device"] = d_out.cpu().numpy()
        got["device->host"] = h_out.copy()
        # in place: the input buffer becomes the output
        base = h_in.ctypes.data
        tickets = [submit_retry(s, r, base + int(r["offset"]), base + int(r["offset"]))
                   for r in wl.reqs]
        for t in tickets:
            assert s.wait(t)["status"] == 0
        inplace = h_in.copy()
    for form in forms:
        check_requests(wl, inp, got[form], f"{form} engine {engine} xfer {xfer}")
    for r in wl.reqs:
        o, m = int(r["offset"]), int(r["length"])
        msg = first_mismatch(inplace[o:o + m], oracle_request(wl, r, inp[o:o + m]))
        assert msg is None, f"in place: request at {o}: {msg}"
    touched = np.zeros(n, bool)
    for r in wl.reqs:
        touched[int(r["offset"]):int(r["offset"] + r["length"])] = True
    assert np.array_equal(inplace[~touched], inp[~touched])


@pytest.mark.parametrize("engine,xfer", TRANSPORTS)
def test_above_max_request_bytes(ctx, engine, xfer):
    """Requests above max_request_bytes take a normal launch that reads and
    writes the pinned pages directly (no staging buffer is that large)."""
    print(f"[gpu] host payload above max_request_bytes, engine={engine} xfer={xfer}",
          flush=True)
    wl = make_trace(12, seed=23, sizes=(16, 64, 200, 320))
    inp = wl.data()
    with server(ctx, wl, mode=engine, host_xfer=xfer, max_request_bytes=64 << 10) as s:
        h_in = s.host_alloc(inp.size)
        h_out = s.host_alloc(inp.size)
        h_in[:] = inp
        h_out[:] = workloads.sentinel(inp.size)
        tickets = [submit_retry(s, r, h_in.ctypes.data + int(r["offset"]),
                                h_out.ctypes.data + int(r["offset"])) for r in wl.reqs]
        for t in tickets:
            assert s.wait(t)["status"] == 0
        out = h_out.copy()
        if engine == 0:
            big = int((wl.reqs["length"] > (64 << 10)).sum())
            assert s.stats()["fallbacks"] == big
    check_requests(wl, inp, out, f"large engine {engine} xfer {xfer}")


@pytest.mark.parametrize("engine,xfer", TRANSPORTS)
def test_replay_from_host(ctx, engine, xfer):
    print(f"[gpu] trace replay from host buffers, engine={engine} xfer={xfer}", flush=True)
    a = ag()
    wl = make_trace(400, seed=24)
    inp = wl.data()
    arrival = np.cumsum(np.random.default_rng(24).exponential(20e-6, wl.reqs.size))
    with server(ctx, wl, mode=engine, host_xfer=xfer) as s:
        h_in = s.host_alloc(inp.size)
        h_out = s.host_alloc(inp.size)
        h_in[:] = inp
        h_out[:] = workloads.sentinel(inp.size)
        done = s.replay(wl.reqs, arrival, h_in, h_out)
        out = h_out.copy()
    assert (done["status"] == a.AES_OK).all()
    assert (done["t_done_ns"] >= done["t_submit_ns"]).all()
    check_requests(wl, inp, out, f"replay engine {engine} xfer {xfer}")


def test_host_buffer_errors(ctx):
    print("[gpu] host buffer errors", flush=True)
    a = ag()
    wl = make_trace(4, seed=25)
    with server(ctx, wl, mode=0) as s:
        h = s.host_alloc(1 << 20)
        iv = bytes(16)
        # a range that starts inside the buffer and runs past its end
        with pytest.raises(a.AesError) as e:
            s.submit(workloads.OP_CTR, 0, iv, h.ctypes.data + (1 << 20) - 4096,
                     h.ctypes.data + (1 << 20) - 4096, 8192)
        assert e.value.status == a.AES_ERR_RANGE
        # freeing while a request is in flight: a 1 MiB CBC-encrypt chain
        # runs for milliseconds, the free comes microseconds after the submit
        t = s.submit(workloads.OP_CBC_ENC, 1, iv, h.ctypes.data, h.ctypes.data, 1 << 20)
        with pytest.raises(a.AesError) as e:
            s.host_free(h)
        assert e.value.status == a.AES_ERR_STATE
        assert s.wait(t)["status"] == 0
        # not the start of a buffer, then a clean free and a double free
        addr = h.ctypes.data
        assert a.lib().aes_server_host_free(s.handle, addr + 16) == a.AES_ERR_ARG
        s.host_free(h)
        st = a.lib().aes_server_host_free(s.handle, addr)
        assert st == a.AES_ERR_ARG
        with pytest.raises(a.AesError) as e:
            s.host_alloc(0)
        assert e.value.status == a.AES_ERR_ARG
