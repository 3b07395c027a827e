"""GPU tests of size-based CPU/GPU dispatch in the serving engines: requests
below an op's crossover whose payloads both lie in the server's host
buffers run on the host route, every other request on the GPU engine; each
request's bytes equal the oracle's (tolerance 0) whichever way it went, and
the route counts match the rule exactly.  Also: calibration on the machine
(values well formed, ECB sharing CTR's and CBC decryption's), callbacks of
host-routed requests, and calibration errors."""
import numpy as np
import pytest
import torch

from synth import workloads
from tests.gpu_util import ag, first_mismatch
from tests.test_gpu_serving import make_trace, oracle_request, server, submit_retry, sync
from tests.test_gpu_serving_host import check_requests, with_ecb

pytestmark = pytest.mark.gpu

U64_MAX = (1 << 64) - 1


@pytest.fixture(scope="module")
def ctx():
    print("\n[gpu] context for dispatch tests", flush=True)
    c = ag().Context(0)
    yield c
    c.close()


def expected_host(wl, cross):
    return int(sum(int(r["length"]) < int(cross[int(r["op"])]) for r in wl.reqs))


@pytest.mark.parametrize("engine", [0, 1])
def test_manual_crossovers(ctx, engine):
    print(f"[gpu] dispatch with set crossovers, engine={engine}", flush=True)
    wl = with_ecb(make_trace(160, seed=31))
    inp = wl.data()
    cross = [U64_MAX, 0, 16 << 10, 32 << 10, 8 << 10]  # by op
    with server(ctx, wl, mode=engine) as s:
        for op, v in enumerate(cross):
            s.set_crossover(op, v)
            assert s.get_crossover(op) == v
        h_in = s.host_alloc(inp.size)
        h_out = s.host_alloc(inp.size)
        h_in[:] = inp
        h_out[:] = workloads.sentinel(inp.size)
        ts = [submit_retry(s, r, h_in.ctypes.data + int(r["offset"]),
                           h_out.ctypes.data + int(r["offset"])) for r in wl.reqs]
        for t in ts:
            assert s.wait(t)["status"] == 0
        out = h_out.copy()
        st = s.stats()
        assert st["host_routed"] == expected_host(wl, cross)
        assert 0 < st["host_routed"] < wl.reqs.size
        # device payloads never take the host route, whatever the crossover
        d_in = torch.from_numpy(inp).cuda()
        d_out = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
        sync()
        ts = [submit_retry(s, r, d_in.data_ptr() + int(r["offset"]),
                           d_out.data_ptr() + int(r["offset"])) for r in wl.reqs]
        for t in ts:
            assert s.wait(t)["status"] == 0
        assert s.stats()["host_routed"] == st["host_routed"]
        dev_out = d_out.cpu().numpy()
    check_requests(wl, inp, out, f"dispatch engine {engine}")
    check_requests(wl, inp, dev_out, f"device payloads engine {engine}")


@pytest.mark.parametrize("engine", [0, 1])
def test_calibrated_dispatch(ctx, engine):
    print(f"[gpu] calibrate then dispatch a trace, engine={engine}", flush=True)
    a = ag()
    wl = make_trace(300, seed=32, sizes=(4, 16, 64, 256, 1024))
    inp = wl.data()
    with server(ctx, wl, mode=engine) as s:
        cross = s.calibrate(0)
        print(f"[gpu] crossovers by op: {[int(c) for c in cross]}", flush=True)
        for c in cross:
            c = int(c)
            assert c == U64_MAX or (c >= 4096 and c & (c - 1) == 0)
        assert cross[a.AES_OP_ECB_ENC] == cross[a.AES_OP_CTR]
        assert cross[a.AES_OP_ECB_DEC] == cross[a.AES_OP_CBC_DEC]
        assert [s.get_crossover(op) for op in range(5)] == [int(c) for c in cross]
        h_in = s.host_alloc(inp.size)
        h_out = s.host_alloc(inp.size)
        h_in[:] = inp
        h_out[:] = workloads.sentinel(inp.size)
        before = s.stats()["host_routed"]
        arrival = np.cumsum(np.random.default_rng(32).exponential(50e-6, wl.reqs.size))
        done = s.replay(wl.reqs, arrival, h_in, h_out)
        assert (done["status"] == 0).all()
        assert s.stats()["host_routed"] - before == expected_host(wl, cross)
        out = h_out.copy()
    check_requests(wl, inp, out, f"calibrated engine {engine}")


def test_host_routed_callbacks(ctx):
    print("[gpu] callbacks of host-routed requests", flush=True)
    wl = make_trace(20, seed=33, sizes=(4,))
    inp = wl.data()
    got = []
    with server(ctx, wl) as s:
        for op in range(5):
            s.set_crossover(op, U64_MAX)
        h_in = s.host_alloc(inp.size)
        h_out = s.host_alloc(inp.size)
        h_in[:] = inp
        ts = [s.submit(int(r["op"]), int(r["key_idx"]), r["iv"],
                       h_in.ctypes.data + int(r["offset"]), h_out.ctypes.data + int(r["offset"]),
                       int(r["length"]), callback=got.append) for r in wl.reqs]
        assert len(got) == wl.reqs.size  # complete before submit returns
        assert sorted(int(d["ticket"]) for d in got) == sorted(ts)
        assert all(int(d["status"]) == 0 for d in got)
        assert s.stats()["host_routed"] == wl.reqs.size
        out = h_out.copy()
    for r in wl.reqs:
        o, n = int(r["offset"]), int(r["length"])
        assert first_mismatch(out[o:o + n], oracle_request(wl, r, inp[o:o + n])) is None


def test_calibrate_errors(ctx):
    print("[gpu] calibration errors", flush=True)
    a = ag()
    wl = make_trace(4, seed=34)
    with server(ctx, wl) as s:
        with pytest.raises(a.AesError) as e:
            s.calibrate(wl.keys.shape[0])  # out of range
        assert e.value.status == a.AES_ERR_RANGE
    with a.Server(ctx, key_slots=4) as s:  # no key set
        with pytest.raises(a.AesError) as e:
            s.calibrate(0)
        assert e.value.status == a.AES_ERR_RANGE
        with pytest.raises(a.AesError) as e:
            s.set_crossover(5, 1)
        assert e.value.status == a.AES_ERR_ARG
