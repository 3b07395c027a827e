"""GPU tests of the serving form (persistent kernel and per-request-launch
engines): every request's bytes must equal the oracle's and be identical
alone and in the mix (tolerance 0); admission, fallback, idle exit and
relaunch, errors, callbacks and trace replay.

While a persistent kernel runs, tests synchronise only torch's current
stream (a device-wide synchronise would wait for the persistent kernel)."""
import time

import numpy as np
import pytest
import torch

import oracle
from synth import gen, workloads
from tests.gpu_util import ag, first_mismatch

pytestmark = pytest.mark.gpu

ENGINES = [0, 1]  # AES_SERVE_PERSISTENT, AES_SERVE_PER_LAUNCH


@pytest.fixture(scope="module")
def ctx():
    print("\n[gpu] context for serving tests", flush=True)
    c = ag().Context(0)
    yield c
    c.close()


def sync():
    torch.cuda.current_stream().synchronize()


def make_trace(n, seed=0, n_keys=8, sizes=(4, 8, 16, 32, 64), ctr_share=True):
    """n requests over one staged buffer: sizes in KiB, ops CBC-enc/dec (and
    CTR with ragged lengths), key slots 0..n_keys-1 with 128/256-bit keys."""
    r = np.random.default_rng(seed)
    kib = r.choice(np.array(sizes), n)
    reqs = np.zeros(n, workloads.REQ_DTYPE)
    reqs["length"] = kib * 1024
    ops = r.integers(0, 3 if ctr_share else 2, n)
    reqs["op"] = ops
    ctr = reqs["op"] == workloads.OP_CTR
    reqs["length"][ctr] -= r.integers(0, 16, ctr.sum()).astype(np.uint64)
    reqs["offset"][1:] = np.cumsum((reqs["length"] + 15) // 16 * 16 + 64)[:-1]
    reqs["key_idx"] = r.integers(0, n_keys, n)
    reqs["iv"] = gen.bytes_(seed, gen.STREAM_IVS, 16 * n).reshape(n, 16)
    keys, kb = workloads.make_keys(seed, n_keys, [128, 256] * (n_keys // 2))
    buf = int(reqs["offset"][-1] + reqs["length"][-1] + 64)
    return workloads.Workload("serve", reqs, keys, kb, buf, seed)


def server(ctx, wl, **cfg):
    a = ag()
    s = a.Server(ctx, key_slots=wl.keys.shape[0], **cfg)
    for i, sch in enumerate(a.expand_keys(wl.keys, wl.key_bits)):
        s.set_key(i, sch)
    return s


def oracle_request(wl, r, src):
    kb = int(wl.key_bits[r["key_idx"]])
    return oracle.mode(int(r["op"]), wl.keys[r["key_idx"]][: kb // 8], kb, r["iv"], src)


def submit_retry(s, r, d_src, d_dst):
    a = ag()
    while True:
        try:
            return s.submit(int(r["op"]), int(r["key_idx"]), r["iv"], d_src, d_dst,
                            int(r["length"]))
        except a.AesError as e:
            if e.status != a.AES_ERR_AGAIN:
                raise
            time.sleep(20e-6)


@pytest.mark.parametrize("engine", ENGINES)
def test_alone_vs_mix(ctx, engine):
    print(f"[gpu] serving alone vs mix, engine={engine}", flush=True)
    wl = make_trace(120)
    inp = wl.data()
    d_in = torch.from_numpy(inp).cuda()
    sync()
    base = d_in.data_ptr()
    outs = {}
    with server(ctx, wl, mode=engine) as s:
        for form in ("alone", "mix"):
            d_out = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
            sync()
            ob = d_out.data_ptr()
            if form == "alone":
                for r in wl.reqs:
                    t = submit_retry(s, r, base + int(r["offset"]), ob + int(r["offset"]))
                    assert s.wait(t)["status"] == 0
            else:
                tickets = [submit_retry(s, r, base + int(r["offset"]), ob + int(r["offset"]))
                           for r in wl.reqs]
                for t in tickets:
                    assert s.wait(t)["status"] == 0
            outs[form] = d_out.cpu().numpy()
        st = s.stats()
        assert st["completed"] == 2 * wl.reqs.size and st["in_flight"] == 0
    msg = first_mismatch(outs["alone"], outs["mix"])
    assert msg is None, f"alone vs mix: {msg}"
    for r in wl.reqs:
        o, n = int(r["offset"]), int(r["length"])
        want = oracle_request(wl, r, inp[o:o + n])
        msg = first_mismatch(outs["mix"][o:o + n], want)
        assert msg is None, f"request at {o} op {int(r['op'])}: {msg}"
    sent = workloads.sentinel(inp.size)
    touched = np.zeros(inp.size, bool)
    for r in wl.reqs:
        touched[int(r["offset"]):int(r["offset"] + r["length"])] = True
    assert np.array_equal(outs["mix"][~touched], sent[~touched])


@pytest.mark.parametrize("engine", ENGINES)
def test_in_place(ctx, engine):
    print(f"[gpu] serving in place, engine={engine}", flush=True)
    wl = make_trace(40, seed=3, sizes=(16, 64))
    inp = wl.data()
    d = torch.from_numpy(inp.copy()).cuda()
    sync()
    with server(ctx, wl, mode=engine) as s:
        ts = [submit_retry(s, r, d.data_ptr() + int(r["offset"]), d.data_ptr() + int(r["offset"]))
              for r in wl.reqs]
        for t in ts:
            assert s.wait(t)["status"] == 0
        got = d.cpu().numpy()
    for r in wl.reqs:
        o, n = int(r["offset"]), int(r["length"])
        assert first_mismatch(got[o:o + n], oracle_request(wl, r, inp[o:o + n])) is None


def test_admission_backpressure(ctx):
    print("[gpu] admission and backpressure", flush=True)
    a = ag()
    wl = make_trace(300, seed=5, sizes=(64,), ctr_share=False)
    inp = wl.data()
    d_in = torch.from_numpy(inp).cuda()
    d_out = torch.empty_like(d_in)
    sync()
    with server(ctx, wl, ring_slots=64, hbm_cap_bytes=1 << 20) as s:
        tickets, again = [], 0
        for r in wl.reqs:
            while True:
                try:
                    tickets.append(s.submit(int(r["op"]), int(r["key_idx"]), r["iv"],
                                            d_in.data_ptr() + int(r["offset"]),
                                            d_out.data_ptr() + int(r["offset"]), int(r["length"])))
                    break
                except a.AesError as e:
                    assert e.status == a.AES_ERR_AGAIN
                    again += 1
                    st = s.stats()
                    assert st["in_flight"] <= 64 and st["in_flight_bytes"] <= 1 << 20
                    time.sleep(50e-6)
        for t in tickets:
            assert s.wait(t)["status"] == 0
        assert again > 0, "the cap should have refused some submits"
        got = d_out.cpu().numpy()
    for r in wl.reqs[::7]:
        o, n = int(r["offset"]), int(r["length"])
        assert first_mismatch(got[o:o + n], oracle_request(wl, r, inp[o:o + n])) is None


def test_oversize_request_takes_a_normal_launch(ctx):
    print("[gpu] oversize fallback", flush=True)
    wl = make_trace(6, seed=7, sizes=(1024,))
    inp = wl.data()
    d_in = torch.from_numpy(inp).cuda()
    d_out = torch.empty_like(d_in)
    sync()
    with server(ctx, wl, max_request_bytes=256 << 10) as s:
        ts = [submit_retry(s, r, d_in.data_ptr() + int(r["offset"]),
                           d_out.data_ptr() + int(r["offset"])) for r in wl.reqs]
        for t in ts:
            assert s.wait(t)["status"] == 0
        assert s.stats()["fallbacks"] == wl.reqs.size
        got = d_out.cpu().numpy()
    for r in wl.reqs:
        o, n = int(r["offset"]), int(r["length"])
        assert first_mismatch(got[o:o + n], oracle_request(wl, r, inp[o:o + n])) is None


def test_oversize_between_ring_requests(ctx):
    """Normal launches interleaved with ring requests: a launched request
    takes no ring position, so the dispatcher never waits on a gap."""
    print("[gpu] oversize requests between ring requests", flush=True)
    wl = make_trace(40, seed=8, sizes=(4, 16, 64, 512))
    inp = wl.data()
    d_in = torch.from_numpy(inp).cuda()
    d_out = torch.empty_like(d_in)
    sync()
    big = int((wl.reqs["length"] > (256 << 10)).sum())
    assert 0 < big < wl.reqs.size
    with server(ctx, wl, max_request_bytes=256 << 10, ring_slots=64) as s:
        for rnd in range(3):  # 120 tickets through a 64-slot ring
            ts = [submit_retry(s, r, d_in.data_ptr() + int(r["offset"]),
                               d_out.data_ptr() + int(r["offset"])) for r in wl.reqs]
            for t in ts:
                assert s.wait(t)["status"] == 0, f"round {rnd}"
        assert s.stats()["fallbacks"] == 3 * big
        got = d_out.cpu().numpy()
    for r in wl.reqs:
        o, n = int(r["offset"]), int(r["length"])
        assert first_mismatch(got[o:o + n], oracle_request(wl, r, inp[o:o + n])) is None


def test_idle_exit_and_relaunch(ctx):
    print("[gpu] idle exit and relaunch", flush=True)
    wl = make_trace(10, seed=9)
    inp = wl.data()
    d_in = torch.from_numpy(inp).cuda()
    d_out = torch.empty_like(d_in)
    sync()
    with server(ctx, wl, idle_timeout_ms=30) as s:
        for i, r in enumerate(wl.reqs):
            t = submit_retry(s, r, d_in.data_ptr() + int(r["offset"]),
                             d_out.data_ptr() + int(r["offset"]))
            assert s.wait(t)["status"] == 0
            if i % 3 == 2:
                time.sleep(0.15)  # the kernel exits; the next submit relaunches it
        assert s.stats()["kernel_launches"] >= 3
        got = d_out.cpu().numpy()
    for r in wl.reqs:
        o, n = int(r["offset"]), int(r["length"])
        assert first_mismatch(got[o:o + n], oracle_request(wl, r, inp[o:o + n])) is None


def test_errors_and_callbacks(ctx):
    print("[gpu] serving errors and callbacks", flush=True)
    a = ag()
    wl = make_trace(20, seed=11)
    inp = wl.data()
    d_in = torch.from_numpy(inp).cuda()
    d_out = torch.empty_like(d_in)
    sync()
    iv = np.zeros(16, np.uint8)
    with server(ctx, wl) as s:
        p, q = d_in.data_ptr(), d_out.data_ptr()
        for args, status in (((0, 99, iv, p, q, 4096), a.AES_ERR_RANGE),
                             ((1, 0, iv, p, q, 4008), a.AES_ERR_LENGTH),
                             ((2, 0, iv, p, q, 0), a.AES_ERR_ARG),
                             ((5, 0, iv, p, q, 4096), a.AES_ERR_ARG),
                             ((2, 0, iv, p, p + 16, 4096), a.AES_ERR_OVERLAP)):
            with pytest.raises(a.AesError) as e:
                s.submit(*args)
            assert e.value.status == status
        with pytest.raises(a.AesError) as e:
            s.set_key(10_000, a.expand_key(bytes(16), 128))
        assert e.value.status == a.AES_ERR_RANGE
        seen = []
        for r in wl.reqs:
            while True:
                try:
                    s.submit(int(r["op"]), int(r["key_idx"]), r["iv"], p + int(r["offset"]),
                             q + int(r["offset"]), int(r["length"]),
                             callback=lambda rec: seen.append((int(rec["ticket"]),
                                                               int(rec["status"]))))
                    break
                except a.AesError as e2:
                    assert e2.status == a.AES_ERR_AGAIN
                    time.sleep(1e-4)
        deadline = time.time() + 20
        while len(seen) < wl.reqs.size and time.time() < deadline:
            time.sleep(1e-3)
        assert sorted(t for t, _ in seen) == list(range(wl.reqs.size))
        assert all(st == 0 for _, st in seen)
        got = d_out.cpu().numpy()
    for r in wl.reqs:
        o, n = int(r["offset"]), int(r["length"])
        assert first_mismatch(got[o:o + n], oracle_request(wl, r, inp[o:o + n])) is None


@pytest.mark.parametrize("engine", ENGINES)
def test_replay_poisson_trace(ctx, engine):
    print(f"[gpu] replay of a Poisson trace, engine={engine}", flush=True)
    tr = workloads.config4(20000.0, 400, n_slots=16)
    wl = workloads.Workload("cfg4", tr.reqs, tr.keys, tr.key_bits, tr.buf_bytes)
    inp = wl.data()
    d_in = torch.from_numpy(inp).cuda()
    d_out = torch.empty_like(d_in)
    sync()
    with server(ctx, wl, mode=engine) as s:
        done = s.replay(tr.reqs, tr.arrivals_s, d_in, d_out)
        got = d_out.cpu().numpy()
    assert (done["status"] == 0).all()
    lat = (done["t_done_ns"] - done["t_submit_ns"]) / 1e3
    assert (lat > 0).all() and np.median(lat) < 1e5
    for r in tr.reqs[::5]:
        o, n = int(r["offset"]), int(r["length"])
        assert first_mismatch(got[o:o + n], oracle_request(wl, r, inp[o:o + n])) is None


def expected_units(op, length, tile=4096, cap=128):
    """Work units of one request in the persistent engine: one per tile, or
    units of ceil(tiles / cap) tiles when it has more than cap tiles; one
    chain for CBC encryption."""
    if op == workloads.OP_CBC_ENC:
        return 1
    tiles = -(-length // tile)
    per_unit = -(-tiles // cap) if tiles > cap else 1
    return -(-length // (tile * per_unit))


@pytest.mark.parametrize("inplace", [False, True])
def test_large_requests_multi_tile_units(ctx, inplace):
    """Requests of more than 128 tiles through the persistent engine, which
    cuts them into about 128 units of several tiles each: every op, ragged CTR
    tails, a CTR counter that wraps mod 2^64 inside the request (across a unit
    boundary), sizes from 520 KiB to just under the 4 MiB request limit, each
    equal to the oracle byte for byte (in place as well)."""
    a = ag()
    print(f"\n[gpu] persistent engine, large requests, in place={inplace}", flush=True)
    sizes = [520 << 10, 1 << 20, (3 << 20) + 4096, (4 << 20) - 16]
    ops = [0, 1, 2, 3, 4]  # CBC-enc, CBC-dec, CTR, ECB-enc, ECB-dec
    n = len(sizes) * len(ops)
    reqs = np.zeros(n, workloads.REQ_DTYPE)
    for i in range(n):
        reqs["op"][i] = ops[i % len(ops)]
        ln = sizes[i // len(ops)]
        if reqs["op"][i] == workloads.OP_CTR:
            ln -= 5 + i  # ragged tail
        reqs["length"][i] = ln
    reqs["offset"][1:] = np.cumsum((reqs["length"] + 15) // 16 * 16 + 48)[:-1]
    reqs["key_idx"] = np.arange(n) % 4
    reqs["iv"] = gen.bytes_(9, gen.STREAM_IVS, 16 * n).reshape(n, 16)
    # A CTR request whose counter wraps 1,000 blocks in (inside its second unit).
    wrap = [i for i in range(n) if reqs["op"][i] == workloads.OP_CTR][1]
    reqs["iv"][wrap, 8:] = np.frombuffer(((1 << 64) - 1000).to_bytes(8, "big"), np.uint8)
    keys, kb = workloads.make_keys(9, 4, [128, 256, 192, 128])
    buf = int(reqs["offset"][-1] + reqs["length"][-1] + 64)
    wl = workloads.Workload("serve_large", reqs, keys, kb, buf, 9)
    src = wl.data()
    d_in = torch.from_numpy(src.copy()).cuda()
    d_out = d_in if inplace else torch.zeros_like(d_in)
    with server(ctx, wl, mode=a.AES_SERVE_PERSISTENT) as s:
        for r in wl.reqs:
            t = submit_retry(s, r, d_in.data_ptr() + int(r["offset"]),
                             d_out.data_ptr() + int(r["offset"]))
            done = s.wait(t)
            assert done["status"] == 0
            assert done["units"] == expected_units(int(r["op"]), int(r["length"]))
        st = s.stats()
    sync()
    got = d_out.cpu().numpy()
    for r in wl.reqs:
        o, ln = int(r["offset"]), int(r["length"])
        msg = first_mismatch(got[o:o + ln], oracle_request(wl, r, src[o:o + ln]))
        assert msg is None, f"op {int(r['op'])} length {ln}: {msg}"
    assert st["host_routed"] == 0


def make_all_ops_trace(n, seed):
    """n requests cycling through all five ops (CBC-enc, CBC-dec, CTR with a
    ragged tail, ECB-enc, ECB-dec), 4..64 KiB, four 128/256-bit key slots."""
    wl = make_trace(n, seed=seed, n_keys=4)
    r = wl.reqs
    r["op"] = np.arange(n) % 5
    r["length"] = (r["length"] + 15) // 16 * 16
    ctr = r["op"] == workloads.OP_CTR
    r["length"][ctr] -= np.uint64(7)
    r["offset"][1:] = np.cumsum((r["length"] + 15) // 16 * 16 + 64)[:-1]
    wl.buf_bytes = int(r["offset"][-1] + r["length"][-1] + 64)
    return wl


@pytest.mark.parametrize("n_wg", [1, 2, 4])
def test_small_persistent_grids(ctx, n_wg):
    """The persistent engine at 512, 1,024 and 2,048 threads (one, two and
    four 512-thread workgroups; section 3.1 of the paper measures its
    Non-Stop Kernel at those sizes): every op against the oracle, alone and
    in the mix.  One workgroup holds the encryption tables only, so its
    decryption requests take a normal launch (counted as fallbacks); from
    two workgroups on, every request runs in the persistent kernel."""
    print(f"[gpu] persistent grid of {n_wg} workgroup(s)", flush=True)
    wl = make_all_ops_trace(40, seed=41 + n_wg)
    inp = wl.data()
    d_in = torch.from_numpy(inp).cuda()
    sync()
    outs = {}
    with server(ctx, wl, mode=0, n_workgroups=n_wg) as s:
        for form in ("alone", "mix"):
            d_out = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
            sync()
            if form == "alone":
                for r in wl.reqs:
                    t = submit_retry(s, r, d_in.data_ptr() + int(r["offset"]),
                                     d_out.data_ptr() + int(r["offset"]))
                    assert s.wait(t)["status"] == 0
            else:
                ts = [submit_retry(s, r, d_in.data_ptr() + int(r["offset"]),
                                   d_out.data_ptr() + int(r["offset"])) for r in wl.reqs]
                for t in ts:
                    assert s.wait(t)["status"] == 0
            outs[form] = d_out.cpu().numpy()
        st = s.stats()
    n_dec = int(np.isin(wl.reqs["op"], [workloads.OP_CBC_DEC, 4]).sum())
    assert st["fallbacks"] == (2 * n_dec if n_wg == 1 else 0)
    assert st["kernel_launches"] >= 1
    assert first_mismatch(outs["alone"], outs["mix"]) is None
    for r in wl.reqs:
        o, n = int(r["offset"]), int(r["length"])
        msg = first_mismatch(outs["mix"][o:o + n], oracle_request(wl, r, inp[o:o + n]))
        assert msg is None, f"op {int(r['op'])} at {o}: {msg}"


def test_persistent_grid_limits(ctx):
    """Grids the device cannot hold at once, and table splits that leave a
    side without workgroups, are refused when the server is created (no
    kernel is launched before the first submit)."""
    print("[gpu] persistent grid limits", flush=True)
    a = ag()
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    for cfg in ({"n_workgroups": n_cu + 1}, {"n_workgroups": 4 * n_cu},
                {"n_workgroups": 1, "dec_workgroups": 1},
                {"n_workgroups": 2, "dec_workgroups": 2},
                {"n_workgroups": 8, "dec_workgroups": 8}):
        with pytest.raises(a.AesError) as e:
            a.Server(ctx, mode=0, **cfg)
        assert e.value.status == a.AES_ERR_ARG, cfg
    # the largest grid the device holds is accepted (and not launched here)
    a.Server(ctx, mode=0, n_workgroups=n_cu).close()


@pytest.mark.parametrize("engine", ENGINES)
def test_unloaded_key_slot(ctx, engine):
    """A key slot never loaded with aes_server_set_key is refused at submit
    (AES_ERR_STATE) rather than reaching the kernels with an empty schedule;
    loaded slots of the same server keep working."""
    print(f"[gpu] unloaded key slot, engine={engine}", flush=True)
    a = ag()
    wl = make_trace(6, seed=44, n_keys=4)
    inp = wl.data()
    d_in = torch.from_numpy(inp).cuda()
    d_out = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
    sync()
    scheds = a.expand_keys(wl.keys, wl.key_bits)
    with a.Server(ctx, mode=engine, key_slots=8) as s:
        for i in range(4):
            s.set_key(i, scheds[i])
        for slot in (4, 7):
            with pytest.raises(a.AesError) as e:
                s.submit(workloads.OP_CTR, slot, bytes(16), d_in.data_ptr(), d_out.data_ptr(),
                         4096)
            assert e.value.status == a.AES_ERR_STATE
        assert s.stats()["submitted"] == 0
        ts = [submit_retry(s, r, d_in.data_ptr() + int(r["offset"]),
                           d_out.data_ptr() + int(r["offset"])) for r in wl.reqs]
        for t in ts:
            assert s.wait(t)["status"] == 0
        got = d_out.cpu().numpy()
    for r in wl.reqs:
        o, n = int(r["offset"]), int(r["length"])
        assert first_mismatch(got[o:o + n], oracle_request(wl, r, inp[o:o + n])) is None


def test_batch_runs_beside_default_persistent_grid(ctx):
    """A batch launch issued while a persistent kernel of the default grid is
    live runs beside it (on the compute units the grid leaves free) instead
    of waiting for the kernel's idle exit; its bytes equal the oracle's.  The
    idle timeout is 10 s, so a launch held back until the exit would take
    that long; the bound here is 3 s."""
    print("[gpu] batch launch beside a live default persistent grid", flush=True)
    a = ag()
    wl = workloads.config2(workloads.OP_CTR, 128, n_pages=16384)
    inp = wl.data()
    d_in = torch.from_numpy(inp).cuda()
    d_out = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
    scheds = a.expand_keys(wl.keys, wl.key_bits)
    d_s = a.schedules_to_device(scheds, torch.device("cuda:0"))
    plan = a.Plan(ctx, wl.reqs, wl.keys.shape[0], wl.buf_bytes)
    small = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    sync()
    with a.Server(ctx, mode=a.AES_SERVE_PERSISTENT, key_slots=1, idle_timeout_ms=10000) as srv:
        srv.set_key(0, scheds[0])
        done = srv.wait(srv.submit(workloads.OP_CTR, 0, bytes(16), small, small, 4096))
        assert done["status"] == 0
        t0 = time.perf_counter()
        plan.launch(d_s, d_in, d_out)
        sync()
        took = time.perf_counter() - t0
    plan.close()
    assert took < 3.0, f"the batch launch waited {took:.2f} s beside the persistent kernel"
    want = workloads.sentinel(inp.size)
    oracle.batch(inp, want, wl.reqs, wl.keys, wl.key_bits, n_threads=0)
    msg = first_mismatch(d_out.cpu().numpy(), want)
    assert msg is None, msg


def test_set_key_rejects_a_mismatched_round_count(ctx):
    """aes_server_set_key refuses a schedule whose round count does not match
    its key size (AES_ERR_KEYSIZE): the persistent engine takes the round
    count recorded at set_key with every request."""
    print("[gpu] set_key round-count check", flush=True)
    a = ag()
    keys, kb = workloads.make_keys(0, 1, 128)
    sch = a.expand_keys(keys, kb)
    bad = sch.copy()
    bad["nr"] = 12
    with a.Server(ctx, mode=a.AES_SERVE_PERSISTENT, key_slots=1) as srv:
        with pytest.raises(a.AesError) as e:
            srv.set_key(0, bad[0])
        assert e.value.status == a.AES_ERR_KEYSIZE
        srv.set_key(0, sch[0])
