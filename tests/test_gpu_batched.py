"""GPU parity of the batched forms: the fused one-launch kernel for mixed
batches, every tile/chain launch shape, per-request launches, HIP graphs of
both, and the autotuner -- all byte for byte against the CPU oracle."""
import numpy as np
import pytest
import torch

from synth import gen, workloads
from tests.gpu_util import ag, device_schedules, first_mismatch, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("\n[gpu] context for batched tests", flush=True)
    c = ag().Context(0)
    yield c
    c.close()


@pytest.fixture()
def fresh(ctx):
    """Restores the default launch configuration after a test."""
    cfg = ctx.get_config()
    yield ctx
    ctx.set_config(**cfg)


def check(got, want, what):
    msg = first_mismatch(got, want)
    assert msg is None, f"{what}: {msg}"


def mixed_workload(n=300, max_pages=12, three_sizes=True):
    wl = workloads.config3(n_reqs=n, max_pages=max_pages)
    if three_sizes:  # use 192-bit keys as well
        wl.key_bits[::3] = 192
    # ragged CTR lengths
    ctr = wl.reqs["op"] == workloads.OP_CTR
    wl.reqs["length"][ctr] -= (np.arange(ctr.sum()) * 5 % 16).astype(np.uint64)
    return wl


@pytest.mark.parametrize("fuse", [1, 0])
@pytest.mark.parametrize("mixed_nb", [1, 2])
@pytest.mark.parametrize("chain_lanes", [16, 64])
def test_mixed_batch_fused_and_split(fresh, fuse, mixed_nb, chain_lanes):
    print(f"[gpu] mixed fuse={fuse} nb={mixed_nb} lanes={chain_lanes}", flush=True)
    fresh.set_config(fuse=fuse, mixed_nb=mixed_nb, chain_lanes=chain_lanes, chain_quad=0)
    wl = mixed_workload()
    inp = wl.data()
    want = run_oracle(wl, inp)
    for form in ("batch", "plan"):
        check(run_gpu(fresh, wl, inp, form=form), want, f"mixed {form}")


@pytest.mark.parametrize("fuse", [1, 0])
def test_chains_on_four_lanes(fresh, fuse):
    """CBC-encrypt chains 16 per wave on four lanes each (chain_quad = 1):
    uneven chains of all three key sizes, alone and inside a mixed batch."""
    print(f"[gpu] four-lane chains, fuse={fuse}", flush=True)
    fresh.set_config(chain_quad=1, fuse=fuse)
    wl = mixed_workload()
    inp = wl.data()
    want = run_oracle(wl, inp)
    for form in ("batch", "plan"):
        check(run_gpu(fresh, wl, inp, form=form), want, f"mixed {form}")
    enc = wl.reqs[wl.reqs["op"] == workloads.OP_CBC_ENC][:37]
    check(run_gpu(fresh, wl, inp, reqs=enc), run_oracle(wl, inp, reqs=enc), "chains only")
    check(run_gpu(fresh, wl, inp, reqs=enc, inplace=True),
          run_oracle(wl, inp, reqs=enc, inplace=True), "chains in place")


@pytest.mark.parametrize("ops", [(0, 1), (0, 2), (1, 2), (0,), (1,), (2,)])
def test_fused_kernel_op_subsets(fresh, ops):
    """Subsets with CBC-encrypt chains run fused; (1, 2) has none and runs as
    one launch per table set."""
    print(f"[gpu] op subset {ops}", flush=True)
    wl = mixed_workload(n=160, max_pages=6)
    r = np.random.default_rng(len(ops)).integers(0, len(ops), wl.reqs.size)
    wl.reqs["op"] = np.array(ops, np.uint32)[r]
    cbc = wl.reqs["op"] != workloads.OP_CTR
    wl.reqs["length"][cbc] = (wl.reqs["length"][cbc] + 15) // 16 * 16
    wl.reqs["length"][cbc] = np.minimum(wl.reqs["length"][cbc],
                                        np.diff(np.append(wl.reqs["offset"], wl.buf_bytes))[cbc])
    inp = wl.data()
    check(run_gpu(fresh, wl, inp), run_oracle(wl, inp), f"ops {ops}")


def test_mixed_in_place_fused(fresh):
    print("[gpu] mixed in place, fused", flush=True)
    wl = workloads.config3(n_reqs=200, max_pages=10)
    inp = wl.data()
    want = run_oracle(wl, inp, inplace=True)
    for form in ("batch", "plan"):
        check(run_gpu(fresh, wl, inp, form=form, inplace=True), want, f"in-place {form}")


@pytest.mark.parametrize("nb,wg", [(1, 256), (1, 512), (1, 1024), (2, 256), (2, 512), (2, 1024),
                                   (4, 256), (4, 512)])
@pytest.mark.parametrize("tile", [4096, 8192, 16384])
def test_tile_shapes(fresh, nb, wg, tile):
    print(f"[gpu] tile shape nb={nb} wg={wg} tile={tile}", flush=True)
    fresh.set_config(ctr_nb=nb, ctr_wg=wg, dec_nb=nb, dec_wg=wg, tile_bytes=tile, fuse=0)
    wl = mixed_workload(n=120, max_pages=9)
    inp = wl.data()
    check(run_gpu(fresh, wl, inp), run_oracle(wl, inp), f"nb={nb} wg={wg} tile={tile}")


def test_per_request_launches(fresh):
    print("[gpu] per-request launches", flush=True)
    a = ag()
    wl = mixed_workload(n=80, max_pages=20)
    inp = wl.data()
    d_s = device_schedules(wl)
    d_in = torch.from_numpy(inp).cuda()
    d_out = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
    for r in wl.reqs:
        a.request_launch(fresh, d_s, d_in, d_out, r)
    torch.cuda.synchronize()
    check(d_out.cpu().numpy(), run_oracle(wl, inp), "per-request")


def test_per_request_in_place_multi_tile_cbc_decrypt(fresh):
    print("[gpu] per-request in place CBC-dec", flush=True)
    a = ag()
    reqs = np.zeros(3, workloads.REQ_DTYPE)
    reqs["length"] = [5 * 4096, 4096, 37 * 16]
    reqs["offset"] = [0, 5 * 4096, 6 * 4096]
    reqs["op"] = workloads.OP_CBC_DEC
    reqs["key_idx"] = [0, 1, 0]
    reqs["iv"] = gen.bytes_(0, gen.STREAM_IVS, 48).reshape(3, 16)
    keys, kb = workloads.make_keys(0, 2, [128, 256])
    wl = workloads.Workload("pr", reqs, keys, kb, 7 * 4096)
    inp = wl.data()
    d_s = device_schedules(wl)
    d = torch.from_numpy(inp.copy()).cuda()
    for r in reqs:
        a.request_launch(fresh, d_s, d, d, r)
    torch.cuda.synchronize()
    check(d.cpu().numpy(), run_oracle(wl, inp, inplace=True), "per-request in place")


def test_graphs_replay(fresh):
    """Each replay is checked, with eager GPU work and synchronisation between."""
    print("[gpu] graph replays", flush=True)
    a = ag()
    wl = mixed_workload(n=150, max_pages=8)
    inp = wl.data()
    want = run_oracle(wl, inp)
    d_s = device_schedules(wl)
    d_in = torch.from_numpy(inp).cuda()
    d_out = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
    sentinel = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
    plan = a.Plan(fresh, wl.reqs, wl.keys.shape[0], wl.buf_bytes)
    g1 = a.Graph.of_plan(plan, d_s, d_in, d_out)
    g2 = a.Graph.of_requests(fresh, d_s, d_in, d_out, wl.reqs)
    for rep in range(3):
        for name, g in (("plan graph", g1), ("requests graph", g2)):
            d_out.copy_(sentinel)  # eager work between replays
            torch.cuda.synchronize()
            g.launch()
            torch.cuda.synchronize()
            check(d_out.cpu().numpy(), want, f"{name} replay {rep}")
    g1.close()
    g2.close()
    plan.close()


def test_tune_then_plan(fresh):
    print("[gpu] autotuner", flush=True)
    a = ag()
    wl = mixed_workload(n=200, max_pages=16)
    inp = wl.data()
    want = run_oracle(wl, inp)
    d_s = device_schedules(wl)
    d_in = torch.from_numpy(inp).cuda()
    d_out = torch.empty_like(d_in)
    best = a.tune(fresh, wl.reqs, d_s, d_in, d_out, iters=2)
    assert fresh.get_config() == best
    check(run_gpu(fresh, wl, inp, form="plan"), want, f"after tuning {best}")
    with pytest.raises(a.AesError):
        a.tune(fresh, wl.reqs, d_s, d_in, d_in, iters=1)


def test_tune_leaves_unused_knobs():
    """The tuner tries only knobs the batch's launch uses: with chains and
    tiles in one fused launch the tile-kernel shapes keep their starting
    values; a batch without chains keeps its chain and fused-kernel
    settings."""
    print("[gpu] tuner skips unused knobs", flush=True)
    a = ag()
    shapes = ("ctr_nb", "ctr_wg", "dec_nb", "dec_wg")
    wl = mixed_workload(n=120, max_pages=8)
    inp = wl.data()
    d_s = device_schedules(wl)
    d_in = torch.from_numpy(inp).cuda()
    d_out = torch.empty_like(d_in)
    c = a.Context(0)
    c.set_config(ctr_nb=1, ctr_wg=512, dec_nb=1, dec_wg=512)
    start = c.get_config()
    best = a.tune(c, wl.reqs, d_s, d_in, d_out, iters=1)
    if best["fuse"]:
        assert {k: best[k] for k in shapes} == {k: start[k] for k in shapes}
    c.close()
    par = wl.reqs[wl.reqs["op"] != workloads.OP_CBC_ENC]
    c = a.Context(0)
    c.set_config(chain_lanes=32, chain_quad=0, mixed_nb=2)
    best = a.tune(c, par, d_s, d_in, d_out, iters=1)
    assert (best["chain_lanes"], best["chain_quad"], best["mixed_nb"]) == (32, 0, 2)
    check(run_gpu(c, wl, inp, form="plan", reqs=par), run_oracle(wl, inp, reqs=par),
          f"tuned {best}")
    c.close()


def test_tune_cache_store_then_hit(tmp_path, monkeypatch):
    """With AESGPU_TUNE_CACHE set, a tuning run stores its result under the
    batch's signature; a new context tuning a batch of the same shape gets the
    stored configuration without a tuning run (the file is not rewritten),
    and its plan still matches the oracle."""
    print("[gpu] tune cache", flush=True)
    import time
    a = ag()
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("AESGPU_TUNE_CACHE", str(path))
    wl = mixed_workload(n=200, max_pages=16)
    inp = wl.data()
    d_s = device_schedules(wl)
    d_in = torch.from_numpy(inp).cuda()
    d_out = torch.empty_like(d_in)
    c1 = a.Context(0)
    c1.set_config(ctr_nb=1, ctr_wg=512)  # a start the tuner may or may not keep
    t0 = time.perf_counter()
    best = a.tune(c1, wl.reqs, d_s, d_in, d_out, iters=2)
    t_tune = time.perf_counter() - t0
    sig = a.tune_key(c1, wl.reqs, wl.keys.shape[0])
    assert sig.startswith("arch=gfx")
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].split("\t")[0] == sig
    assert [int(x) for x in lines[0].split("\t")[1].split()] == [
        best[k] for k in ("tile_bytes", "ctr_nb", "ctr_wg", "dec_nb", "dec_wg", "chain_lanes",
                          "chain_wg", "mixed_nb", "fuse", "grid", "ctr_variant", "chain_quad")]
    mtime = path.stat().st_mtime_ns
    c2 = a.Context(0)
    t0 = time.perf_counter()
    hit = a.tune(c2, wl.reqs, d_s, d_in, d_out, iters=2)
    t_hit = time.perf_counter() - t0
    assert hit == best and c2.get_config() == best
    assert path.stat().st_mtime_ns == mtime
    print(f"[gpu] tuning {t_tune * 1e3:.1f} ms, cache hit {t_hit * 1e3:.2f} ms", flush=True)
    assert t_hit < t_tune
    check(run_gpu(c2, wl, inp, form="plan"), run_oracle(wl, inp), f"cached config {hit}")
    c1.close()
    c2.close()


def test_config3_full_size(fresh):
    """The full config-3 batch (10,000 requests, about 1.75 GiB) in one fused
    launch, every request against the oracle (its threaded batch over the
    whole buffer, CBC-encrypt chains included)."""
    print("[gpu] config 3 full size", flush=True)
    import os

    import oracle
    a = ag()
    wl = workloads.config3()
    d_in = gen.bytes_torch(0, gen.STREAM_DATA, (wl.buf_bytes + 7) // 8 * 8, "cuda")[: wl.buf_bytes]
    d_out = torch.empty_like(d_in)
    d_s = device_schedules(wl)
    plan = a.Plan(fresh, wl.reqs, wl.keys.shape[0], wl.buf_bytes)
    plan.launch(d_s, d_in, d_out)
    torch.cuda.synchronize()
    plan.close()
    got = d_out.cpu().numpy()
    del d_out
    inp = gen.bytes_(0, gen.STREAM_DATA, wl.buf_bytes)
    assert np.array_equal(d_in[:4096].cpu().numpy(), inp[:4096])  # same seeded bytes
    del d_in
    print("[gpu] config 3: oracle over the whole batch", flush=True)
    want = np.zeros_like(inp)  # config 3 packs requests back to back: no gaps
    oracle.batch(inp, want, wl.reqs, wl.keys, wl.key_bits, n_threads=len(os.sched_getaffinity(0)))
    check(got, want, "all 10,000 requests")
