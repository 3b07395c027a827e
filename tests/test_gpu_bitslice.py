"""GPU parity of the bitsliced CTR variant (launch config ctr_variant =
AES_CTR_BITSLICE): byte for byte against the CPU oracle (tolerance 0), and
against the table variant on the full 65,536-page workload.

Cases: all three key sizes, ragged lengths (1..15-byte final blocks), zero-
length requests, counters that wrap mod 2^64 inside a lane's blocks, tiles of
4, 8 and 16 KiB (the kernel works units in 4 KiB chunks), waves whose 8 units
carry different keys (one pass per key), in-place runs, and CTR inside mixed
batches with the fused kernel on and off."""
import numpy as np
import pytest
import torch

import oracle
from synth import gen, workloads
from tests.gpu_util import ag, device_schedules, first_mismatch, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("\n[gpu] context for bitsliced tests", flush=True)
    c = ag().Context(0)
    yield c
    c.close()


@pytest.fixture()
def bs(ctx):
    """The context switched to the bitsliced CTR variant for one test."""
    cfg = ctx.get_config()
    ctx.set_config(ctr_variant=ag().AES_CTR_BITSLICE)
    yield ctx
    ctx.set_config(**cfg)


def check(got, want, what):
    msg = first_mismatch(got, want)
    assert msg is None, f"{what}: {msg}"


def ctr_workload(lengths, key_idx, key_bits, seed=0, wrap_at=()):
    """CTR requests with the given lengths and key indices over one buffer
    (64-byte gaps); requests listed in wrap_at get a counter 3 blocks short
    of 2^64."""
    n = len(lengths)
    reqs = np.zeros(n, workloads.REQ_DTYPE)
    reqs["length"] = np.asarray(lengths, np.uint64)
    reqs["offset"][1:] = np.cumsum((reqs["length"] + 15) // 16 * 16 + 64)[:-1]
    reqs["op"] = workloads.OP_CTR
    reqs["key_idx"] = np.asarray(key_idx, np.uint32)
    reqs["iv"] = gen.bytes_(seed, gen.STREAM_IVS, 16 * n).reshape(n, 16)
    for i in wrap_at:
        reqs["iv"][i, 8:] = np.frombuffer(((1 << 64) - 3).to_bytes(8, "big"), np.uint8)
    keys, kb = workloads.make_keys(seed, len(key_bits), list(key_bits))
    buf = int(reqs["offset"][-1] + reqs["length"][-1] + 64)
    return workloads.Workload("ctr_bs", reqs, keys, kb, buf, seed)


def test_config_switch_round_trips(ctx):
    a = ag()
    cfg = ctx.get_config()
    assert cfg["ctr_variant"] == a.AES_CTR_TABLE
    ctx.set_config(ctr_variant=a.AES_CTR_BITSLICE)
    assert ctx.get_config()["ctr_variant"] == a.AES_CTR_BITSLICE
    with pytest.raises(a.AesError) as e:
        ctx.set_config(ctr_variant=2)
    assert e.value.status == a.AES_ERR_ARG
    ctx.set_config(**cfg)


@pytest.mark.parametrize("bits", [128, 192, 256])
@pytest.mark.parametrize("form", ["batch", "plan", "single"])
def test_pages_all_key_sizes(bs, bits, form):
    print(f"[gpu] bitsliced pages bits={bits} form={form}", flush=True)
    wl = workloads.config2(workloads.OP_CTR, bits, n_pages=700)
    inp = wl.data()
    check(run_gpu(bs, wl, inp, form=form), run_oracle(wl, inp), f"{bits} {form}")


def test_ragged_zero_and_wrap(bs):
    print("[gpu] bitsliced ragged, zero-length, wrap", flush=True)
    lengths = [1, 15, 16, 17, 4095, 4096, 4097, 3 * 4096 + 5, 0, 16 * 1000 + 9, 127, 4096 * 2]
    n = len(lengths)
    wl = ctr_workload(lengths, np.arange(n) % 3, [128, 192, 256], seed=4, wrap_at=(2, 5, 9))
    inp = wl.data()
    want = run_oracle(wl, inp)
    for form in ("batch", "plan"):
        check(run_gpu(bs, wl, inp, form=form), want, form)


@pytest.mark.parametrize("tile", [4096, 8192, 16384])
def test_tile_sizes_chunk_loop(bs, tile):
    print(f"[gpu] bitsliced tile={tile}", flush=True)
    bs.set_config(tile_bytes=tile)
    r = np.random.default_rng(tile)
    lengths = r.integers(1, 40000, 90)
    wl = ctr_workload(lengths, r.integers(0, 4, 90), [128, 256, 192, 128], seed=tile,
                      wrap_at=(7,))
    inp = wl.data()
    check(run_gpu(bs, wl, inp, form="plan"), run_oracle(wl, inp), f"tile {tile}")


def test_waves_with_mixed_keys(bs):
    """Runs of 3 units per key: most waves' 8 units span three keys, so the
    kernel makes several key passes per chunk and stores each lane once."""
    print("[gpu] bitsliced mixed keys per wave", flush=True)
    n = 150
    wl = ctr_workload([4096] * n, np.arange(n) // 3 % 50, [128, 192, 256] * 16 + [128, 256],
                      seed=8)
    inp = wl.data()
    check(run_gpu(bs, wl, inp, form="batch"), run_oracle(wl, inp), "mixed keys")


def test_in_place(bs):
    print("[gpu] bitsliced in place", flush=True)
    wl = ctr_workload([5000, 4096, 77, 12288, 33], [0, 1, 0, 1, 0], [256, 128], seed=12)
    inp = wl.data()
    want = run_oracle(wl, inp, inplace=True)
    for form in ("batch", "plan"):
        check(run_gpu(bs, wl, inp, form=form, inplace=True), want, f"in place {form}")


@pytest.mark.parametrize("fuse", [1, 0])
def test_mixed_batch(bs, fuse):
    """CTR through the bitsliced kernel beside CBC units in the fused (or
    split) table kernels of the same batch."""
    print(f"[gpu] bitsliced in a mixed batch, fuse={fuse}", flush=True)
    bs.set_config(fuse=fuse)
    wl = workloads.config3(n_reqs=240, max_pages=10)
    wl.key_bits[::3] = 192
    ctr = wl.reqs["op"] == workloads.OP_CTR
    wl.reqs["length"][ctr] -= (np.arange(ctr.sum()) * 7 % 16).astype(np.uint64)
    inp = wl.data()
    want = run_oracle(wl, inp)
    for form in ("batch", "plan"):
        check(run_gpu(bs, wl, inp, form=form), want, f"mixed {form}")


@pytest.mark.parametrize("bits", [128, 256])
def test_full_size_equals_table_variant(ctx, bits):
    """65,536 pages of 4 KiB with 16 keys round-robin, in the benchmark's
    plan-launch form: the two variants' outputs are identical over all 256
    MiB, and 200 sampled pages match the oracle."""
    print(f"[gpu] bitsliced vs table, full size, bits={bits}", flush=True)
    a = ag()
    wl = workloads.config2(workloads.OP_CTR, bits)
    inp = wl.data()
    d_s = device_schedules(wl)
    d_in = torch.from_numpy(inp).cuda()
    outs = {}
    cfg = ctx.get_config()
    try:
        for v in (a.AES_CTR_TABLE, a.AES_CTR_BITSLICE):
            ctx.set_config(ctr_variant=v)
            d_out = torch.empty_like(d_in)
            plan = a.Plan(ctx, wl.reqs, 16, wl.buf_bytes)
            plan.launch(d_s, d_in, d_out)
            torch.cuda.synchronize()
            plan.close()
            outs[v] = d_out
    finally:
        ctx.set_config(**cfg)
    assert torch.equal(outs[a.AES_CTR_TABLE], outs[a.AES_CTR_BITSLICE]), "variants differ"
    got = outs[a.AES_CTR_BITSLICE].cpu().numpy()
    rng = np.random.default_rng(5)
    for p in np.unique(np.concatenate([[0, wl.reqs.size - 1],
                                       rng.choice(wl.reqs.size, 200, replace=False)])):
        r = wl.reqs[p]
        o, n = int(r["offset"]), int(r["length"])
        kb = int(wl.key_bits[r["key_idx"]])
        want = oracle.mode(int(r["op"]), wl.keys[r["key_idx"]][: kb // 8], kb, r["iv"],
                           inp[o:o + n])
        check(got[o:o + n], want, f"page {p}")
