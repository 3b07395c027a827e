"""GPU parity of the bitsliced decryption variant (launch config dec_variant
= AES_DEC_BITSLICE): CBC and ECB decryption byte for byte against the CPU
oracle (tolerance 0), and against the table variant at full config-2 size.

Cases: all three key sizes in every form, requests of one block to several
tiles (tiles of 4, 8 and 16 KiB: the kernel works units in 4 KiB chunks and
carries the chaining block from one chunk to the next), zero-length
requests, waves whose 8 units carry different keys (one pass per key), in
place (the stores run from a chunk's last block to its first, and tiles after
the first take their predecessor from the snapshot), ECB decryption, and
decryption inside mixed batches with the fused kernel on and off."""
import os

import numpy as np
import pytest
import torch

import oracle
from synth import gen, workloads
from tests.gpu_util import ag, device_schedules, first_mismatch, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

OP_ECB_DEC = 4


@pytest.fixture(scope="module")
def ctx():
    print("\n[gpu] context for bitsliced decryption tests", flush=True)
    c = ag().Context(0)
    yield c
    c.close()


@pytest.fixture()
def bsd(ctx):
    """The context switched to the bitsliced decryption variant for one test."""
    cfg = ctx.get_config()
    ctx.set_config(dec_variant=ag().AES_DEC_BITSLICE)
    yield ctx
    ctx.set_config(**cfg)


def check(got, want, what):
    msg = first_mismatch(got, want)
    assert msg is None, f"{what}: {msg}"


def dec_workload(lengths, key_idx, key_bits, ops=None, seed=0):
    """Decryption requests (CBC unless ops says otherwise) with the given
    lengths (whole blocks) and key indices over one buffer, 64-byte gaps."""
    n = len(lengths)
    reqs = np.zeros(n, workloads.REQ_DTYPE)
    reqs["length"] = np.asarray(lengths, np.uint64)
    reqs["offset"][1:] = np.cumsum(reqs["length"] + 64)[:-1]
    reqs["op"] = workloads.OP_CBC_DEC if ops is None else np.asarray(ops, np.uint32)
    reqs["key_idx"] = np.asarray(key_idx, np.uint32)
    reqs["iv"] = gen.bytes_(seed, gen.STREAM_IVS, 16 * n).reshape(n, 16)
    keys, kb = workloads.make_keys(seed, len(key_bits), list(key_bits))
    buf = int(reqs["offset"][-1] + reqs["length"][-1] + 64)
    return workloads.Workload("dec_bs", reqs, keys, kb, buf, seed)


def test_config_switch_round_trips(ctx):
    a = ag()
    cfg = ctx.get_config()
    assert cfg["dec_variant"] == a.AES_DEC_TABLE
    ctx.set_config(dec_variant=a.AES_DEC_BITSLICE)
    assert ctx.get_config()["dec_variant"] == a.AES_DEC_BITSLICE
    with pytest.raises(a.AesError) as e:
        ctx.set_config(dec_variant=2)
    assert e.value.status == a.AES_ERR_ARG
    ctx.set_config(**cfg)
    assert ctx.get_config()["dec_variant"] == a.AES_DEC_TABLE


@pytest.mark.parametrize("bits", [128, 192, 256])
@pytest.mark.parametrize("form", ["batch", "plan", "single"])
def test_pages_all_key_sizes(bsd, bits, form):
    print(f"[gpu] bitsliced CBC-dec pages bits={bits} form={form}", flush=True)
    wl = workloads.config2(workloads.OP_CBC_DEC, bits, n_pages=700)
    inp = wl.data()
    check(run_gpu(bsd, wl, inp, form=form), run_oracle(wl, inp), f"{bits} {form}")


@pytest.mark.parametrize("tile", [4096, 8192, 16384])
def test_lengths_and_tile_sizes(bsd, tile):
    """One block up to 13 tiles per request, zero-length requests; with 8
    and 16 KiB tiles a unit spans 2 and 4 chunks of the kernel."""
    print(f"[gpu] bitsliced CBC-dec tile={tile}", flush=True)
    bsd.set_config(tile_bytes=tile)
    u = gen.uniform(tile, gen.STREAM_SIZES, 90)
    lengths = (1 + (u * 3300).astype(np.int64)) * 16
    lengths[[5, 40]] = 0
    lengths[7] = 16
    lengths[8] = 13 * tile
    wl = dec_workload(lengths, np.arange(90) % 4, [128, 256, 192, 128], seed=tile)
    inp = wl.data()
    want = run_oracle(wl, inp)
    for form in ("plan", "batch"):
        check(run_gpu(bsd, wl, inp, form=form), want, f"tile {tile} {form}")


def test_waves_with_mixed_keys(bsd):
    """Keys in runs of 3 units (the planner groups by key, but runs shorter
    than 8 still leave several keys per wave): several key passes per chunk,
    each lane stored once."""
    print("[gpu] bitsliced CBC-dec, mixed keys per wave", flush=True)
    n = 150
    wl = dec_workload([4096] * n, np.arange(n) // 3 % 50, [128, 192, 256] * 16 + [128, 256],
                      seed=8)
    inp = wl.data()
    check(run_gpu(bsd, wl, inp, form="batch"), run_oracle(wl, inp), "mixed keys")


@pytest.mark.parametrize("tile", [4096, 16384])
def test_in_place(bsd, tile):
    print(f"[gpu] bitsliced CBC-dec in place, tile={tile}", flush=True)
    bsd.set_config(tile_bytes=tile)
    wl = dec_workload([5008, 4096, 80, 12288, 32, 65536, 40960 + 16], [0, 1, 0, 1, 0, 1, 0],
                      [256, 128], seed=12)
    inp = wl.data()
    want = run_oracle(wl, inp, inplace=True)
    for form in ("batch", "plan"):
        check(run_gpu(bsd, wl, inp, form=form, inplace=True), want, f"in place {form}")


def test_ecb_decrypt(bsd):
    print("[gpu] bitsliced ECB-dec and CBC-dec together", flush=True)
    lengths = [4096, 16, 8192 + 48, 4096 * 5, 4096]
    wl = dec_workload(lengths, [0, 1, 2, 0, 1], [128, 192, 256],
                      ops=[OP_ECB_DEC, OP_ECB_DEC, workloads.OP_CBC_DEC, OP_ECB_DEC,
                           workloads.OP_CBC_DEC], seed=21)
    inp = wl.data()
    want = run_oracle(wl, inp)
    for form in ("batch", "plan"):
        check(run_gpu(bsd, wl, inp, form=form), want, f"ecb {form}")
    check(run_gpu(bsd, wl, inp, form="batch", inplace=True), run_oracle(wl, inp, inplace=True),
          "ecb in place")


@pytest.mark.parametrize("fuse", [1, 0])
def test_mixed_batch(bsd, fuse):
    """Decryption through the bitsliced kernel beside CBC-encrypt chains and
    CTR tiles in the fused (or split) table kernels of the same batch."""
    print(f"[gpu] bitsliced CBC-dec in a mixed batch, fuse={fuse}", flush=True)
    bsd.set_config(fuse=fuse)
    wl = workloads.config3(n_reqs=240, max_pages=10)
    wl.key_bits[::3] = 192
    inp = wl.data()
    want = run_oracle(wl, inp)
    for form in ("batch", "plan"):
        check(run_gpu(bsd, wl, inp, form=form), want, f"mixed {form}")


@pytest.mark.parametrize("bits", [128, 256])
def test_full_size_against_oracle_and_table(ctx, bits):
    """65,536 pages of 4 KiB with 16 keys round-robin, in the benchmark's
    plan-launch form: every page against the oracle, and the two variants'
    outputs identical over all 256 MiB."""
    print(f"[gpu] bitsliced CBC-dec full size, bits={bits}", flush=True)
    a = ag()
    wl = workloads.config2(workloads.OP_CBC_DEC, bits)
    inp = wl.data()
    d_s = device_schedules(wl)
    d_in = torch.from_numpy(inp).cuda()
    outs = {}
    cfg = ctx.get_config()
    try:
        for v in (a.AES_DEC_TABLE, a.AES_DEC_BITSLICE):
            ctx.set_config(dec_variant=v)
            d_out = torch.empty_like(d_in)
            plan = a.Plan(ctx, wl.reqs, 16, wl.buf_bytes)
            plan.launch(d_s, d_in, d_out)
            torch.cuda.synchronize()
            plan.close()
            outs[v] = d_out
    finally:
        ctx.set_config(**cfg)
    assert torch.equal(outs[a.AES_DEC_TABLE], outs[a.AES_DEC_BITSLICE]), "variants differ"
    want = np.empty_like(inp)
    oracle.batch(inp, want, wl.reqs, wl.keys, wl.key_bits,
                 n_threads=len(os.sched_getaffinity(0)))
    check(outs[a.AES_DEC_BITSLICE].cpu().numpy(), want, "all 65,536 pages")
