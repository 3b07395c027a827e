"""GPU parity: the HIP path through the C ABI against the CPU oracle, byte for
byte (AES is a permutation, so the tolerance is zero bytes).

Sizes span several workgroups and waves and a ragged tail; the benchmark's
full-size shape is checked on every page.
"""
import os

import numpy as np
import pytest
import torch

import oracle
from synth import gen, workloads
from tests.gpu_util import ag, device_schedules, first_mismatch, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("\n[gpu] creating context on device 0", flush=True)
    c = ag().Context(0)
    yield c
    c.close()


def check(got, want, what):
    msg = first_mismatch(got, want)
    assert msg is None, f"{what}: {msg}"


def test_config1_cbc_encrypt_then_decrypt(ctx):
    print("[gpu] config 1: 256 x 4 KiB AES-128-CBC enc then dec", flush=True)
    enc, dec = workloads.config1()
    p = enc.data()
    c_gpu = run_gpu(ctx, enc, p, form="single")
    check(c_gpu, run_oracle(enc, p), "cbc encrypt")
    p_gpu = run_gpu(ctx, dec, c_gpu, form="single")
    check(p_gpu, run_oracle(dec, c_gpu), "cbc decrypt")
    check(p_gpu, p, "round trip")


@pytest.mark.parametrize("op", [workloads.OP_CBC_DEC, workloads.OP_CTR])
@pytest.mark.parametrize("bits", [128, 192, 256])
@pytest.mark.parametrize("form", ["single", "batch", "plan"])
def test_pages_small(ctx, op, bits, form):
    # 1,100 pages: more units than one pass of the grid's waves needs for
    # small grids, with 16 keys round-robin.
    print(f"[gpu] pages op={op} bits={bits} form={form}", flush=True)
    wl = workloads.config2(op, bits, n_pages=1100)
    inp = wl.data()
    check(run_gpu(ctx, wl, inp, form=form), run_oracle(wl, inp), f"{form} op={op} bits={bits}")


@pytest.mark.parametrize("bits", [128, 192, 256])
def test_cbc_encrypt_chains_uneven(ctx, bits):
    print(f"[gpu] uneven CBC-enc chains bits={bits}", flush=True)
    n = 300
    u = gen.uniform(0, gen.STREAM_SIZES, n)
    blocks = (1 + (u * 700).astype(np.uint64))
    reqs = np.zeros(n, workloads.REQ_DTYPE)
    reqs["length"] = blocks * 16
    reqs["offset"][1:] = np.cumsum(reqs["length"] + 32)[:-1]
    reqs["op"] = workloads.OP_CBC_ENC
    reqs["key_idx"] = np.arange(n) % 5
    reqs["iv"] = gen.bytes_(0, gen.STREAM_IVS, 16 * n).reshape(n, 16)
    keys, kb = workloads.make_keys(0, 5, bits)
    buf = int(reqs["offset"][-1] + reqs["length"][-1] + 48)
    wl = workloads.Workload("chains", reqs, keys, kb, buf)
    inp = wl.data()
    check(run_gpu(ctx, wl, inp), run_oracle(wl, inp), "chains")


def test_config3_mixed_small_full_check(ctx):
    print("[gpu] config 3 shape, 400 requests up to 16 pages, full check", flush=True)
    wl = workloads.config3(n_reqs=400, max_pages=16)
    inp = wl.data()
    want = run_oracle(wl, inp)
    for form in ("batch", "plan"):
        check(run_gpu(ctx, wl, inp, form=form), want, f"mixed {form}")


def test_ragged_ctr_tails_and_counter_wrap(ctx):
    print("[gpu] ragged CTR lengths and 64-bit counter wrap", flush=True)
    lens = [1, 15, 16, 17, 100, 1023, 4095, 4096, 4097, 8191, 3 * 4096 + 5, 20000, 65536 + 9]
    n = len(lens)
    reqs = np.zeros(n, workloads.REQ_DTYPE)
    off = 0
    for i, ln in enumerate(lens):
        reqs["offset"][i] = off
        reqs["length"][i] = ln
        off += (ln + 15) // 16 * 16 + 16 * (i % 3)
    reqs["op"] = workloads.OP_CTR
    reqs["key_idx"] = np.arange(n) % 3
    reqs["iv"] = gen.bytes_(0, gen.STREAM_IVS, 16 * n).reshape(n, 16)
    # wrap inside the first tile, at a tile boundary, and inside a later tile
    for i, low in ((5, (1 << 64) - 7), (10, (1 << 64) - 256), (12, (1 << 64) - 4096 // 16 - 3)):
        reqs["iv"][i, 8:] = np.frombuffer(low.to_bytes(8, "big"), np.uint8)
    keys, kb = workloads.make_keys(0, 3, [128, 192, 256])
    wl = workloads.Workload("ragged", reqs, keys, kb, off + 64)
    inp = wl.data()
    check(run_gpu(ctx, wl, inp), run_oracle(wl, inp), "ragged ctr")


@pytest.mark.parametrize("op", [workloads.OP_CBC_DEC, workloads.OP_CTR, workloads.OP_CBC_ENC])
def test_in_place_multi_tile(ctx, op):
    # Requests of several tiles: CBC decryption then needs each tile's
    # predecessor block from before the launch overwrites it.
    print(f"[gpu] in-place multi-tile op={op}", flush=True)
    n = 40
    pages = 1 + np.arange(n) % 9
    reqs = np.zeros(n, workloads.REQ_DTYPE)
    reqs["length"] = pages * 4096
    reqs["offset"][1:] = np.cumsum(reqs["length"])[:-1]
    reqs["op"] = op
    reqs["key_idx"] = np.arange(n) % 4
    reqs["iv"] = gen.bytes_(0, gen.STREAM_IVS, 16 * n).reshape(n, 16)
    keys, kb = workloads.make_keys(0, 4, [128, 256, 192, 128])
    wl = workloads.Workload("inplace", reqs, keys, kb, int(reqs["length"].sum()))
    inp = wl.data()
    want = run_oracle(wl, inp, inplace=True)
    for form in ("batch", "plan"):
        check(run_gpu(ctx, wl, inp, form=form, inplace=True), want, f"in-place {form}")


def test_sentinels_gaps_unsorted_and_zero_length(ctx):
    print("[gpu] gaps, unsorted requests, zero lengths, buffer end", flush=True)
    wl = workloads.config3(n_reqs=120, max_pages=6)
    reqs = wl.reqs.copy()
    reqs["offset"] += (np.arange(reqs.size) * 64).astype(np.uint64)
    ctr = reqs["op"] == workloads.OP_CTR
    reqs["length"][ctr] -= (np.arange(ctr.sum()) % 16).astype(np.uint64)
    reqs["length"][::7] = 0
    buf = int(reqs["offset"][-1] + reqs["length"][-1])  # last request ends at the buffer end
    reqs = reqs[np.random.default_rng(5).permutation(reqs.size)]
    wl2 = workloads.Workload("gaps", reqs, wl.keys, wl.key_bits, buf)
    inp = wl2.data()
    check(run_gpu(ctx, wl2, inp), run_oracle(wl2, inp), "gaps")


def test_plan_relaunch_and_graph_safe_reuse(ctx):
    print("[gpu] plan launched three times on fresh outputs", flush=True)
    a = ag()
    wl = workloads.config3(n_reqs=200, max_pages=8)
    inp = wl.data()
    want = run_oracle(wl, inp)
    d_s = device_schedules(wl)
    plan = a.Plan(ctx, wl.reqs, wl.keys.shape[0], wl.buf_bytes)
    d_in = torch.from_numpy(inp).cuda()
    for _ in range(3):
        d_out = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
        plan.launch(d_s, d_in, d_out)
        torch.cuda.synchronize()
        check(d_out.cpu().numpy(), want, "plan relaunch")
    plan.close()


def test_bad_schedule_leaves_output_untouched(ctx):
    print("[gpu] schedule with an invalid round count", flush=True)
    a = ag()
    wl = workloads.pages(64, workloads.OP_CTR, 128, n_keys=2)
    scheds = a.expand_keys(wl.keys, wl.key_bits)
    scheds[1]["nr"] = 9
    d_s = a.schedules_to_device(scheds)
    inp = wl.data()
    got = run_gpu(ctx, wl, inp, d_scheds=d_s)
    want = run_oracle(wl, inp)
    odd = np.zeros(inp.size, bool)
    for r in wl.reqs[wl.reqs["key_idx"] == 1]:
        odd[int(r["offset"]):int(r["offset"] + r["length"])] = True
    check(got[~odd], want[~odd], "good-key requests")
    check(got[odd], workloads.sentinel(inp.size)[odd], "bad-key requests untouched")


@pytest.mark.parametrize("op,bits", [(workloads.OP_CBC_DEC, 128), (workloads.OP_CTR, 128),
                                     (workloads.OP_CBC_DEC, 256), (workloads.OP_CTR, 256)])
def test_config2_full_size(ctx, op, bits):
    """Full config-2 size (65,536 pages, 256 MiB) in the benchmark's launch
    form, for each of the four runs the benchmark times: every page against
    the oracle (its threaded batch over the whole buffer); then the inverse
    operation over the whole buffer restores the input."""
    print(f"[gpu] config 2 full size op={op} bits={bits}", flush=True)
    a = ag()
    wl = workloads.config2(op, bits)
    inp = wl.data()
    d_s = device_schedules(wl)
    d_in = torch.from_numpy(inp).cuda()
    d_out = torch.empty_like(d_in)
    plan = a.Plan(ctx, wl.reqs, 16, wl.buf_bytes)
    plan.launch(d_s, d_in, d_out)
    torch.cuda.synchronize()
    got = d_out.cpu().numpy()
    want = np.empty_like(inp)
    oracle.batch(inp, want, wl.reqs, wl.keys, wl.key_bits,
                 n_threads=len(os.sched_getaffinity(0)))
    check(got, want, "all 65,536 pages")
    # property over the whole buffer: the inverse operation restores the input
    back = torch.empty_like(d_in)
    inv = wl.reqs.copy()
    if op == workloads.OP_CBC_DEC:
        inv["op"] = workloads.OP_CBC_ENC
    plan2 = a.Plan(ctx, inv, 16, wl.buf_bytes)
    plan2.launch(d_s, d_out, back)
    torch.cuda.synchronize()
    assert torch.equal(back, d_in), "round trip over 256 MiB"
    plan.close()
    plan2.close()
