"""GPU parity of the tile kernels across repeated launches.  A tile launch
leaves its per-workgroup work counters at zero for the next launch that uses
them (a plan's, or the single-call form's on one stream); these tests launch
the same work many times, with eager GPU work between the launches, and check
every output against the CPU oracle byte for byte: plans relaunched on the
default grid, on a grid of 24 and one of 20 workgroups, with unit counts that
do not divide evenly between them; single calls of varying sizes and both
tile sides in turn on one stream; in-place CBC decryption relaunched on its
own output; requests shorter than a tile's step (one unit each, so some
waves of a workgroup start with no unit of their own) on several tile
shapes; and a grid of more workgroups than the counters can give a 128-byte
line each."""
import numpy as np
import pytest
import torch

from synth import workloads
from tests.gpu_util import ag, device_schedules, first_mismatch, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("\n[gpu] context for relaunch tests", flush=True)
    c = ag().Context(0)
    yield c
    c.close()


@pytest.fixture()
def fresh(ctx):
    cfg = ctx.get_config()
    yield ctx
    ctx.set_config(**cfg)


def check(got, want, what):
    msg = first_mismatch(got, want)
    assert msg is None, f"{what}: {msg}"


@pytest.mark.parametrize("grid", [0, 24, 20])
@pytest.mark.parametrize("op,bits,n_pages", [(workloads.OP_CTR, 128, 8191),
                                             (workloads.OP_CBC_DEC, 256, 6007)])
def test_plan_relaunched(fresh, op, bits, n_pages, grid):
    print(f"[gpu] relaunch: plan relaunched op={op} bits={bits} pages={n_pages} grid={grid}",
          flush=True)
    a = ag()
    fresh.set_config(grid=grid)
    wl = workloads.pages(n_pages, op, bits, 16, seed=11)
    inp = wl.data()
    want = run_oracle(wl, inp)
    d_s = device_schedules(wl)
    d_in = torch.from_numpy(inp).cuda()
    sentinel = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
    d_out = sentinel.clone()
    plan = a.Plan(fresh, wl.reqs, wl.keys.shape[0], wl.buf_bytes)
    try:
        for rep in range(12):
            d_out.copy_(sentinel)  # eager work between launches
            torch.cuda.synchronize()
            plan.launch(d_s, d_in, d_out)
            torch.cuda.synchronize()
            check(d_out.cpu().numpy(), want, f"launch {rep}")
    finally:
        plan.close()


def test_single_calls_on_one_stream(fresh):
    """The single-call form keeps its counters per stream: calls of different
    sizes and both tile sides in turn, each checked."""
    print("[gpu] relaunch: single calls of varying size on one stream", flush=True)
    a = ag()
    for rep, n_pages in enumerate([4096, 1000, 8200, 264, 4096]):
        for op in (workloads.OP_CTR, workloads.OP_CBC_DEC):
            wl = workloads.pages(n_pages, op, 128, 16, seed=20 + rep)
            inp = wl.data()
            d_s = device_schedules(wl)
            d_in = torch.from_numpy(inp).cuda()
            d_out = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
            fn = a.ctr_batch if op == workloads.OP_CTR else a.cbc_decrypt_batch
            r = wl.reqs
            fn(fresh, d_s, d_in, d_out, r["offset"], r["length"], r["key_idx"], r["iv"])
            torch.cuda.synchronize()
            check(d_out.cpu().numpy(), run_oracle(wl, inp), f"call {rep} op {op} pages {n_pages}")


def test_in_place_relaunched(fresh):
    """In-place CBC decryption: each launch decrypts the previous launch's
    output, so launch k must equal k decryptions of the input."""
    print("[gpu] relaunch: in-place CBC decryption relaunched", flush=True)
    a = ag()
    wl = workloads.pages(5003, workloads.OP_CBC_DEC, 128, 16, seed=31)
    inp = wl.data()
    d_s = device_schedules(wl)
    d = torch.from_numpy(inp.copy()).cuda()
    plan = a.Plan(fresh, wl.reqs, wl.keys.shape[0], wl.buf_bytes)
    want = inp.copy()
    try:
        for rep in range(4):
            plan.launch(d_s, d, d)
            torch.cuda.synchronize()
            want = run_oracle(wl, want, inplace=True)
            check(d.cpu().numpy(), want, f"in-place launch {rep}")
    finally:
        plan.close()


def small_requests(op, seed, n=300):
    """n requests of 16 B to 4 KiB - 16 B (one unit each, shorter than a
    tile's step for most tile shapes), packed back to back from offset 0 with
    gaps of 16 to 31 bytes, keys of all three sizes."""
    rng = np.random.default_rng(seed)
    lengths = (rng.integers(1, 256, n) * 16).astype(np.uint64)
    if op == workloads.OP_CTR:
        lengths -= (np.arange(n) % 16).astype(np.uint64)  # ragged CTR lengths
        lengths[lengths == 0] = 1
    reqs = np.zeros(n, workloads.REQ_DTYPE)
    reqs["length"] = lengths
    reqs["offset"][1:] = np.cumsum((lengths + 31) // 16 * 16)[:-1]
    reqs["op"] = op
    reqs["key_idx"] = np.arange(n) % 3
    reqs["iv"] = rng.integers(0, 256, (n, 16), dtype=np.uint8)
    keys, kb = workloads.make_keys(seed, 3, [128, 192, 256])
    buf = int(reqs["offset"][-1] + reqs["length"][-1] + 32)
    return workloads.Workload("small", reqs, keys, kb, buf, seed)


@pytest.mark.parametrize("nb,wg", [(1, 256), (2, 1024), (4, 256), (4, 512)])
@pytest.mark.parametrize("op", [workloads.OP_CBC_DEC, workloads.OP_CTR])
def test_units_shorter_than_a_step(fresh, nb, wg, op):
    """Requests shorter than a tile's step on several tile shapes: each is one
    unit, the first starts at offset 0, and a CBC request's only unit takes
    its IV from the record (never from the bytes before it), out of place and
    in place."""
    print(f"[gpu] relaunch: units shorter than a step nb={nb} wg={wg} op={op}", flush=True)
    fresh.set_config(ctr_nb=nb, ctr_wg=wg, dec_nb=nb, dec_wg=wg, fuse=0)
    wl = small_requests(op, seed=40 + nb + wg)
    inp = wl.data()
    for inplace in (False, True):
        check(run_gpu(fresh, wl, inp, form="plan", inplace=inplace),
              run_oracle(wl, inp, inplace=inplace), f"inplace={inplace}")


@pytest.mark.parametrize("op,bits", [(workloads.OP_CTR, 256), (workloads.OP_CBC_DEC, 128)])
def test_grid_beyond_spread_counters(fresh, op, bits):
    """A grid of more than 2,048 workgroups (3,072 of 256 threads), whose
    counters are packed one word apart instead of one per 128-byte line,
    relaunched; every launch checked."""
    print(f"[gpu] relaunch: 3,072-workgroup grid op={op} bits={bits}", flush=True)
    a = ag()
    fresh.set_config(ctr_nb=2, ctr_wg=256, dec_nb=2, dec_wg=256, grid=3072)
    wl = workloads.pages(12289, op, bits, 16, seed=50 + bits)
    inp = wl.data()
    want = run_oracle(wl, inp)
    d_s = device_schedules(wl)
    d_in = torch.from_numpy(inp).cuda()
    sentinel = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
    d_out = sentinel.clone()
    plan = a.Plan(fresh, wl.reqs, wl.keys.shape[0], wl.buf_bytes)
    try:
        for rep in range(4):
            d_out.copy_(sentinel)
            torch.cuda.synchronize()
            plan.launch(d_s, d_in, d_out)
            torch.cuda.synchronize()
            check(d_out.cpu().numpy(), want, f"launch {rep}")
    finally:
        plan.close()
