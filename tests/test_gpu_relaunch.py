"""GPU parity of the tile kernels across repeated launches.  A tile launch
leaves its per-workgroup work counters at zero for the next launch that uses
them (a plan's, or the single-call form's on one stream); these tests launch
the same work many times, with eager GPU work between the launches, and check
every output against the CPU oracle byte for byte: plans relaunched on the
default grid, on a grid of 24 and one of 20 workgroups, with unit counts that
do not divide evenly between them; single calls of varying sizes and both
tile sides in turn on one stream; and in-place CBC decryption relaunched on
its own output."""
import pytest
import torch

from synth import workloads
from tests.gpu_util import ag, device_schedules, first_mismatch, run_oracle

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
