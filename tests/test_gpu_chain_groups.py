"""GPU parity of the CBC-encrypt chain at the edges of its load and store
groups.  The four-lane chain loads its input 8 blocks at a time, one group
ahead, and stores a group's ciphertext while the next group runs, with the
last group stored after the loop; these tests run chains of 1 to 257 blocks
(a group size minus one, equal, plus one, and a few groups) with all three
key sizes against the CPU oracle, byte for byte, out of place and in place,
in every form that runs the chain: batch, plan and the single call (the
chain kernel), a batch that mixes chains with tiles (the fused kernel), one
launch per request, and the persistent serving engine."""
import numpy as np
import pytest
import torch

from synth import gen, workloads
from tests.gpu_util import ag, device_schedules, first_mismatch, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

BLOCKS = [1, 2, 3, 7, 8, 9, 15, 16, 17, 23, 24, 25, 31, 32, 33, 63, 64, 65, 255, 256, 257]


@pytest.fixture(scope="module")
def ctx():
    print("\n[gpu] context for chain group tests", flush=True)
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


def chain_workload(seed=0, tiles=False):
    """One CBC-encrypt request per entry of BLOCKS (keys of 128, 192 and 256
    bits in turn), 48-byte gaps; with tiles, CTR and CBC-decrypt requests of
    one to three pages between them."""
    lengths = [b * 16 for b in BLOCKS]
    ops = [workloads.OP_CBC_ENC] * len(lengths)
    if tiles:
        extra = [(workloads.OP_CTR if i % 2 else workloads.OP_CBC_DEC, 4096 * (1 + i % 3))
                 for i in range(len(lengths))]
        mixed_ops, mixed_len = [], []
        for (o, n), e in zip(extra, lengths):
            mixed_ops += [workloads.OP_CBC_ENC, o]
            mixed_len += [e, n]
        ops, lengths = mixed_ops, mixed_len
    n = len(lengths)
    reqs = np.zeros(n, workloads.REQ_DTYPE)
    reqs["length"] = np.asarray(lengths, np.uint64)
    reqs["offset"][1:] = np.cumsum(reqs["length"] + 48)[:-1]
    reqs["op"] = np.asarray(ops, np.uint32)
    reqs["key_idx"] = np.arange(n) % 3
    reqs["iv"] = gen.bytes_(seed, gen.STREAM_IVS, 16 * n).reshape(n, 16)
    keys, kb = workloads.make_keys(seed, 3, [128, 192, 256])
    buf = int(reqs["offset"][-1] + reqs["length"][-1] + 48)
    return workloads.Workload("chain_groups", reqs, keys, kb, buf, seed)


@pytest.mark.parametrize("inplace", [False, True])
@pytest.mark.parametrize("form", ["batch", "plan", "single"])
def test_chain_kernel(fresh, form, inplace):
    print(f"[gpu] chain group edges form={form} inplace={inplace}", flush=True)
    fresh.set_config(chain_quad=1)
    wl = chain_workload(seed=1)
    inp = wl.data()
    check(run_gpu(fresh, wl, inp, form=form, inplace=inplace),
          run_oracle(wl, inp, inplace=inplace), f"{form} inplace={inplace}")


@pytest.mark.parametrize("inplace", [False, True])
def test_fused_with_tiles(fresh, inplace):
    print(f"[gpu] chain group edges beside tiles, fused, inplace={inplace}", flush=True)
    fresh.set_config(chain_quad=1, fuse=1)
    wl = chain_workload(seed=2, tiles=True)
    inp = wl.data()
    want = run_oracle(wl, inp, inplace=inplace)
    for form in ("batch", "plan"):
        check(run_gpu(fresh, wl, inp, form=form, inplace=inplace), want,
              f"fused {form} inplace={inplace}")


@pytest.mark.parametrize("inplace", [False, True])
def test_per_request_launches(fresh, inplace):
    print(f"[gpu] chain group edges, one launch per request, inplace={inplace}", flush=True)
    a = ag()
    wl = chain_workload(seed=3)
    inp = wl.data()
    d_s = device_schedules(wl)
    d_in = torch.from_numpy(inp.copy()).cuda()
    d_out = d_in if inplace else torch.from_numpy(workloads.sentinel(inp.size)).cuda()
    for r in wl.reqs:
        a.request_launch(fresh, d_s, d_in, d_out, r)
    torch.cuda.synchronize()
    check(d_out.cpu().numpy(), run_oracle(wl, inp, inplace=inplace), "per-request")


def test_persistent_engine(ctx):
    print("[gpu] chain group edges through the persistent engine", flush=True)
    a = ag()
    wl = chain_workload(seed=4)
    inp = wl.data()
    scheds = a.expand_keys(wl.keys, wl.key_bits)
    d_in = torch.from_numpy(inp.copy()).cuda()
    d_out = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
    with a.Server(ctx, mode=a.AES_SERVE_PERSISTENT, key_slots=3) as srv:
        for i, sc in enumerate(scheds):
            srv.set_key(i, sc)
        for r in wl.reqs:
            off = int(r["offset"])
            t = srv.submit(int(r["op"]), int(r["key_idx"]), r["iv"], d_in.data_ptr() + off,
                           d_out.data_ptr() + off, int(r["length"]))
            done = srv.wait(t)
            assert done["status"] == 0, (off, int(done["status"]))
    torch.cuda.synchronize()
    check(d_out.cpu().numpy(), run_oracle(wl, inp), "persistent engine")
