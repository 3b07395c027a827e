"""GPU parity of ECB requests (SP 800-38A 6.1, the paper's service mode):
byte for byte against the CPU oracle (tolerance 0) in every form -- batch,
single-mode calls, plans, per-request launches and their graph, in place,
mixed with the other three ops in the fused and split launches (with either
CTR variant), and through both serving engines."""
import numpy as np
import pytest
import torch

import oracle
from synth import workloads
from tests.gpu_util import ag, device_schedules, first_mismatch, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    print("\n[gpu] context for ECB tests", flush=True)
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


def ecb_pages(op, bits, n_pages=600):
    wl = workloads.config2(workloads.OP_CTR, bits, n_pages=n_pages)
    wl.reqs["op"] = op
    # uneven lengths: whole blocks, some short of a page
    wl.reqs["length"] = 4096 - (np.arange(n_pages, dtype=np.uint64) % 5) * 16 * 37
    return wl


def mixed_all_ops(n=300, seed=0):
    wl = workloads.config3(n_reqs=n, max_pages=10, seed=seed)
    wl.key_bits[::3] = 192
    r = np.random.default_rng(seed).integers(0, 5, n)
    wl.reqs["op"] = r.astype(np.uint32)
    ctr = wl.reqs["op"] == workloads.OP_CTR
    wl.reqs["length"][ctr] -= (np.arange(ctr.sum()) * 3 % 16).astype(np.uint64)
    return wl


@pytest.mark.parametrize("op", [oracle.OP_ECB_ENC, oracle.OP_ECB_DEC])
@pytest.mark.parametrize("bits", [128, 192, 256])
@pytest.mark.parametrize("form", ["batch", "single", "plan"])
def test_ecb_pages(ctx, op, bits, form):
    print(f"[gpu] ECB op={op} bits={bits} form={form}", flush=True)
    wl = ecb_pages(op, bits)
    inp = wl.data()
    check(run_gpu(ctx, wl, inp, form=form), run_oracle(wl, inp), f"ECB {op} {bits} {form}")


@pytest.mark.parametrize("op", [oracle.OP_ECB_ENC, oracle.OP_ECB_DEC])
def test_ecb_in_place(ctx, op):
    print(f"[gpu] ECB in place op={op}", flush=True)
    wl = ecb_pages(op, 256, n_pages=200)
    wl.reqs["length"][::7] = 3 * 4096  # multi-tile requests
    wl.reqs["offset"] = np.concatenate([[0], np.cumsum(wl.reqs["length"][:-1] + 64)]).astype(
        np.uint64)
    wl = workloads.Workload("ecb_inplace", wl.reqs, wl.keys, wl.key_bits,
                            int(wl.reqs["offset"][-1] + wl.reqs["length"][-1]), 0)
    inp = wl.data()
    want = run_oracle(wl, inp, inplace=True)
    for form in ("batch", "plan"):
        check(run_gpu(ctx, wl, inp, form=form, inplace=True), want, f"in place {form}")


@pytest.mark.parametrize("fuse", [1, 0])
@pytest.mark.parametrize("variant", [0, 1])
def test_all_five_ops_in_one_batch(fresh, fuse, variant):
    print(f"[gpu] five ops, fuse={fuse} ctr_variant={variant}", flush=True)
    fresh.set_config(fuse=fuse, ctr_variant=variant)
    wl = mixed_all_ops()
    inp = wl.data()
    want = run_oracle(wl, inp)
    for form in ("batch", "plan"):
        check(run_gpu(fresh, wl, inp, form=form), want, f"five ops {form}")


def test_ecb_per_request_launches_and_graph(ctx):
    print("[gpu] ECB per-request launches and graph", flush=True)
    a = ag()
    wl = mixed_all_ops(n=80, seed=3)
    wl.reqs["op"] = np.where(np.arange(80) % 2 == 0, oracle.OP_ECB_ENC, oracle.OP_ECB_DEC)
    wl.reqs["length"] = wl.reqs["length"] // 16 * 16
    inp = wl.data()
    want = run_oracle(wl, inp)
    d_s = device_schedules(wl)
    d_in = torch.from_numpy(inp).cuda()
    d_out = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
    a.request_launches(ctx, d_s, d_in, d_out, wl.reqs)
    torch.cuda.synchronize()
    check(d_out.cpu().numpy(), want, "per-request launches")
    d_out2 = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
    g = a.Graph.of_requests(ctx, d_s, d_in, d_out2, wl.reqs)
    for _ in range(3):
        g.launch()
        torch.cuda.synchronize()
        check(d_out2.cpu().numpy(), want, "graph replay")
    g.close()


@pytest.mark.parametrize("engine", [0, 1])
def test_ecb_serving_alone_and_in_the_mix(ctx, engine):
    print(f"[gpu] ECB serving, engine={engine}", flush=True)
    a = ag()
    wl = mixed_all_ops(n=60, seed=5)
    wl.reqs["length"] = np.minimum(wl.reqs["length"], 64 * 1024) // 16 * 16
    wl.reqs["offset"] = np.concatenate([[0], np.cumsum(wl.reqs["length"][:-1] + 64)]).astype(
        np.uint64)
    wl = workloads.Workload("ecb_serve", wl.reqs, wl.keys, wl.key_bits,
                            int(wl.reqs["offset"][-1] + wl.reqs["length"][-1] + 64), 0)
    inp = wl.data()
    d_in = torch.from_numpy(inp).cuda()
    torch.cuda.current_stream().synchronize()
    outs = {}
    with a.Server(ctx, mode=engine, key_slots=wl.keys.shape[0]) as s:
        for i, sch in enumerate(a.expand_keys(wl.keys, wl.key_bits)):
            s.set_key(i, sch)
        for form in ("alone", "mix"):
            d_out = torch.from_numpy(workloads.sentinel(inp.size)).cuda()
            torch.cuda.current_stream().synchronize()
            tickets = []
            for r in wl.reqs:
                ecb = int(r["op"]) in (oracle.OP_ECB_ENC, oracle.OP_ECB_DEC)
                t = s.submit(int(r["op"]), int(r["key_idx"]), None if ecb else r["iv"],
                             d_in.data_ptr() + int(r["offset"]),
                             d_out.data_ptr() + int(r["offset"]), int(r["length"]))
                if form == "alone":
                    assert s.wait(t)["status"] == 0
                else:
                    tickets.append(t)
            for t in tickets:
                assert s.wait(t)["status"] == 0
            outs[form] = d_out.cpu().numpy()
    check(outs["alone"], outs["mix"], "alone vs mix")
    check(outs["mix"], run_oracle(wl, inp), "serving vs oracle")
