#!/usr/bin/env python3
"""Benchmark of the batched AES hot path on one MI355X.

Workload (the single-call form at scale): 65,536 independent 4 KiB pages
(256 MiB), 16 keys assigned round-robin, uniform random bytes.  One step runs
the four single calls AES-128 CBC-decrypt, AES-128 CTR (64-bit counter per
page from 0, random nonce), AES-256 CBC-decrypt and AES-256 CTR over the whole
buffer.  Each call is a plan launch: the request list was validated, cut into
work units and uploaded to HBM before the timed region, so data and metadata
are resident when it starts.

Prints one JSON line: GB/s of payload (10^9 bytes/s) over the timed steps,
the roofline record of the dominant kernel (HIP events on the launch stream)
and the CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
UNIT_BYTES = 32  # one work-unit record read per tile
SCHED_BYTES = 512
PROBE = os.path.join(ROOT, "paper_1305_3345_amd", "probe", "lds_gather_probe")


def lds_probe():
    """The LDS gather ceiling of this machine, measured now: conflict-free
    ds_read_b32 lane-gathers per second over the chip, per clock per compute
    unit, and the shader clock during the probe (the probe program is a
    child process, started before this process touches the GPU)."""
    import subprocess
    if not os.path.exists(PROBE):
        raise RuntimeError(f"{PROBE} is missing: build it with "
                           "`python -m paper_1305_3345_amd.build`")
    out = subprocess.run([PROBE, "0"], stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                         text=True, timeout=120)
    if out.returncode != 0:
        raise RuntimeError(f"LDS probe failed: {out.stderr.strip()}")
    return json.loads(out.stdout.strip().splitlines()[-1])


def lds_gathers_per_block(run: str) -> int:
    """Table lookups (LDS gathers) per 16-byte block of a run such as
    "ctr_128" or "cbc_dec_256": 16 per round; CTR's first two rounds take 5
    instead of 32 (their counter-invariant part comes from scalar loads)."""
    nr = {128: 10, 192: 12, 256: 14}[int(run.rsplit("_", 1)[1])]
    return 16 * nr - (27 if run.startswith("ctr") else 0)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--pages", type=int, default=65536)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-pages", type=int, default=65536,
                    help="pages per run timed on the CPU oracle")
    ap.add_argument("--per-call-iters", type=int, default=5,
                    help="iterations of the host-metadata single-call form (0 = skip)")
    ap.add_argument("--runs", default="cbc_dec_128,ctr_128,cbc_dec_256,ctr_256",
                    help="comma-separated subset of the step's runs (for profiling)")
    ap.add_argument("--skip-serving", action="store_true",
                    help="skip the serving (Poisson arrivals, p50/p99) measurement")
    ap.add_argument("--serve-requests", type=int, default=20000,
                    help="measured requests per arrival rate and engine")
    ap.add_argument("--serve-warmup", type=int, default=2000,
                    help="warm-up requests before the measured ones, per rate and engine")
    ap.add_argument("--skip-lds-probe", action="store_true",
                    help="leave out the LDS gather probe (its ceiling is then null); for "
                         "profiler runs, which would also profile the probe's process")
    ap.add_argument("--skip-beside-server", action="store_true",
                    help="skip the batch launch timed beside a live persistent server (it waits "
                         "out the server's idle timeout, about 1 s per launch)")
    ap.add_argument("--skip-host-serving", action="store_true",
                    help="skip serving with payloads in pinned host memory")
    ap.add_argument("--skip-variants", action="store_true",
                    help="skip the table vs bitsliced CTR comparison")
    ap.add_argument("--skip-e2", action="store_true",
                    help="skip the single-request ECB size sweep (4 KiB .. 1 MiB)")
    ap.add_argument("--skip-long", action="store_true",
                    help="skip the 8 GiB CTR stream and the 4,096 CBC-encrypt chains")
    ap.add_argument("--skip-batched", action="store_true",
                    help="skip the mixed-batch (10,000 uneven requests) measurement")
    ap.add_argument("--batched-full-per-request", action="store_true",
                    help="also time all 10,000 mixed requests as one launch each and as a "
                         "graph of those launches (CBC-encrypt chains then run one after "
                         "another: about 20 s per form)")
    ap.add_argument("--batched-no-per-request", action="store_true",
                    help="batched section without the per-request launches of the parallel "
                         "subset (for profiler runs, where each of those launches is slow)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also copy the 256 MiB input once device-to-device (a kernel of "
                         "known traffic for scaling hardware byte counters)")
    return ap.parse_args()


def cpu_baseline(sample_pages: int):
    """The CPU oracle (all host cores) on the first sample_pages pages of each
    of the four runs of a step; GB/s of payload."""
    import numpy as np

    import oracle
    from synth import gen, workloads

    total = 0
    secs = 0.0
    threads = 1
    for bits in (128, 256):
        for op in (workloads.OP_CBC_DEC, workloads.OP_CTR):
            wl = workloads.config2(op, bits, n_pages=sample_pages)
            inp = wl.data()
            out = np.empty_like(inp)
            t0 = time.perf_counter()
            threads = oracle.batch(inp, out, wl.reqs, wl.keys, wl.key_bits,
                                   n_threads=len(os.sched_getaffinity(0)))
            secs += time.perf_counter() - t0
            total += wl.payload_bytes()
    # The size sweep's requests on one core of the oracle (plain scalar C).
    keys, kb = workloads.make_keys(0, 1, 128)
    data = gen.bytes_(0, gen.STREAM_DATA, E2_SIZES[-1])
    e2 = {}
    for n in E2_SIZES:
        t0 = time.perf_counter()
        oracle.mode(oracle.OP_ECB_ENC, keys[0][:16], 128, None, data[:n])
        e2[str(n)] = round((time.perf_counter() - t0) * 1e6, 1)
    return {"value": round(total / secs / 1e9, 4), "unit": "GB/s", "cores": threads,
            "host_cpus": os.cpu_count(), "cpus_allowed": len(os.sched_getaffinity(0)),
            "kind": "oracle",
            "sample": f"first {sample_pages} pages of each of the 4 runs of a step "
                      f"({total >> 20} MiB), same keys/IVs/bytes, {secs:.1f} s",
            "e2_one_core_us": e2}


def cpu_aesni_context(n_pages: int, reps: int = 3):
    """Context, not the oracle: the library's host route (AES-NI) on all host
    threads (aes_host_batch) over the same four runs of a step, host buffers;
    GB/s of payload per run (median of reps) and over the step."""
    import numpy as np

    from paper_1305_3345_amd import aesgpu
    from synth import workloads

    # The CPUs this process may run on (the machine may have more).
    threads = len(os.sched_getaffinity(0))
    per_run = {}
    total_bytes, total_s = 0, 0.0
    for bits in (128, 256):
        for op in (workloads.OP_CBC_DEC, workloads.OP_CTR):
            wl = workloads.config2(op, bits, n_pages=n_pages)
            inp = wl.data()
            out = np.empty_like(inp)
            sch = aesgpu.expand_keys(wl.keys, wl.key_bits)
            aesgpu.host_batch(sch, inp, out, wl.reqs, threads)  # untimed: page in the buffers
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                aesgpu.host_batch(sch, inp, out, wl.reqs, threads)
                ts.append(time.perf_counter() - t0)
            t = sorted(ts)[len(ts) // 2]
            per_run[f"{workloads.OP_NAMES[op]}_{bits}"] = round(wl.payload_bytes() / t / 1e9, 2)
            total_bytes += wl.payload_bytes()
            total_s += t
    return {"value": round(total_bytes / total_s / 1e9, 2), "unit": "GB/s",
            "threads": threads, "kind": "host route (AES-NI), context, not the oracle",
            "per_run": per_run,
            "sample": f"all {n_pages} pages of each of the 4 runs, host memory, median of {reps}"}


# What the tile kernels are built from (sources and per-file compiler flags).
TILE_SOURCES = ("csrc/aes_rounds.h", "csrc/internal.h", "csrc/tile_kernel.h",
                "csrc/aes_tiles_ctr.hip", "csrc/aes_tiles_dec.hip", "build.py")


def profiled_traffic(kernel: str, pages: int):
    """HBM bytes per launch of `kernel` on the 65,536-page workload, from the
    committed rocprofv3 counter summary -- or None when the kernel sources
    have changed since the counters were taken (their SHA-1 is recorded in
    the summary) or the workload differs."""
    import hashlib
    import re

    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "profiles", "tile_kernels_config2_counters.md")
    if pages != 65536 or not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"Kernel sources at the time \(SHA-1 of [^)]*\): `([0-9a-f]{40})`", text)
    src = b"".join(open(os.path.join(here, "paper_1305_3345_amd", f), "rb").read()
                   for f in TILE_SOURCES)
    if not m or hashlib.sha1(src).hexdigest() != m.group(1):
        return None
    m = re.search(r"- `" + re.escape(kernel) + r"`: (\d+)", text)
    return int(m.group(1)) if m else None


def time_gpu(fn, iters, stream):
    """Median milliseconds of fn() over iters runs after one warm-up (HIP events)."""
    import torch
    fn()
    torch.cuda.synchronize()
    ms = []
    for _ in range(iters):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        fn()
        b.record(stream)
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
    ms.sort()
    return ms[len(ms) // 2]


def bench_batched(dev, iters=3, full_per_request=False, per_request=True):
    """The batched form: 10,000 uneven requests (4 KiB..1 MiB, mixed ops, 64
    keys of 128/256 bits) as one autotuned fused launch, against one kernel
    launch per request and a HIP graph of those launches (on the requests of
    the parallel modes; the serial CBC-encrypt chains make per-request
    launches of the whole mix take tens of seconds), plus the chain floor
    (the CBC-encrypt chain with the most block rounds, alone)."""
    import numpy as np
    import torch

    from paper_1305_3345_amd import aesgpu
    from synth import gen, workloads

    wl = workloads.config3()
    nbytes = wl.buf_bytes
    d_in = gen.bytes_torch(0, gen.STREAM_DATA, (nbytes + 7) // 8 * 8, dev)[:nbytes]
    d_out = torch.empty_like(d_in)
    d_s = aesgpu.schedules_to_device(aesgpu.expand_keys(wl.keys, wl.key_bits), dev)
    stream = torch.cuda.current_stream()
    ctx = aesgpu.Context(0)
    t0 = time.perf_counter()
    cfg = aesgpu.tune(ctx, wl.reqs, d_s, d_in, d_out, iters=2)
    tune_s = time.perf_counter() - t0
    plan = aesgpu.Plan(ctx, wl.reqs, wl.keys.shape[0], nbytes)
    info = plan.info()
    full_ms = time_gpu(lambda: plan.launch(d_s, d_in, d_out, stream=stream), iters, stream)
    g_plan = aesgpu.Graph.of_plan(plan, d_s, d_in, d_out)
    full_graph_ms = time_gpu(lambda: g_plan.launch(stream), iters, stream)

    # The chain floor: the CBC-encrypt request with the most rounds in all
    # (blocks x Nr, so an AES-256 chain outweighs an AES-128 one of equal length).
    enc = np.nonzero(wl.reqs["op"] == workloads.OP_CBC_ENC)[0]
    nr = wl.key_bits[wl.reqs["key_idx"][enc]] // 32 + 6
    pick = enc[np.argmax(wl.reqs["length"][enc].astype(np.int64) * nr)]
    longest = wl.reqs[pick:pick + 1]
    p_long = aesgpu.Plan(ctx, longest, wl.keys.shape[0], nbytes)
    chain_ms = time_gpu(lambda: p_long.launch(d_s, d_in, d_out, stream=stream), iters, stream)

    par = wl.reqs[wl.reqs["op"] != workloads.OP_CBC_ENC]
    par_bytes = int(par["length"].sum())
    p_par = aesgpu.Plan(ctx, par, wl.keys.shape[0], nbytes)
    par_batched_ms = time_gpu(lambda: p_par.launch(d_s, d_in, d_out, stream=stream), iters, stream)
    par_each_ms = par_graph_ms = g_each = None
    if per_request:
        par_each_ms = time_gpu(lambda: aesgpu.request_launches(ctx, d_s, d_in, d_out, par,
                                                               stream=stream), iters, stream)
        g_each = aesgpu.Graph.of_requests(ctx, d_s, d_in, d_out, par)
        par_graph_ms = time_gpu(lambda: g_each.launch(stream), iters, stream)
    full = None
    if full_per_request:
        def once(fn):
            a_ev = torch.cuda.Event(enable_timing=True)
            b_ev = torch.cuda.Event(enable_timing=True)
            a_ev.record(stream)
            fn()
            b_ev.record(stream)
            b_ev.synchronize()
            return a_ev.elapsed_time(b_ev)
        print("[batched] all requests, one launch each", file=sys.stderr, flush=True)
        each_ms = once(lambda: aesgpu.request_launches(ctx, d_s, d_in, d_out, wl.reqs,
                                                       stream=stream))
        print("[batched] all requests, graph of per-request launches", file=sys.stderr,
              flush=True)
        g_all = aesgpu.Graph.of_requests(ctx, d_s, d_in, d_out, wl.reqs)
        graph_ms = once(lambda: g_all.launch(stream))
        g_all.close()
        full = {"per_request_launches_ms": round(each_ms, 1),
                "per_request_graph_ms": round(graph_ms, 1),
                "per_request_launches_gbs": round(info["payload_bytes"] / each_ms / 1e6, 2),
                "per_request_graph_gbs": round(info["payload_bytes"] / graph_ms / 1e6, 2),
                "note": "one timed pass each (no warm-up pass)"}
    for o in (g_plan, g_each, plan, p_long, p_par):
        if o is not None:
            o.close()
    ctx.close()
    gbs = lambda b, ms: None if ms is None else round(b / ms / 1e6, 1)
    return {
        "workload": f"{wl.reqs.size} requests, 4 KiB..1 MiB log-uniform, ops "
                    f"{int((wl.reqs['op'] == 0).sum())} CBC-enc / {int((wl.reqs['op'] == 1).sum())} "
                    f"CBC-dec / {int((wl.reqs['op'] == 2).sum())} CTR, 64 keys (128/256)",
        "payload_bytes": info["payload_bytes"],
        "tuned_config": cfg, "tune_s": round(tune_s, 2),
        "one_launch_ms": round(full_ms, 3), "one_launch_gbs": gbs(info["payload_bytes"], full_ms),
        "plan_graph_ms": round(full_graph_ms, 3),
        "chain_floor_ms": round(chain_ms, 3),
        "chain_floor_request_bytes": int(longest["length"][0]),
        "chain_floor_key_bits": int(wl.key_bits[longest["key_idx"][0]]),
        "all_requests_per_request": full,
        "parallel_subset": {
            "requests": int(par.size), "payload_bytes": par_bytes,
            "one_launch_gbs": gbs(par_bytes, par_batched_ms),
            "per_request_launches_gbs": gbs(par_bytes, par_each_ms),
            "per_request_graph_gbs": gbs(par_bytes, par_graph_ms),
            "one_launch_ms": round(par_batched_ms, 3),
            "per_request_launches_ms": None if par_each_ms is None else round(par_each_ms, 3),
            "per_request_graph_ms": None if par_graph_ms is None else round(par_graph_ms, 3),
        },
    }


def bench_variants(ctx, n_pages, d_in, d_out, dev, iters=5):
    """The kernel variants side by side on the 4 KiB-page workload: round
    tables in LDS against the bitsliced kernels, for CTR and for CBC
    decryption, AES-128 and AES-256 (plan launches, median of iters, HIP
    events)."""
    import torch

    from paper_1305_3345_amd import aesgpu
    from synth import workloads

    stream = torch.cuda.current_stream()
    cfg = ctx.get_config()
    out = {}
    try:
        for bits in (128, 256):
            wl = workloads.config2(workloads.OP_CTR, bits, n_pages=n_pages)
            d_s = aesgpu.schedules_to_device(aesgpu.expand_keys(wl.keys, wl.key_bits), dev)
            payload = int(wl.reqs["length"].sum())
            rec = {}
            for v, vname in ((aesgpu.AES_CTR_TABLE, "table"), (aesgpu.AES_CTR_BITSLICE, "bitslice")):
                ctx.set_config(ctr_variant=v)
                plan = aesgpu.Plan(ctx, wl.reqs, wl.keys.shape[0], wl.buf_bytes)
                ms = time_gpu(lambda: plan.launch(d_s, d_in, d_out, stream=stream), iters, stream)
                plan.close()
                rec[vname] = {"ms": round(ms, 4), "gbs_payload": round(payload / ms / 1e6, 1)}
            rec["bitslice_over_table"] = round(rec["table"]["ms"] / rec["bitslice"]["ms"], 3)
            out[f"ctr_{bits}"] = rec
        ctx.set_config(**cfg)
        for bits in (128, 256):
            wl = workloads.config2(workloads.OP_CBC_DEC, bits, n_pages=n_pages)
            d_s = aesgpu.schedules_to_device(aesgpu.expand_keys(wl.keys, wl.key_bits), dev)
            payload = int(wl.reqs["length"].sum())
            rec = {}
            for v, vname in ((aesgpu.AES_DEC_TABLE, "table"), (aesgpu.AES_DEC_BITSLICE, "bitslice")):
                ctx.set_config(dec_variant=v)
                plan = aesgpu.Plan(ctx, wl.reqs, wl.keys.shape[0], wl.buf_bytes)
                ms = time_gpu(lambda: plan.launch(d_s, d_in, d_out, stream=stream), iters, stream)
                plan.close()
                rec[vname] = {"ms": round(ms, 4), "gbs_payload": round(payload / ms / 1e6, 1)}
            rec["bitslice_over_table"] = round(rec["table"]["ms"] / rec["bitslice"]["ms"], 3)
            out[f"cbc_dec_{bits}"] = rec
    finally:
        ctx.set_config(**cfg)
    return out


def bench_long(dev, iters=3):
    """The long-stream workloads: AES-256-CTR over 8 GiB in HBM as 512 chunks
    of 16 MiB (one continuous counter stream), as one plan launch and as 512
    per-request launches; and AES-256-CBC encryption of 4,096 chains of 1 MiB
    (the serial-chain limit) as one launch."""
    import torch

    from paper_1305_3345_amd import aesgpu
    from synth import gen, workloads

    stream = torch.cuda.current_stream()
    ctx = aesgpu.Context(0)
    wl = workloads.config5_ctr()
    nbytes = wl.buf_bytes
    d_in = gen.bytes_torch(0, gen.STREAM_DATA, nbytes, dev)
    d_out = torch.empty_like(d_in)
    d_s = aesgpu.schedules_to_device(aesgpu.expand_keys(wl.keys, wl.key_bits), dev)
    plan = aesgpu.Plan(ctx, wl.reqs, 1, nbytes)
    ctr_ms = time_gpu(lambda: plan.launch(d_s, d_in, d_out, stream=stream), iters, stream)
    plan.close()
    each_ms = time_gpu(lambda: aesgpu.request_launches(ctx, d_s, d_in, d_out, wl.reqs,
                                                       stream=stream), iters, stream)
    wc = workloads.config5_cbc()
    d_sc = aesgpu.schedules_to_device(aesgpu.expand_keys(wc.keys, wc.key_bits), dev)
    pc = aesgpu.Plan(ctx, wc.reqs, 1, wc.buf_bytes)
    cbc_ms = time_gpu(lambda: pc.launch(d_sc, d_in, d_out, stream=stream), 2, stream)
    pc.close()
    ctx.close()
    del d_in, d_out
    torch.cuda.empty_cache()
    gbs = lambda b, ms: round(b / ms / 1e6, 1)
    return {
        "ctr256_8gib": {"chunks": int(wl.reqs.size), "bytes": nbytes,
                        "one_launch_ms": round(ctr_ms, 3), "one_launch_gbs": gbs(nbytes, ctr_ms),
                        "per_chunk_launches_ms": round(each_ms, 3),
                        "per_chunk_launches_gbs": gbs(nbytes, each_ms)},
        "cbcenc256_4096x1mib": {"chains": int(wc.reqs.size), "bytes": wc.buf_bytes,
                                "one_launch_ms": round(cbc_ms, 3),
                                "gbs": gbs(wc.buf_bytes, cbc_ms)},
    }


E2_SIZES = [4096 << k for k in range(9)]  # 4 KiB .. 1 MiB


class _OpenSSLECB:
    """AES-128-ECB encryption on one host core through the system libcrypto
    (EVP interface, AES-NI): the modern stand-in for the paper's optimised
    CPU AES, reported as context -- not the oracle."""

    def __init__(self, key: bytes):
        import ctypes.util

        name = ctypes.util.find_library("crypto") or "libcrypto.so.3"
        lib = ctypes.CDLL(name)
        vp = ctypes.c_void_p
        lib.EVP_CIPHER_CTX_new.restype = vp
        lib.EVP_CIPHER_CTX_free.argtypes = [vp]
        lib.EVP_aes_128_ecb.restype = vp
        lib.EVP_EncryptInit_ex.argtypes = [vp, vp, vp, vp, vp]
        lib.EVP_CIPHER_CTX_set_padding.argtypes = [vp, ctypes.c_int]
        lib.EVP_EncryptUpdate.argtypes = [vp, vp, ctypes.POINTER(ctypes.c_int), vp, ctypes.c_int]
        self.lib = lib
        self.key = ctypes.create_string_buffer(key, 16)
        self.ctx = lib.EVP_CIPHER_CTX_new()
        if lib.EVP_EncryptInit_ex(self.ctx, lib.EVP_aes_128_ecb(), None, self.key, None) != 1:
            raise OSError("EVP_EncryptInit_ex failed")
        lib.EVP_CIPHER_CTX_set_padding(self.ctx, 0)

    def encrypt(self, src_ptr: int, dst_ptr: int, n: int):
        got = ctypes.c_int(0)
        if self.lib.EVP_EncryptUpdate(self.ctx, dst_ptr, ctypes.byref(got), src_ptr, n) != 1:
            raise OSError("EVP_EncryptUpdate failed")

    def close(self):
        self.lib.EVP_CIPHER_CTX_free(self.ctx)


def bench_e2(dev, reps=15):
    """The paper's AES size sweep (section 3.3): one AES-128 ECB-encrypt
    request of 4 KiB .. 1 MiB with the payload resident on the device, timed
    on the host clock from the call to the observed completion -- as one
    kernel launch per request, and through the persistent serving engine --
    against OpenSSL on one host core (context).  Crossover = the smallest
    size at which the GPU form is faster."""
    import numpy as np
    import torch

    from paper_1305_3345_amd import aesgpu
    from synth import gen, workloads

    keys, kb = workloads.make_keys(0, 1, 128)
    nbytes = E2_SIZES[-1]
    d_in = gen.bytes_torch(0, gen.STREAM_DATA, nbytes, dev)
    d_out = torch.empty_like(d_in)
    h_in = d_in.cpu().numpy()
    h_out = np.empty_like(h_in)
    stream = torch.cuda.current_stream()
    ctx = aesgpu.Context(0)
    sched = aesgpu.expand_keys(keys, kb)
    d_s = aesgpu.schedules_to_device(sched, dev)
    cpu = _OpenSSLECB(bytes(keys[0][:16]))
    med = lambda xs: sorted(xs)[len(xs) // 2]
    rows = []
    # One launch per request and the CPU first, with no persistent kernel
    # resident (its workgroups would hold most compute units' LDS).
    for n in E2_SIZES:
        req = np.zeros(1, aesgpu.REQ_DTYPE)
        req["length"] = n
        req["op"] = aesgpu.AES_OP_ECB_ENC
        launch, host = [], []
        for i in range(reps + 2):
            t0 = time.perf_counter()
            aesgpu.request_launch(ctx, d_s, d_in, d_out, req[0], stream=stream)
            stream.synchronize()
            t1 = time.perf_counter()
            cpu.encrypt(h_in.ctypes.data, h_out.ctypes.data, n)
            t2 = time.perf_counter()
            if i >= 2:  # the first rounds warm up caches
                launch.append((t1 - t0) * 1e6)
                host.append((t2 - t1) * 1e6)
        rows.append({"bytes": n, "gpu_launch_us": round(med(launch), 1),
                     "cpu_openssl_us": round(med(host), 1)})
    with aesgpu.Server(ctx, key_slots=1) as srv:
        srv.set_key(0, sched[0])
        for row in rows:
            n = row["bytes"]
            persist = []
            for i in range(reps + 2):
                t0 = time.perf_counter()
                srv.wait(srv.submit(aesgpu.AES_OP_ECB_ENC, 0, None, d_in.data_ptr(),
                                    d_out.data_ptr(), n))
                if i >= 2:
                    persist.append((time.perf_counter() - t0) * 1e6)
            row["gpu_persistent_us"] = round(med(persist), 1)
    # The paper's E1: an (almost) empty service call -- one 16-byte block --
    # through persistent kernels of 512, 1,024 and 2,048 threads (one, two and
    # four 512-thread workgroups; one workgroup holds the encryption tables
    # only) and the default grid, against one normal kernel launch.
    req = np.zeros(1, aesgpu.REQ_DTYPE)
    req["length"] = 16
    req["op"] = aesgpu.AES_OP_ECB_ENC
    launch = []
    for i in range(reps + 2):
        t0 = time.perf_counter()
        aesgpu.request_launch(ctx, d_s, d_in, d_out, req[0], stream=stream)
        stream.synchronize()
        if i >= 2:
            launch.append((time.perf_counter() - t0) * 1e6)
    e1 = {"launch_us": round(med(launch), 1), "persistent_us": {},
          "persistent_library_us": {},
          "note": "launch_us and persistent_us: Python's clock around the call (ctypes and "
                  "torch included); persistent_library_us: the library's own clock from "
                  "entering aes_server_submit to aes_server_wait seeing the completion"}
    for nwg in (1, 2, 4, 0):
        with aesgpu.Server(ctx, key_slots=1, n_workgroups=nwg) as srv:
            srv.set_key(0, sched[0])
            rt, lib_rt = [], []
            for i in range(reps + 2):
                t0 = time.perf_counter()
                rec = srv.wait(srv.submit(aesgpu.AES_OP_ECB_ENC, 0, None, d_in.data_ptr(),
                                          d_out.data_ptr(), 16))
                if i >= 2:
                    rt.append((time.perf_counter() - t0) * 1e6)
                    lib_rt.append((int(rec["t_done_ns"]) - int(rec["t_submit_ns"])) / 1e3)
            label = f"{512 * nwg} threads" if nwg else "default grid"
            e1["persistent_us"][label] = round(med(rt), 1)
            e1["persistent_library_us"][label] = round(med(lib_rt), 1)
    cpu.close()
    ctx.close()

    def crossover(col):
        for r in rows:
            if r[col] < r["cpu_openssl_us"]:
                return r["bytes"]
        return None

    return {"workload": "one AES-128 ECB-encrypt request per size, payload in HBM, "
                        f"median of {reps}; CPU: OpenSSL EVP on one core (context, not the oracle)",
            "sizes": rows,
            "crossover_bytes_launch": crossover("gpu_launch_us"),
            "crossover_bytes_persistent": crossover("gpu_persistent_us"),
            "max_speedup_launch": round(max(r["cpu_openssl_us"] / r["gpu_launch_us"]
                                            for r in rows), 2),
            "max_speedup_persistent": round(max(r["cpu_openssl_us"] / r["gpu_persistent_us"]
                                                for r in rows), 2),
            "e1_empty_call": e1}


def bench_serving(dev, n_measure=2000, n_warm=200):
    """The serving form: Poisson arrivals, sizes uniform in {4,8,16,32,64} KiB,
    AES-128-CBC encrypt/decrypt 50/50 over 256 resident key slots, payloads
    staged in HBM, 256 MiB admission cap.  The per-request-launch engine's
    saturated throughput (a burst of requests) sets the five offered rates
    (0.1, 0.25, 0.5, 0.75, 0.9 of it); both engines replay the same trace at
    each rate; latency = host time from arrival to observed completion."""
    import numpy as np
    import torch

    from paper_1305_3345_amd import aesgpu
    from synth import gen, workloads

    n = n_warm + n_measure
    tr = workloads.config4(1.0, n)  # arrival times at 1 request/s; scaled per rate
    nb = (tr.buf_bytes + 7) // 8 * 8
    d_in = gen.bytes_torch(0, gen.STREAM_DATA, nb, dev)
    d_out = torch.empty_like(d_in)
    torch.cuda.current_stream().synchronize()
    scheds = aesgpu.expand_keys(tr.keys, tr.key_bits)
    ctx = aesgpu.Context(0)
    names = {aesgpu.AES_SERVE_PERSISTENT: "persistent", aesgpu.AES_SERVE_PER_LAUNCH: "per_launch"}

    def replay(engine, arrivals):
        with aesgpu.Server(ctx, mode=engine, key_slots=256) as srv:
            for i, sc in enumerate(scheds):
                srv.set_key(i, sc)
            done = srv.replay(tr.reqs, arrivals, d_in, d_out)
            st = srv.stats()
        assert (done["status"] == 0).all(), "serving request failed"
        return done, st

    def summarize(done):
        m = done[n_warm:]
        lat = (m["t_done_ns"].astype(np.int64) - m["t_submit_ns"].astype(np.int64)) / 1e3
        ops = tr.reqs["op"][n_warm:]
        span = (m["t_done_ns"].max() - m["t_submit_ns"].min()) / 1e9
        out = {"p50_us": round(float(np.percentile(lat, 50)), 1),
               "p99_us": round(float(np.percentile(lat, 99)), 1),
               "p999_us": round(float(np.percentile(lat, 99.9)), 1),
               "gbs": round(float(tr.reqs["length"][n_warm:].sum()) / span / 1e9, 3)}
        for op, nm in ((workloads.OP_CBC_ENC, "enc"), (workloads.OP_CBC_DEC, "dec")):
            sel = lat[ops == op]
            out[f"{nm}_p50_us"] = round(float(np.percentile(sel, 50)), 1)
            out[f"{nm}_p99_us"] = round(float(np.percentile(sel, 99)), 1)
            out[f"{nm}_p999_us"] = round(float(np.percentile(sel, 99.9)), 1)
        gpu = (m["gpu_done_ticks"].astype(np.int64) - m["gpu_dispatch_ticks"].astype(np.int64))
        if gpu.any():  # persistent engine: device clock, 100 MHz, dispatch -> last unit done
            for op, nm in ((workloads.OP_CBC_ENC, "enc"), (workloads.OP_CBC_DEC, "dec")):
                for q in (50, 99, 99.9):
                    out[f"{nm}_gpu_p{str(q).replace('.', '')}_us"] = round(
                        float(np.percentile(gpu[ops == op], q)) / 100, 1)
        return out

    burst = np.zeros(n)
    sat = {}
    for engine in (aesgpu.AES_SERVE_PER_LAUNCH, aesgpu.AES_SERVE_PERSISTENT):
        done, _ = replay(engine, burst)
        span = (done["t_done_ns"].max() - done["t_submit_ns"].min()) / 1e9
        sat[names[engine]] = round(n / span, 1)
    base = sat["per_launch"]
    rates = []
    for frac in (0.1, 0.25, 0.5, 0.75, 0.9):
        rate = frac * base
        row = {"fraction_of_per_launch_saturation": frac, "rate_req_s": round(rate, 1)}
        for engine in (aesgpu.AES_SERVE_PER_LAUNCH, aesgpu.AES_SERVE_PERSISTENT):
            done, st = replay(engine, tr.arrivals_s / rate)
            row[names[engine]] = summarize(done)
            print(f"[serving] {names[engine]} at {frac} of saturation: p50 "
                  f"{row[names[engine]]['p50_us']} us, p99 {row[names[engine]]['p99_us']} us",
                  file=sys.stderr, flush=True)
            if engine == aesgpu.AES_SERVE_PERSISTENT:
                row[names[engine]]["kernel_launches"] = st["kernel_launches"]
        rates.append(row)
    ctx.close()
    return {"workload": f"{n_measure} measured (+{n_warm} warm-up) requests per rate and engine, "
                        "Poisson arrivals, 4..64 KiB, AES-128-CBC enc/dec 50/50, 256 key slots",
            "saturation_req_s": sat, "rates": rates}


def bench_beside_server(dev, n_pages=65536, reps=5):
    """A batch call while a persistent server is live: the server's
    workgroups hold their compute units (each a whole CU's LDS) until its
    idle timeout, so a tile launch issued meanwhile runs on the others.  One
    AES-128 CTR plan launch over n_pages pages, alone and beside an idle
    persistent server of the default grid and of a 4-workgroup grid (a
    request is submitted before each timed launch so the kernel is running)."""
    import numpy as np
    import torch

    from paper_1305_3345_amd import aesgpu
    from synth import gen, workloads

    wl = workloads.config2(workloads.OP_CTR, 128, n_pages=n_pages)
    nbytes = wl.buf_bytes
    d_in = gen.bytes_torch(0, gen.STREAM_DATA, nbytes, dev)
    d_out = torch.empty_like(d_in)
    scheds = aesgpu.expand_keys(wl.keys, wl.key_bits)
    d_s = aesgpu.schedules_to_device(scheds, dev)
    stream = torch.cuda.current_stream()
    ctx = aesgpu.Context(0)
    plan = aesgpu.Plan(ctx, wl.reqs, wl.keys.shape[0], nbytes)
    out = {"workload": f"AES-128 CTR plan launch, {n_pages} x 4 KiB pages, median of {reps}",
           "alone_ms": round(time_gpu(lambda: plan.launch(d_s, d_in, d_out, stream=stream), reps,
                                      stream), 4)}
    small = torch.zeros(4096, dtype=torch.uint8, device=dev)
    for label, nwg in (("beside_default_grid_ms", 0), ("beside_4_workgroups_ms", 4)):
        with aesgpu.Server(ctx, mode=aesgpu.AES_SERVE_PERSISTENT, key_slots=1,
                           n_workgroups=nwg) as srv:
            srv.set_key(0, scheds[0])
            ms = []
            for _ in range(reps + 1):
                t = srv.submit(workloads.OP_CTR, 0, bytes(16), small, small, 4096)
                srv.wait(t)  # the persistent kernel is now running (idle until its timeout)
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                plan.launch(d_s, d_in, d_out, stream=stream)
                b.record(stream)
                b.synchronize()
                ms.append(a.elapsed_time(b))
            ms = sorted(ms[1:])
            out[label] = round(ms[len(ms) // 2], 4)
    plan.close()
    ctx.close()
    return out


def bench_host_serving(dev, n_measure=1000, n_warm=100, reps=15):
    """Serving with payloads in pinned host memory (the paper's request path,
    section 3.2, whose 4 KB measurement includes the copies).  Three
    transports: the persistent kernel reading and writing the pinned pages
    directly; one launch per request with copy-in / kernel / copy-out through
    per-stream HBM staging (the traditional way); one launch per request
    reading the pages directly.  (1) one request at a time, host clock from
    submit to observed completion, median of `reps`; (2) a burst of 256
    AES-128-CTR requests of 1 MiB (GB/s over the host link); (3) the serving
    trace (Poisson, 4..64 KiB, AES-128-CBC enc/dec) at five rates set by the
    copy transport's saturated throughput."""
    import numpy as np

    from paper_1305_3345_amd import aesgpu
    from synth import gen, workloads

    P, L = aesgpu.AES_SERVE_PERSISTENT, aesgpu.AES_SERVE_PER_LAUNCH
    transports = {"persistent_direct": dict(mode=P),
                  "launch_copy": dict(mode=L, host_xfer=aesgpu.AES_XFER_COPY),
                  "launch_direct": dict(mode=L, host_xfer=aesgpu.AES_XFER_DIRECT)}
    ctx = aesgpu.Context(0)
    med = lambda xs: sorted(xs)[len(xs) // 2]

    def make(cfg, scheds, nbytes, data):
        srv = aesgpu.Server(ctx, key_slots=len(scheds), **cfg)
        for i, sc in enumerate(scheds):
            srv.set_key(i, sc)
        h_in = srv.host_alloc(nbytes)
        h_out = srv.host_alloc(nbytes)
        h_in[:] = data[:nbytes]
        return srv, h_in, h_out

    # (1) and (2): one AES-128 key
    keys, kb = workloads.make_keys(0, 1, 128)
    sched = aesgpu.expand_keys(keys, kb)
    big = 256 << 20
    data = gen.bytes_(0, gen.STREAM_DATA, big)
    iv = bytes(16)
    sizes = [4096, 65536, 1 << 20]
    rt = {}
    burst = {}
    for name, cfg in transports.items():
        srv, h_in, h_out = make(cfg, sched, big, data)
        with srv:
            row = {}
            for n in sizes:
                xs = []
                for i in range(reps + 2):
                    t0 = time.perf_counter()
                    srv.wait(srv.submit(aesgpu.AES_OP_CTR, 0, iv, h_in.ctypes.data,
                                        h_out.ctypes.data, n))
                    if i >= 2:
                        xs.append((time.perf_counter() - t0) * 1e6)
                row[f"{n >> 10}KiB_us"] = round(med(xs), 1)
            rt[name] = row
            t0 = time.perf_counter()
            ts = []
            for k in range(256):
                while True:
                    try:
                        ts.append(srv.submit(aesgpu.AES_OP_CTR, 0, iv,
                                             h_in.ctypes.data + k * (1 << 20),
                                             h_out.ctypes.data + k * (1 << 20), 1 << 20))
                        break
                    except aesgpu.AesError as e:
                        if e.status != aesgpu.AES_ERR_AGAIN:
                            raise
            for t in ts:
                srv.wait(t)
            burst[name] = round(big / (time.perf_counter() - t0) / 1e9, 2)

    # (3) the serving trace with host payloads
    n = n_warm + n_measure
    tr = workloads.config4(1.0, n)
    nb = (tr.buf_bytes + 7) // 8 * 8
    tdata = gen.bytes_(0, gen.STREAM_DATA, nb)
    scheds = aesgpu.expand_keys(tr.keys, tr.key_bits)

    def replay(name, arrivals, dispatch=False):
        srv, h_in, h_out = make(transports[name], scheds, nb, tdata)
        with srv:
            cross = srv.calibrate(0) if dispatch else None
            done = srv.replay(tr.reqs, arrivals, h_in, h_out)
            routed = srv.stats()["host_routed"]
        assert (done["status"] == 0).all(), "serving request failed"
        if dispatch:
            return done, cross, routed
        return done

    def summarize(done):
        m = done[n_warm:]
        lat = (m["t_done_ns"].astype(np.int64) - m["t_submit_ns"].astype(np.int64)) / 1e3
        ops = tr.reqs["op"][n_warm:]
        out = {"p50_us": round(float(np.percentile(lat, 50)), 1),
               "p99_us": round(float(np.percentile(lat, 99)), 1)}
        for op, nm in ((workloads.OP_CBC_ENC, "enc"), (workloads.OP_CBC_DEC, "dec")):
            sel = lat[ops == op]
            out[f"{nm}_p50_us"] = round(float(np.percentile(sel, 50)), 1)
            out[f"{nm}_p99_us"] = round(float(np.percentile(sel, 99)), 1)
        return out

    sat = {}
    for name in ("launch_copy", "persistent_direct"):
        done = replay(name, np.zeros(n))
        sat[name] = round(n / ((done["t_done_ns"].max() - done["t_submit_ns"].min()) / 1e9), 1)
    rates = []
    for frac in (0.1, 0.25, 0.5, 0.75, 0.9):
        rate = frac * sat["launch_copy"]
        row = {"fraction_of_launch_copy_saturation": frac, "rate_req_s": round(rate, 1)}
        for name in ("launch_copy", "persistent_direct"):
            row[name] = summarize(replay(name, tr.arrivals_s / rate))
        # size-based dispatch: the persistent engine after start-up calibration
        done, cross, routed = replay("persistent_direct", tr.arrivals_s / rate, dispatch=True)
        row["persistent_dispatch"] = summarize(done)
        row["persistent_dispatch"]["host_routed_frac"] = round(routed / n, 3)
        rates.append(row)
    # Size alone ignores load: at rates set by the persistent engine's own
    # saturation the host route's one submitting core can fall behind.
    high = []
    for frac in (0.1, 0.5):
        rate = frac * sat["persistent_direct"]
        row = {"fraction_of_persistent_saturation": frac, "rate_req_s": round(rate, 1),
               "persistent_direct": summarize(replay("persistent_direct", tr.arrivals_s / rate))}
        done, _, routed = replay("persistent_direct", tr.arrivals_s / rate, dispatch=True)
        row["persistent_dispatch"] = summarize(done)
        row["persistent_dispatch"]["host_routed_frac"] = round(routed / n, 3)
        high.append(row)
    cross_names = ("cbc_enc", "cbc_dec", "ctr", "ecb_enc", "ecb_dec")
    crossovers = {nm: (None if int(c) == (1 << 64) - 1 else int(c))
                  for nm, c in zip(cross_names, cross)}
    ctx.close()
    return {"workload": "payloads in pinned host memory (aes_server_host_alloc); AES-128",
            "round_trip_ctr": rt, "burst_256x1MiB_ctr_gbs": burst,
            "trace": f"{n_measure} measured (+{n_warm} warm-up) requests per rate, Poisson, "
                     "4..64 KiB, AES-128-CBC enc/dec 50/50, 256 key slots",
            "saturation_req_s": sat, "rates": rates,
            "dispatch_crossover_bytes": crossovers, "high_rates": high,
            "dispatch_note": "persistent_dispatch: aes_server_calibrate at start-up, then requests "
                             "below their op's crossover run on the host route (AES-NI on the "
                             "submitting thread); null = the GPU engine was faster at no tested "
                             "size (4 KiB .. 4 MiB; 256 KiB for CBC encryption)"}


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: it measures the single-GPU hot path "
              "(the pages would shard across GPUs with no exchange between them).",
              file=sys.stderr)
        sys.exit(2)

    # The LDS ceiling first, in a child process, before this one uses the GPU.
    probe = None if args.skip_lds_probe else lds_probe()

    import numpy as np
    import torch

    from paper_1305_3345_amd import aesgpu
    from synth import gen, workloads

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = aesgpu.Context(0)

    n_pages = args.pages
    nbytes = n_pages * workloads.PAGE
    d_in = gen.bytes_torch(0, gen.STREAM_DATA, nbytes, dev)  # same bytes as workloads.data()
    d_out = torch.empty_like(d_in)

    runs = []  # (name, kernel, plan, d_scheds, payload, units)
    for bits in (128, 256):
        cfg = ctx.get_config()
        kernels = {workloads.OP_CBC_DEC: f"k_tiles<true, {cfg['dec_nb']}, {cfg['dec_wg']}>",
                   workloads.OP_CTR: (f"k_tiles<false, {cfg['ctr_nb']}, {cfg['ctr_wg']}>"
                                      if cfg["ctr_variant"] == aesgpu.AES_CTR_TABLE
                                      else "k_ctr_bitslice")}
        for op, kname in ((workloads.OP_CBC_DEC, kernels[workloads.OP_CBC_DEC]),
                          (workloads.OP_CTR, kernels[workloads.OP_CTR])):
            name = f"{workloads.OP_NAMES[op]}_{bits}"
            if name not in args.runs.split(","):
                continue
            wl = workloads.config2(op, bits, n_pages=n_pages)
            d_s = aesgpu.schedules_to_device(aesgpu.expand_keys(wl.keys, wl.key_bits), dev)
            plan = aesgpu.Plan(ctx, wl.reqs, wl.keys.shape[0], nbytes)
            info = plan.info()
            units = info["n_units_cbc_dec"] + info["n_units_ctr"]
            runs.append((name, kname, plan, d_s,
                         info["payload_bytes"], units, wl))
    stream = torch.cuda.current_stream()

    def step(events=None):
        for i, (_, _, plan, d_s, _, _, _) in enumerate(runs):
            if events is not None:
                events[i][0].record(stream)
            plan.launch(d_s, d_in, d_out, stream=stream)
            if events is not None:
                events[i][1].record(stream)

    if args.calib_copy:
        d_out.copy_(d_in)
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    ev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)]
           for _ in runs] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(ev[k])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    payload_step = sum(r[4] for r in runs)
    value = payload_step * args.steps / elapsed / 1e9
    # A plain device-to-device copy of the same buffer: the HBM bandwidth this
    # box reaches in practice, to set the runs' traffic against.
    copy_ms = time_gpu(lambda: d_out.copy_(d_in), 5, stream)
    copy_gbs = 2 * nbytes / copy_ms / 1e6

    per_run = {}
    per_kernel = {}
    for i, (name, kname, _, _, payload, units, _) in enumerate(runs):
        ms = [ev[k][i][0].elapsed_time(ev[k][i][1]) for k in range(args.steps)]
        avg = sum(ms) / len(ms)
        med = sorted(ms)[len(ms) // 2]
        algo = 2 * payload + units * UNIT_BYTES + 16 * SCHED_BYTES
        per_run[name] = {"ms": round(avg, 4), "ms_median": round(med, 4),
                         "ms_min": round(min(ms), 4),
                         "gbs_payload": round(payload / avg / 1e6, 1),
                         "hbm_frac": round(algo / avg / 1e6 / HBM_PEAK_GBS, 4),
                         "frac_of_copy": round(algo / avg / 1e6 / copy_gbs, 4)}
        pk = per_kernel.setdefault(kname, {"ms_total": 0.0, "launches": 0, "algo_bytes": 0,
                                           "gathers": 0})
        pk["ms_total"] += sum(ms)
        pk["launches"] += len(ms)
        pk["algo_bytes"] += algo * len(ms)
        pk["gathers"] += payload // 16 * lds_gathers_per_block(name) * len(ms)
    dom = max(per_kernel, key=lambda k: per_kernel[k]["ms_total"])
    d = per_kernel[dom]
    avg_ms = d["ms_total"] / d["launches"]
    algo_per_launch = d["algo_bytes"] / d["launches"]
    achieved = algo_per_launch / avg_ms / 1e6
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": profiled_traffic(f"aesgpu::{dom}", n_pages),
                "kernel": f"aesgpu::{dom}", "avg_launch_ms": round(avg_ms, 4),
                "algo_bytes_per_launch": int(algo_per_launch)}
    # The ceiling that binds the table rounds: LDS gathers (one ds_read_b32
    # lane per table lookup) against the rate a ds_read_b32 probe measured.
    g_rate = d["gathers"] / d["launches"] / avg_ms * 1e3
    ceiling = probe["lane_gathers_per_s"] if probe else None
    roofline["lds_gathers"] = {
        "achieved": float(f"{g_rate:.4g}"),
        "ceiling": float(f"{ceiling:.4g}") if ceiling else None,
        "unit": "lane-gathers/s",
        "frac": round(g_rate / ceiling, 4) if ceiling else None,
        "per_launch": int(d["gathers"] / d["launches"]),
        "ceiling_source": ("lds_gather_probe in this run: "
                           f"{probe['lane_gathers_per_clk_per_cu']} lane-gathers per clock per "
                           f"compute unit at {probe['sclk_ghz']} GHz") if probe else None}

    # Host-metadata single-call form: validation, planning and the unit-table
    # upload happen inside every call (end-to-end, reported beside the value).
    per_call = None
    if args.per_call_iters > 0:
        # The caller's arrays, contiguous as a C caller would hold them.
        calls = []
        for name, _, _, d_s, _, _, wl in runs:
            r = wl.reqs
            fn = aesgpu.ctr_batch if name.startswith("ctr") else aesgpu.cbc_decrypt_batch
            calls.append((fn, d_s, *(np.ascontiguousarray(r[f]) for f in
                                     ("offset", "length", "key_idx", "iv"))))
        for fn, d_s, off, ln, ki, iv in calls:  # one untimed pass
            fn(ctx, d_s, d_in, d_out, off, ln, ki, iv)
        # Then all passes in one window, synchronised only at its ends (as the
        # steps of `value`): each call's host work overlaps the kernels queued
        # before it, as in a caller issuing calls back to back.
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.per_call_iters):
            for fn, d_s, off, ln, ki, iv in calls:
                fn(ctx, d_s, d_in, d_out, off, ln, ki, iv)
        torch.cuda.synchronize()
        t_sum = time.perf_counter() - t1
        per_call = {"value": round(payload_step * args.per_call_iters / t_sum / 1e9, 2),
                    "unit": "GB/s", "calls": len(calls) * args.per_call_iters,
                    "note": "aes_cbc_decrypt_batch / aes_ctr_batch with host request arrays "
                            "(validation + planning + metadata upload in every call), "
                            "back to back in one timed window"}

    variants = None
    if not args.skip_variants:
        variants = bench_variants(ctx, n_pages, d_in, d_out, dev)

    serving = None
    if not args.skip_serving:
        serving = bench_serving(dev, n_measure=args.serve_requests, n_warm=args.serve_warmup)

    beside = None
    if not args.skip_serving and not args.skip_beside_server:
        beside = bench_beside_server(dev, n_pages)

    host_serving = None
    if not args.skip_host_serving:
        host_serving = bench_host_serving(dev)

    batched = None
    if not args.skip_batched:
        batched = bench_batched(dev, full_per_request=args.batched_full_per_request,
                                per_request=not args.batched_no_per_request)

    long_stream = None
    if not args.skip_long:
        long_stream = bench_long(dev)

    e2 = None
    if not args.skip_e2:
        e2 = bench_e2(dev)

    cpu = None
    cpu_aesni = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(min(args.cpu_sample_pages, n_pages))
        cpu_aesni = cpu_aesni_context(n_pages)

    line = {
        "metric": "AES GB/s on 4 KiB pages (batched vs per-call); p50/p99 latency in serving loop",
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": f"the single-call-form-at-scale configuration: {n_pages} x 4 KiB "
                               f"pages ({nbytes >> 20} MiB), 16 keys round-robin, uniform random "
                               "bytes; step = AES-128 CBC-dec, AES-128 CTR, AES-256 CBC-dec, "
                               "AES-256 CTR, timed with the request metadata resident in HBM "
                               "(the single calls, which hand over host request arrays in every "
                               "call, are per_call)",
                   "pages": n_pages, "page_bytes": workloads.PAGE,
                   "form": "plan launch (unit table resident in HBM)"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "cpu_aesni_context": cpu_aesni,
        "per_run": per_run,
        "hbm_copy_gbs": round(copy_gbs, 1),
        "per_call": per_call,
        "ctr_variants": ({k: v for k, v in variants.items() if k.startswith("ctr")}
                         if variants else None),
        "dec_variants": ({k: v for k, v in variants.items() if k.startswith("cbc_dec")}
                         if variants else None),
        "batched": batched,
        "long_stream": long_stream,
        "e2_size_sweep": e2,
        "serving": serving,
        "batch_beside_live_server": beside,
        "host_serving": host_serving,
    }
    for _, _, plan, _, _, _, _ in runs:
        plan.close()
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
