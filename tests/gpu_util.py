"""Helpers shared by the GPU tests: run a workload through the library's C ABI
and through the CPU oracle on the same seeded bytes."""
import numpy as np

import oracle
from synth import workloads


def ag():
    from paper_1305_3345_amd import aesgpu
    aesgpu.lib()
    return aesgpu


def device_schedules(wl):
    a = ag()
    return a.schedules_to_device(a.expand_keys(wl.keys, wl.key_bits))


def run_gpu(ctx, wl, inp: np.ndarray, form: str = "batch", inplace: bool = False,
            reqs=None, d_scheds=None):
    """Runs wl's requests on the GPU; returns the output buffer as numpy.

    form: "batch" (aes_batch), "single" (the single-mode entry point of the
    requests' one op), or "plan" (aes_plan_create + aes_plan_launch)."""
    import torch
    a = ag()
    reqs = wl.reqs if reqs is None else reqs
    d_scheds = device_schedules(wl) if d_scheds is None else d_scheds
    d_in = torch.from_numpy(inp.copy()).cuda()
    d_out = d_in if inplace else torch.from_numpy(workloads.sentinel(inp.size)).cuda()
    if form == "batch":
        a.batch(ctx, d_scheds, d_in, d_out, reqs)
    elif form == "single":
        ops = np.unique(reqs["op"])
        assert ops.size == 1
        fn = {a.AES_OP_CBC_ENC: a.cbc_encrypt_batch, a.AES_OP_CBC_DEC: a.cbc_decrypt_batch,
              a.AES_OP_CTR: a.ctr_batch, a.AES_OP_ECB_ENC: a.ecb_encrypt_batch,
              a.AES_OP_ECB_DEC: a.ecb_decrypt_batch}[int(ops[0])]
        fn(ctx, d_scheds, d_in, d_out, reqs["offset"], reqs["length"], reqs["key_idx"],
           reqs["iv"])
    elif form == "plan":
        plan = a.Plan(ctx, reqs, wl.keys.shape[0], inp.size)
        plan.launch(d_scheds, d_in, d_out)
        torch.cuda.synchronize()
        plan.close()
    else:
        raise ValueError(form)
    torch.cuda.synchronize()
    return d_out.cpu().numpy()


def run_oracle(wl, inp: np.ndarray, inplace: bool = False, reqs=None) -> np.ndarray:
    reqs = wl.reqs if reqs is None else reqs
    out = inp.copy() if inplace else workloads.sentinel(inp.size)
    oracle.batch(inp, out, reqs, wl.keys, wl.key_bits, n_threads=0)
    return out


def first_mismatch(a: np.ndarray, b: np.ndarray):
    d = np.nonzero(a != b)[0]
    if d.size == 0:
        return None
    return f"{d.size} bytes differ, first at {int(d[0])} (block {int(d[0]) // 16})"
