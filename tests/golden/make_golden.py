"""Writes oracle_digests.json: SHA-256 digests of the CPU oracle's output on
small seeded workloads.  It calls only the oracle and the input generator.

The paper prints no AES input/output pair, and no standards vector file is
present, so these digests are regression pins of the oracle itself: its
correctness is pinned by the tests in test_oracle.py.

Run:  python -m tests.golden.make_golden
"""
import hashlib
import json
import os

import numpy as np

import oracle
from synth import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(HERE, "oracle_digests.json")


def _run(wl, inp=None):
    inp = wl.data() if inp is None else inp
    out = workloads.sentinel(wl.buf_bytes)
    oracle.batch(inp, out, wl.reqs, wl.keys, wl.key_bits, n_threads=0)
    return out


def compute() -> dict:
    d = {}
    enc, dec = workloads.config1()
    c = _run(enc)
    d["cfg1_cbc_enc_128"] = hashlib.sha256(c.tobytes()).hexdigest()
    p = _run(dec, c)
    assert np.array_equal(p, enc.data())
    for op in (workloads.OP_CBC_DEC, workloads.OP_CTR):
        for bits in (128, 192, 256):
            wl = workloads.config2(op, bits, n_pages=64)
            d[f"cfg2_small_{workloads.OP_NAMES[op]}_{bits}"] = hashlib.sha256(
                _run(wl).tobytes()).hexdigest()
    wl = workloads.config3(n_reqs=64, max_pages=8)
    d["cfg3_small"] = hashlib.sha256(_run(wl).tobytes()).hexdigest()
    return d


if __name__ == "__main__":
    with open(OUT, "w") as f:
        json.dump(compute(), f, indent=1, sort_keys=True)
        f.write("\n")
    print("wrote", OUT)
