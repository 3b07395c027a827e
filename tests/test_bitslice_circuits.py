"""The generated bitsliced S-box circuits (host only): the generator's own
checks on all 256 inputs pass, and the committed header is exactly what it
writes, so the kernels compile the circuits that were checked.  The
circuits are also evaluated here, independently of the generator's
simulator, from the emitted C expressions, against the oracle's S-box."""
import importlib.util
import os
import re

import numpy as np

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1305_3345_amd", "csrc")


def load_generator():
    spec = importlib.util.spec_from_file_location(
        "gen_bitslice_sbox", os.path.join(CSRC, "gen_bitslice_sbox.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_committed_header_matches_generator(tmp_path):
    gen = load_generator()
    gen.OUT = str(tmp_path / "bitslice_sbox.h")
    gen.main()  # asserts both circuits on all 256 inputs before writing
    assert open(gen.OUT).read() == open(os.path.join(CSRC, "bitslice_sbox.h")).read()


def _eval_function(text, name, x):
    """Evaluates the emitted function `name` on all 256 bytes at once: bit
    i of lane word j is bit i of byte j (numpy uint32 arrays of 8 words
    over 256 lanes)."""
    body = text[text.index(f"void {name}("):]
    body = body[body.index("{") + 1: body.index("\n}\n")]
    env = {f"u{i}": ((x >> i) & 1).astype(np.uint32) * np.uint32(0xFFFFFFFF) for i in range(8)}
    out = {}

    def bitop3(a, b, c, tt):
        r = np.zeros_like(a)
        for idx in range(8):
            if (tt >> idx) & 1:
                m0 = a if idx & 4 else ~a
                m1 = b if idx & 2 else ~b
                m2 = c if idx & 1 else ~c
                r |= m0 & m1 & m2
        return r
    for line in body.strip().splitlines():
        line = line.strip().rstrip(";")
        m = re.match(r"const uint32_t (t\d+) = (.*)", line)
        if m:
            expr = m.group(2).replace("__builtin_amdgcn_bitop3_b32", "bitop3")
            env[m.group(1)] = eval(expr, {"bitop3": bitop3}, env).astype(np.uint32)
            continue
        m = re.match(r"(s\d) = (t\d+|u\d)", line)
        assert m, line
        out[m.group(1)] = env[m.group(2)]
    return sum(((out[f"s{i}"] & 1).astype(np.int64) << i) for i in range(8))


def test_circuits_against_the_oracle_sbox():
    text = open(os.path.join(CSRC, "bitslice_sbox.h")).read()
    x = np.arange(256, dtype=np.uint32)
    s = _eval_function(text, "bitslice_sbox", x)
    si = _eval_function(text, "bitslice_inv_sbox", x)
    want_s, want_si = (a.astype(np.int64) for a in oracle.sbox())
    assert np.array_equal(s, want_s)
    assert np.array_equal(si, want_si)
