"""GPU parity of the CTR tile path that computes the first two rounds' shared
part once per group of counters (one set before and one after the carry out
of counter byte 15), byte for byte against the CPU oracle (tolerance 0).

The counters are placed where that split can go wrong: low byte 0 (no carry
in a group), 1, 128, 192 and 255 (carry after the first block), carries that
ripple through every counter byte, the wrap of the 64-bit counter at a group
boundary and inside a later group of a 16 KiB tile, and requests shorter than
a group.  Every key size, tile size (4, 8 and 16 KiB: one to four groups per
tile) and tile-kernel shape (1, 2 or 4 blocks per lane: four, two or one
step per group)."""
import numpy as np
import pytest

from synth import gen, workloads
from tests.gpu_util import ag, first_mismatch, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

M64 = 1 << 64
# (counter of the request's first block, length in bytes)
CASES = [
    (0, 16384), (1, 16384), (128, 16384), (192, 8192), (255, 16384),
    (0x00FF_FFFF_FFFF_FF80, 16384),  # the carry ripples through bytes 9..14
    (M64 - 0x80, 16384),             # wraps to 0 in the middle of the first group
    (M64 - 256, 16384),              # wraps at the first group boundary
    (M64 - 256 - 5, 16384 - 7),      # wraps inside the second group, ragged tail
    (M64 - 3 * 256 + 17, 16384),     # wraps inside the third group
    (250, 300), (7, 4096 + 16 * 7), (255, 1), (200, 4096 * 3 + 9),
]


def heads_workload(seed=0):
    n = len(CASES) * 3
    reqs = np.zeros(n, workloads.REQ_DTYPE)
    reqs["iv"] = gen.bytes_(seed, gen.STREAM_IVS, 16 * n).reshape(n, 16)
    off = 0
    for i in range(n):
        ctr, ln = CASES[i % len(CASES)]
        reqs["offset"][i] = off
        reqs["length"][i] = ln
        reqs["iv"][i, 8:] = np.frombuffer(ctr.to_bytes(8, "big"), np.uint8)
        off += (ln + 15) // 16 * 16 + 48
    reqs["op"] = workloads.OP_CTR
    reqs["key_idx"] = np.arange(n) // len(CASES)  # each case under every key size
    keys, kb = workloads.make_keys(seed, 3, [128, 192, 256])
    return workloads.Workload("ctr_heads", reqs, keys, kb, off + 64, seed)


@pytest.fixture(scope="module")
def fresh():
    print("\n[gpu] context for shared-head CTR tests", flush=True)
    c = ag().Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("nb,wg", [(1, 1024), (2, 1024), (2, 512), (4, 512), (4, 256)])
@pytest.mark.parametrize("tile", [4096, 8192, 16384])
def test_ctr_heads(fresh, nb, wg, tile):
    print(f"[gpu] CTR heads nb={nb} wg={wg} tile={tile}", flush=True)
    fresh.set_config(ctr_nb=nb, ctr_wg=wg, tile_bytes=tile, fuse=0)
    wl = heads_workload()
    inp = wl.data()
    want = run_oracle(wl, inp)
    for form in ("batch", "plan"):
        msg = first_mismatch(run_gpu(fresh, wl, inp, form=form), want)
        assert msg is None, f"{form} nb={nb} wg={wg} tile={tile}: {msg}"


def test_ctr_heads_in_place(fresh):
    print("[gpu] CTR heads in place", flush=True)
    fresh.set_config(ctr_nb=2, ctr_wg=1024, tile_bytes=16384, fuse=0)
    wl = heads_workload(seed=3)
    inp = wl.data()
    msg = first_mismatch(run_gpu(fresh, wl, inp, form="plan", inplace=True),
                         run_oracle(wl, inp, inplace=True))
    assert msg is None, msg
