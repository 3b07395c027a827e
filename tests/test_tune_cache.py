"""Host-side tests of the autotuner's cache (AESGPU_TUNE_CACHE) on a host-only
context: the batch signature (aes_tune_key), a cached entry applied without
any launch, comment and malformed lines skipped, the last entry of a
signature winning, and a miss or an unsupported entry falling through to the
tuner (which a host-only context refuses with AES_ERR_DEVICE)."""
import os

import numpy as np
import pytest

from synth import workloads


@pytest.fixture(scope="module")
def ag():
    from paper_1305_3345_amd import aesgpu
    if not os.path.exists(aesgpu.LIB_PATH):
        from paper_1305_3345_amd import build
        build.build()
    aesgpu.lib()
    return aesgpu


@pytest.fixture()
def hctx(ag):
    c = ag.Context(ag.AES_DEVICE_NONE)
    yield c
    c.close()


FIELDS = ["tile_bytes", "ctr_nb", "ctr_wg", "dec_nb", "dec_wg", "chain_lanes", "chain_wg",
          "mixed_nb", "fuse", "grid", "ctr_variant", "chain_quad"]

# Dummy device addresses: a host-only context validates them but never
# dereferences them.
D_SCHED, D_IN, D_OUT = 0x10000, 1 << 32, 1 << 33


def pages_reqs(n=65536, op=workloads.OP_CBC_DEC):
    return workloads.pages(n, op, 128, 16).reqs


def raw_tune(ag, ctx, reqs, n_scheds=16, buf=1 << 30):
    best = np.zeros(1, ag.CONFIG_DTYPE)
    st = ag.lib().aes_tune(ctx.handle, reqs.ctypes.data, reqs.size, n_scheds, buf, D_SCHED,
                           D_IN, D_OUT, 1, best.ctypes.data)
    return st, {k: int(best[0][k]) for k in ag.CONFIG_DTYPE.names if k != "reserved"}


def entry(sig, cfg):
    return sig + "\t" + " ".join(str(cfg[k]) for k in FIELDS)


def test_signature(ag, hctx):
    reqs = pages_reqs()
    assert ag.tune_key(hctx, reqs, 16) == (
        "arch=host cu=0 n=2^16 ops=-,2^16,-,-,- bytes=2^28 len=2^12..2^12 keys=2^4")
    mixed = np.concatenate([pages_reqs(3, workloads.OP_CTR), pages_reqs(5, workloads.OP_CBC_ENC)])
    mixed["length"][0] = 0       # empty requests count as requests, not as sizes
    mixed["length"][1] = 100
    mixed["length"][3] = 1 << 20
    assert ag.tune_key(hctx, mixed, 64) == (
        "arch=host cu=0 n=2^3 ops=2^2,-,2^1,-,- bytes=2^20 len=2^6..2^20 keys=2^6")
    assert ag.tune_key(hctx, mixed[:0], 1) == (
        "arch=host cu=0 n=- ops=-,-,-,-,- bytes=- len=-..- keys=2^0")


def test_signature_buffer_too_small(ag, hctx):
    import ctypes
    reqs = pages_reqs(4)
    n = ctypes.c_size_t(0)
    buf = ctypes.create_string_buffer(8)
    st = ag.lib().aes_tune_key(hctx.handle, reqs.ctypes.data, reqs.size, 1, buf, 8,
                               ctypes.byref(n))
    assert st == ag.AES_ERR_ARG and n.value == len(ag.tune_key(hctx, reqs, 1))


def test_cache_hit_applies_config(ag, hctx, tmp_path, monkeypatch):
    reqs = pages_reqs()
    sig = ag.tune_key(hctx, reqs, 16)
    want = dict(hctx.get_config(), tile_bytes=8192, ctr_nb=1, ctr_wg=1024, dec_nb=4, dec_wg=512,
                fuse=0)
    other = dict(want, dec_nb=1)
    path = tmp_path / "tune.txt"
    path.write_text("# comment line\n" + "not an entry\n" + entry("arch=host other", other)
                    + "\n" + entry(sig, other) + "\n" + sig + "\t1 2 3\n" + entry(sig, want)
                    + "\n")
    monkeypatch.setenv("AESGPU_TUNE_CACHE", str(path))
    st, got = raw_tune(ag, hctx, reqs)
    assert st == ag.AES_OK
    assert got == want                      # the last complete entry of the signature
    assert hctx.get_config() == want         # and set in the context
    assert "not an entry" in path.read_text()  # a hit does not rewrite the file


def test_cache_hit_keeps_decryption_variant(ag, hctx, tmp_path, monkeypatch):
    """The cache holds the twelve tuned knobs; the context's decryption
    variant (not tuned) stays as the caller set it across a hit."""
    reqs = pages_reqs()
    sig = ag.tune_key(hctx, reqs, 16)
    hctx.set_config(dec_variant=ag.AES_DEC_BITSLICE)
    want = dict(hctx.get_config(), tile_bytes=8192)
    path = tmp_path / "tune.txt"
    path.write_text(entry(sig, want) + "\n")
    monkeypatch.setenv("AESGPU_TUNE_CACHE", str(path))
    st, got = raw_tune(ag, hctx, reqs)
    assert st == ag.AES_OK and got == want
    assert hctx.get_config()["dec_variant"] == ag.AES_DEC_BITSLICE


def test_cache_miss_and_unsupported_entry(ag, hctx, tmp_path, monkeypatch):
    reqs = pages_reqs()
    sig = ag.tune_key(hctx, reqs, 16)
    path = tmp_path / "tune.txt"
    bad = dict(hctx.get_config(), ctr_nb=3)  # no such tile kernel
    text = entry("arch=host something else", hctx.get_config()) + "\n" + entry(sig, bad) + "\n"
    path.write_text(text)
    monkeypatch.setenv("AESGPU_TUNE_CACHE", str(path))
    before = hctx.get_config()
    st, _ = raw_tune(ag, hctx, reqs)
    assert st == ag.AES_ERR_DEVICE           # falls through to the tuner
    assert hctx.get_config() == before
    assert path.read_text() == text          # nothing stored without a tuning run
    monkeypatch.setenv("AESGPU_TUNE_CACHE", str(tmp_path / "missing.txt"))
    assert raw_tune(ag, hctx, reqs)[0] == ag.AES_ERR_DEVICE
    assert not (tmp_path / "missing.txt").exists()


def test_validation_precedes_cache(ag, hctx, tmp_path, monkeypatch):
    reqs = pages_reqs(8)
    reqs["offset"][3] += 8                   # misaligned: rejected before the cache is read
    path = tmp_path / "tune.txt"
    path.write_text(entry(ag.tune_key(hctx, reqs, 16), hctx.get_config()) + "\n")
    monkeypatch.setenv("AESGPU_TUNE_CACHE", str(path))
    assert raw_tune(ag, hctx, reqs)[0] == ag.AES_ERR_RANGE



def test_concurrent_hits(ag, tmp_path, monkeypatch):
    """Eight threads, each with its own host-only context and batch shape,
    look their entries up in one cache file at the same time: every call hits
    and sets its own entry's configuration."""
    import threading
    ctxs = [ag.Context(ag.AES_DEVICE_NONE) for _ in range(8)]
    reqs = [pages_reqs(1 << (4 + i)) for i in range(8)]
    sigs = [ag.tune_key(c, r, 16) for c, r in zip(ctxs, reqs)]
    assert len(set(sigs)) == 8
    base = ctxs[0].get_config()
    cfgs = [dict(base, chain_lanes=8 * (i + 1)) for i in range(8)]
    path = tmp_path / "tune.txt"
    path.write_text("".join(entry(s, c) + "\n" for s, c in zip(sigs, cfgs)))
    monkeypatch.setenv("AESGPU_TUNE_CACHE", str(path))
    errs = []

    def hit(i):
        for _ in range(50):
            st, got = raw_tune(ag, ctxs[i], reqs[i])
            if st != ag.AES_OK or got != cfgs[i] or ctxs[i].get_config() != cfgs[i]:
                errs.append((i, st))

    ts = [threading.Thread(target=hit, args=(i,)) for i in range(8)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    for c in ctxs:
        c.close()
    assert not errs
