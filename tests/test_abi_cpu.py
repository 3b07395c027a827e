"""Host-side tests of the C ABI (no GPU): exports, key expansion, validation
errors and the work-unit planner, run on a host-only (AES_DEVICE_NONE) context."""
import os
import re

import numpy as np
import pytest

import oracle
from synth import gen, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


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


def declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(aes_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol(ag):
    import ctypes
    names = declared_functions()
    assert {"aes_expand_key", "aes_cbc_encrypt_batch", "aes_cbc_decrypt_batch",
            "aes_ctr_batch", "aes_batch"} <= names
    L = ctypes.CDLL(ag.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.parametrize("bits", (128, 192, 256))
def test_expand_key_matches_oracle(ag, bits):
    r = np.random.default_rng(bits)
    for _ in range(5):
        key = r.integers(0, 256, bits // 8, dtype=np.uint8)
        s = ag.expand_key(key, bits)
        nr = {128: 10, 192: 12, 256: 14}[bits]
        assert s["key_bits"] == bits and s["nr"] == nr
        w = oracle.expand_key(key, bits)  # (4(nr+1), 4) bytes
        ek = s["ek"][: 4 * (nr + 1)].astype("<u4").view(np.uint8).reshape(-1, 4)
        assert np.array_equal(ek, w)
        assert not s["ek"][4 * (nr + 1):].any() and not s["dk"][4 * (nr + 1):].any()
        # equivalent inverse cipher: first and last round keys are swapped, unchanged
        assert np.array_equal(s["dk"][:4], s["ek"][4 * nr: 4 * nr + 4])
        assert np.array_equal(s["dk"][4 * nr: 4 * nr + 4], s["ek"][:4])


def test_expand_key_rejects_bad_sizes(ag):
    with pytest.raises(ag.AesError) as e:
        ag.expand_key(bytes(16), 100)
    assert e.value.status == ag.AES_ERR_KEYSIZE


def _reqs(n=4, op=2, length=4096):
    r = np.zeros(n, workloads.REQ_DTYPE)
    r["offset"] = np.arange(n) * length
    r["length"] = length
    r["op"] = op
    return r


FAKE = 1 << 40  # host-only context: device pointers are never dereferenced


@pytest.mark.parametrize("case,status", [
    ("cbc_len", "AES_ERR_LENGTH"),
    ("unaligned", "AES_ERR_RANGE"),
    ("past_end", "AES_ERR_RANGE"),
    ("key_idx", "AES_ERR_RANGE"),
    ("overlap", "AES_ERR_OVERLAP"),
    ("overlap_unsorted", "AES_ERR_OVERLAP"),
    ("bad_op", "AES_ERR_ARG"),
    ("huge", "AES_ERR_LENGTH"),
    ("alias", "AES_ERR_OVERLAP"),
    ("null", "AES_ERR_ARG"),
    ("ok", "AES_ERR_DEVICE"),
])
def test_validation_errors(ag, hctx, case, status):
    reqs = _reqs(op=1)
    d_in, d_out, buf = FAKE, FAKE + (1 << 30), 4 * 4096
    if case == "cbc_len":
        reqs["length"][2] = 4008
    elif case == "unaligned":
        reqs["offset"][1] += 8
    elif case == "past_end":
        reqs["length"][3] = 8192
    elif case == "key_idx":
        reqs["key_idx"][0] = 1
    elif case == "overlap":
        reqs["offset"][2] = 4096 + 16
        reqs["length"][2] = 1024
    elif case == "overlap_unsorted":
        reqs = reqs[[3, 0, 2, 1]].copy()
        reqs["offset"][0] = 4096 * 2 + 4096 - 16
        reqs["length"][0] = 32
        reqs["offset"][2] = 0
    elif case == "bad_op":
        reqs["op"][1] = 5
    elif case == "huge":
        reqs["length"][0] = 1 << 32
    elif case == "alias":
        d_out = d_in + 16
    elif case == "null":
        d_in = 0
    with pytest.raises(ag.AesError) as e:
        ag.batch(hctx, FAKE + (2 << 30), d_in, d_out, reqs, buf_bytes=buf, n_scheds=1)
    assert e.value.status == getattr(ag, status)


def test_empty_and_zero_length_are_noops(ag, hctx):
    ag.batch(hctx, 0, 0, 0, np.zeros(0, workloads.REQ_DTYPE), buf_bytes=0, n_scheds=0)
    reqs = _reqs()
    reqs["length"] = 0
    ag.batch(hctx, FAKE, FAKE, FAKE + (1 << 30), reqs, buf_bytes=4 * 4096, n_scheds=1)


def test_single_mode_entry_points_validate(ag, hctx):
    n = 3
    off = np.arange(n, dtype=np.uint64) * 4096
    ln = np.full(n, 4096, np.uint64)
    ki = np.zeros(n, np.uint32)
    iv = np.zeros((n, 16), np.uint8)
    for fn in (ag.cbc_encrypt_batch, ag.cbc_decrypt_batch, ag.ctr_batch):
        with pytest.raises(ag.AesError) as e:
            fn(hctx, FAKE, FAKE, FAKE + (1 << 30), off, ln, ki, iv, buf_bytes=n * 4096,
               n_scheds=1)
        assert e.value.status == ag.AES_ERR_DEVICE  # valid, but no device
    ln[1] = 17
    with pytest.raises(ag.AesError) as e:
        ag.cbc_decrypt_batch(hctx, FAKE, FAKE, FAKE + (1 << 30), off, ln, ki, iv,
                             buf_bytes=n * 4096, n_scheds=1)
    assert e.value.status == ag.AES_ERR_LENGTH
    ag.ctr_batch  # CTR takes any length: only the device is missing
    with pytest.raises(ag.AesError) as e:
        ag.ctr_batch(hctx, FAKE, FAKE, FAKE + (1 << 30), off, ln, ki, iv, buf_bytes=n * 4096,
                     n_scheds=1)
    assert e.value.status == ag.AES_ERR_DEVICE


# ------------------------------------------------------------------- planner

def _check_plan(ag, plan, reqs, tile, grouped=False):
    units = plan.units()
    info = plan.info()
    assert info["payload_bytes"] == int(reqs["length"].sum())
    op_of = (units["meta"] >> 24) & 7
    covered = {}
    for u in units:
        covered.setdefault(int(u["offset"]), []).append(u)
    # every request's bytes are covered exactly once by units of its op and key
    total = 0
    for r in reqs:
        off, ln, op = int(r["offset"]), int(r["length"]), int(r["op"])
        if ln == 0:
            continue
        pos = 0
        while pos < ln:
            us = covered.get(off + pos)
            assert us and len(us) == 1, (off, pos)
            u = us[0]
            assert ((int(u["meta"]) >> 24) & 7) == op
            assert (int(u["meta"]) & 0xFFFFFF) == int(r["key_idx"])
            n = int(u["nbytes"])
            if op == ag.AES_OP_CBC_ENC:
                assert n == ln and pos == 0
                assert np.array_equal(u["w"].astype("<u4").view(np.uint8), r["iv"])
            else:
                assert n == min(tile, ln - pos)
                if op == ag.AES_OP_CTR:
                    assert np.array_equal(u["w"][:2].astype("<u4").view(np.uint8), r["iv"][:8])
                    low = int.from_bytes(r["iv"][8:].tobytes(), "big")
                    ctr = int(u["w"][2]) | (int(u["w"][3]) << 32)
                    assert ctr == (low + pos // 16) % (1 << 64)
                elif op in (ag.AES_OP_ECB_ENC, ag.AES_OP_ECB_DEC):
                    assert not (int(u["meta"]) & (1 << 27)) and not u["w"].any()
                else:
                    pred_in = bool(int(u["meta"]) & (1 << 27))
                    assert pred_in == (pos > 0)
                    if pos == 0:
                        assert np.array_equal(u["w"].astype("<u4").view(np.uint8), r["iv"])
            pos += n
            total += n
    assert total == info["payload_bytes"]
    assert len(units) == info["n_units_cbc_dec"] + info["n_units_ctr"] + info["n_chains_cbc_enc"]
    # order: CBC- and ECB-decrypt tiles, CTR tiles, ECB-encrypt tiles, then chains
    k = info["n_units_cbc_dec"]
    assert np.isin(op_of[:k], (ag.AES_OP_CBC_DEC, ag.AES_OP_ECB_DEC)).all()
    enc_ops = op_of[k:k + info["n_units_ctr"]]
    assert np.isin(enc_ops, (ag.AES_OP_CTR, ag.AES_OP_ECB_ENC)).all()
    assert (np.diff((enc_ops == ag.AES_OP_ECB_ENC).astype(np.int64)) >= 0).all()
    ch = units[k + info["n_units_ctr"]:]
    ch_key = (ch["meta"] & 0xFFFFFF).astype(np.int64)
    ch_len = ch["nbytes"].astype(np.int64)
    assert (np.diff(ch_len) <= 0).all()  # chains longest first ...
    for ln in np.unique(ch_len):  # ... those of equal length by key
        assert (np.diff(ch_key[ch_len == ln]) >= 0).all()
    # CTR tiles, then ECB-encrypt tiles: each group in request order, or
    # (grouped) by key with request order kept within a key
    enc = units[k:k + info["n_units_ctr"]]
    order = np.argsort(reqs["offset"], kind="stable")
    for o in (ag.AES_OP_CTR, ag.AES_OP_ECB_ENC):
        mine = enc[((enc["meta"] >> 24) & 7) == o]
        # index of each tile's request in the caller's order
        pos = np.searchsorted(reqs["offset"][order], mine["offset"], side="right") - 1
        req_of = order[pos].astype(np.int64)
        key_of = (mine["meta"] & 0xFFFFFF).astype(np.int64)
        if grouped:
            assert (np.diff(key_of) >= 0).all()
            for key in np.unique(key_of):
                assert (np.diff(req_of[key_of == key]) >= 0).all()
        else:
            assert (np.diff(req_of) >= 0).all()


def test_plan_covers_config3_batch(ag, hctx):
    wl = workloads.config3(n_reqs=600, max_pages=64)
    plan = ag.Plan(hctx, wl.reqs, wl.keys.shape[0], wl.buf_bytes)
    _check_plan(ag, plan, wl.reqs, 4096)
    info = plan.info()
    assert info["extent_bytes"] == wl.buf_bytes and info["tile_bytes"] == 4096
    with pytest.raises(ag.AesError) as e:
        plan.launch(FAKE, FAKE, FAKE + (1 << 40))
    assert e.value.status == ag.AES_ERR_DEVICE
    plan.close()


def test_plan_ragged_ctr_and_counter_wrap(ag, hctx):
    r = np.zeros(5, workloads.REQ_DTYPE)
    lens = [1, 4095, 4097, 3 * 4096 + 5, 16 * 1000]
    off = 0
    for i, ln in enumerate(lens):
        r["offset"][i] = off
        r["length"][i] = ln
        off += (ln + 15) // 16 * 16 + 32
    r["op"] = ag.AES_OP_CTR
    r["iv"] = gen.bytes_(0, 2, 80).reshape(5, 16)
    r["iv"][3, 8:] = np.frombuffer(((1 << 64) - 3).to_bytes(8, "big"), np.uint8)
    plan = ag.Plan(hctx, r, 1, off)
    _check_plan(ag, plan, r, 4096)
    plan.close()


def test_plan_with_ecb_requests(ag, hctx):
    wl = workloads.config3(n_reqs=300, max_pages=16)
    wl.reqs["op"][::5] = ag.AES_OP_ECB_ENC
    wl.reqs["op"][2::5] = ag.AES_OP_ECB_DEC
    wl.reqs["length"][::5] = wl.reqs["length"][::5] // 16 * 16
    wl.reqs["length"][2::5] = wl.reqs["length"][2::5] // 16 * 16
    plan = ag.Plan(hctx, wl.reqs, wl.keys.shape[0], wl.buf_bytes)
    _check_plan(ag, plan, wl.reqs, 4096)
    plan.close()
    bad = wl.reqs.copy()
    bad["length"][0] = 4008 + 1
    with pytest.raises(ag.AesError) as e:
        ag.Plan(hctx, bad, wl.keys.shape[0], wl.buf_bytes)
    assert e.value.status == ag.AES_ERR_LENGTH


def test_plan_unsorted_requests(ag, hctx):
    wl = workloads.config3(n_reqs=50, max_pages=8)
    perm = np.random.default_rng(1).permutation(50)
    plan = ag.Plan(hctx, wl.reqs[perm], wl.keys.shape[0], wl.buf_bytes)
    _check_plan(ag, plan, wl.reqs[perm], 4096)
    plan.close()


def test_plan_chains_longest_first_across_keys(ag, hctx):
    """More CBC-encrypt chains than a launch starts in its first pass: the
    longest chain comes first even under the highest key index and last in
    request order, and chains of equal length follow key order (and request
    order within a key)."""
    n = 300
    r = np.random.default_rng(7)
    reqs = np.zeros(n, workloads.REQ_DTYPE)
    reqs["length"] = r.choice([4096, 16384, 65536], n).astype(np.uint64)
    reqs["length"][-1] = 1 << 20  # the longest chain: last request, highest key
    reqs["offset"][1:] = np.cumsum(reqs["length"])[:-1]
    reqs["key_idx"] = r.integers(0, 63, n)
    reqs["key_idx"][-1] = 63
    reqs["op"] = workloads.OP_CBC_ENC
    reqs["iv"] = gen.bytes_(0, gen.STREAM_IVS, 16 * n).reshape(n, 16)
    plan = ag.Plan(hctx, reqs, 64, int(reqs["offset"][-1] + reqs["length"][-1]))
    _check_plan(ag, plan, reqs, 4096)
    ch = plan.units()
    plan.close()
    assert int(ch["nbytes"][0]) == 1 << 20 and int(ch["meta"][0] & 0xFFFFFF) == 63
    want = sorted(range(n), key=lambda i: (-int(reqs["length"][i]), int(reqs["key_idx"][i]), i))
    assert [int(o) for o in ch["offset"]] == [int(reqs["offset"][i]) for i in want]


def test_launch_config_validation(ag, hctx):
    """Launch configurations are checked and stored without a device."""
    cfg = hctx.get_config()
    assert cfg["tile_bytes"] == 4096 and cfg["ctr_variant"] == ag.AES_CTR_TABLE
    hctx.set_config(ctr_variant=ag.AES_CTR_BITSLICE, tile_bytes=8192)
    got = hctx.get_config()
    assert got["ctr_variant"] == ag.AES_CTR_BITSLICE and got["tile_bytes"] == 8192
    hctx.set_config(dec_variant=ag.AES_DEC_BITSLICE)
    assert hctx.get_config()["dec_variant"] == ag.AES_DEC_BITSLICE
    got = hctx.get_config()
    for bad in ({"ctr_variant": 2}, {"dec_variant": 2}, {"chain_quad": 2}, {"tile_bytes": 1000},
                {"ctr_nb": 3},
                {"chain_lanes": 0},
                {"mixed_nb": 4}, {"fuse": 2}):
        with pytest.raises(ag.AesError) as e:
            hctx.set_config(**bad)
        assert e.value.status == ag.AES_ERR_ARG
        assert hctx.get_config() == got  # nothing changes on error
    hctx.set_config(**cfg)
    assert hctx.get_config() == cfg


@pytest.mark.parametrize("variant", ["table", "bitslice"])
@pytest.mark.parametrize("spread", [8, 200000])
def test_plan_orders_encryption_tiles(ag, hctx, spread, variant):
    """CTR tiles, then ECB-encrypt tiles: in request order under the table
    variant; grouped by key (ascending, request order kept within a key)
    under the bitsliced variant -- with few distinct key indices (the
    planner's counting sort) and with sparse ones (its stable-sort path)."""
    r = np.random.default_rng(spread)
    n = 120
    reqs = np.zeros(n, workloads.REQ_DTYPE)
    reqs["length"] = r.integers(1, 5, n) * 4096
    reqs["offset"][1:] = np.cumsum(reqs["length"])[:-1]
    reqs["op"] = np.where(r.random(n) < 0.3, ag.AES_OP_ECB_ENC, ag.AES_OP_CTR)
    keys = r.choice(spread, min(spread, 10), replace=False)
    reqs["key_idx"] = keys[r.integers(0, keys.size, n)]
    reqs["iv"] = gen.bytes_(spread, 2, 16 * n).reshape(n, 16)
    perm = r.permutation(n)  # callers' order need not be offset order
    reqs = reqs[perm]
    v = ag.AES_CTR_BITSLICE if variant == "bitslice" else ag.AES_CTR_TABLE
    hctx.set_config(ctr_variant=v)
    plan = ag.Plan(hctx, reqs, int(keys.max()) + 1, int(reqs["offset"].max() + 4 * 4096))
    _check_plan(ag, plan, reqs, 4096, grouped=variant == "bitslice")
    units = plan.units()
    plan.close()
    op = (units["meta"] >> 24) & 7
    assert np.flatnonzero(op == ag.AES_OP_CTR).max() < np.flatnonzero(op == ag.AES_OP_ECB_ENC).min()


@pytest.mark.parametrize("variant", ["table", "bitslice"])
@pytest.mark.parametrize("spread", [8, 200000])
def test_plan_orders_decryption_tiles(ag, hctx, spread, variant):
    """CBC- and ECB-decrypt tiles: in request order under the table variant;
    grouped by key (ascending, request order kept within a key) under the
    bitsliced decryption variant; snapshots flags and IVs as always."""
    r = np.random.default_rng(spread + 1)
    n = 120
    reqs = np.zeros(n, workloads.REQ_DTYPE)
    reqs["length"] = r.integers(1, 5, n) * 4096
    reqs["offset"][1:] = np.cumsum(reqs["length"])[:-1]
    reqs["op"] = np.where(r.random(n) < 0.3, ag.AES_OP_ECB_DEC, ag.AES_OP_CBC_DEC)
    keys = r.choice(spread, min(spread, 10), replace=False)
    reqs["key_idx"] = keys[r.integers(0, keys.size, n)]
    reqs["iv"] = gen.bytes_(spread, 2, 16 * n).reshape(n, 16)
    reqs = reqs[r.permutation(n)]
    v = ag.AES_DEC_BITSLICE if variant == "bitslice" else ag.AES_DEC_TABLE
    hctx.set_config(dec_variant=v)
    plan = ag.Plan(hctx, reqs, int(keys.max()) + 1, int(reqs["offset"].max() + 4 * 4096))
    _check_plan(ag, plan, reqs, 4096)
    units = plan.units()
    info = plan.info()
    plan.close()
    dec = units[:info["n_units_cbc_dec"]]
    order = np.argsort(reqs["offset"], kind="stable")
    pos = np.searchsorted(reqs["offset"][order], dec["offset"], side="right") - 1
    req_of = order[pos].astype(np.int64)
    key_of = (dec["meta"] & 0xFFFFFF).astype(np.int64)
    if variant == "bitslice":
        assert (np.diff(key_of) >= 0).all()
        for key in np.unique(key_of):
            mine = req_of[key_of == key]
            assert (np.diff(mine) >= 0).all()
    else:
        assert (np.diff(req_of) >= 0).all()


def _status(fn, *a, **k):
    from paper_1305_3345_amd import aesgpu
    try:
        fn(*a, **k)
    except aesgpu.AesError as e:
        return e.status
    return 0


@pytest.mark.parametrize("op", ["cbc_dec", "ctr", "ecb_enc", "ecb_dec"])
def test_large_single_calls_validate_like_plans(ag, hctx, op):
    """Single-op calls of 20,000 requests take the chunked parallel path
    (chunks of 4,096); every rule violation, overlap and ordering case --
    inside a chunk, across a chunk boundary, and two errors at once -- must
    give the status the serial validator of aes_plan_create gives."""
    n, page = 20000, 4096
    opnum = {"cbc_dec": ag.AES_OP_CBC_DEC, "ctr": ag.AES_OP_CTR, "ecb_enc": ag.AES_OP_ECB_ENC,
             "ecb_dec": ag.AES_OP_ECB_DEC}[op]
    fn = {"cbc_dec": ag.cbc_decrypt_batch, "ctr": ag.ctr_batch, "ecb_enc": ag.ecb_encrypt_batch,
          "ecb_dec": ag.ecb_decrypt_batch}[op]
    buf = n * page

    def base():
        r = np.zeros(n, workloads.REQ_DTYPE)
        r["offset"] = np.arange(n, dtype=np.uint64) * page
        r["length"] = page
        r["op"] = opnum
        r["key_idx"] = np.arange(n) % 16
        r["iv"] = gen.bytes_(7, 2, 16 * n).reshape(n, 16)
        r["length"][::97] = 0
        return r

    cases = {"valid": lambda r: None}
    for k in (3, 4095, 4096, 12000, n - 1):
        cases[f"misaligned@{k}"] = lambda r, k=k: r["offset"].__setitem__(k, r["offset"][k] + 8)
        cases[f"past_end@{k}"] = lambda r, k=k: r["length"].__setitem__(k, buf)
        cases[f"bad_key@{k}"] = lambda r, k=k: r["key_idx"].__setitem__(k, 16)
        cases[f"overlap@{k}"] = lambda r, k=k: r["length"].__setitem__(k - 1, 2 * page)
        cases[f"ragged@{k}"] = lambda r, k=k: r["length"].__setitem__(k, page - 8)
    cases["permuted"] = lambda r: r.__setitem__(slice(None), r[np.random.default_rng(1).permutation(n)])

    def permuted_overlap(r):
        r["length"][5000] = 2 * page
        r[:] = r[np.random.default_rng(2).permutation(n)]
    cases["permuted_overlap"] = permuted_overlap

    def two_errors_a(r):  # range error before a length error
        r["key_idx"][9000] = 99
        r["length"][15000] = page - 8

    def two_errors_b(r):  # overlap early, range error late: rules come first
        r["length"][100] = 2 * page
        r["offset"][19000] += 8
    cases["two_errors_a"] = two_errors_a
    cases["two_errors_b"] = two_errors_b
    for name, mutate in cases.items():
        r = base()
        mutate(r)
        want = _status(ag.Plan, hctx, r, 16, buf)
        want = ag.AES_ERR_DEVICE if want == 0 else want  # a plan is made; a call needs the GPU
        got = _status(fn, hctx, FAKE, FAKE, FAKE + (1 << 40), r["offset"], r["length"],
                      r["key_idx"], r["iv"], buf_bytes=buf, n_scheds=16)
        assert got == want, f"{op} {name}: call {got}, plan {want}"
