// aes_abi.cpp -- the C ABI: validation, planning, contexts, plans, launches.
//
// A call follows the service-request path of the paper (section 3.2): the
// caller hands over input and output buffers and a request list; the library
// checks every request on the host, cuts the requests into work units
// (section 2: one launch carries one large task or many small tasks), copies
// the unit table to the device through pinned staging and launches the round
// kernels on the caller's stream.
#include <hip/hip_runtime.h>
#include <sched.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "host_pool.h"
#include "internal.h"
#include "tune_cache.h"

using namespace aesgpu;

namespace {

thread_local int g_last_hip = 0;

int hip_fail(hipError_t e) {
    g_last_hip = (int)e;
    return AES_ERR_DEVICE;
}

}  // namespace

int aesgpu::hip_fail_status(int hip_error) { return hip_fail((hipError_t)hip_error); }

namespace {

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return hip_fail(e_);                                                                   \
    } while (0)

constexpr uint64_t MAX_REQ_BYTES = (1ull << 32) - 16;
constexpr uint32_t DEFAULT_TILE = 4096;

// ------------------------------------------------------------- validation

// The rules one request must meet (op already known to be valid), in the
// order whose first failure a call reports.
inline int check_request(uint32_t op, uint64_t off, uint64_t len, uint32_t key,
                         uint32_t n_scheds, uint64_t buf_bytes) {
    if (len > MAX_REQ_BYTES || (op != AES_OP_CTR && (len & 15)))
        return AES_ERR_LENGTH;
    if ((off & 15) || off > buf_bytes || len > buf_bytes - off || key >= n_scheds ||
        key >= MAX_KEYS)
        return AES_ERR_RANGE;
    return AES_OK;
}

// Checks one request list against buffer size and schedule count, and that
// the written byte ranges are pairwise disjoint.
int validate(const aes_req_t *reqs, uint64_t n, uint32_t n_scheds, uint64_t buf_bytes) {
    if (n && !reqs)
        return AES_ERR_ARG;
    bool sorted = true;
    uint64_t last_off = 0;
    for (uint64_t i = 0; i < n; i++) {
        const aes_req_t &r = reqs[i];
        if (r.op > AES_OP_ECB_DEC)
            return AES_ERR_ARG;
        const int st = check_request(r.op, r.offset, r.length, r.key_idx, n_scheds, buf_bytes);
        if (st)
            return st;
        if (r.length) {
            if (r.offset < last_off)
                sorted = false;
            last_off = r.offset;
        }
    }
    // Disjointness: a linear scan when the requests come in offset order
    // (the common case), else a sort of (offset, end) pairs.
    if (sorted) {
        uint64_t end = 0;
        bool any = false;
        for (uint64_t i = 0; i < n; i++) {
            if (!reqs[i].length)
                continue;
            if (any && reqs[i].offset < end)
                return AES_ERR_OVERLAP;
            end = reqs[i].offset + reqs[i].length;
            any = true;
        }
        return AES_OK;
    }
    std::vector<std::pair<uint64_t, uint64_t>> ranges;
    try {
        ranges.reserve(n);
    } catch (const std::bad_alloc &) {
        return AES_ERR_NOMEM;
    }
    for (uint64_t i = 0; i < n; i++)
        if (reqs[i].length)
            ranges.emplace_back(reqs[i].offset, reqs[i].offset + reqs[i].length);
    std::sort(ranges.begin(), ranges.end());
    for (size_t i = 1; i < ranges.size(); i++)
        if (ranges[i].first < ranges[i - 1].second)
            return AES_ERR_OVERLAP;
    return AES_OK;
}

int check_buffers(const uint8_t *d_in, const uint8_t *d_out, uint64_t buf_bytes, uint64_t n,
                  const void *d_scheds) {
    if (!n)
        return AES_OK;
    if (!d_in || !d_out || !d_scheds)
        return AES_ERR_ARG;
    if (d_in != d_out) {
        const uintptr_t a = (uintptr_t)d_in, b = (uintptr_t)d_out;
        if (a < b + buf_bytes && b < a + buf_bytes)
            return AES_ERR_OVERLAP;
    }
    return AES_OK;
}

// ---------------------------------------------------------------- planner

inline uint32_t le32(const uint8_t *p) {
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

inline uint64_t be64(const uint8_t *p) {
    uint64_t v = 0;
    for (int i = 0; i < 8; i++)
        v = (v << 8) | p[i];
    return v;
}

struct Planned {
    std::vector<Unit> dec;     // CBC- and ECB-decrypt tiles
    std::vector<Unit> ctr;     // CTR tiles, then ECB-encrypt tiles (the last n_ecb)
    std::vector<Unit> chains;  // CBC-encrypt chains, longest first, ties by key
    uint64_t payload = 0;
    uint64_t extent = 0;
    uint64_t dec_bytes = 0, ctr_bytes = 0, chain_bytes = 0;
    bool dec_has_pred_in = false;
    size_t n_ecb = 0;  // ECB-encrypt tiles at the end of ctr
    std::vector<Unit> ecb;       // ECB-encrypt tiles while planning (appended to ctr)
    std::vector<Unit> sort_buf;  // scratch of the key grouping

    // Empties the plan and keeps the vectors' storage: a context reuses one
    // Planned for every single-call batch, so a call touches no fresh pages.
    void reset() {
        dec.clear();
        ctr.clear();
        ecb.clear();
        chains.clear();
        payload = extent = 0;
        dec_bytes = ctr_bytes = chain_bytes = 0;
        dec_has_pred_in = false;
        n_ecb = 0;
    }
};

bool is_dec_tile_op(uint32_t op) { return op == AES_OP_CBC_DEC || op == AES_OP_ECB_DEC; }
bool is_enc_tile_op(uint32_t op) { return op == AES_OP_CTR || op == AES_OP_ECB_ENC; }

// Stable grouping of tiles by key index.  A counting sort over the key
// indices in use (one pass to count, one to place; buf is scratch) when they
// are dense enough, else a stable sort.
void group_by_key(std::vector<Unit> &t, std::vector<Unit> &buf) {
    uint32_t max_key = 0;
    for (const Unit &u : t)
        max_key = std::max(max_key, u.meta & META_KEY_MASK);
    const uint64_t n_keys = (uint64_t)max_key + 1;
    if (n_keys > 4 * (uint64_t)t.size() + 64) {
        std::stable_sort(t.begin(), t.end(), [](const Unit &a, const Unit &b) {
            return (a.meta & META_KEY_MASK) < (b.meta & META_KEY_MASK);
        });
        return;
    }
    std::vector<uint64_t> start(n_keys + 1, 0);
    for (const Unit &u : t)
        start[(u.meta & META_KEY_MASK) + 1]++;
    for (uint64_t i = 0; i < n_keys; i++)
        start[i + 1] += start[i];
    buf.resize(t.size());
    for (const Unit &u : t)
        buf[start[u.meta & META_KEY_MASK]++] = u;
    t.swap(buf);
}

// Cuts every request into units: CTR, ECB and CBC-decrypt into tile_bytes
// tiles (a multiple of 16), CBC-encrypt into one chain each.  p is emptied
// first (its storage kept).  Encryption-side tiles: CTR tiles, then
// ECB-encrypt tiles (the bitsliced kernel takes only the CTR range); with
// group_ctr each of the two groups is ordered by key (request order kept
// within a key), and with group_dec the decryption tiles are, which the
// bitsliced kernels need to share one schedule across a wave's tiles -- the
// table kernels read a schedule per tile.
int plan_units(const aes_req_t *reqs, uint64_t n, uint32_t tile_bytes, bool group_ctr,
               bool group_dec, Planned &p) {
    p.reset();
    try {
        uint64_t n_tiles_ctr = 0, n_tiles_dec = 0, n_chain = 0;
        for (uint64_t i = 0; i < n; i++) {
            const uint64_t t = (reqs[i].length + tile_bytes - 1) / tile_bytes;
            if (is_enc_tile_op(reqs[i].op))
                n_tiles_ctr += t;
            else if (is_dec_tile_op(reqs[i].op))
                n_tiles_dec += t;
            else if (reqs[i].length)
                n_chain++;
        }
        if (n_tiles_ctr >= (1ull << 32) || n_tiles_dec >= (1ull << 32) || n_chain >= (1ull << 32))
            return AES_ERR_RANGE;
        p.ctr.reserve(n_tiles_ctr);
        p.dec.reserve(n_tiles_dec);
        p.chains.reserve(n_chain);
        for (uint64_t i = 0; i < n; i++) {
            const aes_req_t &r = reqs[i];
            if (!r.length)
                continue;
            p.payload += r.length;
            p.extent = std::max(p.extent, r.offset + r.length);
            (r.op == AES_OP_CBC_ENC ? p.chain_bytes
                                    : is_enc_tile_op(r.op) ? p.ctr_bytes : p.dec_bytes) += r.length;
            const uint32_t meta_base = r.key_idx | (r.op << META_OP_SHIFT);
            if (r.op == AES_OP_CBC_ENC) {
                Unit u;
                u.off = r.offset;
                u.nbytes = (uint32_t)r.length;
                u.meta = meta_base;
                for (int w = 0; w < 4; w++)
                    u.w[w] = le32(r.iv + 4 * w);
                p.chains.push_back(u);
                continue;
            }
            const uint64_t ctr0 = be64(r.iv + 8);
            for (uint64_t pos = 0; pos < r.length; pos += tile_bytes) {
                Unit u;
                u.off = r.offset + pos;
                u.nbytes = (uint32_t)std::min<uint64_t>(tile_bytes, r.length - pos);
                u.meta = meta_base;
                if (r.op == AES_OP_CTR) {
                    const uint64_t c = ctr0 + pos / 16;  // mod 2^64, nonce untouched
                    u.w[0] = le32(r.iv);
                    u.w[1] = le32(r.iv + 4);
                    u.w[2] = (uint32_t)c;
                    u.w[3] = (uint32_t)(c >> 32);
                    p.ctr.push_back(u);
                } else if (r.op == AES_OP_ECB_ENC || r.op == AES_OP_ECB_DEC) {
                    u.w[0] = u.w[1] = u.w[2] = u.w[3] = 0;  // every block on its own
                    (r.op == AES_OP_ECB_ENC ? p.ecb : p.dec).push_back(u);
                } else {
                    if (pos == 0) {
                        for (int w = 0; w < 4; w++)
                            u.w[w] = le32(r.iv + 4 * w);
                    } else {
                        u.meta |= FLAG_PRED_IN;
                        u.w[0] = u.w[1] = u.w[2] = u.w[3] = 0;
                        p.dec_has_pred_in = true;
                    }
                    p.dec.push_back(u);
                }
            }
        }
        if (group_ctr) {
            group_by_key(p.ctr, p.sort_buf);
            group_by_key(p.ecb, p.sort_buf);
        }
        if (group_dec)
            group_by_key(p.dec, p.sort_buf);
        p.n_ecb = p.ecb.size();
        p.ctr.insert(p.ctr.end(), p.ecb.begin(), p.ecb.end());
        // Chains longest first across the batch, so that when there are more
        // chains than chain slots the longest start in the first pass and the
        // batch's makespan is as short as the chains allow; chains of equal
        // length are grouped by key (a wave runs the largest round count
        // among its chains for all of them, so same-key chains share waves).
        std::stable_sort(p.chains.begin(), p.chains.end(), [](const Unit &a, const Unit &b) {
            const uint32_t ka = a.meta & META_KEY_MASK, kb = b.meta & META_KEY_MASK;
            return a.nbytes != b.nbytes ? a.nbytes > b.nbytes : ka < kb;
        });
    } catch (const std::bad_alloc &) {
        return AES_ERR_NOMEM;
    }
    return AES_OK;
}

}  // namespace

// ---------------------------------------------------------------- context

struct Slot {
    void *h_stage = nullptr;  // pinned host staging for the unit table
    size_t h_cap = 0;
    void *d_units = nullptr;  // device unit table + in-place predecessor snapshots
    size_t d_cap = 0;
    hipEvent_t ev = nullptr;  // recorded after the last launch that used the slot
    bool ev_pending = false;
    hipEvent_t copied = nullptr;  // the unit table's upload on the copy stream
    uint32_t *d_ctrs = nullptr;   // tile-kernel counters: decryption side, then encryption
};

struct aes_ctx {
    int device = AES_DEVICE_NONE;
    int n_cu = 0;
    char arch[32] = "host";  // device architecture (gcnArchName up to ':'), for the tune cache
    uint32_t *d_timg = nullptr;
    static constexpr int N_SLOTS = 4;
    Slot slots[N_SLOTS];
    int next_slot = 0;
    uint32_t tile_bytes = DEFAULT_TILE;
    TileLaunch tile_ctr;
    TileLaunch tile_dec;
    ChainLaunch chain{256, 64, true, 0};  // four lanes per chain
    int mixed_nb = 1;        // fused kernel: 1 block per lane (its chain path takes the VGPRs)
    bool fuse = true;        // one launch for batches that mix ops
    int grid = 0;            // tile / fused kernel workgroups, 0 = one per compute unit
    uint32_t ctr_variant = AES_CTR_TABLE;
    uint32_t dec_variant = AES_DEC_TABLE;
    hipStream_t capture = nullptr;  // private stream for graph capture and tuning
    // Scratch of the single-call forms, reused from call to call (a context
    // is used by one thread at a time): requests built from the caller's
    // arrays, and the plan of the batch.
    std::vector<aes_req_t> scratch_reqs;
    Planned scratch_plan;
    std::unique_ptr<HostPool> pool;  // large single-op calls (created on first use)
    hipStream_t copy = nullptr;      // unit-table uploads of the single-call forms
};

struct aes_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
    uint64_t n_nodes = 0;
};

struct aes_plan {
    aes_ctx *ctx = nullptr;
    Planned p;
    uint32_t n_scheds = 0;
    uint64_t buf_bytes = 0;
    void *d_units = nullptr;  // [dec | ctr | chains] units, then dec predecessor snapshots
    uint32_t *d_ctrs = nullptr;  // tile-kernel counters: decryption side, then encryption
    size_t n_dec = 0, n_ctr = 0, n_chain = 0;
    uint32_t tile_bytes = DEFAULT_TILE;
};

int aesgpu::ctx_info(const aes_ctx_t *ctx, CtxInfo *out) {
    if (!ctx || !out)
        return AES_ERR_ARG;
    out->device = ctx->device;
    out->n_cu = ctx->n_cu;
    out->d_timg = ctx->d_timg;
    return AES_OK;
}

namespace {

size_t units_bytes(size_t n_dec, size_t n_ctr, size_t n_chain) {
    return (n_dec + n_ctr + n_chain) * sizeof(Unit) + n_dec * 16;
}

struct PlanView {
    void *d_units;
    uint32_t *d_ctrs;  // 2 x TILE_CTRS zeroed counters of the tile launches
    size_t n_dec, n_ctr, n_chain;
    bool pred_in;
    uint64_t dec_bytes, ctr_bytes;
    size_t n_ecb;  // ECB-encrypt tiles: the last n_ecb of the n_ctr encryption tiles
};

PlanView view_of(const Planned &p, void *d_units, uint32_t *d_ctrs) {
    return PlanView{d_units, d_ctrs, p.dec.size(), p.ctr.size(), p.chains.size(), p.dec_has_pred_in,
                    p.dec_bytes, p.ctr_bytes, p.n_ecb};
}

// Zeroed tile-kernel counters for one plan or staging slot (the kernels
// leave them zeroed after every launch).
int alloc_tile_ctrs(uint32_t **out) {
    const size_t bytes = 2 * (size_t)TILE_CTRS * sizeof(uint32_t);
    if (hipMalloc((void **)out, bytes) != hipSuccess) {
        *out = nullptr;
        return AES_ERR_NOMEM;
    }
    const hipError_t e = hipMemset(*out, 0, bytes);
    if (e != hipSuccess) {
        (void)hipFree(*out);
        *out = nullptr;
        return hip_fail(e);
    }
    return AES_OK;
}

// Takes the context's next staging slot for a call whose unit table has
// ubytes bytes (need = device bytes with the in-place snapshots): waits for
// the slot's last launch, then grows its pinned and device buffers if needed.
int take_slot(aes_ctx *ctx, size_t ubytes, size_t need, Slot **out) {
    HIP_TRY(hipSetDevice(ctx->device));
    Slot &s = ctx->slots[ctx->next_slot];
    ctx->next_slot = (ctx->next_slot + 1) % aes_ctx::N_SLOTS;
    if (s.ev_pending) {
        HIP_TRY(hipEventSynchronize(s.ev));
        s.ev_pending = false;
    }
    if (s.h_cap < ubytes) {
        if (s.h_stage)
            (void)hipHostFree(s.h_stage);
        s.h_stage = nullptr;
        s.h_cap = 0;
        if (hipHostMalloc(&s.h_stage, ubytes, hipHostMallocDefault) != hipSuccess)
            return AES_ERR_NOMEM;
        s.h_cap = ubytes;
    }
    if (s.d_cap < need) {
        if (s.d_units)
            (void)hipFree(s.d_units);
        s.d_units = nullptr;
        s.d_cap = 0;
        if (hipMalloc(&s.d_units, need) != hipSuccess)
            return AES_ERR_NOMEM;
        s.d_cap = need;
    }
    if (!s.d_ctrs) {
        const int st = alloc_tile_ctrs(&s.d_ctrs);
        if (st)
            return st;
    }
    *out = &s;
    return AES_OK;
}

// Uploads a slot's unit table for a launch on `stream`.  When the stream is
// not being captured, the copy goes on the context's copy stream and the
// launch waits for it by event, so the upload of one call overlaps the
// kernels of the call before; under capture it stays on `stream`.  The slot
// is free of earlier uploads and launches (its event was waited for).
int upload_units(aes_ctx *ctx, Slot &s, size_t ubytes, void *stream) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing((hipStream_t)stream, &cap));
    if (cap == hipStreamCaptureStatusNone && !ctx->copy &&
        hipStreamCreateWithFlags(&ctx->copy, hipStreamNonBlocking) != hipSuccess)
        ctx->copy = nullptr;
    if (cap != hipStreamCaptureStatusNone || !ctx->copy) {
        HIP_TRY(hipMemcpyAsync(s.d_units, s.h_stage, ubytes, hipMemcpyHostToDevice,
                               (hipStream_t)stream));
        return AES_OK;
    }
    HIP_TRY(hipMemcpyAsync(s.d_units, s.h_stage, ubytes, hipMemcpyHostToDevice, ctx->copy));
    HIP_TRY(hipEventRecord(s.copied, ctx->copy));
    HIP_TRY(hipStreamWaitEvent((hipStream_t)stream, s.copied, 0));
    return AES_OK;
}

// Workgroups of the fused kernel that hold the decryption tables: a share of
// the grid proportional to the CBC-decrypt bytes among the parallel bytes.
uint32_t dec_workgroups(const PlanView &v, int grid) {
    if (!v.n_dec)
        return 0;
    if (!v.n_ctr && !v.n_chain)
        return (uint32_t)grid;
    const double share = (double)v.dec_bytes / (double)(v.dec_bytes + v.ctr_bytes + 1);
    long k = std::lround(share * grid);
    if (k < 1)
        k = 1;
    if (k > grid - 1)
        k = grid - 1;
    return (uint32_t)k;
}

// Launches the kernels of one planned batch whose unit table is at v.d_units.
int launch_planned(aes_ctx *ctx, const PlanView &v, const aes_schedule_t *d_scheds,
                   uint32_t n_scheds, const uint8_t *d_in, uint8_t *d_out, void *stream) {
    Unit *u = (Unit *)v.d_units;
    Unit *u_dec = u;
    Unit *u_ctr = u + v.n_dec;
    Unit *u_chain = u + v.n_dec + v.n_ctr;
    void *d_preds = nullptr;
    int e;
    if (v.n_dec && v.pred_in && d_in == d_out) {
        d_preds = (void *)(u + v.n_dec + v.n_ctr + v.n_chain);
        if ((e = launch_snapshot_preds(u_dec, (uint32_t)v.n_dec, d_in, d_preds, stream)))
            return hip_fail((hipError_t)e);
    }
    // The bitsliced decryption kernel takes every decryption tile in a launch
    // of its own (the predecessor snapshots above included).
    size_t n_dec = v.n_dec;
    if (n_dec && ctx->dec_variant == AES_DEC_BITSLICE) {
        if ((e = launch_dec_bitslice(u_dec, (uint32_t)n_dec, d_scheds, n_scheds, d_preds, d_in,
                                     d_out, stream)))
            return hip_fail((hipError_t)e);
        n_dec = 0;
    }
    // The bitsliced CTR kernel has a launch of its own for the CTR tiles; the
    // table kernels then take only the ECB-encrypt tiles of that range.
    const size_t n_ctr_only = v.n_ctr - v.n_ecb;
    const bool bitslice = ctx->ctr_variant == AES_CTR_BITSLICE && n_ctr_only;
    if (bitslice && (e = launch_ctr_bitslice(u_ctr, (uint32_t)n_ctr_only, d_scheds, n_scheds,
                                             d_in, d_out, ctx->n_cu, stream)))
        return hip_fail((hipError_t)e);
    if (bitslice)
        u_ctr += n_ctr_only;
    const size_t n_ctr_tab = bitslice ? v.n_ecb : v.n_ctr;
    const int kinds = (n_dec > 0) + (n_ctr_tab > 0) + (v.n_chain > 0);
    // One fused launch when CBC-encrypt chains share the batch with tiles: the
    // long chains then run beside the tiles on the workgroups the split gives
    // them.  Without chains, one launch per table set is faster (the tile
    // kernels carry no chain registers).
    if (ctx->fuse && v.n_chain > 0 && kinds > 1) {
        const int grid = ctx->grid > 0 ? ctx->grid : ctx->n_cu;
        MixedArgs a;
        a.dec = u_dec;
        a.ctr = u_ctr;
        a.chains = u_chain;
        a.preds = (const uint32_t *)d_preds;
        a.sched = d_scheds;
        a.timg = ctx->d_timg;
        a.in = d_in;
        a.out = d_out;
        a.n_dec = (uint32_t)n_dec;
        a.n_ctr = (uint32_t)n_ctr_tab;
        a.n_chain = (uint32_t)v.n_chain;
        a.n_sched = n_scheds;
        PlanView fused = v;
        fused.n_dec = n_dec;
        fused.n_ctr = n_ctr_tab;
        fused.ctr_bytes = bitslice ? (v.n_ctr ? v.ctr_bytes * v.n_ecb / v.n_ctr : 0)
                                   : v.ctr_bytes;
        a.n_dec_wg = dec_workgroups(fused, grid);
        a.chain_lanes = (uint32_t)ctx->chain.lanes;
        a.chain_quad = ctx->chain.quad ? 1u : 0u;
        if ((e = launch_mixed(a, ctx->mixed_nb, grid, stream)))
            return hip_fail((hipError_t)e);
        return AES_OK;
    }
    if ((e = launch_cbcdec_tiles(u_dec, (uint32_t)n_dec, d_scheds, n_scheds, ctx->d_timg,
                                 d_preds, d_in, d_out, v.d_ctrs, ctx->tile_dec, ctx->n_cu,
                                 stream)))
        return hip_fail((hipError_t)e);
    if ((e = launch_ctr_tiles(u_ctr, (uint32_t)n_ctr_tab, d_scheds, n_scheds, ctx->d_timg, d_in,
                              d_out, v.d_ctrs + TILE_CTRS, ctx->tile_ctr, ctx->n_cu, stream)))
        return hip_fail((hipError_t)e);
    if ((e = launch_cbcenc_chains(u_chain, (uint32_t)v.n_chain, d_scheds, n_scheds, ctx->d_timg,
                                  d_in, d_out, ctx->chain, ctx->n_cu, stream)))
        return hip_fail((hipError_t)e);
    return AES_OK;
}

void pack_units(const Planned &p, void *dst) {
    Unit *u = (Unit *)dst;
    if (!p.dec.empty())
        memcpy(u, p.dec.data(), p.dec.size() * sizeof(Unit));
    u += p.dec.size();
    if (!p.ctr.empty())
        memcpy(u, p.ctr.data(), p.ctr.size() * sizeof(Unit));
    u += p.ctr.size();
    if (!p.chains.empty())
        memcpy(u, p.chains.data(), p.chains.size() * sizeof(Unit));
}

int run_batch(aes_ctx *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
              const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes, const aes_req_t *reqs,
              uint64_t n, void *stream) {
    if (!ctx)
        return AES_ERR_ARG;
    int st = check_buffers(d_in, d_out, buf_bytes, n, d_scheds);
    if (st)
        return st;
    if ((st = validate(reqs, n, n_scheds, buf_bytes)))
        return st;
    Planned &p = ctx->scratch_plan;
    if ((st = plan_units(reqs, n, ctx->tile_bytes, ctx->ctr_variant == AES_CTR_BITSLICE,
                         ctx->dec_variant == AES_DEC_BITSLICE, p)))
        return st;
    if (!p.payload)
        return AES_OK;
    if (ctx->device == AES_DEVICE_NONE)
        return AES_ERR_DEVICE;
    const size_t ubytes = (p.dec.size() + p.ctr.size() + p.chains.size()) * sizeof(Unit);
    const size_t need = units_bytes(p.dec.size(), p.ctr.size(), p.chains.size());
    Slot *sp = nullptr;
    if ((st = take_slot(ctx, ubytes, need, &sp)))
        return st;
    Slot &s = *sp;
    pack_units(p, s.h_stage);
    if ((st = upload_units(ctx, s, ubytes, stream)))
        return st;
    st = launch_planned(ctx, view_of(p, s.d_units, s.d_ctrs), d_scheds, n_scheds, d_in, d_out,
                        stream);
    if (st)
        return st;
    HIP_TRY(hipEventRecord(s.ev, (hipStream_t)stream));
    s.ev_pending = true;
    return AES_OK;
}

// ------------------------------------------------- batches without allocation

// aes_batch_noalloc keeps its unit table, in-place predecessor snapshots and
// tile counters in one fixed device array per GPU (`scratch`), and plans on
// the host into fixed static arrays, so that a call allocates nothing.  Its
// device address is taken once per device when a context is created there
// (host code never uses the array's name for device memory).  Every call on a
// device shares that device's array: calls that overlap in time on one device
// (other streams, or other host threads) race on it.
constexpr uint64_t NOALLOC_UNITS_BYTES = (uint64_t)AES_NOALLOC_MAX_UNITS * sizeof(Unit);
constexpr uint64_t NOALLOC_PREDS_BYTES = (uint64_t)AES_NOALLOC_MAX_UNITS * 16;
constexpr uint64_t NOALLOC_CTRS_OFF = NOALLOC_UNITS_BYTES + NOALLOC_PREDS_BYTES;
constexpr uint64_t NOALLOC_SCRATCH_BYTES =
    NOALLOC_CTRS_OFF + 2 * (uint64_t)TILE_CTRS * sizeof(uint32_t);

static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES];  // device address of `scratch`, per device

// Host side of a call: the unit table is built here and copied from here;
// the ranges hold the disjointness check of unsorted requests.  Guarded by
// g_noalloc_mu for the whole of a call's host work.
std::mutex g_noalloc_mu;
Unit g_noalloc_units[AES_NOALLOC_MAX_UNITS];
std::pair<uint64_t, uint64_t> g_noalloc_ranges[AES_NOALLOC_MAX_UNITS];

// Takes the device address of `scratch` on the current device (once per
// device).  The caller has made `device` current.
int noalloc_setup(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES)
        return AES_OK;  // such a device has no scratch; its no-allocation calls fail
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device])
        return AES_OK;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol);
    g_scratch_ptr[device] = p;
    return AES_OK;
}

int run_batch_noalloc(aes_ctx *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                      const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                      const aes_req_t *reqs, uint64_t n, void *stream) {
    if (!ctx)
        return AES_ERR_ARG;
    int st = check_buffers(d_in, d_out, buf_bytes, n, d_scheds);
    if (st)
        return st;
    if (n && !reqs)
        return AES_ERR_ARG;
    // 1. The per-request rules (as validate), order, and the unit counts.
    const uint32_t tile = ctx->tile_bytes;
    uint64_t n_dec = 0, n_ctr = 0, n_ecb = 0, n_chain = 0, n_live = 0, payload = 0;
    uint64_t dec_bytes = 0, ctr_bytes = 0, last_off = 0;
    bool sorted = true, pred_in = false;
    for (uint64_t i = 0; i < n; i++) {
        const aes_req_t &r = reqs[i];
        if (r.op > AES_OP_ECB_DEC)
            return AES_ERR_ARG;
        if ((st = check_request(r.op, r.offset, r.length, r.key_idx, n_scheds, buf_bytes)))
            return st;
        if (!r.length)
            continue;
        if (r.offset < last_off)
            sorted = false;
        last_off = r.offset;
        n_live++;
        payload += r.length;
        const uint64_t t = (r.length + tile - 1) / tile;
        if (r.op == AES_OP_CBC_ENC) {
            n_chain++;
        } else if (is_dec_tile_op(r.op)) {
            n_dec += t;
            dec_bytes += r.length;
            pred_in |= r.op == AES_OP_CBC_DEC && t > 1;
        } else {
            (r.op == AES_OP_CTR ? n_ctr : n_ecb) += t;
            ctr_bytes += r.length;
        }
    }
    const uint64_t n_units = n_dec + n_ctr + n_ecb + n_chain;
    if (n_units > AES_NOALLOC_MAX_UNITS)
        return AES_ERR_RANGE;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    // 2. Disjoint output ranges: a linear scan in offset order, else a sort
    //    of (offset, end) pairs in the static array (n_live <= n_units).
    if (sorted) {
        uint64_t end = 0;
        bool any = false;
        for (uint64_t i = 0; i < n; i++) {
            if (!reqs[i].length)
                continue;
            if (any && reqs[i].offset < end)
                return AES_ERR_OVERLAP;
            end = reqs[i].offset + reqs[i].length;
            any = true;
        }
    } else {
        uint64_t k = 0;
        for (uint64_t i = 0; i < n; i++)
            if (reqs[i].length)
                g_noalloc_ranges[k++] = {reqs[i].offset, reqs[i].offset + reqs[i].length};
        std::sort(g_noalloc_ranges, g_noalloc_ranges + k);
        for (uint64_t i = 1; i < k; i++)
            if (g_noalloc_ranges[i].first < g_noalloc_ranges[i - 1].second)
                return AES_ERR_OVERLAP;
    }
    if (!payload)
        return AES_OK;
    if (ctx->device == AES_DEVICE_NONE)
        return AES_ERR_DEVICE;
    void *d_scratch =
        ctx->device < NOALLOC_MAX_DEVICES ? g_scratch_ptr[ctx->device] : nullptr;
    if (!d_scratch)
        return AES_ERR_DEVICE;
    // 3. Unit records, as plan_units cuts them: [CBC/ECB-decrypt tiles | CTR
    //    tiles | ECB-encrypt tiles | chains], tiles in request order, chains
    //    longest first (equal lengths by key index, then offset).
    Unit *w_dec = g_noalloc_units, *w_ctr = w_dec + n_dec, *w_ecb = w_ctr + n_ctr;
    Unit *w_chain = w_ecb + n_ecb;
    for (uint64_t i = 0; i < n; i++) {
        const aes_req_t &r = reqs[i];
        if (!r.length)
            continue;
        const uint32_t meta = r.key_idx | (r.op << META_OP_SHIFT);
        if (r.op == AES_OP_CBC_ENC) {
            Unit &u = *w_chain++;
            u.off = r.offset;
            u.nbytes = (uint32_t)r.length;
            u.meta = meta;
            for (int j = 0; j < 4; j++)
                u.w[j] = le32(r.iv + 4 * j);
            continue;
        }
        const uint64_t ctr0 = be64(r.iv + 8);
        for (uint64_t pos = 0; pos < r.length; pos += tile) {
            Unit &u = r.op == AES_OP_CTR ? *w_ctr++ : r.op == AES_OP_ECB_ENC ? *w_ecb++ : *w_dec++;
            u.off = r.offset + pos;
            u.nbytes = (uint32_t)std::min<uint64_t>(tile, r.length - pos);
            u.meta = meta;
            if (r.op == AES_OP_CTR) {
                const uint64_t c = ctr0 + pos / 16;  // mod 2^64, nonce untouched
                u.w[0] = le32(r.iv);
                u.w[1] = le32(r.iv + 4);
                u.w[2] = (uint32_t)c;
                u.w[3] = (uint32_t)(c >> 32);
            } else if (r.op == AES_OP_CBC_DEC && pos == 0) {
                for (int j = 0; j < 4; j++)
                    u.w[j] = le32(r.iv + 4 * j);
            } else {
                if (r.op == AES_OP_CBC_DEC)
                    u.meta |= FLAG_PRED_IN;
                u.w[0] = u.w[1] = u.w[2] = u.w[3] = 0;
            }
        }
    }
    Unit *chains = g_noalloc_units + n_dec + n_ctr + n_ecb;
    std::sort(chains, chains + n_chain, [](const Unit &a, const Unit &b) {
        const uint32_t ka = a.meta & META_KEY_MASK, kb = b.meta & META_KEY_MASK;
        if (a.nbytes != b.nbytes)
            return a.nbytes > b.nbytes;
        return ka != kb ? ka < kb : a.off < b.off;
    });
    // 4. Upload (the static host array is read before the copy call returns,
    //    as for any copy from pageable memory), zero the tile counters, launch.
    HIP_TRY(hipSetDevice(ctx->device));
    HIP_TRY(hipMemcpyAsync(d_scratch, g_noalloc_units, n_units * sizeof(Unit),
                           hipMemcpyHostToDevice, (hipStream_t)stream));
    uint32_t *d_ctrs = (uint32_t *)((uint8_t *)d_scratch + NOALLOC_CTRS_OFF);
    int e = launch_zero_words(d_ctrs, 2 * TILE_CTRS, stream);
    if (e)
        return hip_fail((hipError_t)e);
    const PlanView v{d_scratch, d_ctrs, (size_t)n_dec, (size_t)(n_ctr + n_ecb), (size_t)n_chain,
                     pred_in, dec_bytes, ctr_bytes, (size_t)n_ecb};
    return launch_planned(ctx, v, d_scheds, n_scheds, d_in, d_out, stream);
}

// --------------------------------------------- large single-op calls, in parallel

// Requests per chunk of the parallel single-call path, and the smallest call
// it takes (below that, thread hand-off costs more than it saves).
constexpr uint64_t PAR_CHUNK = 4096;
constexpr uint64_t PAR_MIN_REQS = 2 * PAR_CHUNK;
constexpr int PAR_MAX_THREADS = 8;

struct ChunkScan {
    uint64_t err_at = UINT64_MAX;  // first request that breaks a rule
    int err = AES_OK;
    bool ordered = true;  // nonzero requests in offset order and disjoint
    uint64_t first_off = UINT64_MAX, last_end = 0;
    uint64_t tiles = 0, payload = 0, extent = 0;
    bool pred_in = false;
};

// A single-op call over tiles (CBC decryption, CTR, ECB) with many requests:
// the requests are checked in chunks on the context's threads (same rules and
// error precedence as validate), then each chunk writes its unit records
// straight into the pinned staging buffer at offsets from a prefix sum, in
// request order.  Returns 1 when the call is not for this path.
int single_parallel(uint32_t op, aes_ctx *ctx, const aes_schedule_t *d_scheds,
                    uint32_t n_scheds, const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                    const uint64_t *offsets, const uint64_t *lengths, const uint32_t *key_idx,
                    const uint8_t *ivs, uint64_t n, void *stream) {
    if (n < PAR_MIN_REQS || op == AES_OP_CBC_ENC ||
        (op == AES_OP_CTR && ctx->ctr_variant == AES_CTR_BITSLICE) ||
        (is_dec_tile_op(op) && ctx->dec_variant == AES_DEC_BITSLICE) ||
        n / PAR_CHUNK >= (1ull << 30))
        return 1;
    int st = check_buffers(d_in, d_out, buf_bytes, n, d_scheds);
    if (st)
        return st;
    if (!ctx->pool) {
        const unsigned hw = std::thread::hardware_concurrency();
        const int t = (int)std::min<unsigned>(hw ? hw : 1, PAR_MAX_THREADS);
        try {
            ctx->pool.reset(new HostPool(t - 1));
        } catch (...) {
            return 1;
        }
    }
    const uint32_t tile = ctx->tile_bytes;
    const bool dec = is_dec_tile_op(op);
    const uint64_t n_chunks = (n + PAR_CHUNK - 1) / PAR_CHUNK;
    std::vector<ChunkScan> sc;
    std::vector<uint64_t> base;
    try {
        sc.resize(n_chunks);
        base.resize(n_chunks + 1);
    } catch (const std::bad_alloc &) {
        return AES_ERR_NOMEM;
    }
    // 1. Rules, order and unit counts per chunk.
    ctx->pool->run((int)n_chunks, [&](int c) {
        ChunkScan &k = sc[c];
        const uint64_t lo = (uint64_t)c * PAR_CHUNK, hi = std::min(n, lo + PAR_CHUNK);
        for (uint64_t i = lo; i < hi; i++) {
            const uint64_t off = offsets[i], len = lengths[i];
            const int e = check_request(op, off, len, key_idx[i], n_scheds, buf_bytes);
            if (e) {
                k.err_at = i;
                k.err = e;
                return;
            }
            if (!len)
                continue;
            if (off < k.last_end || (k.first_off != UINT64_MAX && off < k.first_off))
                k.ordered = false;
            if (k.first_off == UINT64_MAX)
                k.first_off = off;
            k.last_end = std::max(k.last_end, off + len);
            k.tiles += (len + tile - 1) / tile;
            k.payload += len;
            k.extent = std::max(k.extent, off + len);
            k.pred_in |= dec && op == AES_OP_CBC_DEC && len > tile;
        }
    });
    // 2. The first error in request order, then disjointness.
    uint64_t err_at = UINT64_MAX, payload = 0;
    bool ordered = true, pred_in = false;
    uint64_t prev_end = 0;
    base[0] = 0;
    for (uint64_t c = 0; c < n_chunks; c++) {
        if (sc[c].err_at < err_at) {
            err_at = sc[c].err_at;
            st = sc[c].err;
        }
        ordered = ordered && sc[c].ordered &&
                  (sc[c].first_off == UINT64_MAX || sc[c].first_off >= prev_end);
        if (sc[c].first_off != UINT64_MAX)
            prev_end = sc[c].last_end;
        payload += sc[c].payload;
        pred_in |= sc[c].pred_in;
        base[c + 1] = base[c] + sc[c].tiles;
    }
    if (err_at != UINT64_MAX)
        return st;
    if (!ordered) {  // unsorted (or overlapping): the sort-based check
        std::vector<std::pair<uint64_t, uint64_t>> ranges;
        try {
            ranges.reserve(n);
        } catch (const std::bad_alloc &) {
            return AES_ERR_NOMEM;
        }
        for (uint64_t i = 0; i < n; i++)
            if (lengths[i])
                ranges.emplace_back(offsets[i], offsets[i] + lengths[i]);
        std::sort(ranges.begin(), ranges.end());
        for (size_t i = 1; i < ranges.size(); i++)
            if (ranges[i].first < ranges[i - 1].second)
                return AES_ERR_OVERLAP;
    }
    const uint64_t n_tiles = base[n_chunks];
    if (n_tiles >= (1ull << 32))
        return AES_ERR_RANGE;
    if (!payload)
        return AES_OK;
    if (ctx->device == AES_DEVICE_NONE)
        return AES_ERR_DEVICE;
    const size_t n_dec = dec ? n_tiles : 0, n_enc = dec ? 0 : n_tiles;
    const size_t ubytes = n_tiles * sizeof(Unit);
    const size_t need = units_bytes(n_dec, n_enc, 0);
    Slot *sp = nullptr;
    if ((st = take_slot(ctx, ubytes, need, &sp)))
        return st;
    Slot &s = *sp;
    // 3. Unit records, in request order, into the staging buffer.
    Unit *out = (Unit *)s.h_stage;
    ctx->pool->run((int)n_chunks, [&](int c) {
        const uint64_t lo = (uint64_t)c * PAR_CHUNK, hi = std::min(n, lo + PAR_CHUNK);
        Unit *u = out + base[c];
        for (uint64_t i = lo; i < hi; i++) {
            const uint64_t off = offsets[i], len = lengths[i];
            if (!len)
                continue;
            const uint32_t meta = key_idx[i] | (op << META_OP_SHIFT);
            const uint8_t *iv = ivs ? ivs + 16 * i : nullptr;
            const uint64_t ctr0 = op == AES_OP_CTR ? be64(iv + 8) : 0;
            for (uint64_t pos = 0; pos < len; pos += tile, u++) {
                u->off = off + pos;
                u->nbytes = (uint32_t)std::min<uint64_t>(tile, len - pos);
                u->meta = meta;
                if (op == AES_OP_CTR) {
                    const uint64_t ctr = ctr0 + pos / 16;  // mod 2^64, nonce untouched
                    u->w[0] = le32(iv);
                    u->w[1] = le32(iv + 4);
                    u->w[2] = (uint32_t)ctr;
                    u->w[3] = (uint32_t)(ctr >> 32);
                } else if (op == AES_OP_CBC_DEC && pos == 0) {
                    for (int w = 0; w < 4; w++)
                        u->w[w] = le32(iv + 4 * w);
                } else {
                    if (op == AES_OP_CBC_DEC)
                        u->meta |= FLAG_PRED_IN;
                    u->w[0] = u->w[1] = u->w[2] = u->w[3] = 0;
                }
            }
        }
    });
    if ((st = upload_units(ctx, s, ubytes, stream)))
        return st;
    PlanView v{s.d_units, s.d_ctrs, n_dec, n_enc, 0, pred_in, dec ? payload : 0, dec ? 0 : payload,
               op == AES_OP_ECB_ENC ? n_enc : 0};
    st = launch_planned(ctx, v, d_scheds, n_scheds, d_in, d_out, stream);
    if (st)
        return st;
    HIP_TRY(hipEventRecord(s.ev, (hipStream_t)stream));
    s.ev_pending = true;
    return AES_OK;
}

int single_mode(uint32_t op, aes_ctx *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes, const uint64_t *offsets,
                const uint64_t *lengths, const uint32_t *key_idx, const uint8_t *ivs, uint64_t n,
                void *stream) {
    if (!ctx)
        return AES_ERR_ARG;
    const bool ecb = op == AES_OP_ECB_ENC || op == AES_OP_ECB_DEC;  // no IVs
    if (n && (!offsets || !lengths || !key_idx || (!ivs && !ecb)))
        return AES_ERR_ARG;
    const int pst = single_parallel(op, ctx, d_scheds, n_scheds, d_in, d_out, buf_bytes, offsets,
                                    lengths, key_idx, ecb ? nullptr : ivs, n, stream);
    if (pst != 1)
        return pst;
    std::vector<aes_req_t> &reqs = ctx->scratch_reqs;
    try {
        reqs.resize(n);
    } catch (const std::bad_alloc &) {
        return AES_ERR_NOMEM;
    }
    for (uint64_t i = 0; i < n; i++) {
        reqs[i].offset = offsets[i];
        reqs[i].length = lengths[i];
        reqs[i].key_idx = key_idx[i];
        reqs[i].op = op;
        if (ecb)
            memset(reqs[i].iv, 0, 16);
        else
            memcpy(reqs[i].iv, ivs + 16 * i, 16);
    }
    return run_batch(ctx, d_scheds, n_scheds, d_in, d_out, buf_bytes, reqs.data(), n, stream);
}

}  // namespace

// ============================================================ exported API

extern "C" {

const char *aes_strerror(int status) {
    switch (status) {
    case AES_OK: return "ok";
    case AES_ERR_ARG: return "invalid argument";
    case AES_ERR_KEYSIZE: return "key size must be 128, 192 or 256 bits";
    case AES_ERR_LENGTH: return "bad length (CBC needs whole 16-byte blocks; requests < 4 GiB)";
    case AES_ERR_RANGE: return "offset, range or key index out of bounds";
    case AES_ERR_OVERLAP: return "requests or buffers overlap";
    case AES_ERR_DEVICE: return "HIP device error or no device";
    case AES_ERR_NOMEM: return "out of memory";
    case AES_ERR_AGAIN: return "resource temporarily unavailable";
    case AES_ERR_TIMEOUT: return "timed out";
    case AES_ERR_STATE: return "invalid state for this call";
    default: return "unknown status";
    }
}

int aes_last_hip_error(void) { return g_last_hip; }

int aes_expand_key(const uint8_t *key, uint32_t key_bits, aes_schedule_t *out) {
    return expand_key(key, key_bits, out);
}

int aes_ctx_create(int hip_device, aes_ctx_t **out) {
    if (!out)
        return AES_ERR_ARG;
    *out = nullptr;
    if (hip_device < AES_DEVICE_NONE)
        return AES_ERR_ARG;
    aes_ctx *ctx = new (std::nothrow) aes_ctx();
    if (!ctx)
        return AES_ERR_NOMEM;
    ctx->device = hip_device;
    if (hip_device != AES_DEVICE_NONE) {
        int ndev = 0;
        hipError_t e = hipGetDeviceCount(&ndev);
        if (e != hipSuccess || hip_device >= ndev) {
            delete ctx;
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidDevice);
        }
        hipDeviceProp_t prop;
        if ((e = hipSetDevice(hip_device)) != hipSuccess ||
            (e = hipGetDeviceProperties(&prop, hip_device)) != hipSuccess) {
            delete ctx;
            return hip_fail(e);
        }
        ctx->n_cu = prop.multiProcessorCount;
        size_t an = strcspn(prop.gcnArchName, ":");
        an = an < sizeof(ctx->arch) - 1 ? an : sizeof(ctx->arch) - 1;
        memcpy(ctx->arch, prop.gcnArchName, an);
        ctx->arch[an] = '\0';
        uint32_t img[TIMG_WORDS];
        make_table_image(img);
        if (hipMalloc((void **)&ctx->d_timg, sizeof(img)) != hipSuccess) {
            delete ctx;
            return AES_ERR_NOMEM;
        }
        if ((e = hipMemcpy(ctx->d_timg, img, sizeof(img), hipMemcpyHostToDevice)) != hipSuccess) {
            (void)hipFree(ctx->d_timg);
            delete ctx;
            return hip_fail(e);
        }
        if (int st = noalloc_setup(hip_device)) {
            (void)hipFree(ctx->d_timg);
            delete ctx;
            return st;
        }
        for (Slot &s : ctx->slots) {
            if ((e = hipEventCreateWithFlags(&s.ev, hipEventDisableTiming)) != hipSuccess ||
                (e = hipEventCreateWithFlags(&s.copied, hipEventDisableTiming)) != hipSuccess) {
                aes_ctx_destroy(ctx);
                return hip_fail(e);
            }
        }
    }
    *out = ctx;
    return AES_OK;
}

void aes_ctx_destroy(aes_ctx_t *ctx) {
    if (!ctx)
        return;
    if (ctx->device != AES_DEVICE_NONE) {
        (void)hipSetDevice(ctx->device);
        for (Slot &s : ctx->slots) {
            if (s.ev) {
                if (s.ev_pending)
                    (void)hipEventSynchronize(s.ev);
                (void)hipEventDestroy(s.ev);
            }
            if (s.copied)
                (void)hipEventDestroy(s.copied);
            if (s.h_stage)
                (void)hipHostFree(s.h_stage);
            if (s.d_units)
                (void)hipFree(s.d_units);
            if (s.d_ctrs)
                (void)hipFree(s.d_ctrs);
        }
        if (ctx->d_timg)
            (void)hipFree(ctx->d_timg);
        if (ctx->capture)
            (void)hipStreamDestroy(ctx->capture);
        if (ctx->copy) {
            (void)hipStreamSynchronize(ctx->copy);
            (void)hipStreamDestroy(ctx->copy);
        }
    }
    delete ctx;
}

int aes_batch(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
              const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes, const aes_req_t *reqs,
              uint64_t n_reqs, void *stream) {
    return run_batch(ctx, d_scheds, n_scheds, d_in, d_out, buf_bytes, reqs, n_reqs, stream);
}

int aes_batch_noalloc(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                      const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                      const aes_req_t *reqs, uint64_t n_reqs, void *stream) {
    return run_batch_noalloc(ctx, d_scheds, n_scheds, d_in, d_out, buf_bytes, reqs, n_reqs,
                             stream);
}

int aes_cbc_encrypt_batch(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                          const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                          const uint64_t *offsets, const uint64_t *lengths,
                          const uint32_t *key_idx, const uint8_t *ivs, uint64_t n, void *stream) {
    return single_mode(AES_OP_CBC_ENC, ctx, d_scheds, n_scheds, d_in, d_out, buf_bytes, offsets,
                       lengths, key_idx, ivs, n, stream);
}

int aes_cbc_decrypt_batch(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                          const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                          const uint64_t *offsets, const uint64_t *lengths,
                          const uint32_t *key_idx, const uint8_t *ivs, uint64_t n, void *stream) {
    return single_mode(AES_OP_CBC_DEC, ctx, d_scheds, n_scheds, d_in, d_out, buf_bytes, offsets,
                       lengths, key_idx, ivs, n, stream);
}

int aes_ctr_batch(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                  const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                  const uint64_t *offsets, const uint64_t *lengths, const uint32_t *key_idx,
                  const uint8_t *ivs, uint64_t n, void *stream) {
    return single_mode(AES_OP_CTR, ctx, d_scheds, n_scheds, d_in, d_out, buf_bytes, offsets,
                       lengths, key_idx, ivs, n, stream);
}

int aes_ecb_encrypt_batch(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                          const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                          const uint64_t *offsets, const uint64_t *lengths,
                          const uint32_t *key_idx, const uint8_t *ivs, uint64_t n,
                          void *stream) {
    return single_mode(AES_OP_ECB_ENC, ctx, d_scheds, n_scheds, d_in, d_out, buf_bytes, offsets,
                       lengths, key_idx, ivs, n, stream);
}

int aes_ecb_decrypt_batch(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                          const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                          const uint64_t *offsets, const uint64_t *lengths,
                          const uint32_t *key_idx, const uint8_t *ivs, uint64_t n,
                          void *stream) {
    return single_mode(AES_OP_ECB_DEC, ctx, d_scheds, n_scheds, d_in, d_out, buf_bytes, offsets,
                       lengths, key_idx, ivs, n, stream);
}

// ------------------------------------------------------------------ plans

int aes_plan_create(aes_ctx_t *ctx, const aes_req_t *reqs, uint64_t n, uint32_t n_scheds,
                    uint64_t buf_bytes, aes_plan_t **out) {
    if (!ctx || !out)
        return AES_ERR_ARG;
    *out = nullptr;
    int st = validate(reqs, n, n_scheds, buf_bytes);
    if (st)
        return st;
    aes_plan *pl = new (std::nothrow) aes_plan();
    if (!pl)
        return AES_ERR_NOMEM;
    pl->ctx = ctx;
    pl->tile_bytes = ctx->tile_bytes;
    pl->n_scheds = n_scheds;
    pl->buf_bytes = buf_bytes;
    if ((st = plan_units(reqs, n, ctx->tile_bytes, ctx->ctr_variant == AES_CTR_BITSLICE,
                         ctx->dec_variant == AES_DEC_BITSLICE, pl->p))) {
        delete pl;
        return st;
    }
    pl->n_dec = pl->p.dec.size();
    pl->n_ctr = pl->p.ctr.size();
    pl->n_chain = pl->p.chains.size();
    if (ctx->device != AES_DEVICE_NONE && pl->p.payload) {
        hipError_t e;
        const size_t need = units_bytes(pl->n_dec, pl->n_ctr, pl->n_chain);
        const size_t ubytes = (pl->n_dec + pl->n_ctr + pl->n_chain) * sizeof(Unit);
        std::vector<Unit> host;
        try {
            host.resize(pl->n_dec + pl->n_ctr + pl->n_chain);
        } catch (const std::bad_alloc &) {
            delete pl;
            return AES_ERR_NOMEM;
        }
        pack_units(pl->p, host.data());
        if ((e = hipSetDevice(ctx->device)) != hipSuccess) {
            delete pl;
            return hip_fail(e);
        }
        if (hipMalloc(&pl->d_units, need) != hipSuccess) {
            delete pl;
            return AES_ERR_NOMEM;
        }
        if ((e = hipMemcpy(pl->d_units, host.data(), ubytes, hipMemcpyHostToDevice)) !=
            hipSuccess) {
            (void)hipFree(pl->d_units);
            delete pl;
            return hip_fail(e);
        }
        if ((st = alloc_tile_ctrs(&pl->d_ctrs))) {
            (void)hipFree(pl->d_units);
            delete pl;
            return st;
        }
    }
    *out = pl;
    return AES_OK;
}

int aes_plan_launch(aes_plan_t *plan, const aes_schedule_t *d_scheds, const uint8_t *d_in,
                    uint8_t *d_out, void *stream) {
    if (!plan)
        return AES_ERR_ARG;
    const uint64_t n = plan->n_dec + plan->n_ctr + plan->n_chain;
    int st = check_buffers(d_in, d_out, plan->buf_bytes, n, d_scheds);
    if (st)
        return st;
    if (!plan->p.payload)
        return AES_OK;
    aes_ctx *ctx = plan->ctx;
    if (ctx->device == AES_DEVICE_NONE)
        return AES_ERR_DEVICE;
    HIP_TRY(hipSetDevice(ctx->device));
    return launch_planned(ctx, view_of(plan->p, plan->d_units, plan->d_ctrs), d_scheds, plan->n_scheds, d_in,
                          d_out, stream);
}

int aes_plan_info(const aes_plan_t *plan, aes_plan_info_t *info) {
    if (!plan || !info)
        return AES_ERR_ARG;
    memset(info, 0, sizeof(*info));
    info->n_units_cbc_dec = plan->n_dec;
    info->n_units_ctr = plan->n_ctr;
    info->n_chains_cbc_enc = plan->n_chain;
    info->payload_bytes = plan->p.payload;
    info->extent_bytes = plan->p.extent;
    info->tile_bytes = plan->tile_bytes;
    return AES_OK;
}

int aes_plan_units(const aes_plan_t *plan, aes_unit_t *out, uint64_t max, uint64_t *n_out) {
    if (!plan || !n_out || (max && !out))
        return AES_ERR_ARG;
    static_assert(sizeof(aes_unit_t) == sizeof(Unit), "unit record layout");
    const uint64_t total = plan->n_dec + plan->n_ctr + plan->n_chain;
    *n_out = total;
    uint64_t k = 0;
    for (const auto *v : {&plan->p.dec, &plan->p.ctr, &plan->p.chains})
        for (const Unit &u : *v) {
            if (k >= max)
                return AES_OK;
            memcpy(&out[k++], &u, sizeof(Unit));
        }
    return AES_OK;
}

void aes_plan_destroy(aes_plan_t *plan) {
    if (!plan)
        return;
    if (plan->d_units || plan->d_ctrs) {
        (void)hipSetDevice(plan->ctx->device);
        (void)hipDeviceSynchronize();
        if (plan->d_units)
            (void)hipFree(plan->d_units);
        if (plan->d_ctrs)
            (void)hipFree(plan->d_ctrs);
    }
    delete plan;
}

// ----------------------------------------------------------- launch config

int aes_ctx_get_config(const aes_ctx_t *ctx, aes_launch_config_t *cfg) {
    if (!ctx || !cfg)
        return AES_ERR_ARG;
    memset(cfg, 0, sizeof(*cfg));
    cfg->tile_bytes = ctx->tile_bytes;
    cfg->ctr_nb = (uint32_t)ctx->tile_ctr.nb;
    cfg->ctr_wg = (uint32_t)ctx->tile_ctr.wg_threads;
    cfg->dec_nb = (uint32_t)ctx->tile_dec.nb;
    cfg->dec_wg = (uint32_t)ctx->tile_dec.wg_threads;
    cfg->chain_lanes = (uint32_t)ctx->chain.lanes;
    cfg->chain_wg = (uint32_t)ctx->chain.wg_threads;
    cfg->chain_quad = ctx->chain.quad ? 1u : 0u;
    cfg->mixed_nb = (uint32_t)ctx->mixed_nb;
    cfg->fuse = ctx->fuse ? 1u : 0u;
    cfg->grid = (uint32_t)ctx->grid;
    cfg->ctr_variant = ctx->ctr_variant;
    cfg->dec_variant = ctx->dec_variant;
    return AES_OK;
}

int aes_ctx_set_config(aes_ctx_t *ctx, const aes_launch_config_t *cfg) {
    if (!ctx || !cfg)
        return AES_ERR_ARG;
    if (cfg->tile_bytes < 1024 || cfg->tile_bytes > (1u << 24) || (cfg->tile_bytes & 1023))
        return AES_ERR_ARG;
    if (!tile_shape_supported((int)cfg->ctr_nb, (int)cfg->ctr_wg) ||
        !tile_shape_supported((int)cfg->dec_nb, (int)cfg->dec_wg))
        return AES_ERR_ARG;
    if (cfg->chain_lanes < 1 || cfg->chain_lanes > 64 || cfg->chain_wg < 64 ||
        cfg->chain_wg > 1024 || (cfg->chain_wg & 63))
        return AES_ERR_ARG;
    if (cfg->mixed_nb != 1 && cfg->mixed_nb != 2)
        return AES_ERR_ARG;
    if (cfg->fuse > 1 || cfg->grid > 65535)
        return AES_ERR_ARG;
    if (cfg->ctr_variant != AES_CTR_TABLE && cfg->ctr_variant != AES_CTR_BITSLICE)
        return AES_ERR_ARG;
    if (cfg->dec_variant != AES_DEC_TABLE && cfg->dec_variant != AES_DEC_BITSLICE)
        return AES_ERR_ARG;
    if (cfg->chain_quad > 1)
        return AES_ERR_ARG;
    ctx->tile_bytes = cfg->tile_bytes;
    ctx->tile_ctr.nb = (int)cfg->ctr_nb;
    ctx->tile_ctr.wg_threads = (int)cfg->ctr_wg;
    ctx->tile_ctr.grid = (int)cfg->grid;
    ctx->tile_dec.nb = (int)cfg->dec_nb;
    ctx->tile_dec.wg_threads = (int)cfg->dec_wg;
    ctx->tile_dec.grid = (int)cfg->grid;
    ctx->chain.lanes = (int)cfg->chain_lanes;
    ctx->chain.wg_threads = (int)cfg->chain_wg;
    ctx->chain.quad = cfg->chain_quad != 0;
    ctx->mixed_nb = (int)cfg->mixed_nb;
    ctx->fuse = cfg->fuse != 0;
    ctx->grid = (int)cfg->grid;
    ctx->ctr_variant = cfg->ctr_variant;
    ctx->dec_variant = cfg->dec_variant;
    return AES_OK;
}

// ---------------------------------------------------- one request, one launch

int aes_request_launch(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                       const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                       const aes_req_t *req, void *stream) {
    if (!ctx || !req)
        return AES_ERR_ARG;
    int st = check_buffers(d_in, d_out, buf_bytes, 1, d_scheds);
    if (st)
        return st;
    if ((st = validate(req, 1, n_scheds, buf_bytes)))
        return st;
    if (!req->length)
        return AES_OK;
    if (ctx->device == AES_DEVICE_NONE)
        return AES_ERR_DEVICE;
    HIP_TRY(hipSetDevice(ctx->device));
    // In place, a multi-tile CBC decryption stays in one wave, which carries
    // each predecessor block in registers before overwriting it.
    uint32_t tile = ctx->tile_bytes;
    if (req->op == AES_OP_CBC_DEC && d_in == d_out && req->length > tile)
        tile = (uint32_t)req->length;
    const int e = launch_request(*req, tile, d_scheds, n_scheds, ctx->d_timg, d_in, d_out,
                                 ctx->n_cu, stream);
    if (e)
        return hip_fail((hipError_t)e);
    return AES_OK;
}

int aes_request_launches(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                         const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                         const aes_req_t *reqs, uint64_t n_reqs, void *stream) {
    if (!ctx)
        return AES_ERR_ARG;
    int st = check_buffers(d_in, d_out, buf_bytes, n_reqs, d_scheds);
    if (st)
        return st;
    if ((st = validate(reqs, n_reqs, n_scheds, buf_bytes)))
        return st;
    for (uint64_t i = 0; i < n_reqs && !st; i++)
        st = aes_request_launch(ctx, d_scheds, n_scheds, d_in, d_out, buf_bytes, &reqs[i],
                                stream);
    return st;
}

// -------------------------------------------------------------- HIP graphs

namespace {

int capture_stream(aes_ctx *ctx) {
    if (!ctx->capture)
        HIP_TRY(hipStreamCreateWithFlags(&ctx->capture, hipStreamNonBlocking));
    return AES_OK;
}

// Ends a capture on ctx->capture and instantiates it into *out.
int finish_capture(aes_ctx *ctx, int launch_status, uint64_t nodes, aes_graph_t **out) {
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->capture, &g);
    if (launch_status) {
        if (g)
            (void)hipGraphDestroy(g);
        return launch_status;
    }
    if (e != hipSuccess)
        return hip_fail(e);
    aes_graph *gr = new (std::nothrow) aes_graph();
    if (!gr) {
        (void)hipGraphDestroy(g);
        return AES_ERR_NOMEM;
    }
    gr->graph = g;
    gr->device = ctx->device;
    gr->n_nodes = nodes;
    if ((e = hipGraphInstantiate(&gr->exec, g, nullptr, nullptr, 0)) != hipSuccess) {
        (void)hipGraphDestroy(g);
        delete gr;
        return hip_fail(e);
    }
    *out = gr;
    return AES_OK;
}

}  // namespace

int aes_plan_graph(aes_plan_t *plan, const aes_schedule_t *d_scheds, const uint8_t *d_in,
                   uint8_t *d_out, aes_graph_t **out) {
    if (!plan || !out)
        return AES_ERR_ARG;
    *out = nullptr;
    aes_ctx *ctx = plan->ctx;
    const uint64_t n = plan->n_dec + plan->n_ctr + plan->n_chain;
    int st = check_buffers(d_in, d_out, plan->buf_bytes, n, d_scheds);
    if (st)
        return st;
    if (ctx->device == AES_DEVICE_NONE)
        return AES_ERR_DEVICE;
    HIP_TRY(hipSetDevice(ctx->device));
    if ((st = capture_stream(ctx)))
        return st;
    HIP_TRY(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
    st = plan->p.payload ? launch_planned(ctx, view_of(plan->p, plan->d_units, plan->d_ctrs), d_scheds,
                                          plan->n_scheds, d_in, d_out, ctx->capture)
                         : AES_OK;
    return finish_capture(ctx, st, 1, out);
}

int aes_requests_graph(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                       const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                       const aes_req_t *reqs, uint64_t n_reqs, aes_graph_t **out) {
    if (!ctx || !out)
        return AES_ERR_ARG;
    *out = nullptr;
    int st = check_buffers(d_in, d_out, buf_bytes, n_reqs, d_scheds);
    if (st)
        return st;
    if ((st = validate(reqs, n_reqs, n_scheds, buf_bytes)))
        return st;
    if (ctx->device == AES_DEVICE_NONE)
        return AES_ERR_DEVICE;
    HIP_TRY(hipSetDevice(ctx->device));
    if ((st = capture_stream(ctx)))
        return st;
    HIP_TRY(hipStreamBeginCapture(ctx->capture, hipStreamCaptureModeThreadLocal));
    uint64_t nodes = 0;
    for (uint64_t i = 0; i < n_reqs && !st; i++) {
        if (!reqs[i].length)
            continue;
        st = aes_request_launch(ctx, d_scheds, n_scheds, d_in, d_out, buf_bytes, &reqs[i],
                                ctx->capture);
        nodes++;
    }
    return finish_capture(ctx, st, nodes, out);
}

int aes_graph_launch(aes_graph_t *g, void *stream) {
    if (!g)
        return AES_ERR_ARG;
    HIP_TRY(hipSetDevice(g->device));
    HIP_TRY(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return AES_OK;
}

void aes_graph_destroy(aes_graph_t *g) {
    if (!g)
        return;
    (void)hipSetDevice(g->device);
    if (g->exec)
        (void)hipGraphExecDestroy(g->exec);
    if (g->graph)
        (void)hipGraphDestroy(g->graph);
    delete g;
}

// ----------------------------------------------------------------- tuning

namespace {

// Median time in ms of `iters` launches of plan (after one warm-up).
int time_plan(aes_plan *plan, const aes_schedule_t *d_scheds, const uint8_t *d_in,
              uint8_t *d_out, int iters, double *ms_out) {
    aes_ctx *ctx = plan->ctx;
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    std::vector<double> ms;
    int st = AES_OK;
    for (int i = 0; i <= iters && !st; i++) {
        hipError_t e = hipEventRecord(a, ctx->capture);
        if (e == hipSuccess) {
            st = launch_planned(ctx, view_of(plan->p, plan->d_units, plan->d_ctrs), d_scheds, plan->n_scheds,
                                d_in, d_out, ctx->capture);
            if (!st)
                e = hipEventRecord(b, ctx->capture);
        }
        if (!st && e == hipSuccess)
            e = hipEventSynchronize(b);
        if (!st && e != hipSuccess)
            st = hip_fail(e);
        float t = 0.f;
        if (!st && (e = hipEventElapsedTime(&t, a, b)) != hipSuccess)
            st = hip_fail(e);
        if (!st && i > 0)
            ms.push_back(t);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st)
        return st;
    std::sort(ms.begin(), ms.end());
    *ms_out = ms[ms.size() / 2];
    return AES_OK;
}

}  // namespace

// Relative gain a tuning candidate needs to replace the best so far.
constexpr double TUNE_MARGIN = 0.02;

int aes_tune(aes_ctx_t *ctx, const aes_req_t *reqs, uint64_t n_reqs, uint32_t n_scheds,
             uint64_t buf_bytes, const aes_schedule_t *d_scheds, const uint8_t *d_in,
             uint8_t *d_out, uint32_t iters, aes_launch_config_t *best_out) {
    if (!ctx || (n_reqs && !reqs) || iters < 1 || iters > 1000)
        return AES_ERR_ARG;
    int st = check_buffers(d_in, d_out, buf_bytes, n_reqs, d_scheds);
    if (st)
        return st;
    if (n_reqs && d_in == d_out)
        return AES_ERR_OVERLAP;  // repeated runs must not feed on their own output
    if ((st = validate(reqs, n_reqs, n_scheds, buf_bytes)))
        return st;
    // The tune cache: a stored configuration for a batch of this shape is
    // applied without timing (if the library still supports it).
    const char *cache = getenv("AESGPU_TUNE_CACHE");
    std::string sig;
    if (cache && *cache) {
        sig = tune_signature(ctx->arch, ctx->n_cu, reqs, n_reqs, n_scheds);
        aes_launch_config_t c;
        // The cache holds the tuned knobs; the decryption variant is the
        // caller's and stays as set.
        if (tune_cache_lookup(cache, sig, &c) && ((c.dec_variant = ctx->dec_variant), true) &&
            aes_ctx_set_config(ctx, &c) == AES_OK) {
            if (best_out)
                aes_ctx_get_config(ctx, best_out);
            return AES_OK;
        }
    }
    if (ctx->device == AES_DEVICE_NONE)
        return AES_ERR_DEVICE;
    HIP_TRY(hipSetDevice(ctx->device));
    if ((st = capture_stream(ctx)))
        return st;
    aes_launch_config_t best;
    aes_ctx_get_config(ctx, &best);
    double best_ms = 1e30;
    // One candidate: set it, (re)plan when the tile size or the CTR variant
    // (which decides the key grouping of CTR tiles) changed, time it.
    aes_plan *plan = nullptr;
    uint32_t plan_tile = 0, plan_variant = 0;
    auto trial = [&](const aes_launch_config_t &c) -> int {
        int s2 = aes_ctx_set_config(ctx, &c);
        if (s2)
            return AES_OK;  // shape not available: skip
        if (!plan || plan_tile != c.tile_bytes || plan_variant != c.ctr_variant) {
            aes_plan_destroy(plan);
            plan = nullptr;
            if ((s2 = aes_plan_create(ctx, reqs, n_reqs, n_scheds, buf_bytes, &plan)))
                return s2;
            plan_tile = c.tile_bytes;
            plan_variant = c.ctr_variant;
        }
        double ms = 0;
        if ((s2 = time_plan(plan, d_scheds, d_in, d_out, (int)iters, &ms)))
            return s2;
        // A candidate must beat the best by more than run-to-run noise: where
        // a knob does not matter (a batch bound by one long CBC-enc chain
        // times the same under every tile shape) the starting value stays,
        // instead of whichever shape a timing fluctuation favoured.
        if (ms < best_ms * (1.0 - TUNE_MARGIN)) {
            best_ms = ms;
            best = c;
        }
        return AES_OK;
    };
    // Coordinate descent from the starting configuration, one knob at a time
    // from the best point so far, and only over knobs the batch's launch uses
    // (a knob the launch ignores would be set by timing noise alone): tile
    // size; the fusion switch (batches mixing CBC-encrypt chains with tiles);
    // tile-kernel shapes (unfused launches with tiles); the fused kernel's
    // blocks per lane (fused launches); chain mode (batches with chains); the
    // CTR variant (batches with CTR requests).
    aes_launch_config_t c = best;
    st = trial(c);
    if (!st && !plan)
        st = AES_ERR_ARG;  // the context's own configuration did not apply
    if (st) {
        aes_plan_destroy(plan);
        (void)aes_ctx_set_config(ctx, &best);
        return st;
    }
    // Which unit kinds the batch has (the plan is rebuilt by later trials;
    // only whether each kind is present is kept, which no knob changes).
    const bool has_dec = !plan->p.dec.empty();
    const bool has_ctr = plan->p.ctr.size() > plan->p.n_ecb;
    const bool has_ecb_enc = plan->p.n_ecb > 0;
    const bool has_chains = !plan->p.chains.empty();
    const bool has_tiles = has_dec || has_ctr || has_ecb_enc;
    // Whether the table tile kernels run, and whether one fused launch takes
    // the batch, under k (as launch_planned decides: the bitsliced variant
    // launches the CTR tiles on their own).
    auto table_tiles = [&](const aes_launch_config_t &k) {
        return (has_dec && k.dec_variant != AES_DEC_BITSLICE) || has_ecb_enc ||
               (has_ctr && k.ctr_variant != AES_CTR_BITSLICE);
    };
    auto fused = [&](const aes_launch_config_t &k) {
        const bool ctr_tab = has_ecb_enc || (has_ctr && k.ctr_variant != AES_CTR_BITSLICE);
        const bool dec_tab = has_dec && k.dec_variant != AES_DEC_BITSLICE;
        const int kinds = (int)dec_tab + (int)ctr_tab + (int)has_chains;
        return k.fuse && has_chains && kinds > 1;
    };
    const uint32_t tiles[] = {4096, 8192, 16384};
    for (uint32_t t : tiles) {
        if (st || !has_tiles)
            break;
        c = best;
        c.tile_bytes = t;
        st = trial(c);
    }
    for (uint32_t f = 0; f <= 1 && !st && has_chains && has_tiles; f++) {
        c = best;
        c.fuse = f;
        st = trial(c);
    }
    const uint32_t shapes[][2] = {{1, 1024}, {2, 1024}, {2, 512}, {4, 512}, {4, 256}, {1, 512}};
    for (auto &sh : shapes) {
        if (st || fused(best) || !table_tiles(best))
            break;
        c = best;
        c.ctr_nb = c.dec_nb = sh[0];
        c.ctr_wg = c.dec_wg = sh[1];
        st = trial(c);
    }
    for (uint32_t mnb = 1; mnb <= 2 && !st && fused(best); mnb++) {
        c = best;
        c.mixed_nb = mnb;
        st = trial(c);
    }
    const uint32_t lanes[] = {16, 32, 64};
    for (uint32_t l : lanes) {
        if (st || !has_chains)
            break;
        c = best;
        c.chain_lanes = l;
        c.chain_quad = 0;
        st = trial(c);
    }
    if (!st && has_chains) {  // four lanes per chain
        c = best;
        c.chain_quad = 1;
        st = trial(c);
    }
    for (uint32_t v = AES_CTR_TABLE; v <= AES_CTR_BITSLICE && has_ctr && !st; v++) {
        c = best;
        c.ctr_variant = v;
        st = trial(c);
    }
    aes_plan_destroy(plan);
    (void)aes_ctx_set_config(ctx, &best);
    if (st)
        return st;
    if (cache && *cache)
        (void)tune_cache_store(cache, sig, best);  // a cache that cannot be written is skipped
    if (best_out)
        *best_out = best;
    return AES_OK;
}

int aes_host_batch(const aes_schedule_t *scheds, uint32_t n_scheds, const uint8_t *in,
                   uint8_t *out, uint64_t buf_bytes, const aes_req_t *reqs, uint64_t n_reqs,
                   uint32_t n_threads) {
    if (n_threads > 1024)
        return AES_ERR_ARG;
    int st = check_buffers(in, out, buf_bytes, n_reqs, scheds);
    if (st)
        return st;
    if ((st = validate(reqs, n_reqs, n_scheds, buf_bytes)))
        return st;
    if (!n_reqs)
        return AES_OK;
    uint64_t nt = n_threads;
    if (!nt) {  // the CPUs this process may run on (a machine may have more)
        cpu_set_t set;
        nt = sched_getaffinity(0, sizeof(set), &set) == 0 ? (uint64_t)CPU_COUNT(&set)
                                                          : std::thread::hardware_concurrency();
    }
    nt = std::max<uint64_t>(1, std::min<uint64_t>(nt, n_reqs));
    // Requests are claimed one at a time (their sizes differ; k at a time
    // only past 2^31 requests).  The error reported is the one of the
    // lowest-numbered request that failed; the others still run.
    const uint64_t k = (n_reqs + INT32_MAX - 1) / INT32_MAX;
    std::mutex m;
    uint64_t bad_i = UINT64_MAX;
    int bad_code = AES_OK;
    HostPool pool((int)nt - 1);
    pool.run((int)((n_reqs + k - 1) / k), [&](int c) {
        const uint64_t end = std::min<uint64_t>(n_reqs, ((uint64_t)c + 1) * k);
        for (uint64_t i = (uint64_t)c * k; i < end; i++) {
            const aes_req_t &r = reqs[i];
            const int e = aes_host_route_crypt(&scheds[r.key_idx], r.op, r.iv, in + r.offset,
                                               out + r.offset, r.length);
            if (e) {
                std::lock_guard<std::mutex> lk(m);
                if (i < bad_i) {
                    bad_i = i;
                    bad_code = e;
                }
            }
        }
    });
    return bad_code;
}

int aes_tune_key(const aes_ctx_t *ctx, const aes_req_t *reqs, uint64_t n_reqs, uint32_t n_scheds,
                 char *buf, size_t cap, size_t *len_out) {
    if (!ctx || (n_reqs && !reqs) || (cap && !buf))
        return AES_ERR_ARG;
    const std::string sig = tune_signature(ctx->arch, ctx->n_cu, reqs, n_reqs, n_scheds);
    if (len_out)
        *len_out = sig.size();
    if (cap < sig.size() + 1)
        return AES_ERR_ARG;
    memcpy(buf, sig.c_str(), sig.size() + 1);
    return AES_OK;
}

}  // extern "C"
