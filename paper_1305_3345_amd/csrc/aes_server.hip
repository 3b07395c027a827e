// aes_server.hip -- the serving form: a persistent kernel fed through a ring of
// request descriptors in pinned host-mapped memory (the paper's Non-Stop
// Kernel, section 3.1, with the request path of section 3.2), and the
// per-request-launch engine it is compared with.
//
// Device side.  One wave of the grid (the dispatcher) polls the host ring with
// system-scope acquire loads, 64 descriptors per round trip, cuts each
// request into work units and publishes them to a device queue (one queue per
// LDS table set: encryption tables for CTR tiles and CBC-encrypt chains,
// decryption tables for CBC-decrypt tiles).  Every other wave claims units
// from its workgroup's queue, runs them with the batch kernels' round code,
// releases its output at system scope and decrements the request's unit
// count; the wave that finishes the last unit writes the completion record
// into host-mapped memory.  The dispatcher snapshots each CBC-decrypt tile's
// predecessor block before publishing, so tiles run in any order and
// in-place requests are safe.  The kernel ends when the host raises the stop
// flag or no descriptor arrives for idle_timeout_ms; the host relaunches it
// on demand.
//
// Host side.  aes_server_submit writes the descriptor fields, then its
// sequence word with a release store; a completion thread watches the
// completion records (or, in the per-launch engine, HIP events), applies
// admission accounting, and runs callbacks or queues completions for
// poll/wait.  Ring positions are numbered apart from tickets: a request that
// takes a normal launch gets a ticket but no ring position, so the
// dispatcher, which consumes positions in order, never waits on a gap.
//
// Payloads may sit in pinned host buffers that the server allocates and
// maps into the device (fine-grained, so system-scope fences order them).
// The persistent kernel reads and writes those pages in place over the host
// link: its acquire before reading a unit and its release before counting
// the unit done are system-scope already.  The per-launch engine either does
// the same or, by default, moves them with copy commands through one HBM
// staging buffer per stream.
//
// Size-based dispatch: with a crossover set for an op, a request of that op
// below it whose payloads both sit in the server's host buffers runs on the
// host route (aes_host.cpp) on the submitting thread instead; calibration
// measures the crossovers with round trips through this server.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "aes_chain.h"
#include "aes_rounds.h"
#include "internal.h"

namespace aesgpu {

// Ring descriptor, 64 bytes, host-mapped.  seq = ring position + 1 once every
// other field is written.
struct ServeDesc {
    uint64_t seq;
    uint64_t src;
    uint64_t dst;
    uint32_t length;
    uint32_t key_slot;
    uint32_t op;
    uint32_t nr;  // the key slot's round count, recorded by the host at set_key
    uint32_t iv[4];
    uint64_t t_submit;
};
static_assert(sizeof(ServeDesc) == 64, "descriptor is 64 bytes");

// Completion record, 32 bytes, host-mapped, in the request's ring slot;
// seq = ring position + 1 written last.
struct ServeDone {
    uint64_t seq;
    int32_t status;
    uint32_t units;
    uint64_t t_dispatch;
    uint64_t t_done;
};
static_assert(sizeof(ServeDone) == 32, "completion is 32 bytes");

// Work unit in a device queue, 64 bytes.
struct ServeUnit {
    Unit u;  // off = the tile's byte position inside the request
    uint64_t src;
    uint64_t dst;
    uint64_t pos;  // ring position of the request
    uint32_t slot;
    uint32_t info;  // bits 0..7 the round count; UNIT_ONLY: the request's only unit
};
static_assert(sizeof(ServeUnit) == 64, "queue unit is 64 bytes");
constexpr uint32_t UNIT_ONLY = 1u << 8;

// Queue counters, each on its own 128-byte line.
struct ServeQueue {
    uint64_t head;  // next unit to claim
    uint64_t pad0[15];
    uint64_t tail;  // units published
    uint64_t pad1[15];
};

// Host-mapped control block.
struct ServeCtl {
    uint32_t stop;  // host -> device
    uint32_t pad0[31];
    uint64_t consumed;  // device -> host: ring positions taken
    uint64_t pad1[15];
};

struct ServeArgs {
    ServeDesc *ring;  // host-mapped (device address)
    ServeDone *done;  // host-mapped (device address)
    ServeCtl *ctl;    // host-mapped (device address)
    ServeUnit *qunits[2];
    ServeQueue *q;        // [2], device memory
    uint32_t *closed;     // device memory
    uint32_t *remaining;  // [ring_slots], device memory
    const aes_schedule_t *keys;
    const uint32_t *timg;
    uint64_t start_pos;
    uint64_t idle_ticks;  // 100 MHz ticks
    uint32_t ring_mask;
    uint32_t qmask;
    uint32_t n_keys;
    uint32_t n_dec_wg;
    uint32_t tile;
    uint32_t max_bytes;
};

#define SYS __HIP_MEMORY_SCOPE_SYSTEM
#define AGT __HIP_MEMORY_SCOPE_AGENT

__device__ __forceinline__ uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

__device__ __forceinline__ void complete(const ServeArgs &a, uint32_t slot, uint64_t pos,
                                         int32_t status) {
    ServeDone *d = a.done + slot;
    __hip_atomic_store(&d->status, status, __ATOMIC_RELAXED, SYS);
    __hip_atomic_store(&d->t_done, now_ticks(), __ATOMIC_RELAXED, SYS);
    __hip_atomic_store(&d->seq, pos + 1, __ATOMIC_RELEASE, SYS);
}

// Tiles above which a request's work units span several tiles.  The last of
// k units is claimed about 0.085 k us after the first (claims on one queue
// head serialise) and then runs for about 0.7 us per KiB, so a 1 MiB request
// finishes soonest with about 90 units; requests up to 512 KiB keep one tile
// per unit.
constexpr uint32_t UNITS_CAP = 128;

// The dispatcher: one full wave.
__device__ void dispatch_loop(const ServeArgs &a) {
    const uint32_t lane = threadIdx.x & 63u;
    uint64_t next = a.start_pos;
    uint64_t tail[2] = {__hip_atomic_load(&a.q[0].tail, __ATOMIC_RELAXED, AGT),
                        __hip_atomic_load(&a.q[1].tail, __ATOMIC_RELAXED, AGT)};
    uint64_t last_work = now_ticks();
    for (;;) {
        const uint64_t t = next + lane;
        ServeDesc *d = a.ring + (t & a.ring_mask);
        const uint64_t seq = __hip_atomic_load(&d->seq, __ATOMIC_RELAXED, SYS);
        const uint64_t ready = __ballot(seq == t + 1);
        const uint32_t n_ready = ~ready ? (uint32_t)__builtin_ctzll(~ready) : 64u;
        if (n_ready)
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        if (n_ready == 0) {
            const uint32_t stop = __hip_atomic_load(&a.ctl->stop, __ATOMIC_RELAXED, SYS);
            if (stop || now_ticks() - last_work > a.idle_ticks)
                break;
            __builtin_amdgcn_s_sleep(2);
            continue;
        }
        // Lane i < n_ready reads descriptor next + i.
        uint64_t src = 0, dst = 0, misc = 0, ivlo = 0, ivhi = 0;
        uint32_t len = 0;
        if (lane < n_ready) {
            src = __hip_atomic_load(&d->src, __ATOMIC_RELAXED, SYS);
            dst = __hip_atomic_load(&d->dst, __ATOMIC_RELAXED, SYS);
            len = __hip_atomic_load(&d->length, __ATOMIC_RELAXED, SYS);
            const uint32_t key = __hip_atomic_load(&d->key_slot, __ATOMIC_RELAXED, SYS);
            const uint32_t op = __hip_atomic_load(&d->op, __ATOMIC_RELAXED, SYS);
            const uint32_t nr = __hip_atomic_load(&d->nr, __ATOMIC_RELAXED, SYS);
            misc = ((uint64_t)op << 32) | ((uint64_t)(nr & 0xFFu) << 24) | (key & 0xFFFFFFu);
            ivlo = (uint64_t)__hip_atomic_load(&d->iv[0], __ATOMIC_RELAXED, SYS) |
                   ((uint64_t)__hip_atomic_load(&d->iv[1], __ATOMIC_RELAXED, SYS) << 32);
            ivhi = (uint64_t)__hip_atomic_load(&d->iv[2], __ATOMIC_RELAXED, SYS) |
                   ((uint64_t)__hip_atomic_load(&d->iv[3], __ATOMIC_RELAXED, SYS) << 32);
        }
        for (uint32_t i = 0; i < n_ready; i++) {
            const uint64_t pos = next + i;
            const uint32_t slot = (uint32_t)(pos & a.ring_mask);
            const uint64_t r_src = __shfl(src, (int)i);
            const uint64_t r_dst = __shfl(dst, (int)i);
            const uint32_t r_len = __shfl(len, (int)i);
            const uint64_t r_misc = __shfl(misc, (int)i);
            const uint64_t r_ivlo = __shfl(ivlo, (int)i);
            const uint64_t r_ivhi = __shfl(ivhi, (int)i);
            const uint32_t key = (uint32_t)r_misc & 0xFFFFFFu;
            const uint32_t nr = ((uint32_t)r_misc >> 24) & 0xFFu;
            const uint32_t op = (uint32_t)(r_misc >> 32);
            const uint64_t t_disp = now_ticks();
            if (lane == 0)
                __hip_atomic_store(&a.done[slot].t_dispatch, t_disp, __ATOMIC_RELAXED, SYS);
            // Work units of whole tiles: one tile each, except that a request of
            // more than UNITS_CAP tiles is cut into about UNITS_CAP units of
            // several tiles, because waves claim units one at a time from one
            // queue head and same-address claims serialise.
            const uint32_t n_tiles = (r_len + a.tile - 1) / a.tile;
            const uint32_t ub =
                a.tile * (n_tiles > UNITS_CAP ? (n_tiles + UNITS_CAP - 1) / UNITS_CAP : 1u);
            const uint32_t k_units = op == AES_OP_CBC_ENC ? 1u : (r_len + ub - 1) / ub;
            if (lane == 0)
                __hip_atomic_store(&a.done[slot].units, k_units, __ATOMIC_RELAXED, SYS);
            // The host validates every request; these checks keep a bad
            // descriptor from reaching the kernels.
            const int qi = op == AES_OP_CBC_DEC || op == AES_OP_ECB_DEC ? 1 : 0;
            const bool ok = op <= AES_OP_ECB_DEC && key < a.n_keys && r_len > 0 &&
                            (nr == 10 || nr == 12 || nr == 14) &&
                            r_len <= a.max_bytes && (op == AES_OP_CTR || (r_len & 15u) == 0) &&
                            r_src && r_dst && (qi == 0 || a.n_dec_wg > 0);
            if (!ok) {
                if (lane == 0)
                    complete(a, slot, pos, AES_ERR_ARG);
                continue;
            }
            const uint32_t k = k_units;
            // No wait for room: the host admits at most queue_units units
            // per queue in flight, so published units are never overwritten
            // before a worker has taken them.
            if (lane == 0)
                __hip_atomic_store(&a.remaining[slot], k, __ATOMIC_RELAXED, AGT);
            const uint32_t w0 = (uint32_t)r_ivlo, w1 = (uint32_t)(r_ivlo >> 32);
            const uint32_t w2 = (uint32_t)r_ivhi, w3 = (uint32_t)(r_ivhi >> 32);
            for (uint32_t j = lane; j < k; j += 64u) {
                ServeUnit su;
                const uint32_t at = j * ub;  // the unit's byte offset
                su.u.off = at;
                su.u.nbytes = op == AES_OP_CBC_ENC ? r_len : min(ub, r_len - at);
                su.u.meta = key | (op << META_OP_SHIFT);
                if (op == AES_OP_CTR) {
                    const uint64_t c0 = ((uint64_t)__builtin_bswap32(w2) << 32) | __builtin_bswap32(w3);
                    const uint64_t c = c0 + at / 16u;
                    su.u.w[0] = w0;
                    su.u.w[1] = w1;
                    su.u.w[2] = (uint32_t)c;
                    su.u.w[3] = (uint32_t)(c >> 32);
                } else if (op == AES_OP_ECB_ENC || op == AES_OP_ECB_DEC) {
                    su.u.w[0] = su.u.w[1] = su.u.w[2] = su.u.w[3] = 0u;
                } else if (j == 0) {
                    su.u.w[0] = w0;
                    su.u.w[1] = w1;
                    su.u.w[2] = w2;
                    su.u.w[3] = w3;
                } else {
                    // CBC decryption: the ciphertext block before this tile.
                    const uint4 p =
                        *reinterpret_cast<const uint4 *>((const uint8_t *)r_src + at - 16);
                    su.u.w[0] = p.x;
                    su.u.w[1] = p.y;
                    su.u.w[2] = p.z;
                    su.u.w[3] = p.w;
                }
                su.src = r_src;
                su.dst = r_dst;
                su.pos = pos;
                su.slot = slot;
                su.info = nr | (k == 1u ? UNIT_ONLY : 0u);
                a.qunits[qi][(tail[qi] + j) & a.qmask] = su;
            }
            tail[qi] += k;
            // The fence orders the unit records before the tail (a release
            // store after it would write the cache back a second time).
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            if (lane == 0)
                __hip_atomic_store(&a.q[qi].tail, tail[qi], __ATOMIC_RELAXED, AGT);
        }
        next += n_ready;
        if (lane == 0)
            __hip_atomic_store(&a.ctl->consumed, next, __ATOMIC_RELAXED, SYS);
        last_work = now_ticks();
    }
    if (lane == 0) {
        __hip_atomic_store(&a.ctl->consumed, next, __ATOMIC_RELAXED, SYS);
        __hip_atomic_store(a.closed, 1u, __ATOMIC_RELEASE, AGT);
    }
}

// Wave-uniform relaxed read of a device-scope counter.  Polling loops use
// relaxed loads: an acquire at agent or system scope invalidates caches, and
// hundreds of idle waves doing that continuously would evict the working
// waves' data.  The acquire fence comes once, after progress is seen.
__device__ __forceinline__ uint64_t poll_u64(uint64_t *p) {
    const uint64_t v = __hip_atomic_load(p, __ATOMIC_RELAXED, AGT);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Takes the next queue position (lane 0 adds 1 to head; every lane gets the
// value) and waits, with the whole wave, until the dispatcher has published
// it.  Returns false once the queue is closed and the position lies past the
// last published unit.  All control flow here is wave-uniform: the unit
// code that follows runs on all 64 lanes.
__device__ __forceinline__ bool claim(const ServeArgs &a, int qi, uint64_t *idx) {
    const uint32_t lane = threadIdx.x & 63u;
    ServeQueue *q = a.q + qi;
    uint64_t got = 0;
    if (lane == 0)
        got = __hip_atomic_fetch_add(&q->head, 1ull, __ATOMIC_RELAXED, AGT);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)got);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(got >> 32));
    const uint64_t pos = ((uint64_t)hi << 32) | lo;
    uint32_t nap = 1;
    for (;;) {
        // the tail and the closed flag in one round trip
        const uint64_t t = poll_u64(&q->tail);
        const uint32_t closed =
            __builtin_amdgcn_readfirstlane(__hip_atomic_load(a.closed, __ATOMIC_RELAXED, AGT));
        if (pos < t)
            break;
        if (closed) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (pos < poll_u64(&q->tail))
                break;
            return false;
        }
        // The waves holding the next four positions poll back to back; the
        // others back off from about 0.03 to 1 microsecond between polls.
        if (pos - t < 4u || nap < 16) {
            __builtin_amdgcn_s_sleep(1);
            nap++;
        } else {
            __builtin_amdgcn_s_sleep(32);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    *idx = pos;
    return true;
}

// One queue unit.  Its round count comes with it (the host records each key
// slot's at aes_server_set_key and the dispatcher copies it into the unit),
// so the round keys and the unit's data are requested together instead of
// after a load of the schedule's round count, one memory round trip fewer.
template <bool DEC>
__device__ __forceinline__ void serve_unit(const uint32_t *lds, uint32_t L0, uint32_t L2,
                                           uint32_t lane, const Unit &un, uint32_t nr,
                                           const ServeArgs &a, const uint8_t *src,
                                           uint8_t *dst) {
    const uint32_t key = un.meta & META_KEY_MASK;
    if (key >= a.n_keys)
        return;
    const aes_schedule_t *ks = a.keys + key;
    const uint32_t op = unit_op(un.meta);
    if (DEC) {
        if (op == AES_OP_ECB_DEC) {
            if (nr == 10)
                cbcdec_unit<1, 10, true>(lds, L0, L2, lane, un, nullptr, ks->dk, src, dst);
            else if (nr == 12)
                cbcdec_unit<1, 12, true>(lds, L0, L2, lane, un, nullptr, ks->dk, src, dst);
            else if (nr == 14)
                cbcdec_unit<1, 14, true>(lds, L0, L2, lane, un, nullptr, ks->dk, src, dst);
        } else {
            if (nr == 10)
                cbcdec_unit<1, 10, false>(lds, L0, L2, lane, un, nullptr, ks->dk, src, dst);
            else if (nr == 12)
                cbcdec_unit<1, 12, false>(lds, L0, L2, lane, un, nullptr, ks->dk, src, dst);
            else if (nr == 14)
                cbcdec_unit<1, 14, false>(lds, L0, L2, lane, un, nullptr, ks->dk, src, dst);
        }
    } else if (op == AES_OP_CBC_ENC) {
        // One serial chain, on four lanes (one state column each).
        if (lane >= 4u)
            return;
        if (nr == 10)
            chain_quad_run<10>(lds, L0, lane, un, ks->ek, 10u, src, dst);
        else if (nr == 12)
            chain_quad_run<12>(lds, L0, lane, un, ks->ek, 12u, src, dst);
        else if (nr == 14)
            chain_quad_run<14>(lds, L0, lane, un, ks->ek, 14u, src, dst);
    } else if (op == AES_OP_ECB_ENC) {
        if (nr == 10)
            ecb_enc_unit<1, 10>(lds, L0, lane, un, ks->ek, src, dst);
        else if (nr == 12)
            ecb_enc_unit<1, 12>(lds, L0, lane, un, ks->ek, src, dst);
        else if (nr == 14)
            ecb_enc_unit<1, 14>(lds, L0, lane, un, ks->ek, src, dst);
    } else {
        if (nr == 10)
            ctr_unit<1, 10>(lds, L0, lane, un, ks->ek, src, dst);
        else if (nr == 12)
            ctr_unit<1, 12>(lds, L0, lane, un, ks->ek, src, dst);
        else if (nr == 14)
            ctr_unit<1, 14>(lds, L0, lane, un, ks->ek, src, dst);
    }
}

template <bool DEC>
__device__ void worker_loop(const ServeArgs &a, const uint32_t *lds) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t L0 = (lane & 31u) << 2;
    const uint32_t L2 = L0 | SI_BASE;
    const int qi = DEC ? 1 : 0;
    uint64_t idx;
    while (claim(a, qi, &idx)) {
        // Input written by other agents must be re-read: acquire at system scope.
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
        const ServeUnit *p = a.qunits[qi] + (idx & a.qmask);
        Unit un;
        un.off = __hip_atomic_load(&p->u.off, __ATOMIC_RELAXED, AGT);
        un.nbytes = __hip_atomic_load(&p->u.nbytes, __ATOMIC_RELAXED, AGT);
        un.meta = __hip_atomic_load(&p->u.meta, __ATOMIC_RELAXED, AGT);
        for (int w = 0; w < 4; w++)
            un.w[w] = __hip_atomic_load(&p->u.w[w], __ATOMIC_RELAXED, AGT);
        const uint8_t *src = (const uint8_t *)__hip_atomic_load(&p->src, __ATOMIC_RELAXED, AGT);
        uint8_t *dst = (uint8_t *)__hip_atomic_load(&p->dst, __ATOMIC_RELAXED, AGT);
        const uint64_t pos = __hip_atomic_load(&p->pos, __ATOMIC_RELAXED, AGT);
        const uint32_t slot = __hip_atomic_load(&p->slot, __ATOMIC_RELAXED, AGT);
        const uint32_t info =
            __builtin_amdgcn_readfirstlane(__hip_atomic_load(&p->info, __ATOMIC_RELAXED, AGT));
        serve_unit<DEC>(lds, L0, L2, lane, un, info & 0xFFu, a, src, dst);
        // Make this unit's output visible beyond the device, then count it
        // (a request's only unit completes it without the count).
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        if (info & UNIT_ONLY) {
            if (lane == 0)
                complete(a, slot, pos, AES_OK);
            continue;
        }
        // The release fence above orders this unit's output before the count;
        // the last unit acquires the others' before completing the request.
        uint32_t left = 0;
        if (lane == 0)
            left = __hip_atomic_fetch_sub(&a.remaining[slot], 1u, __ATOMIC_RELAXED, AGT);
        left = __builtin_amdgcn_readfirstlane(left);
        if (left == 1u) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (lane == 0)
                complete(a, slot, pos, AES_OK);
        }
    }
}

// Run before every launch of k_serve (same stream): reopens the queues and
// drops positions taken by waves of the previous run that found no unit.
__global__ void k_serve_reset(ServeQueue *q, uint32_t *closed) {
    if (threadIdx.x == 0) {
        for (int i = 0; i < 2; i++)
            q[i].head = q[i].tail;
        *closed = 0u;
    }
}

// The grid: workgroup 0 (encryption tables) carries the dispatcher on its
// first wave, so that the one wave every other wave waits for is the first
// placed; the last n_dec_wg workgroups hold the decryption tables (none in a
// one-workgroup grid, whose decryption requests the host sends to a normal
// launch).  Every workgroup takes a whole compute unit's LDS, and the host
// never launches more workgroups than the device holds at once.
__global__ __launch_bounds__(512) void k_serve(ServeArgs a) {
    __shared__ uint32_t lds[LDS_DEC_WORDS];
    const bool dec = blockIdx.x >= gridDim.x - a.n_dec_wg;
    if (dec)
        fill_tables<true>(lds, a.timg);
    else
        fill_tables<false>(lds, a.timg);
    __syncthreads();
    if (blockIdx.x == 0 && (threadIdx.x >> 6) == 0) {
        dispatch_loop(a);
        return;
    }
    if (dec)
        worker_loop<true>(a, lds);
    else
        worker_loop<false>(a, lds);
}

}  // namespace aesgpu

// ======================================================================= host

using aesgpu::ServeArgs;
using aesgpu::ServeCtl;
using aesgpu::ServeDesc;
using aesgpu::ServeDone;
using aesgpu::ServeQueue;
using aesgpu::ServeUnit;

namespace {

uint64_t host_ns() {
    return (uint64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

inline void cpu_relax() { __builtin_ia32_pause(); }

// A pinned host buffer from aes_server_host_alloc: host and device views.
struct HostBuf {
    uint8_t *h;
    uint8_t *d;
    uint64_t n;
};

struct SlotInfo {
    uint64_t ticket = 0;
    uint64_t ring_pos = 0;  // persistent engine: the request's ring position
    uint64_t length = 0;
    uint32_t units = 0;  // work units admitted to queue `queue` (persistent engine)
    int queue = 0;
    aes_done_cb cb = nullptr;
    void *user = nullptr;
    uint64_t t_submit = 0;
    bool busy = false;
    bool by_launch = false;   // completion comes from a HIP event
    bool host_route = false;  // ran on the host route
};

}  // namespace

struct aes_server {
    aes_ctx_t *ctx = nullptr;
    aes_server_config_t cfg;
    int device = 0;
    uint32_t mask = 0;
    uint32_t n_wg = 0, n_dec_wg = 0;
    // host-mapped (host and device views)
    ServeDesc *ring = nullptr, *ring_d = nullptr;
    ServeDone *done = nullptr, *done_d = nullptr;
    ServeCtl *ctl = nullptr, *ctl_d = nullptr;
    // device memory
    aes_schedule_t *keys_d = nullptr;
    std::vector<aes_schedule_t> keys_h;  // host copies for the host route
    // Slots loaded by aes_server_set_key (read without mu by submits).
    std::unique_ptr<std::atomic<uint8_t>[]> key_set;
    uint64_t crossover[5] = {0, 0, 0, 0, 0};  // by op; 0 = never the host route
    ServeUnit *qunits_d[2] = {nullptr, nullptr};
    ServeQueue *q_d = nullptr;
    uint32_t *closed_d = nullptr;
    uint32_t *remaining_d = nullptr;
    const uint32_t *timg_d = nullptr;
    hipStream_t kstream = nullptr;     // the persistent kernel
    hipStream_t fbstream = nullptr;    // requests that take a normal launch
    std::vector<hipStream_t> streams;  // per-launch engine
    std::vector<uint8_t *> stage;      // per-launch engine: HBM staging, one per stream
    std::vector<hipEvent_t> events;    // one per ticket slot
    bool running = false;
    // bookkeeping (under mu)
    std::mutex mu;
    std::condition_variable cv;       // completions (waiters)
    std::condition_variable work_cv;  // submits (the idle completion thread)
    uint64_t next_ticket = 0;
    uint64_t ring_next = 0;          // next ring position (persistent engine)
    std::vector<uint8_t> ring_busy;  // ring slot holds an unfinished request
    uint64_t inflight_bytes = 0;
    uint32_t inflight = 0;
    uint64_t inflight_units[2] = {0, 0};
    std::vector<SlotInfo> slots;
    std::vector<uint64_t> live;
    std::vector<HostBuf> hostbufs;
    std::unordered_map<uint64_t, aes_done_t> finished;
    std::deque<uint64_t> finished_order;
    aes_server_stats_t stats{};
    std::thread poller;
    std::atomic<bool> quit{false};
    // Change counters read without mu: submits (the completion thread spins
    // on it before sleeping) and completion rounds (aes_server_wait spins on
    // it before sleeping).
    std::atomic<uint64_t> n_submits{0};
    std::atomic<uint64_t> n_finish_rounds{0};
};

// Spin budgets before a thread sleeps on a condition variable: a wake-up
// through the OS costs tens of microseconds, more than a request's round
// trip through the persistent kernel.
constexpr uint64_t POLLER_SPIN_NS = 200000;  // the completion thread, after its last request
constexpr uint64_t WAIT_SPIN_NS = 200000;    // aes_server_wait
// How long stop_persistent waits for the kernel after raising the stop flag.
// Once the dispatcher sees the flag it publishes nothing more, and the
// workers finish the units already published (at most queue_units units of
// at most 4 MiB in all), which takes milliseconds.
constexpr uint64_t STOP_WAIT_NS = 10000000000ull;

namespace {

using aesgpu::hip_fail_status;

// Launches the persistent kernel from the ring position the last one reached.
int launch_persistent(aes_server *s) {
    hipError_t e;
    hipLaunchKernelGGL(aesgpu::k_serve_reset, dim3(1), dim3(64), 0, s->kstream, s->q_d,
                       s->closed_d);
    if ((e = hipGetLastError()) != hipSuccess)
        return hip_fail_status(e);
    __atomic_store_n(&s->ctl->stop, 0u, __ATOMIC_RELEASE);
    ServeArgs a;
    a.ring = s->ring_d;
    a.done = s->done_d;
    a.ctl = s->ctl_d;
    a.qunits[0] = s->qunits_d[0];
    a.qunits[1] = s->qunits_d[1];
    a.q = s->q_d;
    a.closed = s->closed_d;
    a.remaining = s->remaining_d;
    a.keys = s->keys_d;
    a.timg = s->timg_d;
    a.start_pos = __atomic_load_n(&s->ctl->consumed, __ATOMIC_ACQUIRE);
    a.idle_ticks = (uint64_t)s->cfg.idle_timeout_ms * 100000ull;
    a.ring_mask = s->mask;
    a.qmask = s->cfg.queue_units - 1;
    a.n_keys = s->cfg.key_slots;
    a.n_dec_wg = s->n_dec_wg;
    a.tile = 4096;
    a.max_bytes = (uint32_t)s->cfg.max_request_bytes;
    hipLaunchKernelGGL(aesgpu::k_serve, dim3(s->n_wg), dim3(512), 0, s->kstream, a);
    if ((e = hipGetLastError()) != hipSuccess)
        return hip_fail_status(e);
    s->running = true;
    s->stats.kernel_launches++;
    return AES_OK;
}

// Asks the persistent kernel to exit and waits for it, for at most
// STOP_WAIT_NS (caller holds mu).  AES_ERR_TIMEOUT: the kernel is still
// running (the stop flag stays raised and the server still counts it as
// running).
int stop_persistent(aes_server *s) {
    if (!s->running)
        return AES_OK;
    __atomic_store_n(&s->ctl->stop, 1u, __ATOMIC_RELEASE);
    const uint64_t deadline = host_ns() + STOP_WAIT_NS;
    hipError_t e;
    while ((e = hipStreamQuery(s->kstream)) == hipErrorNotReady) {
        if (host_ns() > deadline)
            return AES_ERR_TIMEOUT;
        std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    s->running = false;
    __atomic_store_n(&s->ctl->stop, 0u, __ATOMIC_RELEASE);
    return e == hipSuccess ? AES_OK : hip_fail_status(e);
}

void finish_slot(aes_server *s, uint32_t slot, int32_t status, uint32_t units, uint64_t gd,
                 uint64_t gt, std::vector<std::pair<SlotInfo, aes_done_t>> &cbs) {
    SlotInfo &si = s->slots[slot];
    aes_done_t d;
    d.ticket = si.ticket;
    d.status = status;
    d.units = units;
    d.t_submit_ns = si.t_submit;
    d.t_done_ns = host_ns();
    d.gpu_dispatch_ticks = gd;
    d.gpu_done_ticks = gt;
    s->inflight--;
    s->inflight_bytes -= si.length;
    s->inflight_units[si.queue] -= si.units;
    if (!si.by_launch && !si.host_route && s->cfg.mode == AES_SERVE_PERSISTENT)
        s->ring_busy[si.ring_pos & s->mask] = 0;
    s->stats.completed++;
    if (si.cb) {
        cbs.emplace_back(si, d);
    } else {
        s->finished[si.ticket] = d;
        s->finished_order.push_back(si.ticket);
    }
    si.busy = false;
}

// The completion thread.
void poll_loop(aes_server *s) {
    std::vector<std::pair<SlotInfo, aes_done_t>> cbs;
    uint64_t last_check = host_ns();
    while (!s->quit.load(std::memory_order_acquire)) {
        bool progressed = false;
        bool busy;
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (size_t i = 0; i < s->live.size();) {
                const uint64_t t = s->live[i];
                const uint32_t slot = (uint32_t)(t & s->mask);
                SlotInfo &si = s->slots[slot];
                bool fin = false;
                int32_t st = AES_OK;
                uint32_t units = 0;
                uint64_t gd = 0, gt = 0;
                if (si.by_launch) {
                    const hipError_t e = hipEventQuery(s->events[slot]);
                    if (e == hipSuccess) {
                        fin = true;
                    } else if (e != hipErrorNotReady) {
                        fin = true;
                        st = hip_fail_status(e);
                    }
                } else {
                    const ServeDone &dr = s->done[si.ring_pos & s->mask];
                    if (__atomic_load_n(&dr.seq, __ATOMIC_ACQUIRE) == si.ring_pos + 1) {
                        fin = true;
                        st = dr.status;
                        units = dr.units;
                        gd = dr.t_dispatch;
                        gt = dr.t_done;
                    }
                }
                if (fin) {
                    finish_slot(s, slot, st, units, gd, gt, cbs);
                    s->live[i] = s->live.back();
                    s->live.pop_back();
                    progressed = true;
                } else {
                    i++;
                }
            }
            busy = !s->live.empty();
            // The persistent kernel may have exited on idle between a submit
            // and its launch check: relaunch it while descriptors wait.
            const uint64_t now = host_ns();
            if (s->cfg.mode == AES_SERVE_PERSISTENT && s->running && busy && !progressed &&
                now - last_check > 1000000ull) {
                last_check = now;
                if (hipStreamQuery(s->kstream) == hipSuccess) {
                    s->running = false;
                    if (__atomic_load_n(&s->ctl->consumed, __ATOMIC_ACQUIRE) < s->ring_next)
                        (void)launch_persistent(s);
                }
            }
        }
        if (progressed) {
            s->n_finish_rounds.fetch_add(1, std::memory_order_release);
            s->cv.notify_all();
        }
        for (auto &c : cbs)
            c.first.cb(&c.second, c.first.user);
        cbs.clear();
        if (!progressed) {
            if (busy) {
                for (int k = 0; k < 16; k++)
                    cpu_relax();
            } else {
                // Idle: spin a little for the next submit (back-to-back
                // callers then never wait for this thread to wake), then
                // sleep until a submit (or shutdown) rather than for a fixed
                // time, so that the first completion after an idle period is
                // seen as soon as it lands.  A submit between the check
                // above and the spin is caught by the wait's predicate.
                const uint64_t seen = s->n_submits.load(std::memory_order_acquire);
                const uint64_t until = host_ns() + POLLER_SPIN_NS;
                bool woke = false;
                while (!s->quit.load(std::memory_order_relaxed) && host_ns() < until) {
                    if (s->n_submits.load(std::memory_order_acquire) != seen) {
                        woke = true;
                        break;
                    }
                    cpu_relax();
                }
                if (woke)
                    continue;
                std::unique_lock<std::mutex> lk(s->mu);
                s->work_cv.wait_for(lk, std::chrono::milliseconds(5), [s] {
                    return !s->live.empty() || s->quit.load(std::memory_order_acquire);
                });
            }
        }
    }
}

int check_request(aes_server *s, uint32_t op, uint32_t key_slot, const uint8_t *iv,
                  const uint8_t *src, uint8_t *dst, uint64_t length) {
    const bool ecb = op == AES_OP_ECB_ENC || op == AES_OP_ECB_DEC;  // no IV
    if (op > AES_OP_ECB_DEC || (!iv && !ecb) || !src || !dst || !length)
        return AES_ERR_ARG;
    if (length > (1ull << 32) - 16 || (op != AES_OP_CTR && (length & 15)))
        return AES_ERR_LENGTH;
    if (key_slot >= s->cfg.key_slots)
        return AES_ERR_RANGE;
    // A slot never loaded holds no schedule: the kernels would skip the
    // request and leave its output unwritten.
    if (!s->key_set[key_slot].load(std::memory_order_acquire))
        return AES_ERR_STATE;
    if (src != dst) {
        const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
        if (a < b + length && b < a + length)
            return AES_ERR_OVERLAP;
    }
    return AES_OK;
}

// Looks [p, p + len) up among the server's host buffers (caller holds mu):
// returns 1 with *buf set when it starts inside one, 0 when it does not
// (device memory), AES_ERR_RANGE when it starts inside one and runs past
// its end.
int find_host(const aes_server *s, const uint8_t *p, uint64_t len, const HostBuf **buf) {
    for (const HostBuf &b : s->hostbufs) {
        if (p >= b.h && p < b.h + b.n) {
            if (len > (uint64_t)(b.h + b.n - p))
                return AES_ERR_RANGE;
            *buf = &b;
            return 1;
        }
    }
    return 0;
}

// Posts one request (caller holds mu).
int submit_locked(aes_server *s, uint32_t op, uint32_t key_slot, const uint8_t *iv,
                  const uint8_t *src, uint8_t *dst, uint64_t length, aes_done_cb cb, void *user,
                  uint64_t t_submit, uint64_t *ticket_out) {
    const HostBuf *hs = nullptr, *hd = nullptr;
    const int src_host = find_host(s, src, length, &hs);
    const int dst_host = find_host(s, dst, length, &hd);
    if (src_host < 0 || dst_host < 0)
        return AES_ERR_RANGE;
    // Device views of the payload (host buffers are mapped into the device).
    const uint8_t *src_d = src_host ? hs->d + (src - hs->h) : src;
    uint8_t *dst_d = dst_host ? hd->d + (dst - hd->h) : dst;
    const uint64_t ticket = s->next_ticket;
    const uint32_t slot = (uint32_t)(ticket & s->mask);
    const bool dec_op = op == AES_OP_CBC_DEC || op == AES_OP_ECB_DEC;
    // A persistent grid without decryption workgroups sends decryption to a
    // normal launch, as it does requests above max_request_bytes.
    const bool by_launch = s->cfg.mode == AES_SERVE_PER_LAUNCH ||
                           length > s->cfg.max_request_bytes || (dec_op && !s->n_dec_wg);
    const uint64_t ring_pos = s->ring_next;
    const uint32_t rslot = (uint32_t)(ring_pos & s->mask);
    if (s->slots[slot].busy || (!by_launch && s->ring_busy[rslot]) ||
        (s->inflight && s->inflight_bytes + length > s->cfg.hbm_cap_bytes)) {
        s->stats.rejected_again++;
        return AES_ERR_AGAIN;
    }
    // Units this request adds to its device queue; the queue never holds
    // more than queue_units unconsumed units (see the dispatcher).
    const int queue = dec_op ? 1 : 0;
    const uint32_t units =
        by_launch ? 0u : (op == AES_OP_CBC_ENC ? 1u : (uint32_t)((length + 4095) / 4096));
    if (s->inflight_units[queue] + units > s->cfg.queue_units) {
        s->stats.rejected_again++;
        return AES_ERR_AGAIN;
    }
    if (by_launch) {
        aes_req_t r;
        r.offset = 0;
        r.length = length;
        r.key_idx = key_slot;
        r.op = op;
        if (iv)
            memcpy(r.iv, iv, 16);
        else
            memset(r.iv, 0, 16);
        const size_t si = s->cfg.mode == AES_SERVE_PER_LAUNCH ? ticket % s->streams.size() : 0;
        hipStream_t st = s->cfg.mode == AES_SERVE_PER_LAUNCH ? s->streams[si] : s->fbstream;
        // Copy transport: host sides go through this stream's staging buffer
        // (in stream order: copy in, rounds in place or into it, copy out).
        const bool staged = !s->stage.empty() && (src_host || dst_host) &&
                            length <= s->cfg.max_request_bytes;
        const uint8_t *ksrc = src_d;
        uint8_t *kdst = dst_d;
        hipError_t e;
        if (staged && src_host) {
            if ((e = hipMemcpyAsync(s->stage[si], src, length, hipMemcpyHostToDevice, st)) !=
                hipSuccess)
                return hip_fail_status(e);
            ksrc = s->stage[si];
        }
        if (staged && dst_host)
            kdst = s->stage[si];
        int rc = aes_request_launch(s->ctx, s->keys_d, s->cfg.key_slots, ksrc, kdst, length, &r,
                                    st);
        if (rc)
            return rc;
        if (staged && dst_host &&
            (e = hipMemcpyAsync(dst, s->stage[si], length, hipMemcpyDeviceToHost, st)) !=
                hipSuccess)
            return hip_fail_status(e);
        if ((e = hipEventRecord(s->events[slot], st)) != hipSuccess)
            return hip_fail_status(e);
        if (s->cfg.mode == AES_SERVE_PERSISTENT)
            s->stats.fallbacks++;
    } else {
        ServeDesc *d = s->ring + rslot;
        d->src = (uint64_t)(uintptr_t)src_d;
        d->dst = (uint64_t)(uintptr_t)dst_d;
        d->length = (uint32_t)length;
        d->key_slot = key_slot;
        d->op = op;
        d->nr = s->keys_h[key_slot].nr;
        if (iv)
            memcpy(d->iv, iv, 16);
        else
            memset(d->iv, 0, 16);
        d->t_submit = t_submit;
        __atomic_store_n(&d->seq, ring_pos + 1, __ATOMIC_RELEASE);
        s->ring_busy[rslot] = 1;
        s->ring_next++;
        if (!s->running) {
            int rc = launch_persistent(s);
            if (rc)
                return rc;
        }
    }
    SlotInfo &si = s->slots[slot];
    si.ticket = ticket;
    si.ring_pos = ring_pos;
    si.length = length;
    si.cb = cb;
    si.user = user;
    si.t_submit = t_submit;
    si.busy = true;
    si.by_launch = by_launch;
    si.host_route = false;
    si.units = units;
    si.queue = queue;
    s->next_ticket++;
    s->inflight++;
    s->inflight_bytes += length;
    s->inflight_units[queue] += units;
    s->live.push_back(ticket);
    s->n_submits.fetch_add(1, std::memory_order_release);
    s->work_cv.notify_one();  // the completion thread may be idle
    s->stats.submitted++;
    if (ticket_out)
        *ticket_out = ticket;
    return AES_OK;
}

// The host route (caller does not hold mu).  Returns 1 when the request is
// not for it (it goes to the GPU engine), else its submit status: AES_OK
// with *ticket_out set once the request has completed (its own status is in
// its completion), or AES_ERR_AGAIN when its ticket slot is still busy.
int try_host_route(aes_server *s, uint32_t op, uint32_t key_slot, const uint8_t *iv,
                   const uint8_t *src, uint8_t *dst, uint64_t length, aes_done_cb cb,
                   void *user, uint64_t t_submit, uint64_t *ticket_out) {
    aes_schedule_t sched;
    uint64_t ticket;
    uint32_t slot;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        const HostBuf *b;
        if (length >= s->crossover[op] || !s->key_set[key_slot].load(std::memory_order_relaxed) ||
            find_host(s, src, length, &b) != 1 || find_host(s, dst, length, &b) != 1)
            return 1;
        ticket = s->next_ticket;
        slot = (uint32_t)(ticket & s->mask);
        SlotInfo &si = s->slots[slot];
        if (si.busy) {
            s->stats.rejected_again++;
            return AES_ERR_AGAIN;
        }
        sched = s->keys_h[key_slot];
        si = SlotInfo();
        si.ticket = ticket;
        si.length = length;
        si.cb = cb;
        si.user = user;
        si.t_submit = t_submit;
        si.busy = true;
        si.host_route = true;
        s->next_ticket++;
        s->inflight++;
        s->inflight_bytes += length;
        s->stats.submitted++;
        s->stats.host_routed++;
    }
    const int st = aes_host_route_crypt(&sched, op, iv, src, dst, length);
    std::vector<std::pair<SlotInfo, aes_done_t>> cbs;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        finish_slot(s, slot, st, 0, 0, 0, cbs);
    }
    s->cv.notify_all();
    if (ticket_out)
        *ticket_out = ticket;
    for (auto &c : cbs)
        c.first.cb(&c.second, c.first.user);
    return AES_OK;
}

// Frees a server.  kernel_alive: its persistent kernel did not stop, so the
// memory and streams that kernel may still touch (ring, completions,
// control block, queues, key slots, payload buffers, its stream) are left
// allocated rather than freed under it; the host-side state is freed.
void free_server(aes_server *s, bool kernel_alive = false) {
    if (s->poller.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);  // no lost wakeup of the idle wait
            s->quit.store(true, std::memory_order_release);
        }
        s->work_cv.notify_all();
        s->poller.join();
    }
    (void)hipSetDevice(s->device);
    if (kernel_alive) {
        delete s;
        return;
    }
    for (hipEvent_t e : s->events)
        (void)hipEventDestroy(e);
    for (hipStream_t st : s->streams)
        (void)hipStreamDestroy(st);
    if (s->kstream)
        (void)hipStreamDestroy(s->kstream);
    if (s->fbstream)
        (void)hipStreamDestroy(s->fbstream);
    if (s->ring)
        (void)hipHostFree(s->ring);
    if (s->done)
        (void)hipHostFree(s->done);
    if (s->ctl)
        (void)hipHostFree(s->ctl);
    for (void *p : {(void *)s->keys_d, (void *)s->qunits_d[0], (void *)s->qunits_d[1],
                    (void *)s->q_d, (void *)s->closed_d, (void *)s->remaining_d})
        if (p)
            (void)hipFree(p);
    for (uint8_t *p : s->stage)
        if (p)
            (void)hipFree(p);
    for (const HostBuf &b : s->hostbufs)
        (void)hipHostFree(b.h);
    delete s;
}

bool pow2(uint32_t v) { return v && !(v & (v - 1)); }

}  // namespace

extern "C" {

int aes_server_create(aes_ctx_t *ctx, const aes_server_config_t *cfg_in, aes_server_t **out) {
    if (!ctx || !out)
        return AES_ERR_ARG;
    *out = nullptr;
    aes_server_config_t cfg;
    memset(&cfg, 0, sizeof(cfg));
    if (cfg_in)
        cfg = *cfg_in;
    if (!cfg.ring_slots)
        cfg.ring_slots = 4096;
    if (!cfg.key_slots)
        cfg.key_slots = 256;
    if (!cfg.n_streams)
        cfg.n_streams = 8;
    if (!cfg.queue_units)
        cfg.queue_units = 65536;
    if (!cfg.idle_timeout_ms)
        cfg.idle_timeout_ms = 1000;
    if (!cfg.hbm_cap_bytes)
        cfg.hbm_cap_bytes = 256ull << 20;
    if (!cfg.max_request_bytes)
        cfg.max_request_bytes = 4ull << 20;
    if (cfg.mode > AES_SERVE_PER_LAUNCH || cfg.host_xfer > AES_XFER_DIRECT ||
        !pow2(cfg.ring_slots) || cfg.ring_slots < 64 ||
        cfg.ring_slots > 65536 || cfg.key_slots > 65536 || !pow2(cfg.queue_units) ||
        cfg.queue_units < 1024 || cfg.n_streams > 64 ||
        cfg.max_request_bytes > (uint64_t)(cfg.queue_units) * 4096 ||
        cfg.max_request_bytes > (1ull << 32) - 16)
        return AES_ERR_ARG;
    aesgpu::CtxInfo ci;
    int st = aesgpu::ctx_info(ctx, &ci);
    if (st)
        return st;
    if (ci.device == AES_DEVICE_NONE)
        return AES_ERR_DEVICE;
    aes_server *s = new (std::nothrow) aes_server();
    if (!s)
        return AES_ERR_NOMEM;
    s->ctx = ctx;
    s->cfg = cfg;
    s->device = ci.device;
    s->mask = cfg.ring_slots - 1;
    s->timg_d = ci.d_timg;
    // Every workgroup of the persistent grid must be resident at once (the
    // workers wait on the dispatcher's wave): at most the compute units times
    // the workgroups of k_serve one compute unit holds (one: each takes a
    // whole compute unit's LDS).  One workgroup holds the encryption tables
    // only; from two on, dec_workgroups of them (default half) hold the
    // decryption tables.
    hipError_t e;
    int per_cu = 0;
    if ((e = hipSetDevice(s->device)) != hipSuccess ||
        (e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, aesgpu::k_serve, 512, 0)) !=
            hipSuccess) {
        delete s;
        return hip_fail_status(e);
    }
    const long max_wg = (long)ci.n_cu * per_cu;
    // The default grid leaves one compute unit in eight free.  The hardware
    // places a kernel's workgroups on the shader engines in turn, in order;
    // once a persistent grid fills any shader engine, the first workgroup of
    // a kernel launched beside it that is sent there waits, and every
    // workgroup behind it, until the persistent kernel exits.  On a 256-CU
    // MI355X (32 shader engines of 8 CUs) grids of up to 224 workgroups let
    // other kernels run beside them; 228 and more held them back.
    long n_wg = cfg.n_workgroups ? (long)cfg.n_workgroups : (long)ci.n_cu - (long)ci.n_cu / 8;
    if (!cfg.n_workgroups && n_wg < 2)
        n_wg = max_wg < 2 ? max_wg : 2;
    long n_dec = n_wg == 1 ? 0 : (cfg.dec_workgroups ? (long)cfg.dec_workgroups : n_wg / 2);
    if (cfg.mode == AES_SERVE_PERSISTENT &&
        (n_wg < 1 || n_wg > max_wg || (n_wg == 1 && cfg.dec_workgroups) ||
         (n_wg > 1 && (n_dec < 1 || n_dec > n_wg - 1)))) {
        delete s;
        return AES_ERR_ARG;
    }
    s->n_wg = (uint32_t)n_wg;
    s->n_dec_wg = (uint32_t)n_dec;
#define SRV_TRY(expr)                                                                              \
    do {                                                                                           \
        if ((e = (expr)) != hipSuccess) {                                                          \
            free_server(s);                                                                        \
            return hip_fail_status(e);                                                             \
        }                                                                                          \
    } while (0)
    const unsigned hflags = hipHostMallocMapped | hipHostMallocCoherent;
    SRV_TRY(hipHostMalloc((void **)&s->ring, sizeof(ServeDesc) * cfg.ring_slots, hflags));
    SRV_TRY(hipHostMalloc((void **)&s->done, sizeof(ServeDone) * cfg.ring_slots, hflags));
    SRV_TRY(hipHostMalloc((void **)&s->ctl, sizeof(ServeCtl), hflags));
    memset(s->ring, 0, sizeof(ServeDesc) * cfg.ring_slots);
    memset(s->done, 0, sizeof(ServeDone) * cfg.ring_slots);
    memset(s->ctl, 0, sizeof(ServeCtl));
    SRV_TRY(hipHostGetDevicePointer((void **)&s->ring_d, s->ring, 0));
    SRV_TRY(hipHostGetDevicePointer((void **)&s->done_d, s->done, 0));
    SRV_TRY(hipHostGetDevicePointer((void **)&s->ctl_d, s->ctl, 0));
    SRV_TRY(hipMalloc((void **)&s->keys_d, sizeof(aes_schedule_t) * cfg.key_slots));
    SRV_TRY(hipMemset(s->keys_d, 0, sizeof(aes_schedule_t) * cfg.key_slots));
    if (cfg.mode == AES_SERVE_PERSISTENT) {
        for (int i = 0; i < 2; i++)
            SRV_TRY(hipMalloc((void **)&s->qunits_d[i], sizeof(ServeUnit) * cfg.queue_units));
        SRV_TRY(hipMalloc((void **)&s->q_d, sizeof(ServeQueue) * 2));
        SRV_TRY(hipMemset(s->q_d, 0, sizeof(ServeQueue) * 2));
        SRV_TRY(hipMalloc((void **)&s->closed_d, sizeof(uint32_t)));
        SRV_TRY(hipMalloc((void **)&s->remaining_d, sizeof(uint32_t) * cfg.ring_slots));
        SRV_TRY(hipMemset(s->remaining_d, 0, sizeof(uint32_t) * cfg.ring_slots));
        SRV_TRY(hipStreamCreateWithFlags(&s->kstream, hipStreamNonBlocking));
        SRV_TRY(hipStreamCreateWithFlags(&s->fbstream, hipStreamNonBlocking));
    } else {
        s->streams.resize(cfg.n_streams, nullptr);
        for (auto &st2 : s->streams)
            SRV_TRY(hipStreamCreateWithFlags(&st2, hipStreamNonBlocking));
        if (cfg.host_xfer == AES_XFER_COPY) {
            s->stage.resize(cfg.n_streams, nullptr);
            for (auto &p : s->stage)
                SRV_TRY(hipMalloc((void **)&p, cfg.max_request_bytes));
        }
    }
    s->events.resize(cfg.ring_slots, nullptr);
    for (auto &ev : s->events)
        SRV_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
#undef SRV_TRY
    s->slots.resize(cfg.ring_slots);
    s->ring_busy.assign(cfg.ring_slots, 0);
    s->keys_h.assign(cfg.key_slots, aes_schedule_t());
    s->key_set.reset(new (std::nothrow) std::atomic<uint8_t>[cfg.key_slots]);
    if (!s->key_set) {
        free_server(s);
        return AES_ERR_NOMEM;
    }
    for (uint32_t i = 0; i < cfg.key_slots; i++)
        s->key_set[i].store(0, std::memory_order_relaxed);
    s->live.reserve(cfg.ring_slots);
    try {
        s->poller = std::thread(poll_loop, s);
    } catch (...) {
        free_server(s);
        return AES_ERR_NOMEM;
    }
    *out = s;
    return AES_OK;
}

int aes_server_set_key(aes_server_t *s, uint32_t slot, const aes_schedule_t *host_sched) {
    if (!s || !host_sched)
        return AES_ERR_ARG;
    if (slot >= s->cfg.key_slots)
        return AES_ERR_RANGE;
    // The persistent engine takes the round count from here with each request.
    const uint32_t kb = host_sched->key_bits, nr = host_sched->nr;
    if (!((kb == 128 && nr == 10) || (kb == 192 && nr == 12) || (kb == 256 && nr == 14)))
        return AES_ERR_KEYSIZE;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->inflight)
        return AES_ERR_STATE;
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess)
        return hip_fail_status(e);
    int st = stop_persistent(s);
    if (st)
        return st;
    if ((e = hipMemcpy(s->keys_d + slot, host_sched, sizeof(aes_schedule_t),
                       hipMemcpyHostToDevice)) != hipSuccess)
        return hip_fail_status(e);
    s->keys_h[slot] = *host_sched;
    s->key_set[slot].store(1, std::memory_order_release);
    return AES_OK;
}

int aes_server_submit(aes_server_t *s, uint32_t op, uint32_t key_slot, const uint8_t iv[16],
                      const uint8_t *d_src, uint8_t *d_dst, uint64_t length, aes_done_cb cb,
                      void *user, uint64_t *ticket) {
    if (!s)
        return AES_ERR_ARG;
    int st = check_request(s, op, key_slot, iv, d_src, d_dst, length);
    if (st)
        return st;
    const uint64_t t_submit = host_ns();
    st = try_host_route(s, op, key_slot, iv, d_src, d_dst, length, cb, user, t_submit, ticket);
    if (st != 1)
        return st;
    std::lock_guard<std::mutex> lk(s->mu);
    if (hipSetDevice(s->device) != hipSuccess)
        return AES_ERR_DEVICE;
    return submit_locked(s, op, key_slot, iv, d_src, d_dst, length, cb, user, t_submit, ticket);
}

int aes_server_poll(aes_server_t *s, aes_done_t *out, uint32_t max, uint32_t *n_out) {
    if (!s || !n_out || (max && !out))
        return AES_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    uint32_t n = 0;
    while (n < max && !s->finished_order.empty()) {
        const uint64_t t = s->finished_order.front();
        s->finished_order.pop_front();
        auto it = s->finished.find(t);
        if (it == s->finished.end())
            continue;  // already taken by aes_server_wait
        out[n++] = it->second;
        s->finished.erase(it);
    }
    *n_out = n;
    return AES_OK;
}

int aes_server_wait(aes_server_t *s, uint64_t ticket, uint64_t timeout_ns, aes_done_t *out) {
    if (!s)
        return AES_ERR_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::nanoseconds(timeout_ns);
    const uint64_t spin_until = host_ns() + std::min<uint64_t>(WAIT_SPIN_NS, timeout_ns);
    for (;;) {
        auto it = s->finished.find(ticket);
        if (it != s->finished.end()) {
            if (out)
                *out = it->second;
            s->finished.erase(it);
            return AES_OK;
        }
        const SlotInfo &si = s->slots[ticket & s->mask];
        if (ticket >= s->next_ticket || !si.busy || si.ticket != ticket || si.cb)
            return AES_ERR_ARG;
        // Spin first (without mu) until the completion thread finishes a
        // round or the spin budget ends; then sleep on cv.
        const uint64_t seen = s->n_finish_rounds.load(std::memory_order_acquire);
        if (host_ns() < spin_until) {
            lk.unlock();
            while (s->n_finish_rounds.load(std::memory_order_acquire) == seen &&
                   host_ns() < spin_until)
                cpu_relax();
            lk.lock();
            continue;
        }
        if (s->cv.wait_until(lk, deadline) == std::cv_status::timeout &&
            s->finished.find(ticket) == s->finished.end())
            return AES_ERR_TIMEOUT;
    }
}

int aes_server_replay(aes_server_t *s, const aes_req_t *reqs, const double *arrival_s, uint64_t n,
                      const uint8_t *d_src_base, uint8_t *d_dst_base, aes_done_t *out) {
    if (!s || (n && (!reqs || !arrival_s || !out || !d_src_base || !d_dst_base)))
        return AES_ERR_ARG;
    for (uint64_t i = 0; i < n; i++) {
        int st = check_request(s, reqs[i].op, reqs[i].key_idx, reqs[i].iv,
                               d_src_base + reqs[i].offset, d_dst_base + reqs[i].offset,
                               reqs[i].length);
        if (st)
            return st;
    }
    std::vector<uint64_t> tickets(n, ~0ull);
    const uint64_t t0 = host_ns() + 1000000ull;
    for (uint64_t i = 0; i < n; i++) {
        const uint64_t target = t0 + (uint64_t)(arrival_s[i] * 1e9);
        while (host_ns() < target)
            cpu_relax();
        for (;;) {
            int st = try_host_route(s, reqs[i].op, reqs[i].key_idx, reqs[i].iv,
                                    d_src_base + reqs[i].offset, d_dst_base + reqs[i].offset,
                                    reqs[i].length, nullptr, nullptr, target, &tickets[i]);
            if (st == 1) {
                std::lock_guard<std::mutex> lk(s->mu);
                st = submit_locked(s, reqs[i].op, reqs[i].key_idx, reqs[i].iv,
                                   d_src_base + reqs[i].offset, d_dst_base + reqs[i].offset,
                                   reqs[i].length, nullptr, nullptr, target, &tickets[i]);
            }
            if (st == AES_OK)
                break;
            if (st != AES_ERR_AGAIN) {
                memset(&out[i], 0, sizeof(out[i]));
                out[i].status = st;
                out[i].ticket = ~0ull;
                break;
            }
            cpu_relax();
        }
    }
    int rc = AES_OK;
    for (uint64_t i = 0; i < n; i++) {
        if (tickets[i] == ~0ull)
            continue;
        int st = aes_server_wait(s, tickets[i], 60ull * 1000000000ull, &out[i]);
        if (st && !rc)
            rc = st;
    }
    return rc;
}

int aes_server_stats(aes_server_t *s, aes_server_stats_t *out) {
    if (!s || !out)
        return AES_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->in_flight = s->inflight;
    out->in_flight_bytes = s->inflight_bytes;
    return AES_OK;
}

int aes_server_host_alloc(aes_server_t *s, uint64_t bytes, void **host_ptr) {
    if (!s || !bytes || !host_ptr)
        return AES_ERR_ARG;
    *host_ptr = nullptr;
    std::lock_guard<std::mutex> lk(s->mu);
    hipError_t e = hipSetDevice(s->device);
    if (e != hipSuccess)
        return hip_fail_status(e);
    HostBuf b;
    b.n = bytes;
    if (hipHostMalloc((void **)&b.h, bytes, hipHostMallocMapped | hipHostMallocCoherent) !=
        hipSuccess)
        return AES_ERR_NOMEM;
    if ((e = hipHostGetDevicePointer((void **)&b.d, b.h, 0)) != hipSuccess) {
        (void)hipHostFree(b.h);
        return hip_fail_status(e);
    }
    try {
        s->hostbufs.push_back(b);
    } catch (...) {
        (void)hipHostFree(b.h);
        return AES_ERR_NOMEM;
    }
    *host_ptr = b.h;
    return AES_OK;
}

int aes_server_host_free(aes_server_t *s, void *host_ptr) {
    if (!s || !host_ptr)
        return AES_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    for (size_t i = 0; i < s->hostbufs.size(); i++) {
        if (s->hostbufs[i].h != host_ptr)
            continue;
        if (s->inflight)
            return AES_ERR_STATE;
        hipError_t e = hipHostFree(host_ptr);
        s->hostbufs.erase(s->hostbufs.begin() + (ptrdiff_t)i);
        return e == hipSuccess ? AES_OK : hip_fail_status(e);
    }
    return AES_ERR_ARG;
}

int aes_server_set_crossover(aes_server_t *s, uint32_t op, uint64_t bytes) {
    if (!s || op > AES_OP_ECB_DEC)
        return AES_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    s->crossover[op] = bytes;
    return AES_OK;
}

int aes_server_get_crossover(aes_server_t *s, uint32_t op, uint64_t *bytes) {
    if (!s || !bytes || op > AES_OP_ECB_DEC)
        return AES_ERR_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    *bytes = s->crossover[op];
    return AES_OK;
}

int aes_server_calibrate(aes_server_t *s, uint32_t key_slot, uint64_t out[5]) {
    if (!s)
        return AES_ERR_ARG;
    if (key_slot >= s->cfg.key_slots)
        return AES_ERR_RANGE;
    aes_schedule_t sched;
    uint64_t saved[5];
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->inflight)
            return AES_ERR_STATE;
        if (!s->key_set[key_slot].load(std::memory_order_relaxed))
            return AES_ERR_RANGE;
        sched = s->keys_h[key_slot];
        memcpy(saved, s->crossover, sizeof(saved));
        memset(s->crossover, 0, sizeof(s->crossover));  // measure the GPU engine itself
    }
    if (!__builtin_cpu_supports("aes"))
        return AES_ERR_DEVICE;
    const uint64_t top = std::min<uint64_t>(s->cfg.max_request_bytes, 4ull << 20);
    uint8_t *in = nullptr, *outb = nullptr;
    int rc = aes_server_host_alloc(s, top, (void **)&in);
    if (!rc)
        rc = aes_server_host_alloc(s, top, (void **)&outb);
    const uint8_t iv[16] = {0};
    const uint32_t ops[3] = {AES_OP_CTR, AES_OP_CBC_DEC, AES_OP_CBC_ENC};
    uint64_t found[3] = {0, 0, 0};
    constexpr int REPS = 5;
    for (int oi = 0; oi < 3 && !rc; oi++) {
        const uint32_t op = ops[oi];
        const uint64_t cap = op == AES_OP_CBC_ENC ? std::min<uint64_t>(top, 256u << 10) : top;
        std::vector<uint64_t> sizes;
        std::vector<bool> gpu_wins;
        for (uint64_t n = 4096; n <= cap && !rc; n *= 2) {
            uint64_t tg[REPS + 1], th[REPS + 1];
            for (int r = 0; r <= REPS && !rc; r++) {  // round 0 warms up
                uint64_t t0 = host_ns(), ticket = 0;
                rc = aes_server_submit(s, op, key_slot, iv, in, outb, n, nullptr, nullptr, &ticket);
                aes_done_t d;
                if (!rc)
                    rc = aes_server_wait(s, ticket, 10ull * 1000000000ull, &d);
                if (!rc)
                    rc = d.status;
                tg[r] = host_ns() - t0;
                t0 = host_ns();
                if (!rc)
                    rc = aes_host_route_crypt(&sched, op, iv, in, outb, n);
                th[r] = host_ns() - t0;
            }
            std::sort(tg + 1, tg + REPS + 1);
            std::sort(th + 1, th + REPS + 1);
            sizes.push_back(n);
            gpu_wins.push_back(tg[1 + REPS / 2] < th[1 + REPS / 2]);
        }
        if (rc)
            break;
        size_t k0 = sizes.size();
        while (k0 > 0 && gpu_wins[k0 - 1])
            k0--;
        found[oi] = k0 == sizes.size() ? UINT64_MAX : sizes[k0];
    }
    if (in)
        (void)aes_server_host_free(s, in);
    if (outb)
        (void)aes_server_host_free(s, outb);
    std::lock_guard<std::mutex> lk(s->mu);
    if (rc) {
        memcpy(s->crossover, saved, sizeof(saved));
        return rc;
    }
    s->crossover[AES_OP_CTR] = s->crossover[AES_OP_ECB_ENC] = found[0];
    s->crossover[AES_OP_CBC_DEC] = s->crossover[AES_OP_ECB_DEC] = found[1];
    s->crossover[AES_OP_CBC_ENC] = found[2];
    if (out)
        memcpy(out, s->crossover, sizeof(s->crossover));
    return AES_OK;
}

int aes_server_destroy(aes_server_t *s) {
    if (!s)
        return AES_OK;
    int rc = AES_OK;
    bool kernel_alive = false;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        const auto deadline = std::chrono::steady_clock::now() + std::chrono::seconds(10);
        while (s->inflight) {
            if (s->cv.wait_until(lk, deadline) == std::cv_status::timeout && s->inflight) {
                rc = AES_ERR_TIMEOUT;
                break;
            }
        }
        (void)hipSetDevice(s->device);
        int st = stop_persistent(s);
        if (st == AES_ERR_TIMEOUT)
            kernel_alive = true;
        if (st && !rc)
            rc = st;
        if (s->fbstream)
            (void)hipStreamSynchronize(s->fbstream);
        for (hipStream_t st2 : s->streams)
            (void)hipStreamSynchronize(st2);
    }
    free_server(s, kernel_alive);
    return rc;
}

}  // extern "C"
