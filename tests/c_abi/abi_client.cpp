// abi_client.cpp -- a client of libaesgpu.so written against include/aesgpu.h
// alone: no Python, no torch.  Device buffers come from hipMalloc, every call
// goes through the C ABI, and each form's output is checked byte for byte
// against the CPU oracle (liboracle.so, test infrastructure), request by
// request, with the bytes outside every request checked unchanged.
//
// Forms: the mixed batch (aes_batch), the single-op calls for CTR and CBC
// decryption, a plan launch and two replays of its graph, the persistent
// serving engine (submit and wait per request), and the host route's batch
// (aes_host_batch) on host buffers.  Prints one "c abi ok" line and returns 0,
// or prints the first mismatch and returns 1.
#include <hip/hip_runtime.h>

#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "aesgpu.h"

extern "C" int oracle_mode(uint32_t op, const uint8_t *key, uint32_t key_bits,
                           const uint8_t iv[16], const uint8_t *in, uint8_t *out, uint64_t len);

namespace {

#define AES_CHECK(call)                                                                          \
    do {                                                                                         \
        const int st_ = (call);                                                                  \
        if (st_ != AES_OK) {                                                                     \
            fprintf(stderr, "%s:%d %s: %s (%d)\n", __FILE__, __LINE__, #call, aes_strerror(st_), \
                    st_);                                                                        \
            exit(1);                                                                             \
        }                                                                                        \
    } while (0)

#define HIP_CHECK(call)                                                                      \
    do {                                                                                     \
        const hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) {                                                              \
            fprintf(stderr, "%s:%d %s: %s\n", __FILE__, __LINE__, #call,                     \
                    hipGetErrorString(e_));                                                  \
            exit(1);                                                                         \
        }                                                                                    \
    } while (0)

// SplitMix64 (seeded input bytes only).
struct Rng {
    uint64_t x;
    uint64_t next() {
        uint64_t z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    void fill(uint8_t *p, size_t n) {
        for (size_t i = 0; i < n; i++)
            p[i] = (uint8_t)next();
    }
};

constexpr int N_KEYS = 3;
const uint32_t KEY_BITS[N_KEYS] = {128, 192, 256};
constexpr uint8_t SENTINEL = 0xA5;

uint8_t g_keys[N_KEYS][32];

// The oracle's output for reqs over in (sentinel bytes elsewhere).
std::vector<uint8_t> expected(const std::vector<aes_req_t> &reqs, const std::vector<uint8_t> &in) {
    std::vector<uint8_t> out(in.size(), SENTINEL);
    for (const aes_req_t &r : reqs) {
        if (oracle_mode(r.op, g_keys[r.key_idx], KEY_BITS[r.key_idx], r.iv, in.data() + r.offset,
                        out.data() + r.offset, r.length) != 0) {
            fprintf(stderr, "oracle rejected a request\n");
            exit(1);
        }
    }
    return out;
}

int compare(const char *form, const std::vector<uint8_t> &got, const std::vector<uint8_t> &want) {
    for (size_t i = 0; i < got.size(); i++) {
        if (got[i] != want[i]) {
            fprintf(stderr, "%s: byte %zu is %02x, expected %02x\n", form, i, got[i], want[i]);
            return 1;
        }
    }
    return 0;
}

}  // namespace

int main() {
    Rng rng{2024};
    aes_ctx_t *ctx = nullptr;
    AES_CHECK(aes_ctx_create(0, &ctx));

    aes_schedule_t sch[N_KEYS];
    for (int k = 0; k < N_KEYS; k++) {
        rng.fill(g_keys[k], sizeof(g_keys[k]));
        AES_CHECK(aes_expand_key(g_keys[k], KEY_BITS[k], &sch[k]));
    }
    aes_schedule_t *d_sch = nullptr;
    HIP_CHECK(hipMalloc((void **)&d_sch, sizeof(sch)));
    HIP_CHECK(hipMemcpy(d_sch, sch, sizeof(sch), hipMemcpyHostToDevice));

    // 240 requests of every op, 1..300 blocks (CTR lengths ragged), gaps
    // between them, every key size.
    std::vector<aes_req_t> reqs(240);
    uint64_t off = 0;
    for (size_t i = 0; i < reqs.size(); i++) {
        aes_req_t &r = reqs[i];
        r.op = (uint32_t)(i % 5);
        r.key_idx = (uint32_t)((i / 5) % N_KEYS);
        r.length = 16 * (1 + rng.next() % 300);
        if (r.op == AES_OP_CTR)
            r.length -= rng.next() % 16;
        rng.fill(r.iv, 16);
        r.offset = off;
        off += (r.length + 15) / 16 * 16 + 16 * (rng.next() % 4);
    }
    const uint64_t buf = off + 64;
    std::vector<uint8_t> in(buf);
    rng.fill(in.data(), buf);
    uint8_t *d_in = nullptr, *d_out = nullptr;
    HIP_CHECK(hipMalloc((void **)&d_in, buf));
    HIP_CHECK(hipMalloc((void **)&d_out, buf));
    HIP_CHECK(hipMemcpy(d_in, in.data(), buf, hipMemcpyHostToDevice));
    const std::vector<uint8_t> sentinel(buf, SENTINEL);
    std::vector<uint8_t> got(buf);

    auto reset = [&] { HIP_CHECK(hipMemcpy(d_out, sentinel.data(), buf, hipMemcpyHostToDevice)); };
    auto fetch = [&] {
        HIP_CHECK(hipDeviceSynchronize());
        HIP_CHECK(hipMemcpy(got.data(), d_out, buf, hipMemcpyDeviceToHost));
    };
    int bad = 0;
    const std::vector<uint8_t> want_all = expected(reqs, in);

    // 1. One mixed batch.
    reset();
    AES_CHECK(aes_batch(ctx, d_sch, N_KEYS, d_in, d_out, buf, reqs.data(), reqs.size(), nullptr));
    fetch();
    bad |= compare("aes_batch", got, want_all);

    // 2. Single-op calls with the caller's arrays (CTR, then CBC decryption).
    for (uint32_t op : {(uint32_t)AES_OP_CTR, (uint32_t)AES_OP_CBC_DEC}) {
        std::vector<aes_req_t> sub;
        std::vector<uint64_t> offs, lens;
        std::vector<uint32_t> kidx;
        std::vector<uint8_t> ivs;
        for (const aes_req_t &r : reqs) {
            if (r.op != op)
                continue;
            sub.push_back(r);
            offs.push_back(r.offset);
            lens.push_back(r.length);
            kidx.push_back(r.key_idx);
            ivs.insert(ivs.end(), r.iv, r.iv + 16);
        }
        reset();
        if (op == AES_OP_CTR)
            AES_CHECK(aes_ctr_batch(ctx, d_sch, N_KEYS, d_in, d_out, buf, offs.data(), lens.data(),
                                    kidx.data(), ivs.data(), sub.size(), nullptr));
        else
            AES_CHECK(aes_cbc_decrypt_batch(ctx, d_sch, N_KEYS, d_in, d_out, buf, offs.data(),
                                            lens.data(), kidx.data(), ivs.data(), sub.size(),
                                            nullptr));
        fetch();
        bad |= compare(op == AES_OP_CTR ? "aes_ctr_batch" : "aes_cbc_decrypt_batch", got,
                       expected(sub, in));
    }

    // 3. A plan, then two replays of its graph.
    aes_plan_t *plan = nullptr;
    AES_CHECK(aes_plan_create(ctx, reqs.data(), reqs.size(), N_KEYS, buf, &plan));
    reset();
    AES_CHECK(aes_plan_launch(plan, d_sch, d_in, d_out, nullptr));
    fetch();
    bad |= compare("aes_plan_launch", got, want_all);
    aes_graph_t *graph = nullptr;
    AES_CHECK(aes_plan_graph(plan, d_sch, d_in, d_out, &graph));
    for (int rep = 0; rep < 2; rep++) {
        reset();
        AES_CHECK(aes_graph_launch(graph, nullptr));
        fetch();
        bad |= compare("aes_graph_launch", got, want_all);
    }
    aes_graph_destroy(graph);
    aes_plan_destroy(plan);

    // 4. The persistent serving engine, one request at a time.
    aes_server_config_t cfg;
    memset(&cfg, 0, sizeof(cfg));
    cfg.mode = AES_SERVE_PERSISTENT;
    cfg.key_slots = N_KEYS;
    aes_server_t *srv = nullptr;
    AES_CHECK(aes_server_create(ctx, &cfg, &srv));
    for (int k = 0; k < N_KEYS; k++)
        AES_CHECK(aes_server_set_key(srv, (uint32_t)k, &sch[k]));
    reset();
    for (const aes_req_t &r : reqs) {
        uint64_t ticket = 0;
        AES_CHECK(aes_server_submit(srv, r.op, r.key_idx, r.iv, d_in + r.offset, d_out + r.offset,
                                    r.length, nullptr, nullptr, &ticket));
        aes_done_t done;
        AES_CHECK(aes_server_wait(srv, ticket, 10000000000ull, &done));
        AES_CHECK(done.status);
    }
    AES_CHECK(aes_server_destroy(srv));
    fetch();
    bad |= compare("aes_server", got, want_all);

    // 5. The host route's batch on host buffers.
    std::vector<uint8_t> host_out(buf, SENTINEL);
    AES_CHECK(aes_host_batch(sch, N_KEYS, in.data(), host_out.data(), buf, reqs.data(),
                             reqs.size(), 0));
    bad |= compare("aes_host_batch", host_out, want_all);

    HIP_CHECK(hipFree(d_in));
    HIP_CHECK(hipFree(d_out));
    HIP_CHECK(hipFree(d_sch));
    aes_ctx_destroy(ctx);
    if (bad)
        return 1;
    uint64_t payload = 0;
    for (const aes_req_t &r : reqs)
        payload += r.length;
    printf("c abi ok: %zu requests, %llu bytes, every form equal to the oracle\n", reqs.size(),
           (unsigned long long)payload);
    return 0;
}
