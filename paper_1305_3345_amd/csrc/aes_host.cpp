// aes_host.cpp -- the host route of size-based CPU/GPU dispatch.  The paper
// (section 4) notes that the fixed cost of calling the GPU makes small tasks
// finish sooner on the CPU, with the crossover depending on the task and the
// machine, best found by a micro-benchmark at start-up.  The serving engine
// routes a request here only when the caller has set or calibrated a
// crossover for its op, its length is below it, and both payload sides are
// in the server's pinned host buffers; no GPU entry point calls this code.
//
// AES-NI on the calling core, over the schedules the kernels use: ek round r
// holds the 16 bytes FIPS-197 lists for w[4r..4r+3], and dk round r is the
// equivalent inverse cipher's key for decryption round r (FIPS-197 5.3.5),
// which is the form the AESDEC instruction takes.  Modes per SP 800-38A:
// ECB 6.1, CBC 6.2, CTR 6.5 with the low 64 bits of the counter block as a
// big-endian counter (no carry into the nonce half).
#include <stdint.h>
#include <string.h>
#include <wmmintrin.h>

#include "aesgpu.h"

#define AESNI __attribute__((target("aes,sse4.1")))

namespace {

constexpr int LANES = 8;  // blocks in flight: AESENC latency over its issue rate

struct Keys {
    __m128i k[15];
};

AESNI inline void load_keys(const uint32_t *w, int nr, Keys *out) {
    for (int r = 0; r <= nr; r++)
        out->k[r] = _mm_loadu_si128(reinterpret_cast<const __m128i *>(w + 4 * r));
}

AESNI inline __m128i enc1(const Keys &K, int nr, __m128i x) {
    x = _mm_xor_si128(x, K.k[0]);
    for (int r = 1; r < nr; r++)
        x = _mm_aesenc_si128(x, K.k[r]);
    return _mm_aesenclast_si128(x, K.k[nr]);
}

AESNI inline __m128i dec1(const Keys &K, int nr, __m128i x) {
    x = _mm_xor_si128(x, K.k[0]);
    for (int r = 1; r < nr; r++)
        x = _mm_aesdec_si128(x, K.k[r]);
    return _mm_aesdeclast_si128(x, K.k[nr]);
}

// LANES independent blocks through the cipher together.
template <bool DEC>
AESNI inline void crypt8(const Keys &K, int nr, __m128i *x) {
    for (int j = 0; j < LANES; j++)
        x[j] = _mm_xor_si128(x[j], K.k[0]);
    for (int r = 1; r < nr; r++)
        for (int j = 0; j < LANES; j++)
            x[j] = DEC ? _mm_aesdec_si128(x[j], K.k[r]) : _mm_aesenc_si128(x[j], K.k[r]);
    for (int j = 0; j < LANES; j++)
        x[j] = DEC ? _mm_aesdeclast_si128(x[j], K.k[nr]) : _mm_aesenclast_si128(x[j], K.k[nr]);
}

inline __m128i ld(const uint8_t *p) { return _mm_loadu_si128(reinterpret_cast<const __m128i *>(p)); }
inline void st(uint8_t *p, __m128i v) { _mm_storeu_si128(reinterpret_cast<__m128i *>(p), v); }

// Counter block for block j: nonce half unchanged, low half + j mod 2^64.
inline __m128i ctr_block(uint64_t nonce_le, uint64_t c0, uint64_t j) {
    return _mm_set_epi64x((long long)__builtin_bswap64(c0 + j), (long long)nonce_le);
}

template <bool DEC>
AESNI void ecb(const Keys &K, int nr, const uint8_t *src, uint8_t *dst, uint64_t nblk) {
    uint64_t i = 0;
    __m128i x[LANES];
    for (; i + LANES <= nblk; i += LANES) {
        for (int j = 0; j < LANES; j++)
            x[j] = ld(src + 16 * (i + j));
        crypt8<DEC>(K, nr, x);
        for (int j = 0; j < LANES; j++)
            st(dst + 16 * (i + j), x[j]);
    }
    for (; i < nblk; i++)
        st(dst + 16 * i, DEC ? dec1(K, nr, ld(src + 16 * i)) : enc1(K, nr, ld(src + 16 * i)));
}

AESNI void ctr(const Keys &K, int nr, const uint8_t *iv, const uint8_t *src, uint8_t *dst,
               uint64_t length) {
    uint64_t nonce, cbe;
    memcpy(&nonce, iv, 8);
    memcpy(&cbe, iv + 8, 8);
    const uint64_t c0 = __builtin_bswap64(cbe);
    const uint64_t full = length / 16;
    uint64_t i = 0;
    __m128i x[LANES];
    for (; i + LANES <= full; i += LANES) {
        for (int j = 0; j < LANES; j++)
            x[j] = ctr_block(nonce, c0, i + j);
        crypt8<false>(K, nr, x);
        for (int j = 0; j < LANES; j++)
            st(dst + 16 * (i + j), _mm_xor_si128(x[j], ld(src + 16 * (i + j))));
    }
    for (; i < full; i++)
        st(dst + 16 * i, _mm_xor_si128(enc1(K, nr, ctr_block(nonce, c0, i)), ld(src + 16 * i)));
    const uint64_t tail = length % 16;
    if (tail) {
        uint8_t ks[16];
        st(ks, enc1(K, nr, ctr_block(nonce, c0, full)));
        for (uint64_t b = 0; b < tail; b++)
            dst[16 * full + b] = src[16 * full + b] ^ ks[b];
    }
}

AESNI void cbc_enc(const Keys &K, int nr, const uint8_t *iv, const uint8_t *src, uint8_t *dst,
                   uint64_t nblk) {
    __m128i c = ld(iv);
    for (uint64_t i = 0; i < nblk; i++) {
        c = enc1(K, nr, _mm_xor_si128(ld(src + 16 * i), c));
        st(dst + 16 * i, c);
    }
}

// In place is allowed: each group's ciphertext (the next group's chaining
// values) is read before the group's plaintext overwrites it.
AESNI void cbc_dec(const Keys &K, int nr, const uint8_t *iv, const uint8_t *src, uint8_t *dst,
                   uint64_t nblk) {
    __m128i prev = ld(iv);
    uint64_t i = 0;
    __m128i x[LANES], c[LANES];
    for (; i + LANES <= nblk; i += LANES) {
        for (int j = 0; j < LANES; j++)
            x[j] = c[j] = ld(src + 16 * (i + j));
        crypt8<true>(K, nr, x);
        st(dst + 16 * i, _mm_xor_si128(x[0], prev));
        for (int j = 1; j < LANES; j++)
            st(dst + 16 * (i + j), _mm_xor_si128(x[j], c[j - 1]));
        prev = c[LANES - 1];
    }
    for (; i < nblk; i++) {
        const __m128i cj = ld(src + 16 * i);
        st(dst + 16 * i, _mm_xor_si128(dec1(K, nr, cj), prev));
        prev = cj;
    }
}

}  // namespace

extern "C" int aes_host_route_crypt(const aes_schedule_t *sched, uint32_t op, const uint8_t *iv,
                                    const uint8_t *src, uint8_t *dst, uint64_t length) {
    const bool ecb_op = op == AES_OP_ECB_ENC || op == AES_OP_ECB_DEC;
    if (!sched || op > AES_OP_ECB_DEC || (!iv && !ecb_op) || (length && (!src || !dst)))
        return AES_ERR_ARG;
    const int nr = (int)sched->nr;
    if (!((nr == 10 && sched->key_bits == 128) || (nr == 12 && sched->key_bits == 192) ||
          (nr == 14 && sched->key_bits == 256)))
        return AES_ERR_KEYSIZE;
    if (op != AES_OP_CTR && (length & 15))
        return AES_ERR_LENGTH;
    if (src != dst && length) {
        const uintptr_t a = (uintptr_t)src, b = (uintptr_t)dst;
        if (a < b + length && b < a + length)
            return AES_ERR_OVERLAP;
    }
    if (!__builtin_cpu_supports("aes"))
        return AES_ERR_DEVICE;
    if (!length)
        return AES_OK;
    const bool dec = op == AES_OP_CBC_DEC || op == AES_OP_ECB_DEC;
    Keys K;
    load_keys(dec ? sched->dk : sched->ek, nr, &K);
    switch (op) {
    case AES_OP_CBC_ENC:
        cbc_enc(K, nr, iv, src, dst, length / 16);
        break;
    case AES_OP_CBC_DEC:
        cbc_dec(K, nr, iv, src, dst, length / 16);
        break;
    case AES_OP_CTR:
        ctr(K, nr, iv, src, dst, length);
        break;
    case AES_OP_ECB_ENC:
        ecb<false>(K, nr, src, dst, length / 16);
        break;
    default:
        ecb<true>(K, nr, src, dst, length / 16);
        break;
    }
    return AES_OK;
}
