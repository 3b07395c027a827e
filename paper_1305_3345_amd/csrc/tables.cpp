// tables.cpp -- the library's host-side AES constants: S-box, round tables and
// key schedules, built at run time from the field arithmetic of FIPS-197.
//
// GF(2^8) (FIPS-197 4.2, modulus x^8+x^4+x^3+x+1) is handled through log and
// antilog tables over the generator 0x03; the multiplicative inverse of a is
// 0x03^(255 - log a).  The S-box affine map (FIPS-197 5.1.1) is applied in its
// rotation form b ^ rotl(b,1) ^ rotl(b,2) ^ rotl(b,3) ^ rotl(b,4) ^ 0x63.
//
// Words are little-endian column words: byte r of a column (row r of the
// state) sits in bits 8r..8r+7, which is what a 32-bit load of the byte
// stream gives on the GPU.
#include <string.h>

#include "internal.h"

namespace aesgpu {
namespace {

struct Field {
    uint8_t log[256];
    uint8_t alog[256];
    uint8_t sbox[256];
    uint8_t inv_sbox[256];

    Field() {
        uint8_t x = 1;
        for (int i = 0; i < 255; i++) {
            alog[i] = x;
            log[x] = (uint8_t)i;
            uint8_t x2 = (uint8_t)((x << 1) ^ ((x & 0x80) ? 0x1b : 0));
            x = (uint8_t)(x2 ^ x);  // x * 0x03
        }
        alog[255] = alog[0];
        log[0] = 0;
        for (int a = 0; a < 256; a++) {
            uint8_t inv = a ? alog[(255 - log[a]) % 255] : 0;
            uint8_t s = inv;
            for (int k = 1; k <= 4; k++)
                s ^= (uint8_t)((inv << k) | (inv >> (8 - k)));
            s ^= 0x63;
            sbox[a] = s;
        }
        for (int a = 0; a < 256; a++)
            inv_sbox[sbox[a]] = (uint8_t)a;
    }

    uint8_t mul(uint8_t a, uint8_t b) const {
        if (!a || !b)
            return 0;
        return alog[(log[a] + log[b]) % 255];
    }
};

const Field &field() {
    static const Field f;
    return f;
}

inline uint32_t rotl32(uint32_t v, int k) { return k ? (v << k) | (v >> (32 - k)) : v; }

inline uint32_t bytes4(uint8_t b0, uint8_t b1, uint8_t b2, uint8_t b3) {
    return (uint32_t)b0 | ((uint32_t)b1 << 8) | ((uint32_t)b2 << 16) | ((uint32_t)b3 << 24);
}

uint32_t sub_word(uint32_t w) {
    const Field &f = field();
    return bytes4(f.sbox[w & 0xff], f.sbox[(w >> 8) & 0xff], f.sbox[(w >> 16) & 0xff],
                  f.sbox[w >> 24]);
}

// InvMixColumns of one column word (FIPS-197 5.3.3).
uint32_t inv_mix_column(uint32_t w) {
    const Field &f = field();
    uint8_t a[4] = {(uint8_t)w, (uint8_t)(w >> 8), (uint8_t)(w >> 16), (uint8_t)(w >> 24)};
    static const uint8_t m[4] = {0x0e, 0x0b, 0x0d, 0x09};
    uint8_t o[4];
    for (int r = 0; r < 4; r++) {
        uint8_t acc = 0;
        for (int k = 0; k < 4; k++)
            acc ^= f.mul(m[(k - r + 4) % 4], a[k]);
        o[r] = acc;
    }
    return bytes4(o[0], o[1], o[2], o[3]);
}

}  // namespace

void make_table_image(uint32_t img[TIMG_WORDS]) {
    const Field &f = field();
    for (int x = 0; x < 256; x++) {
        uint8_t s = f.sbox[x];
        // MixColumns column 0 of the circulant (02 03 01 01): rows get 2s, s, s, 3s.
        uint32_t te0 = bytes4(f.mul(s, 2), s, s, f.mul(s, 3));
        uint8_t si = f.inv_sbox[x];
        // InvMixColumns column 0 of (0e 0b 0d 09): rows get e*si, 9*si, d*si, b*si.
        uint32_t td0 = bytes4(f.mul(si, 0x0e), f.mul(si, 0x09), f.mul(si, 0x0d), f.mul(si, 0x0b));
        for (int t = 0; t < 4; t++) {
            img[t * 256 + x] = rotl32(te0, 8 * t);
            img[1024 + t * 256 + x] = rotl32(td0, 8 * t);
        }
        img[2048 + x] = 0x01010101u * si;
    }
}

int expand_key(const uint8_t *key, uint32_t key_bits, aes_schedule_t *out) {
    if (!key || !out)
        return AES_ERR_ARG;
    int nk, nr;
    switch (key_bits) {
    case 128: nk = 4; nr = 10; break;
    case 192: nk = 6; nr = 12; break;
    case 256: nk = 8; nr = 14; break;
    default: return AES_ERR_KEYSIZE;
    }
    memset(out, 0, sizeof(*out));
    out->key_bits = key_bits;
    out->nr = (uint32_t)nr;
    uint32_t *w = out->ek;
    for (int i = 0; i < nk; i++)
        w[i] = bytes4(key[4 * i], key[4 * i + 1], key[4 * i + 2], key[4 * i + 3]);
    uint32_t rcon = 1;
    const int total = 4 * (nr + 1);
    for (int i = nk; i < total; i++) {
        uint32_t t = w[i - 1];
        if (i % nk == 0) {
            // RotWord moves the first byte last: a right rotation of the LE word.
            t = sub_word((t >> 8) | (t << 24)) ^ rcon;
            rcon = field().mul((uint8_t)rcon, 2);
        } else if (nk > 6 && i % nk == 4) {
            t = sub_word(t);
        }
        w[i] = w[i - nk] ^ t;
    }
    // Equivalent inverse cipher schedule (FIPS-197 5.3.5), in application order.
    for (int c = 0; c < 4; c++) {
        out->dk[c] = w[4 * nr + c];
        out->dk[4 * nr + c] = w[c];
    }
    for (int r = 1; r < nr; r++)
        for (int c = 0; c < 4; c++)
            out->dk[4 * r + c] = inv_mix_column(w[4 * (nr - r) + c]);
    return AES_OK;
}

}  // namespace aesgpu
