// bitslice_aes.h -- the bitsliced AES cipher (FIPS-197 section 5.1) on 32
// blocks held as 128 bit planes, for CTR keystream on CDNA4.
//
// Plane layout: P[w][8 r + k] is bit k of byte r of state word w (the word of
// column w, little-endian), one bit per block across a 32-bit register, so
// every Boolean operation works on 32 blocks at once:
//   SubBytes    -- the generated tower-field S-box circuit (bitslice_sbox.h);
//   ShiftRows   -- register moves;
//   MixColumns  -- out_r = xtime(a_r ^ a_(r+1)) ^ (a_(r+1) ^ a_(r+2) ^ a_(r+3));
//   AddRoundKey -- each key bit becomes an all-ones or all-zero mask.
#pragma once
#include <stdint.h>

#include "bitslice_sbox.h"

namespace aesgpu {

// One transpose stage: exchange the j-bit fields that differ between words k
// and k + j (m selects the fields that stay).
template <int J>
__device__ __forceinline__ void swap_stage(uint32_t a[32], uint32_t m) {
#pragma unroll
    for (int k = 0; k < 32; k++) {
        if (k & J)
            continue;
        const uint32_t x = a[k], y = a[k + J];
        a[k] = (x & m) | ((y << J) & ~m);
        a[k + J] = ((x >> J) & m) | (y & ~m);
    }
}

// In-place 32x32 bit transpose: afterwards bit j of a[i] is the old bit i of
// a[j].  Halfword and byte stages are single v_perm_b32 operations.
__device__ __forceinline__ void transpose32(uint32_t a[32]) {
#pragma unroll
    for (int k = 0; k < 16; k++) {
        const uint32_t x = a[k], y = a[k + 16];
        a[k] = __builtin_amdgcn_perm(y, x, 0x05040100u);
        a[k + 16] = __builtin_amdgcn_perm(y, x, 0x07060302u);
    }
#pragma unroll
    for (int k = 0; k < 32; k++) {
        if (k & 8)
            continue;
        const uint32_t x = a[k], y = a[k + 8];
        a[k] = __builtin_amdgcn_perm(y, x, 0x06020400u);
        a[k + 8] = __builtin_amdgcn_perm(y, x, 0x07030501u);
    }
    swap_stage<4>(a, 0x0F0F0F0Fu);
    swap_stage<2>(a, 0x33333333u);
    swap_stage<1>(a, 0x55555555u);
}

__device__ __forceinline__ uint32_t key_mask(uint32_t word, int bit) {
    return 0u - ((word >> bit) & 1u);
}

// Plane k of state byte b (b = row + 4 * column).
#define PL(P, b, k) P[(b) >> 2][((b) & 3) * 8 + (k)]

__device__ __forceinline__ void bs_add_round_key(uint32_t P[4][32],
                                                 const uint32_t *__restrict__ rk) {
#pragma unroll
    for (int w = 0; w < 4; w++) {
        const uint32_t kw = rk[w];
#pragma unroll
        for (int i = 0; i < 32; i++)
            P[w][i] ^= key_mask(kw, i);
    }
}

__device__ __forceinline__ void bs_sub_bytes(uint32_t P[4][32]) {
#pragma unroll
    for (int b = 0; b < 16; b++)
        bitslice_sbox(PL(P, b, 0), PL(P, b, 1), PL(P, b, 2), PL(P, b, 3), PL(P, b, 4),
                      PL(P, b, 5), PL(P, b, 6), PL(P, b, 7), PL(P, b, 0), PL(P, b, 1),
                      PL(P, b, 2), PL(P, b, 3), PL(P, b, 4), PL(P, b, 5), PL(P, b, 6),
                      PL(P, b, 7));
}

// ShiftRows (FIPS-197 5.1.2): row r of the state rotates left by r columns.
// A renaming of planes; done as register moves so that every round leaves the
// state in the same registers.
__device__ __forceinline__ void bs_shift_rows(uint32_t P[4][32]) {
#pragma unroll
    for (int k = 0; k < 8; k++) {
        uint32_t t = PL(P, 1, k);  // row 1: one column
        PL(P, 1, k) = PL(P, 5, k);
        PL(P, 5, k) = PL(P, 9, k);
        PL(P, 9, k) = PL(P, 13, k);
        PL(P, 13, k) = t;
        t = PL(P, 2, k);  // row 2: two columns
        PL(P, 2, k) = PL(P, 10, k);
        PL(P, 10, k) = t;
        t = PL(P, 6, k);
        PL(P, 6, k) = PL(P, 14, k);
        PL(P, 14, k) = t;
        t = PL(P, 15, k);  // row 3: three columns (one to the right)
        PL(P, 15, k) = PL(P, 11, k);
        PL(P, 11, k) = PL(P, 7, k);
        PL(P, 7, k) = PL(P, 3, k);
        PL(P, 3, k) = t;
    }
}

// MixColumns and AddRoundKey (FIPS-197 5.1.3-5.1.4), in place, column by
// column: out_r = xtime(a_r ^ a_(r+1)) ^ (a_0 ^ a_1 ^ a_2 ^ a_3) ^ a_r ^ key.
__device__ __forceinline__ void bs_mix_key(uint32_t P[4][32], const uint32_t *__restrict__ rk) {
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const uint32_t kw = rk[c];  // round-key word c holds rows 0..3 of column c
        uint32_t t[4][8], tot[8];
#pragma unroll
        for (int k = 0; k < 8; k++) {
#pragma unroll
            for (int r = 0; r < 4; r++)
                t[r][k] = PL(P, 4 * c + r, k) ^ PL(P, 4 * c + ((r + 1) & 3), k);
            tot[k] = t[0][k] ^ t[2][k];
        }
#pragma unroll
        for (int r = 0; r < 4; r++) {
#pragma unroll
            for (int k = 0; k < 8; k++) {
                // xtime(t)_k = t_(k-1), with t_7 also fed into bits 0, 1, 3 and 4
                const uint32_t xt = k == 0 ? t[r][7] : t[r][k - 1];
                uint32_t v = __builtin_amdgcn_bitop3_b32(xt, tot[k], PL(P, 4 * c + r, k), 0x96);
                const uint32_t km = key_mask(kw, 8 * r + k);
                if (k == 1 || k == 3 || k == 4)
                    v = __builtin_amdgcn_bitop3_b32(v, t[r][7], km, 0x96);
                else
                    v ^= km;
                PL(P, 4 * c + r, k) = v;
            }
        }
    }
}

// The cipher (FIPS-197 5.1) on 32 bitsliced blocks; nr = 10, 12 or 14.
__device__ __forceinline__ void bs_cipher(uint32_t P[4][32], const uint32_t *__restrict__ rk,
                                          uint32_t nr) {
    bs_add_round_key(P, rk);
#pragma unroll 1
    for (uint32_t r = 1; r < nr; r++) {
        bs_sub_bytes(P);
        bs_shift_rows(P);
        bs_mix_key(P, rk + 4 * r);
    }
    bs_sub_bytes(P);
    bs_shift_rows(P);
    bs_add_round_key(P, rk + 4 * nr);
}

// Keystream of the 32 counter blocks ctr + 8 j + sub (j = 0..31) of one lane:
// afterwards P[w][j] is word w of block j's keystream.  The 16-byte counter
// block is nonce words w0, w1 and a 64-bit big-endian counter (SP 800-38A
// section 6.5 with a 64-bit counter field), given as ctr.
__device__ __forceinline__ void bs_ctr_keystream(uint32_t P[4][32], uint32_t w0, uint32_t w1,
                                                 uint64_t ctr, uint32_t sub,
                                                 const uint32_t *__restrict__ rk, uint32_t nr) {
#pragma unroll
    for (int j = 0; j < 32; j++) {
        const uint64_t c = ctr + 8u * j + sub;
        P[2][j] = __builtin_bswap32((uint32_t)(c >> 32));
        P[3][j] = __builtin_bswap32((uint32_t)c);
    }
    transpose32(P[2]);
    transpose32(P[3]);
#pragma unroll
    for (int i = 0; i < 32; i++) {  // the nonce words are the same in all 32 blocks
        P[0][i] = key_mask(w0, i);
        P[1][i] = key_mask(w1, i);
    }
    bs_cipher(P, rk, nr);
#pragma unroll
    for (int w = 0; w < 4; w++)
        transpose32(P[w]);
}

}  // namespace aesgpu
