// bitslice_aes.h -- the bitsliced AES cipher (FIPS-197 section 5.1) and
// inverse cipher (section 5.3) on 32 blocks held as 128 bit planes, for CTR
// keystream and CBC / ECB decryption on CDNA4.
//
// Plane layout: P[w][8 r + k] is bit k of byte r of state word w (the word of
// column w, little-endian), one bit per block across a 32-bit register, so
// every Boolean operation works on 32 blocks at once:
//   SubBytes    -- the generated tower-field S-box circuits (bitslice_sbox.h);
//   ShiftRows   -- register moves;
//   MixColumns  -- out_r = xtime(a_r ^ a_(r+1)) ^ (a_(r+1) ^ a_(r+2) ^ a_(r+3));
//   InvMixColumns -- MixColumns after multiplying each column by {04}x^2 +
//                 {05} (the inverse polynomial {0b}x^3 + {0d}x^2 + {09}x +
//                 {0e} is that product modulo x^4 + 1);
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

// MixColumns (FIPS-197 5.1.3) of column c, in place, then with KEY the
// round-key word kw added (5.1.4): out_r = xtime(a_r ^ a_(r+1)) ^ (a_0 ^ a_1
// ^ a_2 ^ a_3) ^ a_r ^ key.  Rows are rewritten in order 0..3, so only the
// column's total, a copy of row 0 (for row 3's a_(r+1)) and one row's
// xtime input are live beside the state.
template <bool KEY>
__device__ __forceinline__ void bs_mix_col(uint32_t P[4][32], int c, uint32_t kw) {
    uint32_t tot[8], a0[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
        a0[k] = PL(P, 4 * c, k);
        tot[k] = __builtin_amdgcn_bitop3_b32(PL(P, 4 * c, k), PL(P, 4 * c + 1, k),
                                             PL(P, 4 * c + 2, k), 0x96) ^
                 PL(P, 4 * c + 3, k);
    }
#pragma unroll
    for (int r = 0; r < 4; r++) {
        uint32_t t[8];
#pragma unroll
        for (int k = 0; k < 8; k++)
            t[k] = PL(P, 4 * c + r, k) ^ (r == 3 ? a0[k] : PL(P, 4 * c + r + 1, k));
#pragma unroll
        for (int k = 0; k < 8; k++) {
            // xtime(t)_k = t_(k-1), with t_7 also fed into bits 0, 1, 3 and 4
            const uint32_t xt = k == 0 ? t[7] : t[k - 1];
            uint32_t v = __builtin_amdgcn_bitop3_b32(xt, tot[k], PL(P, 4 * c + r, k), 0x96);
            const uint32_t km = KEY ? key_mask(kw, 8 * r + k) : 0u;
            if (k == 1 || k == 3 || k == 4)
                v = KEY ? __builtin_amdgcn_bitop3_b32(v, t[7], km, 0x96) : v ^ t[7];
            else if (KEY)
                v ^= km;
            PL(P, 4 * c + r, k) = v;
        }
    }
}

// MixColumns and AddRoundKey (FIPS-197 5.1.3-5.1.4), in place, column by
// column (round-key word c holds rows 0..3 of column c).
__device__ __forceinline__ void bs_mix_key(uint32_t P[4][32], const uint32_t *__restrict__ rk) {
#pragma unroll
    for (int c = 0; c < 4; c++)
        bs_mix_col<true>(P, c, rk[c]);
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

// ---------------------------------------------------------- inverse cipher

// InvShiftRows (FIPS-197 5.3.1): row r of the state rotates right by r
// columns (the moves of bs_shift_rows reversed).
__device__ __forceinline__ void bs_inv_shift_rows(uint32_t P[4][32]) {
#pragma unroll
    for (int k = 0; k < 8; k++) {
        uint32_t t = PL(P, 13, k);  // row 1: one column to the right
        PL(P, 13, k) = PL(P, 9, k);
        PL(P, 9, k) = PL(P, 5, k);
        PL(P, 5, k) = PL(P, 1, k);
        PL(P, 1, k) = t;
        t = PL(P, 2, k);  // row 2: two columns
        PL(P, 2, k) = PL(P, 10, k);
        PL(P, 10, k) = t;
        t = PL(P, 6, k);
        PL(P, 6, k) = PL(P, 14, k);
        PL(P, 14, k) = t;
        t = PL(P, 3, k);  // row 3: three columns to the right (one to the left)
        PL(P, 3, k) = PL(P, 7, k);
        PL(P, 7, k) = PL(P, 11, k);
        PL(P, 11, k) = PL(P, 15, k);
        PL(P, 15, k) = t;
    }
}

__device__ __forceinline__ void bs_inv_sub_bytes(uint32_t P[4][32]) {
#pragma unroll
    for (int b = 0; b < 16; b++)
        bitslice_inv_sbox(PL(P, b, 0), PL(P, b, 1), PL(P, b, 2), PL(P, b, 3), PL(P, b, 4),
                          PL(P, b, 5), PL(P, b, 6), PL(P, b, 7), PL(P, b, 0), PL(P, b, 1),
                          PL(P, b, 2), PL(P, b, 3), PL(P, b, 4), PL(P, b, 5), PL(P, b, 6),
                          PL(P, b, 7));
}

// {04} * t on one byte's planes: two xtime steps, each moving bit k to k + 1
// and feeding bit 7 back into bits 0, 1, 3 and 4.
__device__ __forceinline__ void bs_times4(const uint32_t t[8], uint32_t o[8]) {
    o[0] = t[6];
    o[1] = t[6] ^ t[7];
    o[2] = t[0] ^ t[7];
    o[3] = t[1] ^ t[6];
    o[4] = __builtin_amdgcn_bitop3_b32(t[2], t[6], t[7], 0x96);
    o[5] = t[3] ^ t[7];
    o[6] = t[4];
    o[7] = t[5];
}

// InvMixColumns (FIPS-197 5.3.3), in place: per column, a_r ^= {04}(a_r ^
// a_(r+2)), then MixColumns.
__device__ __forceinline__ void bs_inv_mix_columns(uint32_t P[4][32]) {
#pragma unroll
    for (int c = 0; c < 4; c++) {
#pragma unroll
        for (int r = 0; r < 2; r++) {
            uint32_t d[8], u[8];
#pragma unroll
            for (int k = 0; k < 8; k++)
                d[k] = PL(P, 4 * c + r, k) ^ PL(P, 4 * c + r + 2, k);
            bs_times4(d, u);
#pragma unroll
            for (int k = 0; k < 8; k++) {
                PL(P, 4 * c + r, k) ^= u[k];
                PL(P, 4 * c + r + 2, k) ^= u[k];
            }
        }
        bs_mix_col<false>(P, c, 0u);
    }
}

// The inverse cipher (FIPS-197 5.3, the straightforward form with the
// encryption schedule, round keys taken from the last): nr = 10, 12 or 14.
__device__ __forceinline__ void bs_inv_cipher(uint32_t P[4][32], const uint32_t *__restrict__ rk,
                                              uint32_t nr) {
    bs_add_round_key(P, rk + 4 * nr);
#pragma unroll 1
    for (uint32_t r = nr - 1; r >= 1; r--) {
        bs_inv_shift_rows(P);
        bs_inv_sub_bytes(P);
        bs_add_round_key(P, rk + 4 * r);
        bs_inv_mix_columns(P);
    }
    bs_inv_shift_rows(P);
    bs_inv_sub_bytes(P);
    bs_add_round_key(P, rk);
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
