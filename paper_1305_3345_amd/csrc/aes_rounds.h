// aes_rounds.h -- AES round and work-unit device functions for CDNA4 (gfx950),
// table variant, shared by the batch kernels and the persistent server (the
// CBC-encrypt chains built on these rounds are in aes_chain.h).
//
// The cipher is FIPS-197 in the round-table ("T-table") form: for encryption
// one round of SubBytes, ShiftRows, MixColumns and AddRoundKey on column c is
//   t_c = Te0[s_c.b0] ^ Te1[s_(c+1).b1] ^ Te2[s_(c+2).b2] ^ Te3[s_(c+3).b3] ^ rk_c,
// with Te_k the S-box output times column k of the MixColumns circulant; the
// equivalent inverse cipher (FIPS-197 5.3.5) has the same shape with Td_k,
// columns c-k and the transformed round keys.  Modes are SP 800-38A: CTR
// (6.5, 64-bit counter) and CBC decryption (6.2) run every block in
// parallel; CBC encryption (6.2) is a serial chain per request.
//
// Layout in LDS (one workgroup per compute unit; tables are filled once per
// workgroup and the grid walks over all work units):
//   Each 1 KiB table is replicated 32 times so that lane l reads only bank
//   l mod 32: entry x of table t lives at byte
//     (t >> 1) << 16 | x << 8 | (t & 1) << 7 | (lane & 31) << 2.
//   One v_perm_b32 builds that address from a state word and a per-lane
//   constant (byte k of the state word into bits 8..15); the table parity is
//   the ds_read immediate offset.  Four tables take 128 KiB.  Decryption adds
//   the inverse S-box (Si4, byte repeated 4 times) at 128 KiB + x << 7 |
//   (lane & 31) << 2, 32 KiB more, for the last round.
//   Round keys are wave-uniform in the parallel kernels (one wave works one
//   unit of one request) and live in SGPRs.

#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

namespace aesgpu {

constexpr uint32_t LDS_ENC_WORDS = 32768;  // 128 KiB
constexpr uint32_t LDS_DEC_WORDS = 40960;  // 160 KiB
constexpr uint32_t SI_BASE = 0x20000u;     // byte address of Si4

// ---------------------------------------------------------------- tables

// Each thread loads table words from the 9 KiB image and writes the word's
// 32 replicas itself, starting at replica (thread mod 32) so that the 32
// threads of a half-wave hit 32 different banks on every store.
template <bool DEC>
__device__ __forceinline__ void fill_tables(uint32_t *lds, const uint32_t *__restrict__ timg) {
    const uint32_t base = DEC ? 1024u : 0u;
    const uint32_t nwords = DEC ? 1280u : 1024u;  // 4 tables (+ Si4)
    const uint32_t rot = threadIdx.x & 31u;
    for (uint32_t w = threadIdx.x; w < nwords; w += blockDim.x) {
        uint32_t v, dst;
        if (w < 1024u) {
            const uint32_t t = w >> 8, x = w & 255u;
            v = timg[base + w];
            dst = (t >> 1) * 16384u + x * 64u + (t & 1u) * 32u;
        } else {
            const uint32_t x = w - 1024u;
            v = timg[2048u + x];
            dst = 32768u + x * 32u;
        }
#pragma unroll
        for (uint32_t j = 0; j < 32u; j++)
            lds[dst + ((j + rot) & 31u)] = v;
    }
}

// Three-input XOR in one VALU op (v_bitop3_b32, truth table 0x96 = a ^ b ^ c).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ uint32_t lds_word(const uint32_t *lds, uint32_t byte_addr) {
    return *reinterpret_cast<const uint32_t *>(reinterpret_cast<const char *>(lds) + byte_addr);
}

// Table T (0..3) looked up at byte K of v.  L0 = (lane & 31) * 4; tables 2
// and 3 live in the second 64 KiB region (L0 | 0x10000, byte 2 = region).
template <int K, int T>
__device__ __forceinline__ uint32_t tlook(const uint32_t *lds, uint32_t v, uint32_t L0) {
    // v_perm_b32 selector: byte0 <- L.byte0, byte1 <- v.byte K, byte2 <- L.byte2, byte3 <- 0
    const uint32_t L = T < 2 ? L0 : (L0 | 0x10000u);
    const uint32_t a = __builtin_amdgcn_perm(v, L, 0x0C020400u | ((4u + K) << 8));
    return lds_word(lds, a + ((T & 1) ? 128u : 0u));
}

// Inverse S-box byte K of v, read from Si4.  L2 = SI_BASE | (lane & 31) * 4.
template <int K>
__device__ __forceinline__ uint32_t silook(const uint32_t *lds, uint32_t v, uint32_t L2) {
    const uint32_t x = (v >> (8 * K)) & 0xffu;
    return lds_word(lds, (x << 7) | L2);
}

// Bytes 0,1 of a,b and bytes 2,3 of c,d: out byte r = (a,b,c,d)[r].byte r.
__device__ __forceinline__ uint32_t pick_diag(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
    const uint32_t lo = __builtin_amdgcn_perm(b, a, 0x0C0C0500u);
    const uint32_t hi = __builtin_amdgcn_perm(d, c, 0x07020C0Cu);
    return lo ^ hi;
}

// One column of an encryption round:
// Te0[a.b0] ^ Te1[b.b1] ^ Te2[c.b2] ^ Te3[d.b3] ^ k.
__device__ __forceinline__ uint32_t round_col(const uint32_t *lds, uint32_t a, uint32_t b,
                                              uint32_t c, uint32_t d, uint32_t k, uint32_t L0) {
    return xor3(xor3(tlook<0, 0>(lds, a, L0), tlook<1, 1>(lds, b, L0), tlook<2, 2>(lds, c, L0)),
                tlook<3, 3>(lds, d, L0), k);
}

// SubBytes of a.b0, b.b1, c.b2, d.b3 gathered into one word (a column of
// the last round before AddRoundKey): Te_((r+3) mod 4) holds S(x) at byte r.
__device__ __forceinline__ uint32_t sub_col(const uint32_t *lds, uint32_t a, uint32_t b,
                                            uint32_t c, uint32_t d, uint32_t L0) {
    return pick_diag(tlook<0, 3>(lds, a, L0), tlook<1, 0>(lds, b, L0), tlook<2, 1>(lds, c, L0),
                     tlook<3, 2>(lds, d, L0));
}

// One full encryption round (SubBytes, ShiftRows, MixColumns, AddRoundKey):
// column c takes row r from column c + r.
__device__ __forceinline__ void enc_round(const uint32_t *lds, uint32_t s[4],
                                          const uint32_t *__restrict__ rk, uint32_t L0) {
    const uint32_t t0 = round_col(lds, s[0], s[1], s[2], s[3], rk[0], L0);
    const uint32_t t1 = round_col(lds, s[1], s[2], s[3], s[0], rk[1], L0);
    const uint32_t t2 = round_col(lds, s[2], s[3], s[0], s[1], rk[2], L0);
    const uint32_t t3 = round_col(lds, s[3], s[0], s[1], s[2], rk[3], L0);
    s[0] = t0;
    s[1] = t1;
    s[2] = t2;
    s[3] = t3;
}

// Last encryption round (no MixColumns):
// o_c = SubBytes/ShiftRows(s)_c ^ rk_c ^ x_c.
__device__ __forceinline__ void enc_last(const uint32_t *lds, const uint32_t s[4],
                                         const uint32_t *__restrict__ rk, uint32_t L0,
                                         const uint32_t x[4], uint32_t o[4]) {
#pragma unroll
    for (int c = 0; c < 4; c++)
        o[c] = xor3(sub_col(lds, s[c], s[(c + 1) & 3], s[(c + 2) & 3], s[(c + 3) & 3], L0),
                    rk[c], x[c]);
}

// One round of the equivalent inverse cipher (InvSubBytes, InvShiftRows,
// InvMixColumns, AddRoundKey with the transformed key): row r of column c
// comes from column c - r.
__device__ __forceinline__ void dec_round(const uint32_t *lds, uint32_t s[4],
                                          const uint32_t *__restrict__ dk, uint32_t L0) {
    const uint32_t t0 = xor3(xor3(tlook<0, 0>(lds, s[0], L0), tlook<1, 1>(lds, s[3], L0),
                                  tlook<2, 2>(lds, s[2], L0)),
                             tlook<3, 3>(lds, s[1], L0), dk[0]);
    const uint32_t t1 = xor3(xor3(tlook<0, 0>(lds, s[1], L0), tlook<1, 1>(lds, s[0], L0),
                                  tlook<2, 2>(lds, s[3], L0)),
                             tlook<3, 3>(lds, s[2], L0), dk[1]);
    const uint32_t t2 = xor3(xor3(tlook<0, 0>(lds, s[2], L0), tlook<1, 1>(lds, s[1], L0),
                                  tlook<2, 2>(lds, s[0], L0)),
                             tlook<3, 3>(lds, s[3], L0), dk[2]);
    const uint32_t t3 = xor3(xor3(tlook<0, 0>(lds, s[3], L0), tlook<1, 1>(lds, s[2], L0),
                                  tlook<2, 2>(lds, s[1], L0)),
                             tlook<3, 3>(lds, s[0], L0), dk[3]);
    s[0] = t0;
    s[1] = t1;
    s[2] = t2;
    s[3] = t3;
}

// Last inverse round: o_c byte r = InvS(s_(c-r).b_r) ^ dk ^ x.
__device__ __forceinline__ void dec_last(const uint32_t *lds, const uint32_t s[4],
                                         const uint32_t *__restrict__ dk, uint32_t L2,
                                         const uint32_t x[4], uint32_t o[4]) {
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const uint32_t a = silook<0>(lds, s[c], L2);
        const uint32_t b = silook<1>(lds, s[(c + 3) & 3], L2);
        const uint32_t d2 = silook<2>(lds, s[(c + 2) & 3], L2);
        const uint32_t d3 = silook<3>(lds, s[(c + 1) & 3], L2);
        o[c] = xor3(pick_diag(a, b, d2, d3), dk[c], x[c]);
    }
}

// ------------------------------------------------------------ block I/O

// A 16-byte vector for the nontemporal builtins (which take no HIP vector
// types).
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// Loads block b of a unit of nbytes bytes; bytes past the end read as zero.
// NT: whole blocks are read with the nontemporal hint (streamed, not kept in
// the caches).
template <bool NT = false>
__device__ __forceinline__ void load_block(const uint8_t *src, uint32_t b, uint32_t nbytes,
                                           uint32_t x[4]) {
    const uint32_t start = b << 4;
    if (start + 16u <= nbytes) {
        if (NT) {
            const u32x4_t v =
                __builtin_nontemporal_load(reinterpret_cast<const u32x4_t *>(src + start));
            x[0] = v.x;
            x[1] = v.y;
            x[2] = v.z;
            x[3] = v.w;
        } else {
            const uint4 v = *reinterpret_cast<const uint4 *>(src + start);
            x[0] = v.x;
            x[1] = v.y;
            x[2] = v.z;
            x[3] = v.w;
        }
    } else {
        x[0] = x[1] = x[2] = x[3] = 0u;
        if (start < nbytes) {
            for (uint32_t k = 0; k < nbytes - start; k++)
                x[k >> 2] |= (uint32_t)src[start + k] << (8 * (k & 3));
        }
    }
}

template <bool NT = false>
__device__ __forceinline__ void store_block(uint8_t *dst, uint32_t b, uint32_t nbytes,
                                            const uint32_t o[4]) {
    const uint32_t start = b << 4;
    if (start + 16u <= nbytes) {
        if (NT) {
            const u32x4_t v = {o[0], o[1], o[2], o[3]};
            __builtin_nontemporal_store(v, reinterpret_cast<u32x4_t *>(dst + start));
        } else {
            *reinterpret_cast<uint4 *>(dst + start) = make_uint4(o[0], o[1], o[2], o[3]);
        }
    } else if (start < nbytes) {
        for (uint32_t k = 0; k < nbytes - start; k++)
            dst[start + k] = (uint8_t)(o[k >> 2] >> (8 * (k & 3)));
    }
}

// ------------------------------------------------------------ round keys

// A wave-uniform word copied into a vector register with one v_mov_b32.
// Written as inline assembly, the result is opaque to the compiler, which
// therefore keeps it in that VGPR instead of folding it back into the scalar
// register it came from.  (An identity-pattern DPP move does the same in the
// compiler's terms but costs three VALU ops: the scalar-to-vector move, the
// tied "old" operand and the DPP move.)
__device__ __forceinline__ uint32_t to_vgpr(uint32_t k) {
    uint32_t v;
    asm("v_mov_b32 %0, %1" : "=v"(v) : "s"(k));
    return v;
}

// Round keys of one schedule for the tile loops.  Keys of rounds
// FIRST..FIRST+NV-1 are copied into vector registers once per unit
// (to_vgpr); the others are read from the schedule into scalar registers.  With every
// round key scalar, keys plus the loop state exceed the scalar registers a
// wave has, and the compiler spills them to VGPR lanes and reads them back
// with v_readlane inside the rounds.
template <int NR, int NV, int FIRST = 1>
struct RoundKeys {
    static constexpr int V = NV < NR - FIRST ? NV : NR - FIRST;
    const uint32_t *rk;
    uint32_t v[V > 0 ? 4 * V : 1];
    __device__ __forceinline__ explicit RoundKeys(const uint32_t *__restrict__ k) : rk(k) {
#pragma unroll
        for (int i = 0; i < 4 * V; i++)
            v[i] = to_vgpr(k[4 * FIRST + i]);
    }
    // Round r's four words (r a compile-time constant after unrolling).
    __device__ __forceinline__ const uint32_t *operator[](int r) const {
        return r >= FIRST && r < FIRST + V ? v + 4 * (r - FIRST) : rk + 4 * r;
    }
};

// Rounds whose keys the 1024-thread tile and per-request kernels hold in
// vector registers, per side: the fewest that leave no scalar-register spills
// with two blocks per lane (113 VGPRs for plain CTR, 103 for decryption, of
// the 128 such workgroups allow).  Measured about 1% faster on every key size
// and side than all-scalar keys with their spills.  CTR tiles with shared
// heads hold rounds 3..7 (rounds 1 and 2 come from the heads); they spill
// some loop state to VGPR lanes, read back once per step, and 5 measured
// ahead of 3 and 4.  AES-256 CTR tiles with shared heads hold rounds 3..10
// (TILE_NV_CTR256): the scalar registers this frees keep a counter group's
// heads live across its steps.
constexpr int TILE_NV_CTR = 5;
constexpr int TILE_NV_CTR256 = 8;
constexpr int TILE_NV_DEC = 8;

// -------------------------------------------------------------- CTR tiles

// SP 800-38A 6.5: block b of the unit uses counter block nonce || BE64(ctr0 + b).
template <int NB, int NR, int NV = 0>
__device__ __forceinline__ void ctr_unit(const uint32_t *lds, uint32_t L0,
                                         uint32_t lane, const Unit &un,
                                         const uint32_t *__restrict__ rk, const uint8_t *in,
                                         uint8_t *out) {
    const RoundKeys<NR, NV> K(rk);
    const uint32_t nbytes = un.nbytes;
    const uint32_t nblk = (nbytes + 15u) >> 4;
    const uint64_t ctr0 = ((uint64_t)un.w[3] << 32) | un.w[2];
    const uint32_t n0 = un.w[0] ^ rk[0];
    const uint32_t n1 = un.w[1] ^ rk[1];
    const uint8_t *src = in + un.off;
    uint8_t *dst = out + un.off;
    for (uint32_t base = 0; base < nblk; base += 64u * NB) {
        uint32_t s[NB][4], x[NB][4];
#pragma unroll
        for (int i = 0; i < NB; i++) {
            const uint32_t b = base + 64u * i + lane;
            const uint64_t c = ctr0 + b;
            s[i][0] = n0;
            s[i][1] = n1;
            s[i][2] = __builtin_bswap32((uint32_t)(c >> 32)) ^ rk[2];
            s[i][3] = __builtin_bswap32((uint32_t)c) ^ rk[3];
            load_block(src, b, nbytes, x[i]);
        }
#pragma unroll
        for (int r = 1; r < NR; r++) {
#pragma unroll
            for (int i = 0; i < NB; i++)
                enc_round(lds, s[i], K[r], L0);
        }
#pragma unroll
        for (int i = 0; i < NB; i++) {
            uint32_t o[4];
            enc_last(lds, s[i], K[NR], L0, x[i], o);
            store_block(dst, base + 64u * i + lane, nbytes, o);
        }
    }
}

// ------------------------------------------- CTR tiles, shared first rounds
//
// Counter blocks differ only in byte 15 until a carry.  With the initial
// state words s0..s3 (counter byte 15 is byte 3 of s3), round 1 gives
//   t0 = U0 ^ Te3[s3.b3],  t1, t2, t3 independent of byte 15,
// and round 2 takes one byte of t0 per output column:
//   u0 = P0 ^ Te0[t0.b0], u1 = P1 ^ Te3[t0.b3], u2 = P2 ^ Te2[t0.b2],
//   u3 = P3 ^ Te1[t0.b1],
// where U0 and P0..P3 depend only on counter bytes 0..14 (and the key).  A
// group of 256 consecutive counters sees at most two values of those bytes
// (one carry out of byte 15).  Once per group the wave computes U0, P0..P3
// for both (heads A and B) with scalar loads from the table image in device
// memory, off the LDS pipe, and each lane takes the head of its block:
// rounds 1 and 2 cost 5 LDS lookups per block instead of 32.  (Caching the
// counter's constant part across the first rounds is Bernstein and
// Schwabe's idea, "New AES software speed records", INDOCRYPT 2008.)

// U0, P0..P3 for the counter blocks whose bits 8..63 equal h.  n0, n1: nonce
// words already XORed with round key 0; te: Te0..Te3 in device memory.
__device__ __forceinline__ void ctr_head(const uint32_t *__restrict__ te, uint32_t n0, uint32_t n1,
                                         uint64_t h, const uint32_t *__restrict__ rk,
                                         uint32_t out[5]) {
    const uint64_t c = h << 8;
    const uint32_t s0 = n0, s1 = n1;
    const uint32_t s2 = __builtin_bswap32((uint32_t)(c >> 32)) ^ rk[2];
    const uint32_t s3 = __builtin_bswap32((uint32_t)c) ^ rk[3];  // byte 3 is not used
    auto T = [te](int t, uint32_t w, int k) { return te[t * 256 + ((w >> (8 * k)) & 255u)]; };
    const uint32_t *k1 = rk + 4, *k2 = rk + 8;
    const uint32_t t1 = T(0, s1, 0) ^ T(1, s2, 1) ^ T(2, s3, 2) ^ T(3, s0, 3) ^ k1[1];
    const uint32_t t2 = T(0, s2, 0) ^ T(1, s3, 1) ^ T(2, s0, 2) ^ T(3, s1, 3) ^ k1[2];
    const uint32_t t3 = T(0, s3, 0) ^ T(1, s0, 1) ^ T(2, s1, 2) ^ T(3, s2, 3) ^ k1[3];
    out[0] = T(0, s0, 0) ^ T(1, s1, 1) ^ T(2, s2, 2) ^ k1[0];
    out[1] = T(1, t1, 1) ^ T(2, t2, 2) ^ T(3, t3, 3) ^ k2[0];
    out[2] = T(0, t1, 0) ^ T(1, t2, 1) ^ T(2, t3, 2) ^ k2[1];
    out[3] = T(0, t2, 0) ^ T(1, t3, 1) ^ T(3, t1, 3) ^ k2[2];
    out[4] = T(0, t3, 0) ^ T(2, t1, 2) ^ T(3, t2, 3) ^ k2[3];
}

// Both heads of the counters ctr0 + g .. ctr0 + g + n - 1 (n <= 256): A for
// those before the carry out of byte 15, D = A ^ B (zero without a carry).
__device__ __forceinline__ void ctr_heads(const uint32_t *__restrict__ te, uint32_t n0, uint32_t n1,
                                          uint64_t cf, uint32_t n,
                                          const uint32_t *__restrict__ rk, uint32_t A[5],
                                          uint32_t D[5]) {
    ctr_head(te, n0, n1, cf >> 8, rk, A);
    // Keep the two heads' scalar loads apart (scalar registers are short).
    __builtin_amdgcn_sched_barrier(0);
    if (((uint32_t)cf & 255u) + n - 1u >= 256u) {
        // Bits 8..63 one higher (mod 2^56, as the 64-bit counter wraps).
        uint32_t B[5];
        ctr_head(te, n0, n1, (cf >> 8) + 1u, rk, B);
#pragma unroll
        for (int j = 0; j < 5; j++)
            D[j] = A[j] ^ B[j];
    } else {
#pragma unroll
        for (int j = 0; j < 5; j++)
            D[j] = 0u;
    }
    __builtin_amdgcn_sched_barrier(0);
}

// One step of ctr_unit_head: blocks base + 64 i + lane; lo0 = the low byte of
// the heads' first counter plus base minus that counter's block.
template <int NB, int NR, int NV>
__device__ __forceinline__ void ctr_head_step(const uint32_t *lds, uint32_t L0, uint32_t lane,
                                              const RoundKeys<NR, NV, 3> &K,
                                              const uint32_t A[5], const uint32_t D[5],
                                              uint32_t lo0, uint32_t rk3, uint32_t base,
                                              uint32_t nbytes, const uint8_t *src, uint8_t *dst) {
    uint32_t s[NB][4], x[NB][4];
#pragma unroll
    for (int i = 0; i < NB; i++) {
        const uint32_t lo = lo0 + 64u * i + lane;  // < 512
        const uint32_t m = lo >= 256u ? ~0u : 0u;  // this block takes head B
        const uint32_t t0 = (A[0] ^ (D[0] & m)) ^ tlook<3, 3>(lds, (lo << 24) ^ rk3, L0);
        s[i][0] = (A[1] ^ (D[1] & m)) ^ tlook<0, 0>(lds, t0, L0);
        s[i][1] = (A[2] ^ (D[2] & m)) ^ tlook<3, 3>(lds, t0, L0);
        s[i][2] = (A[3] ^ (D[3] & m)) ^ tlook<2, 2>(lds, t0, L0);
        s[i][3] = (A[4] ^ (D[4] & m)) ^ tlook<1, 1>(lds, t0, L0);
        load_block(src, base + 64u * i + lane, nbytes, x[i]);
    }
#pragma unroll
    for (int r = 3; r < NR; r++) {
#pragma unroll
        for (int i = 0; i < NB; i++)
            enc_round(lds, s[i], K[r], L0);
    }
#pragma unroll
    for (int i = 0; i < NB; i++) {
        uint32_t o[4];
        enc_last(lds, s[i], K[NR], L0, x[i], o);
        store_block(dst, base + 64u * i + lane, nbytes, o);
    }
}

// ctr_unit with rounds 1 and 2 from the shared heads (same output), computed
// once per group of 256 counters (a 4 KiB unit: once).  For AES-256 this
// needs its round keys 3..10 in vector registers (TILE_NV_CTR256): with keys
// 8..14 in scalar registers the heads live across steps pushed them to VGPR
// lanes and the form ran 10% slower than computing the heads once per step,
// which it now beats by 1.2-1.6%.
template <int NB, int NR, int NV = 0>
__device__ __forceinline__ void ctr_unit_head(const uint32_t *lds, uint32_t L0, uint32_t lane,
                                              const Unit &un, const uint32_t *__restrict__ rk,
                                              const uint32_t *__restrict__ te, const uint8_t *in,
                                              uint8_t *out) {
    static_assert(256 % (64 * NB) == 0, "steps tile a group of 256 counters");
    const RoundKeys<NR, NV, 3> K(rk);
    const uint32_t nbytes = un.nbytes;
    const uint32_t nblk = (nbytes + 15u) >> 4;
    const uint64_t ctr0 = ((uint64_t)un.w[3] << 32) | un.w[2];
    const uint32_t n0 = un.w[0] ^ rk[0];
    const uint32_t n1 = un.w[1] ^ rk[1];
    const uint8_t *src = in + un.off;
    uint8_t *dst = out + un.off;
    uint32_t A[5], D[5];
    for (uint32_t g = 0; g < nblk; g += 256u) {
        const uint64_t cf = ctr0 + g;  // the group's first counter (wave-uniform)
        const uint32_t gend = nblk - g < 256u ? nblk : g + 256u;
        ctr_heads(te, n0, n1, cf, gend - g, rk, A, D);
        for (uint32_t base = g; base < gend; base += 64u * NB)
            ctr_head_step<NB, NR, NV>(lds, L0, lane, K, A, D,
                                      ((uint32_t)cf & 255u) + (base - g), rk[3], base, nbytes,
                                      src, dst);
    }
}

// SP 800-38A 6.1: ECB encryption, every block on its own (whole blocks).
template <int NB, int NR, int NV = 0>
__device__ __forceinline__ void ecb_enc_unit(const uint32_t *lds, uint32_t L0, uint32_t lane,
                                             const Unit &un, const uint32_t *__restrict__ rk,
                                             const uint8_t *in, uint8_t *out) {
    const RoundKeys<NR, NV> K(rk);
    const uint32_t nbytes = un.nbytes;
    const uint32_t nblk = nbytes >> 4;
    const uint8_t *src = in + un.off;
    uint8_t *dst = out + un.off;
    const uint32_t zero[4] = {0u, 0u, 0u, 0u};
    for (uint32_t base = 0; base < nblk; base += 64u * NB) {
        uint32_t s[NB][4];
#pragma unroll
        for (int i = 0; i < NB; i++) {
            load_block(src, base + 64u * i + lane, nbytes, s[i]);
#pragma unroll
            for (int w = 0; w < 4; w++)
                s[i][w] ^= rk[w];
        }
#pragma unroll
        for (int r = 1; r < NR; r++) {
#pragma unroll
            for (int i = 0; i < NB; i++)
                enc_round(lds, s[i], K[r], L0);
        }
#pragma unroll
        for (int i = 0; i < NB; i++) {
            uint32_t o[4];
            enc_last(lds, s[i], K[NR], L0, zero, o);
            store_block(dst, base + 64u * i + lane, nbytes, o);
        }
    }
}

// Key checks and round-count dispatch for one encryption-table tile (CTR
// or ECB encryption; wave-uniform).
// With te (Te0..Te3 in device memory) CTR units take the shared-head path.
template <int NB, int NV = 0>
__device__ __forceinline__ void run_ctr_unit(const uint32_t *lds, uint32_t L0,
                                             uint32_t lane, const Unit &un,
                                             const aes_schedule_t *__restrict__ sched,
                                             uint32_t n_sched, const uint8_t *in, uint8_t *out,
                                             const uint32_t *__restrict__ te = nullptr) {
    const uint32_t key = un.meta & META_KEY_MASK;
    if (key >= n_sched)
        return;
    const aes_schedule_t *ks = sched + key;
    const uint32_t nr = ks->nr;
    if (unit_op(un.meta) == AES_OP_ECB_ENC) {
        if (nr == 10)
            ecb_enc_unit<NB, 10, NV>(lds, L0, lane, un, ks->ek, in, out);
        else if (nr == 12)
            ecb_enc_unit<NB, 12, NV>(lds, L0, lane, un, ks->ek, in, out);
        else if (nr == 14)
            ecb_enc_unit<NB, 14, NV>(lds, L0, lane, un, ks->ek, in, out);
        return;
    }
    if (te) {
        if (nr == 10)
            ctr_unit_head<NB, 10, NV>(lds, L0, lane, un, ks->ek, te, in, out);
        else if (nr == 12)
            ctr_unit_head<NB, 12, NV>(lds, L0, lane, un, ks->ek, te, in, out);
        else if (nr == 14)
            ctr_unit_head<NB, 14, (NV > 0 ? TILE_NV_CTR256 : 0)>(lds, L0, lane, un, ks->ek, te,
                                                                  in, out);
        return;
    }
    if (nr == 10)
        ctr_unit<NB, 10, NV>(lds, L0, lane, un, ks->ek, in, out);
    else if (nr == 12)
        ctr_unit<NB, 12, NV>(lds, L0, lane, un, ks->ek, in, out);
    else if (nr == 14)
        ctr_unit<NB, 14, NV>(lds, L0, lane, un, ks->ek, in, out);
}

// ------------------------------------------------------- CBC-decrypt tiles

// DPP wave_shr:1 -- lane l receives lane l-1; lane 0 keeps `old`.
__device__ __forceinline__ uint32_t shift_up(uint32_t old, uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, 0x138, 0xF, 0xF, false);
}

// SP 800-38A 6.2: P_j = D(C_j) ^ C_(j-1).  Lane l of step i decrypts block
// 64i + l; its predecessor is lane l-1's ciphertext, and lane 0 takes lane 63
// of the previous step (or the block before the unit).  ECB (6.1): P_j =
// D(C_j), no chaining.  NT: payload loads and stores with the nontemporal
// hint.
template <int NB, int NR, bool ECB = false, int NV = 0, bool NT = false>
__device__ __forceinline__ void cbcdec_unit(const uint32_t *lds, uint32_t L0,
                                            uint32_t L2, uint32_t lane, const Unit &un,
                                            const uint4 *snap, const uint32_t *__restrict__ dk,
                                            const uint8_t *in, uint8_t *out) {
    const RoundKeys<NR, NV> K(dk);
    const uint32_t nbytes = un.nbytes;
    const uint32_t nblk = nbytes >> 4;
    const uint8_t *src = in + un.off;
    uint8_t *dst = out + un.off;
    uint32_t carry[4];
    if (ECB) {
        carry[0] = carry[1] = carry[2] = carry[3] = 0u;
    } else if (un.meta & FLAG_PRED_IN) {
        const uint4 p = snap ? *snap : *reinterpret_cast<const uint4 *>(src - 16);
        carry[0] = p.x;
        carry[1] = p.y;
        carry[2] = p.z;
        carry[3] = p.w;
    } else {
        // As values (readfirstlane), not memory: otherwise the compiler merges
        // this branch and the load above into one load through a selected
        // pointer, which puts the unit record on the stack.
        carry[0] = __builtin_amdgcn_readfirstlane(un.w[0]);
        carry[1] = __builtin_amdgcn_readfirstlane(un.w[1]);
        carry[2] = __builtin_amdgcn_readfirstlane(un.w[2]);
        carry[3] = __builtin_amdgcn_readfirstlane(un.w[3]);
    }
    for (uint32_t base = 0; base < nblk; base += 64u * NB) {
        uint32_t c[NB][4], s[NB][4], pred[NB][4];
#pragma unroll
        for (int i = 0; i < NB; i++)
            load_block<NT>(src, base + 64u * i + lane, nbytes, c[i]);
#pragma unroll
        for (int i = 0; i < NB; i++) {
#pragma unroll
            for (int w = 0; w < 4; w++) {
                if (ECB) {
                    pred[i][w] = 0u;
                } else {
                    const uint32_t prev_last =
                        i == 0 ? carry[w]
                               : (uint32_t)__builtin_amdgcn_readlane((int)c[i - 1][w], 63);
                    pred[i][w] = shift_up(prev_last, c[i][w]);
                }
                s[i][w] = c[i][w] ^ dk[w];
            }
        }
        if (!ECB) {
#pragma unroll
            for (int w = 0; w < 4; w++)
                carry[w] = (uint32_t)__builtin_amdgcn_readlane((int)c[NB - 1][w], 63);
        }
#pragma unroll
        for (int r = 1; r < NR; r++) {
#pragma unroll
            for (int i = 0; i < NB; i++)
                dec_round(lds, s[i], K[r], L0);
        }
#pragma unroll
        for (int i = 0; i < NB; i++) {
            uint32_t o[4];
            dec_last(lds, s[i], K[NR], L2, pred[i], o);
            store_block<NT>(dst, base + 64u * i + lane, nbytes, o);
        }
    }
}

template <int NB, int NV = 0, bool NT = false>
__device__ __forceinline__ void run_dec_unit(const uint32_t *lds, uint32_t L0,
                                             uint32_t L2, uint32_t lane, const Unit &un,
                                             const uint4 *snap,
                                             const aes_schedule_t *__restrict__ sched,
                                             uint32_t n_sched, const uint8_t *in, uint8_t *out) {
    const uint32_t key = un.meta & META_KEY_MASK;
    if (key >= n_sched)
        return;
    const aes_schedule_t *ks = sched + key;
    const uint32_t nr = ks->nr;
    if (unit_op(un.meta) == AES_OP_ECB_DEC) {
        if (nr == 10)
            cbcdec_unit<NB, 10, true, NV, NT>(lds, L0, L2, lane, un, snap, ks->dk, in, out);
        else if (nr == 12)
            cbcdec_unit<NB, 12, true, NV, NT>(lds, L0, L2, lane, un, snap, ks->dk, in, out);
        else if (nr == 14)
            cbcdec_unit<NB, 14, true, NV, NT>(lds, L0, L2, lane, un, snap, ks->dk, in, out);
        return;
    }
    if (nr == 10)
        cbcdec_unit<NB, 10, false, NV, NT>(lds, L0, L2, lane, un, snap, ks->dk, in, out);
    else if (nr == 12)
        cbcdec_unit<NB, 12, false, NV, NT>(lds, L0, L2, lane, un, snap, ks->dk, in, out);
    else if (nr == 14)
        cbcdec_unit<NB, 14, false, NV, NT>(lds, L0, L2, lane, un, snap, ks->dk, in, out);
}

}  // namespace aesgpu
