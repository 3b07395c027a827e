// aes_bitslice.hip -- bitsliced AES for CTR mode and CBC / ECB decryption on
// CDNA4 (gfx950).
//
// The comparison variant of the round-table kernels: no LDS and no lookups
// (the cipher is in bitslice_aes.h).  A wave works 8 units at once: lane l
// takes unit l / 8 and its blocks 8 j + l % 8 (j = 0..31) of each 4 KiB
// chunk, so each 16-byte load or store instruction touches 128 contiguous
// bytes per unit.  Units of one wave should share a key (the planner sorts
// the units of a bitsliced launch by key); a wave makes one pass per
// distinct key.
#include <hip/hip_runtime.h>

#include "bitslice_aes.h"
#include "internal.h"

namespace aesgpu {

// One pass over a group of up to 8 CTR chunks of 4 KiB with the key `rk`;
// lanes whose chunk uses that key store their blocks.  Lane l covers blocks
// 8 j + l % 8 (j = 0..31) of the chunk of its lane group (l / 8).  w0..w3 are
// the chunk's first counter block as little-endian words (w2, w3: the 64-bit
// counter, low word first).
__device__ __forceinline__ void bs_ctr_pass(uint64_t off, uint32_t nbytes, uint32_t w0,
                                            uint32_t w1, uint32_t w2, uint32_t w3, uint32_t sub,
                                            bool store, const uint32_t *__restrict__ rk,
                                            uint32_t nr, const uint8_t *in, uint8_t *out) {
    uint32_t P[4][32];
    // The block words are rebuilt in every pass: an empty asm makes them
    // opaque, so they are not kept live through the cipher of another pass.
    asm volatile("" : "+v"(w0), "+v"(w1), "+v"(w2), "+v"(w3));
    bs_ctr_keystream(P, w0, w1, ((uint64_t)w3 << 32) | w2, sub, rk, nr);
    if (!store)
        return;
    const uint8_t *src = in + off;
    uint8_t *dst = out + off;
    // Whole blocks are stored in the loop; the ragged final block (at most one
    // per tile) keeps its keystream words for the byte loop after it.
    const uint32_t tail_start = nbytes & ~15u;
    uint32_t r0 = 0, r1 = 0, r2 = 0, r3 = 0;
#pragma unroll
    for (int j = 0; j < 32; j++) {
        const uint32_t start = (8u * j + sub) << 4;
        if (start + 16u <= nbytes) {
            const uint4 v = *reinterpret_cast<const uint4 *>(src + start);
            *reinterpret_cast<uint4 *>(dst + start) =
                make_uint4(v.x ^ P[0][j], v.y ^ P[1][j], v.z ^ P[2][j], v.w ^ P[3][j]);
        }
        const bool ragged = start == tail_start;
        r0 = ragged ? P[0][j] : r0;
        r1 = ragged ? P[1][j] : r1;
        r2 = ragged ? P[2][j] : r2;
        r3 = ragged ? P[3][j] : r3;
    }
    if ((nbytes & 15u) && ((tail_start >> 4) & 7u) == sub) {
        for (uint32_t k = 0; k < (nbytes & 15u); k++) {
            const uint32_t w = k < 4 ? r0 : (k < 8 ? r1 : (k < 12 ? r2 : r3));
            dst[tail_start + k] = src[tail_start + k] ^ (uint8_t)(w >> (8 * (k & 3)));
        }
    }
}

// CTR units in groups of 8 per wave (grid-stride over groups); each unit is
// worked in 4 KiB chunks, one chunk per lane group per step.
__global__ __launch_bounds__(256, 2) void k_ctr_bitslice(const Unit *__restrict__ units,
                                                         uint32_t n_units,
                                                         const aes_schedule_t *__restrict__ sched,
                                                         uint32_t n_sched, const uint8_t *in,
                                                         uint8_t *out) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t g = lane >> 3, sub = lane & 7u;
    const uint32_t wpb = blockDim.x >> 6;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x >> 6));
    const uint32_t nw = __builtin_amdgcn_readfirstlane(gridDim.x * wpb);
    const uint32_t n_groups = (n_units + 7u) / 8u;
    for (uint32_t grp = wave; grp < n_groups; grp += nw) {
        const uint32_t u = grp * 8u + g;
        uint64_t off = 0;
        uint32_t nbytes = 0, key = 0xFFFFFFFFu, w0 = 0, w1 = 0, w2 = 0, w3 = 0;
        if (u < n_units) {
            const Unit un = units[u];
            off = un.off;
            nbytes = un.nbytes;
            // CTR units only (the planner places them first): anything else
            // gets an out-of-range key and is skipped
            key = unit_op(un.meta) == AES_OP_CTR ? un.meta & META_KEY_MASK : 0xFFFFFFFFu;
            w0 = un.w[0];
            w1 = un.w[1];
            w2 = un.w[2];
            w3 = un.w[3];
        }
        const bool keyed = key < n_sched;
        for (uint32_t ci = 0;; ci++) {
            const uint32_t pos = ci << 12;
            const bool has = keyed && pos < nbytes;
            uint64_t pending = __ballot(has);
            if (!pending)
                break;
            const uint64_t c = (((uint64_t)w3 << 32) | w2) + (pos >> 4);
            const uint32_t len = has ? min(nbytes - pos, 4096u) : 0u;
            while (pending) {
                const uint32_t k =
                    __builtin_amdgcn_readlane(key, (uint32_t)__builtin_ctzll(pending));
                const bool mine = has && key == k;
                const aes_schedule_t *ks = sched + k;
                const uint32_t nr = ks->nr;
                if (nr == 10 || nr == 12 || nr == 14)
                    bs_ctr_pass(off + pos, len, w0, w1, (uint32_t)c, (uint32_t)(c >> 32), sub,
                                mine, ks->ek, nr, in, out);
                pending &= ~__ballot(mine);
            }
        }
    }
}

// One pass of CBC (SP 800-38A 6.2: P_j = D(C_j) ^ C_(j-1)) or ECB decryption
// over a chunk of up to 4 KiB of one lane group's unit with the key `rk` (the
// encryption schedule; the inverse cipher runs it backwards).  carry is the
// ciphertext block before the chunk; lanes whose unit uses that key store.
// The stores run from the chunk's last block to its first, and every lane
// loads its predecessor block before the store that may overwrite it: the
// predecessor of block 8 j + s is stored by lane s - 1 in the same step, or
// (s = 0) by lane 7 in the step after, so decryption in place reads
// ciphertext only.
__device__ __forceinline__ void bs_dec_pass(uint64_t off, uint32_t nbytes, uint32_t sub,
                                            bool store, bool ecb, const uint32_t carry[4],
                                            const uint32_t *__restrict__ rk, uint32_t nr,
                                            const uint8_t *in, uint8_t *out) {
    uint32_t P[4][32];
    const uint8_t *src = in + off;
#pragma unroll
    for (int j = 0; j < 32; j++) {
        const uint32_t start = (8u * j + sub) << 4;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        if (start < nbytes)
            v = *reinterpret_cast<const uint4 *>(src + start);
        P[0][j] = v.x;
        P[1][j] = v.y;
        P[2][j] = v.z;
        P[3][j] = v.w;
    }
#pragma unroll
    for (int w = 0; w < 4; w++)
        transpose32(P[w]);
    bs_inv_cipher(P, rk, nr);
#pragma unroll
    for (int w = 0; w < 4; w++)
        transpose32(P[w]);
    if (!store)
        return;
    uint8_t *dst = out + off;
#pragma unroll
    for (int j = 31; j >= 0; j--) {
        const uint32_t start = (8u * j + sub) << 4;
        if (start < nbytes) {
            uint4 pr = make_uint4(0u, 0u, 0u, 0u);
            if (!ecb) {
                if (start == 0u)
                    pr = make_uint4(carry[0], carry[1], carry[2], carry[3]);
                else
                    pr = *reinterpret_cast<const uint4 *>(src + start - 16u);
            }
            *reinterpret_cast<uint4 *>(dst + start) =
                make_uint4(P[0][j] ^ pr.x, P[1][j] ^ pr.y, P[2][j] ^ pr.z, P[3][j] ^ pr.w);
        }
    }
}

// CBC- and ECB-decrypt units in groups of 8 per wave (grid-stride over
// groups), each worked in 4 KiB chunks, one chunk per lane group per step.
// The ciphertext block before a unit: the unit's IV words, the in-place
// snapshot (preds, one per unit) or in[off - 16]; before a later chunk: the
// chunk's predecessor, read before the chunk before it is stored.
__global__ __launch_bounds__(256, 2) void k_dec_bitslice(const Unit *__restrict__ units,
                                                         uint32_t n_units,
                                                         const aes_schedule_t *__restrict__ sched,
                                                         uint32_t n_sched,
                                                         const uint4 *__restrict__ preds,
                                                         const uint8_t *in, uint8_t *out) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t g = lane >> 3, sub = lane & 7u;
    const uint32_t wpb = blockDim.x >> 6;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x >> 6));
    const uint32_t nw = __builtin_amdgcn_readfirstlane(gridDim.x * wpb);
    const uint32_t n_groups = (n_units + 7u) / 8u;
    for (uint32_t grp = wave; grp < n_groups; grp += nw) {
        const uint32_t u = grp * 8u + g;
        uint64_t off = 0;
        uint32_t nbytes = 0, key = 0xFFFFFFFFu;
        bool ecb = false;
        uint32_t carry[4] = {0u, 0u, 0u, 0u};
        if (u < n_units) {
            const Unit un = units[u];
            off = un.off;
            nbytes = un.nbytes;
            const uint32_t op = unit_op(un.meta);
            ecb = op == AES_OP_ECB_DEC;
            // decryption units only: anything else gets an out-of-range key
            key = op == AES_OP_CBC_DEC || ecb ? un.meta & META_KEY_MASK : 0xFFFFFFFFu;
            if (!ecb && (un.meta & FLAG_PRED_IN)) {
                const uint4 p = preds ? preds[u] : *reinterpret_cast<const uint4 *>(in + off - 16);
                carry[0] = p.x;
                carry[1] = p.y;
                carry[2] = p.z;
                carry[3] = p.w;
            } else if (!ecb) {
                carry[0] = un.w[0];
                carry[1] = un.w[1];
                carry[2] = un.w[2];
                carry[3] = un.w[3];
            }
        }
        const bool keyed = key < n_sched;
        for (uint32_t ci = 0;; ci++) {
            const uint32_t pos = ci << 12;
            const bool has = keyed && pos < nbytes;
            uint64_t pending = __ballot(has);
            if (!pending)
                break;
            const uint32_t len = has ? min(nbytes - pos, 4096u) : 0u;
            // The next chunk's predecessor, read before this chunk is stored.
            uint4 nxt = make_uint4(0u, 0u, 0u, 0u);
            if (has && !ecb && pos + 4096u < nbytes)
                nxt = *reinterpret_cast<const uint4 *>(in + off + pos + 4096u - 16u);
            while (pending) {
                const uint32_t k =
                    __builtin_amdgcn_readlane(key, (uint32_t)__builtin_ctzll(pending));
                const bool mine = has && key == k;
                const aes_schedule_t *ks = sched + k;
                const uint32_t nr = ks->nr;
                if (nr == 10 || nr == 12 || nr == 14)
                    bs_dec_pass(off + pos, len, sub, mine, ecb, carry, ks->ek, nr, in, out);
                pending &= ~__ballot(mine);
            }
            carry[0] = nxt.x;
            carry[1] = nxt.y;
            carry[2] = nxt.z;
            carry[3] = nxt.w;
        }
    }
}

int launch_dec_bitslice(const Unit *d_units, uint32_t n_units, const aes_schedule_t *d_sched,
                        uint32_t n_sched, const void *d_preds, const uint8_t *d_in,
                        uint8_t *d_out, void *stream) {
    if (!n_units)
        return hipSuccess;
    const uint32_t groups = (n_units + 7u) / 8u;
    uint32_t grid = (groups + 3u) / 4u;
    if (grid > 65535u)
        grid = 65535u;
    hipLaunchKernelGGL(k_dec_bitslice, dim3(grid), dim3(256), 0, (hipStream_t)stream, d_units,
                       n_units, d_sched, n_sched, (const uint4 *)d_preds, d_in, d_out);
    return hipGetLastError();
}

int launch_ctr_bitslice(const Unit *d_units, uint32_t n_units, const aes_schedule_t *d_sched,
                        uint32_t n_sched, const uint8_t *d_in, uint8_t *d_out, int n_cu,
                        void *stream) {
    if (!n_units)
        return hipSuccess;
    (void)n_cu;
    const uint32_t groups = (n_units + 7u) / 8u;
    // 4 waves (groups) per workgroup; the hardware fills the compute units.
    uint32_t grid = (groups + 3u) / 4u;
    if (grid > 65535u)
        grid = 65535u;
    hipLaunchKernelGGL(k_ctr_bitslice, dim3(grid), dim3(256), 0, (hipStream_t)stream, d_units,
                       n_units, d_sched, n_sched, d_in, d_out);
    return hipGetLastError();
}

}  // namespace aesgpu
