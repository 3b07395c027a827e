// aes_chain.h -- CBC encryption (SP 800-38A 6.2) for CDNA4 (gfx950): each
// request is one serial chain, run on one lane or on four lanes (one state
// column each), with the table-variant rounds of aes_rounds.h.  Used by the
// chain and fused batch kernels, the per-request kernel and the persistent
// server.
#pragma once

#include <hip/hip_runtime.h>

#include "aes_rounds.h"
#include "internal.h"

namespace aesgpu {

// A 32-bit word in global memory (device memory, or host memory mapped into
// the device).
typedef __attribute__((address_space(1))) uint32_t gu32;

// ------------------------------------------------------- CBC-encrypt chains

// SP 800-38A 6.2: C_j = E(P_j ^ C_(j-1)); one chain per lane, strictly serial.
// Round keys differ between lanes, so they live in VGPRs.  Lanes of one wave
// may use different key sizes: rounds run up to MAXNR (the largest Nr in the
// wave) and a lane with fewer rounds sits out the extra ones, so mixed waves
// cost MAXNR rounds per block rather than the sum over key sizes.
template <int MAXNR>
__device__ __forceinline__ void chain_run(const uint32_t *lds, uint32_t L0,
                                          const Unit &un, const uint32_t *ek, uint32_t nr,
                                          const uint8_t *in, uint8_t *out) {
    uint32_t rk[4 * (MAXNR + 1)];
#pragma unroll
    for (int i = 0; i < MAXNR + 1; i++) {
        const uint4 v = reinterpret_cast<const uint4 *>(ek)[i];
        rk[4 * i + 0] = v.x;
        rk[4 * i + 1] = v.y;
        rk[4 * i + 2] = v.z;
        rk[4 * i + 3] = v.w;
    }
    uint32_t rkl[4];  // this lane's last-round key
#pragma unroll
    for (int w = 0; w < 4; w++)
        rkl[w] = nr == 10 ? rk[40 + w] : (nr == 12 && MAXNR >= 12 ? rk[48 + w] : rk[4 * MAXNR + w]);
    uint32_t prev[4] = {un.w[0], un.w[1], un.w[2], un.w[3]};
    const uint32_t nblk = un.nbytes >> 4;
    const uint8_t *src = in + un.off;
    uint8_t *dst = out + un.off;
    constexpr uint32_t PF = 8;  // blocks fetched together: one 128-byte line per lane
    for (uint32_t b = 0; b < nblk; b += PF) {
        uint32_t x[PF][4];
#pragma unroll
        for (uint32_t j = 0; j < PF; j++) {
            if (b + j < nblk) {
                const uint4 v = *reinterpret_cast<const uint4 *>(src + ((b + j) << 4));
                x[j][0] = v.x;
                x[j][1] = v.y;
                x[j][2] = v.z;
                x[j][3] = v.w;
            }
        }
#pragma unroll
        for (uint32_t j = 0; j < PF; j++) {
            if (b + j < nblk) {
                uint32_t s[4];
#pragma unroll
                for (int w = 0; w < 4; w++)
                    s[w] = x[j][w] ^ prev[w] ^ rk[w];
#pragma unroll
                for (int r = 1; r < MAXNR; r++) {
                    if (r < 10 || (uint32_t)r < nr)
                        enc_round(lds, s, rk + 4 * r, L0);
                }
                const uint32_t zero[4] = {0u, 0u, 0u, 0u};
                enc_last(lds, s, rkl, L0, zero, prev);
                *reinterpret_cast<uint4 *>(dst + ((b + j) << 4)) =
                    make_uint4(prev[0], prev[1], prev[2], prev[3]);
            }
        }
    }
}

// One chain per lane; lanes of one wave may have different keys and lengths.
// A lane whose schedule is invalid (bad index or round count) does nothing.
__device__ __forceinline__ void run_chain(const uint32_t *lds, uint32_t L0,
                                          const Unit &un, const aes_schedule_t *__restrict__ sched,
                                          uint32_t n_sched, const uint8_t *in, uint8_t *out) {
    const uint32_t key = un.meta & META_KEY_MASK;
    const aes_schedule_t *ks = sched + (key < n_sched ? key : 0u);
    const uint32_t nr = key < n_sched ? ks->nr : 0u;
    const bool ok = nr == 10 || nr == 12 || nr == 14;
    const uint64_t m12 = __ballot(ok && nr == 12);
    const uint64_t m14 = __ballot(ok && nr == 14);
    if (!ok)
        return;
    if (m14)
        chain_run<14>(lds, L0, un, ks->ek, nr, in, out);
    else if (m12)
        chain_run<12>(lds, L0, un, ks->ek, nr, in, out);
    else
        chain_run<10>(lds, L0, un, ks->ek, nr, in, out);
}

// Chains of a wave: `cl` active lanes per wave (spreading few chains over more
// waves and compute units lowers nothing but the per-CU contention; each lane
// is still one serial chain).  Wave e takes chains e*cl + lane, then strides.
__device__ __forceinline__ void chain_loop(const uint32_t *lds, uint32_t L0,
                                           uint32_t lane, uint32_t e, uint32_t n_waves,
                                           uint32_t cl, const Unit *__restrict__ chains,
                                           uint32_t n_chain,
                                           const aes_schedule_t *__restrict__ sched,
                                           uint32_t n_sched, const uint8_t *in, uint8_t *out) {
    if (lane >= cl)
        return;
    for (uint64_t c = (uint64_t)e * cl + lane; c < n_chain; c += (uint64_t)n_waves * cl) {
        const Unit un = chains[c];
        run_chain(lds, L0, un, sched, n_sched, in, out);
    }
}

// ------------------------------------------------ one chain on four lanes
//
// A single serial chain (the per-request launch and the serving engine)
// runs on lanes 0..3: lane q holds state column q, reads the other three
// columns from its quad neighbours with DPP quad_perm and does its column's
// four lookups, so a round costs four dependent LDS reads per lane instead of
// sixteen.  Round keys: word q of each round key in VGPRs.

// Lane q of each quad receives lane (q + K) mod 4's v.
template <int K>
__device__ __forceinline__ uint32_t quad_next(uint32_t v) {
    // quad_perm selectors [1,2,3,0], [2,3,0,1], [3,0,1,2]
    constexpr int sel = K == 1 ? 0x39 : (K == 2 ? 0x4E : 0x93);
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, sel, 0xF, 0xF, false);
}

// A round of the quad form.  Column j of the round's output takes row r from
// column j + r (ShiftRows), so lane j needs Te_r of byte r of lane (j + r)'s
// column.  Each lane looks up the four bytes of its own column and the quad
// exchanges the looked-up words afterwards: the exchange then reads values
// returned by LDS, not ones a VALU op has just written, and the lookups do not
// wait for it.
// The lookup that needs no exchange goes last: the three exchanged words are
// moved while it is in flight, so only one XOR3 stands between the last LDS
// return and the next round's addresses.
__device__ __forceinline__ uint32_t quad_round_col(const uint32_t *lds, uint32_t st, uint32_t k,
                                                   uint32_t L0) {
    const uint32_t a1 = tlook<1, 1>(lds, st, L0);
    const uint32_t a2 = tlook<2, 2>(lds, st, L0);
    const uint32_t a3 = tlook<3, 3>(lds, st, L0);
    const uint32_t a0 = tlook<0, 0>(lds, st, L0);
    return xor3(xor3(quad_next<1>(a1), quad_next<2>(a2), k), quad_next<3>(a3), a0);
}

// The last round's SubBytes/ShiftRows column in the quad form (byte r of
// column j is S of byte r of lane (j + r)'s column), exchanged after lookup.
__device__ __forceinline__ uint32_t quad_sub_col(const uint32_t *lds, uint32_t st, uint32_t L0) {
    const uint32_t b = quad_next<1>(tlook<1, 0>(lds, st, L0));
    const uint32_t c = quad_next<2>(tlook<2, 1>(lds, st, L0));
    const uint32_t d = quad_next<3>(tlook<3, 2>(lds, st, L0));
    const uint32_t a = tlook<0, 3>(lds, st, L0);  // unexchanged, last
    return pick_diag(a, b, c, d);
}

// One block of a quad's chain: the whitened state st through rounds 1 ..
// MAXNR-1 and the last round.  A quad whose schedule has fewer rounds than
// MAXNR (quads of one wave may mix key sizes) runs the extra rounds too and
// takes the state it had before them into its last round: a select instead of
// a branch around each extra round, which costs two exec-mask updates and two
// taken branches per round.  With nr == MAXNR known at compile time the
// selects fold away.
template <int MAXNR>
__device__ __forceinline__ uint32_t quad_block(const uint32_t *lds, uint32_t st, const uint32_t *rk,
                                               uint32_t rkl, uint32_t nr, uint32_t L0) {
    uint32_t s10 = 0, s12 = 0;  // the state entering round 10 / round 12
#pragma unroll
    for (int r = 1; r < MAXNR; r++) {
        if (r == 10)
            s10 = st;
        if (r == 12)
            s12 = st;
        st = quad_round_col(lds, st, rk[r], L0);
    }
    if (MAXNR > 10)
        st = nr == 10u ? s10 : (MAXNR > 12 && nr == 12u ? s12 : st);
    return quad_sub_col(lds, st, L0) ^ rkl;
}

// Runs a quad's chain.  Lanes of a quad share one chain (un, ek, nr); quads
// of a wave may have different chains, keys and key sizes: rounds run up to
// MAXNR.
template <int MAXNR>
__device__ __forceinline__ void chain_quad_run(const uint32_t *lds, uint32_t L0, uint32_t q,
                                               const Unit &un, const uint32_t *ek, uint32_t nr,
                                               const uint8_t *in, uint8_t *out) {
    uint32_t rk[MAXNR + 1];
#pragma unroll
    for (int r = 0; r <= MAXNR; r++)
        rk[r] = ek[4 * r + q];
    const uint32_t rkl = nr == 10 ? rk[10] : (nr == 12 && MAXNR >= 12 ? rk[12] : rk[MAXNR]);
    // the IV's word q, selected with masks (an indexed read of un.w would
    // put the record in scratch memory)
    uint32_t prev = 0;
#pragma unroll
    for (uint32_t w = 0; w < 4; w++)
        prev |= un.w[w] & (0u - (uint32_t)(q == w));
    const uint32_t nblk = un.nbytes >> 4;
    if (nblk == 0)
        return;
    // Through the global address space: a payload pointer that the compiler
    // cannot trace to a kernel argument (the serving kernel reads it from a
    // queue unit) would otherwise be accessed with flat instructions, which
    // it also counts as LDS operations, and every round's LDS wait would then
    // be for all four lookups instead of the next one.
    const gu32 *src = (const gu32 *)(in + un.off) + q;
    gu32 *dst = (gu32 *)(out + un.off) + q;
    // Blocks go in groups of PF, software-pipelined: group g's words are
    // loaded while group g-1's rounds run, and group g-1's ciphertext is
    // stored while group g's run, so no wait falls on a load or store issued
    // less than a group earlier (waiting on the loads of the group about to
    // run cost about a seventh of a chain's time).  Loads past the chain's
    // end read its last block again (always in bounds, and no branch); the
    // whole groups run without per-block checks, a partial last group after
    // them.
    constexpr uint32_t PF = 8;
    const uint32_t last = nblk - 1u;
    const uint32_t nfull = nblk / PF * PF;
    uint32_t x[PF], y[PF];
#pragma unroll
    for (uint32_t j = 0; j < PF; j++)
        x[j] = src[4 * (j < last ? j : last)];
    uint32_t b = 0;
    for (; b < nfull; b += PF) {
        // Using the group's first word here (an empty asm with a memory
        // clobber keeps it in place) puts the wait for the group's loads
        // before the stores and loads issued below.
        uint32_t st = x[0] ^ prev ^ rk[0];
        asm volatile("" ::"v"(st) : "memory");
        if (b) {
            gu32 *d = dst + 4 * (b - PF);
#pragma unroll
            for (uint32_t j = 0; j < PF; j++)
                d[4 * j] = y[j];
        }
        uint32_t xn[PF];
#pragma unroll
        for (uint32_t j = 0; j < PF; j++) {
            const uint32_t i = b + PF + j;
            xn[j] = src[4 * (i < last ? i : last)];
        }
        // Keeps the loads here, a group ahead of their use (without it the
        // scheduler sinks them to the end of the group, next to the copies
        // into x, and the group ends waiting on them).
        asm volatile("" ::: "memory");
#pragma unroll
        for (uint32_t j = 0; j < PF; j++) {
            if (j)
                st = x[j] ^ prev ^ rk[0];
            prev = quad_block<MAXNR>(lds, st, rk, rkl, nr, L0);
            y[j] = prev;
        }
#pragma unroll
        for (uint32_t j = 0; j < PF; j++)
            x[j] = xn[j];
    }
    if (nfull) {
        gu32 *d = dst + 4 * (nfull - PF);
#pragma unroll
        for (uint32_t j = 0; j < PF; j++)
            d[4 * j] = y[j];
    }
    if (nfull < nblk) {
        gu32 *d = dst + 4 * nfull;
#pragma unroll
        for (uint32_t j = 0; j < PF - 1; j++) {
            if (nfull + j < nblk) {
                prev = quad_block<MAXNR>(lds, x[j] ^ prev ^ rk[0], rk, rkl, nr, L0);
                d[4 * j] = prev;
            }
        }
    }
}

// Key check and round-count dispatch for the chains of a wave's quads (un,
// per quad); MAXNR is the largest round count among them.
__device__ __forceinline__ void run_chains_quad(const uint32_t *lds, uint32_t L0, uint32_t q,
                                                bool active, const Unit &un,
                                                const aes_schedule_t *__restrict__ sched,
                                                uint32_t n_sched, const uint8_t *in,
                                                uint8_t *out) {
    const uint32_t key = un.meta & META_KEY_MASK;
    const bool keyed = active && key < n_sched;
    const aes_schedule_t *ks = sched + (keyed ? key : 0u);
    const uint32_t nr = keyed ? ks->nr : 0u;
    const bool ok = nr == 10 || nr == 12 || nr == 14;
    const uint64_t m12 = __ballot(ok && nr == 12);
    const uint64_t m14 = __ballot(ok && nr == 14);
    const uint64_t mok = __ballot(ok);
    if (!ok)
        return;
    // A wave whose chains all have the largest round count runs it as a
    // constant (no selects before the last round).
    if (m14 == mok)
        chain_quad_run<14>(lds, L0, q, un, ks->ek, 14u, in, out);
    else if (m14)
        chain_quad_run<14>(lds, L0, q, un, ks->ek, nr, in, out);
    else if (m12 == mok)
        chain_quad_run<12>(lds, L0, q, un, ks->ek, 12u, in, out);
    else if (m12)
        chain_quad_run<12>(lds, L0, q, un, ks->ek, nr, in, out);
    else
        chain_quad_run<10>(lds, L0, q, un, ks->ek, nr, in, out);
}

// Runs one CBC-encrypt chain on lanes 0..3 of the calling wave (the other
// lanes take no part).  Key and round count are wave-uniform.
__device__ __forceinline__ void run_chain_quad(const uint32_t *lds, uint32_t L0, uint32_t lane,
                                               const Unit &un,
                                               const aes_schedule_t *__restrict__ sched,
                                               uint32_t n_sched, const uint8_t *in,
                                               uint8_t *out) {
    const uint32_t key = un.meta & META_KEY_MASK;
    if (key >= n_sched || lane >= 4u)
        return;
    const aes_schedule_t *ks = sched + key;
    const uint32_t nr = ks->nr;
    if (nr == 10)
        chain_quad_run<10>(lds, L0, lane, un, ks->ek, 10u, in, out);
    else if (nr == 12)
        chain_quad_run<12>(lds, L0, lane, un, ks->ek, 12u, in, out);
    else if (nr == 14)
        chain_quad_run<14>(lds, L0, lane, un, ks->ek, 14u, in, out);
}

// Chains of a wave in quads: 16 chains per wave, four lanes each.  Wave e
// takes chains 16 e + lane / 4, then strides by 16 n_waves.
__device__ __forceinline__ void chain_loop_quad(const uint32_t *lds, uint32_t L0,
                                                uint32_t lane, uint32_t e, uint32_t n_waves,
                                                const Unit *__restrict__ chains,
                                                uint32_t n_chain,
                                                const aes_schedule_t *__restrict__ sched,
                                                uint32_t n_sched, const uint8_t *in,
                                                uint8_t *out) {
    const uint32_t q = lane & 3u;
    for (uint64_t base = (uint64_t)e * 16u; base < n_chain; base += (uint64_t)n_waves * 16u) {
        const uint64_t c = base + (lane >> 2);
        const bool active = c < n_chain;
        Unit un;
        if (active) {
            un = chains[c];
        } else {
            un.off = 0;
            un.nbytes = 0;
            un.meta = 0;
            un.w[0] = un.w[1] = un.w[2] = un.w[3] = 0u;
        }
        run_chains_quad(lds, L0, q, active, un, sched, n_sched, in, out);
    }
}

}  // namespace aesgpu
