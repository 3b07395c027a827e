// tile_kernel.h -- the parallel-mode tile kernel (CTR and ECB encryption, or
// CBC and ECB decryption) and its launcher.  Each of aes_tiles_ctr.hip and
// aes_tiles_dec.hip instantiates one side, so that each is compiled with the
// instruction-scheduling strategy measured best for it.
#pragma once

#include <hip/hip_runtime.h>

#include "aes_rounds.h"
#include "internal.h"

namespace aesgpu {

// Tile counters: one per workgroup of a tile launch, for each side.
static_assert(TILE_CTRS == 65536, "one counter per workgroup of the largest grid");
constexpr uint32_t TILE_MAX_GRID = TILE_CTRS;
// Grids of up to TILE_SPREAD_GRID workgroups keep each counter on a 128-byte
// line of its own (word 32 g): with the counters packed, 16 workgroups of all
// eight XCDs shared each 64-byte line, and the claims of some XCDs were served
// slower than others' (the slowest XCD's workgroups ended about 4% after the
// average, launch after launch; with a line each, about 2%), and a launch ends
// with its slowest workgroup.  Larger grids pack the counters (word g).
constexpr uint32_t TILE_CTR_STRIDE = 32;
constexpr uint32_t TILE_SPREAD_GRID = TILE_CTRS / TILE_CTR_STRIDE;

// One table set in LDS per workgroup.  Workgroup g owns a contiguous range
// of units.  Wave w starts on unit w of the range without a claim (its record
// is loaded, and its first claim issued, while the tables fill); after that,
// waves claim units wpb, wpb + 1, ... of the range one at a time from the
// workgroup's counter in wg_ctr.  The SIMD arbiter runs the oldest wave first,
// so with a fixed share per wave the first waves of each SIMD finished in
// about half the time of the last and the CUs ran the final third of a launch
// with one or two waves per SIMD; with claims, favoured waves simply take
// more units.  Each claim is made one unit ahead, so its latency overlaps the
// unit before (the counters are spread over 128-byte lines, see
// TILE_CTR_STRIDE).  Every wave ends on exactly one failing claim; the wave whose
// failing claim is the last (value max(range - wpb, 0) + wpb - 1) resets the
// counter, which is zero again when the launch ends, ready for the next
// launch of the same plan on the same stream (or a replay of a graph holding
// it).
template <bool DEC, int NB, int WG>
__global__ __launch_bounds__(WG) void k_tiles(const Unit *__restrict__ units, uint32_t n_units,
                                              const aes_schedule_t *__restrict__ sched,
                                              uint32_t n_sched, const uint32_t *__restrict__ timg,
                                              const uint4 *__restrict__ preds, const uint8_t *in,
                                              uint8_t *out, uint32_t *__restrict__ wg_ctr) {
    __shared__ uint32_t lds[DEC ? LDS_DEC_WORDS : LDS_ENC_WORDS];
    const uint32_t lane = threadIdx.x & 63u;
    // Waves per workgroup from the template (the kernel is launched with WG
    // threads); unit indices are made explicitly uniform, so the unit record
    // and key-schedule loads stay scalar.
    constexpr uint32_t wpb = WG / 64;
    const uint32_t g = blockIdx.x;
    const uint32_t lo = (uint32_t)((uint64_t)n_units * g / gridDim.x);
    const uint32_t range = (uint32_t)((uint64_t)n_units * (g + 1) / gridDim.x) - lo;
    uint32_t *cnt = wg_ctr + (gridDim.x <= TILE_SPREAD_GRID ? g * TILE_CTR_STRIDE : g);
    uint32_t c = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    Unit un;
    if (c < range)
        un = units[lo + c];
    uint32_t got = lane == 0 ? atomicAdd(cnt, 1u) : 0u;
    fill_tables<DEC>(lds, timg);
    __syncthreads();
    const uint32_t L0 = (lane & 31u) << 2;
    const uint32_t L2 = L0 | SI_BASE;
    while (c < range) {
        const uint32_t u = lo + c;
        if (DEC)
            run_dec_unit<NB, TILE_NV_DEC, true>(lds, L0, L2, lane, un,
                                                preds ? preds + u : nullptr, sched, n_sched,
                                                in, out);
        else
            run_ctr_unit<NB, TILE_NV_CTR>(lds, L0, lane, un, sched, n_sched, in, out, timg);
        c = wpb + __builtin_amdgcn_readfirstlane(got);
        if (c < range) {
            got = lane == 0 ? atomicAdd(cnt, 1u) : 0u;  // the next claim, in flight meanwhile
            un = units[lo + c];
        }
    }
    const uint32_t last = (range > wpb ? range - wpb : 0u) + wpb - 1u;
    if (__builtin_amdgcn_readfirstlane(got) == last && lane == 0)
        __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

using TileKernel = void (*)(const Unit *, uint32_t, const aes_schedule_t *, uint32_t,
                            const uint32_t *, const uint4 *, const uint8_t *, uint8_t *,
                            uint32_t *);

// Compiled shapes: blocks per lane NB in {1, 2, 4} x workgroup size WG in
// {256, 512, 1024}.  The launch bound sets the VGPR budget (WG 1024 gives
// 128 VGPRs per lane, 512 gives 256).
template <bool DEC>
inline TileKernel pick_tile_kernel(int nb, int wg) {
#define AESGPU_TK(NB_, WG_)                                                                     \
    if (nb == NB_ && wg <= WG_)                                                                 \
        return (TileKernel)&k_tiles<DEC, NB_, WG_>;
    AESGPU_TK(1, 256) AESGPU_TK(1, 512) AESGPU_TK(1, 1024)
    AESGPU_TK(2, 256) AESGPU_TK(2, 512) AESGPU_TK(2, 1024)
    AESGPU_TK(4, 256) AESGPU_TK(4, 512)
#undef AESGPU_TK
    return nullptr;
}

// d_ctrs: TILE_MAX_GRID zeroed counters (zero again after every launch).
template <bool DEC>
inline int launch_tiles(const Unit *d_units, uint32_t n_units, const aes_schedule_t *d_sched,
                        uint32_t n_sched, const uint32_t *d_timg, const void *d_preds,
                        const uint8_t *d_in, uint8_t *d_out, uint32_t *d_ctrs,
                        const TileLaunch &cfg, int n_cu, void *stream) {
    if (!n_units)
        return hipSuccess;
    const TileKernel k = pick_tile_kernel<DEC>(cfg.nb, cfg.wg_threads);
    if (!k)
        return hipErrorInvalidValue;
    const int waves = cfg.wg_threads / 64;
    int grid = cfg.grid > 0 ? cfg.grid : n_cu;
    const long need = ((long)n_units + waves - 1) / waves;
    if (need < grid)
        grid = (int)need;
    if (grid < 1)
        grid = 1;
    if (!d_ctrs || (uint32_t)grid > TILE_MAX_GRID)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3(grid), dim3(cfg.wg_threads), 0, (hipStream_t)stream, d_units,
                       n_units, d_sched, n_sched, d_timg, (const uint4 *)d_preds, d_in, d_out,
                       d_ctrs);
    return hipGetLastError();
}

}  // namespace aesgpu
