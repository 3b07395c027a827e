// aes_kernels.hip -- batch kernels (chains, one fused launch, one request per
// launch) over the round functions of aes_rounds.h.  The tile kernels live in
// tile_kernel.h, instantiated by aes_tiles_ctr.hip and aes_tiles_dec.hip.
#include <hip/hip_runtime.h>

#include "aes_chain.h"
#include "aes_rounds.h"
#include "internal.h"

namespace aesgpu {

// Wave numbering that spreads consecutive waves over workgroups first.
__device__ __forceinline__ uint32_t spread_wave(uint32_t wg, uint32_t n_wg) {
    return __builtin_amdgcn_readfirstlane((threadIdx.x >> 6) * n_wg + wg);
}

// CBC-encrypt chains: cl chains per wave on one lane each, or (cl = 0) 16
// chains per wave on four lanes each.
__global__ __launch_bounds__(1024) void k_chains(const Unit *__restrict__ chains,
                                                 uint32_t n_chain, uint32_t cl,
                                                 const aes_schedule_t *__restrict__ sched,
                                                 uint32_t n_sched,
                                                 const uint32_t *__restrict__ timg,
                                                 const uint8_t *in, uint8_t *out) {
    __shared__ uint32_t lds[LDS_ENC_WORDS];
    fill_tables<false>(lds, timg);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t L0 = (lane & 31u) << 2;
    const uint32_t n_waves = __builtin_amdgcn_readfirstlane(gridDim.x * (blockDim.x >> 6));
    const uint32_t e = spread_wave(blockIdx.x, gridDim.x);
    if (cl)
        chain_loop(lds, L0, lane, e, n_waves, cl, chains, n_chain, sched, n_sched, in, out);
    else
        chain_loop_quad(lds, L0, lane, e, n_waves, chains, n_chain, sched, n_sched, in, out);
}

// ----------------------------------------------------- one fused launch

// A whole mixed batch in one launch.  Workgroups [0, n_dec_wg) hold the
// decryption tables and work the CBC-decrypt tiles; the others hold the
// encryption tables, start the CBC-encrypt chains (the long serial work)
// on their first waves, and every encryption wave then works CTR tiles.
template <int NB, bool QUAD>
__global__ __launch_bounds__(1024) void k_mixed(MixedArgs a) {
    __shared__ uint32_t lds[LDS_DEC_WORDS];
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t L0 = (lane & 31u) << 2;
    const uint32_t L2 = L0 | SI_BASE;
    const uint32_t wpb = blockDim.x >> 6;
    if (blockIdx.x < a.n_dec_wg) {
        fill_tables<true>(lds, a.timg);
        __syncthreads();
        const uint32_t nw = __builtin_amdgcn_readfirstlane(a.n_dec_wg * wpb);
        for (uint32_t u = spread_wave(blockIdx.x, a.n_dec_wg); u < a.n_dec; u += nw) {
            const Unit un = a.dec[u];
            run_dec_unit<NB>(lds, L0, L2, lane, un,
                             a.preds ? reinterpret_cast<const uint4 *>(a.preds) + u : nullptr,
                             a.sched, a.n_sched, a.in, a.out);
        }
        return;
    }
    fill_tables<false>(lds, a.timg);
    __syncthreads();
    const uint32_t n_enc_wg = gridDim.x - a.n_dec_wg;
    const uint32_t e = spread_wave(blockIdx.x - a.n_dec_wg, n_enc_wg);
    const uint32_t nw = __builtin_amdgcn_readfirstlane(n_enc_wg * wpb);
    // Waves [0, cw) run the chains and stop; the others work the CTR tiles
    // (at least half of the waves when there are any), so the two paths
    // share no registers.
    uint32_t cw = 0;
    if (a.n_chain) {
        const uint32_t per_wave = QUAD ? 16u : a.chain_lanes;
        const uint32_t chain_waves = (uint32_t)(((uint64_t)a.n_chain + per_wave - 1) / per_wave);
        const uint32_t cap = a.n_ctr ? nw / 2u : nw;
        cw = chain_waves < cap ? chain_waves : cap;
        if (cw < 1u)
            cw = 1u;
        if (e < cw) {
            if (QUAD)
                chain_loop_quad(lds, L0, lane, e, cw, a.chains, a.n_chain, a.sched, a.n_sched,
                                a.in, a.out);
            else
                chain_loop(lds, L0, lane, e, cw, a.chain_lanes, a.chains, a.n_chain, a.sched,
                           a.n_sched, a.in, a.out);
            return;
        }
    }
    for (uint32_t u = e - cw; u < a.n_ctr; u += nw - cw) {
        const Unit un = a.ctr[u];
        run_ctr_unit<NB>(lds, L0, lane, un, a.sched, a.n_sched, a.in, a.out);
    }
}

// ------------------------------------------------- one request per launch

// Unit t of a single request passed by value (the per-request launch form).
__device__ __forceinline__ Unit request_unit(const aes_req_t &r, uint32_t t, uint32_t tile) {
    Unit u;
    const uint64_t pos = (uint64_t)t * tile;
    u.off = r.offset + pos;
    const uint64_t left = r.length - pos;
    u.nbytes = (uint32_t)(left < tile ? left : tile);
    u.meta = r.key_idx | (r.op << META_OP_SHIFT);
    uint32_t w[4];
#pragma unroll
    for (int i = 0; i < 4; i++)
        w[i] = (uint32_t)r.iv[4 * i] | ((uint32_t)r.iv[4 * i + 1] << 8) |
               ((uint32_t)r.iv[4 * i + 2] << 16) | ((uint32_t)r.iv[4 * i + 3] << 24);
    if (r.op == AES_OP_CTR) {
        // initial counter: bytes 8..15 of T1 big-endian, plus the tile's first block
        const uint64_t c0 = ((uint64_t)__builtin_bswap32(w[2]) << 32) | __builtin_bswap32(w[3]);
        const uint64_t c = c0 + pos / 16;
        u.w[0] = w[0];
        u.w[1] = w[1];
        u.w[2] = (uint32_t)c;
        u.w[3] = (uint32_t)(c >> 32);
    } else if (r.op == AES_OP_ECB_ENC || r.op == AES_OP_ECB_DEC) {
        u.w[0] = u.w[1] = u.w[2] = u.w[3] = 0u;
    } else if (t == 0 || r.op == AES_OP_CBC_ENC) {
        u.w[0] = w[0];
        u.w[1] = w[1];
        u.w[2] = w[2];
        u.w[3] = w[3];
    } else {
        u.meta |= FLAG_PRED_IN;
        u.w[0] = u.w[1] = u.w[2] = u.w[3] = 0u;
    }
    return u;
}

template <bool DEC, int NB>
__global__ __launch_bounds__(1024) void k_request(aes_req_t r, uint32_t tile,
                                                 const aes_schedule_t *__restrict__ sched,
                                                 uint32_t n_sched,
                                                 const uint32_t *__restrict__ timg,
                                                 const uint8_t *in, uint8_t *out) {
    __shared__ uint32_t lds[DEC ? LDS_DEC_WORDS : LDS_ENC_WORDS];
    fill_tables<DEC>(lds, timg);
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t L0 = (lane & 31u) << 2;
    const uint32_t L2 = L0 | SI_BASE;
    if (!DEC && r.op == AES_OP_CBC_ENC) {
        // One serial chain, on four lanes of the first wave.
        if (blockIdx.x == 0 && threadIdx.x < 64u) {
            const Unit un = request_unit(r, 0, (uint32_t)r.length);
            run_chain_quad(lds, L0, lane, un, sched, n_sched, in, out);
        }
        return;
    }
    const uint32_t wpb = blockDim.x >> 6;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(blockIdx.x * wpb + (threadIdx.x >> 6));
    const uint32_t nw = __builtin_amdgcn_readfirstlane(gridDim.x * wpb);
    const uint32_t n_units = (uint32_t)((r.length + tile - 1) / tile);
    for (uint32_t t = wave; t < n_units; t += nw) {
        const Unit un = request_unit(r, t, tile);
        if (DEC)
            run_dec_unit<NB, TILE_NV_DEC>(lds, L0, L2, lane, un, nullptr, sched, n_sched, in,
                                          out);
        else
            run_ctr_unit<NB, TILE_NV_CTR>(lds, L0, lane, un, sched, n_sched, in, out);
    }
}

// --------------------------------------------------- in-place predecessors

__global__ void k_snapshot_preds(const Unit *__restrict__ units, uint32_t n_units,
                                 const uint8_t *in, uint4 *preds) {
    const uint32_t u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_units)
        return;
    if (units[u].meta & FLAG_PRED_IN)
        preds[u] = *reinterpret_cast<const uint4 *>(in + units[u].off - 16);
}

// --------------------------------------------------------------- launchers

static uint32_t chain_waves_needed(uint32_t n_chain, uint32_t cl) {
    return (uint32_t)(((uint64_t)n_chain + cl - 1) / cl);
}

int launch_cbcenc_chains(const Unit *d_units, uint32_t n_units, const aes_schedule_t *d_sched,
                         uint32_t n_sched, const uint32_t *d_timg, const uint8_t *d_in,
                         uint8_t *d_out, const ChainLaunch &cfg, int n_cu, void *stream) {
    if (!n_units)
        return hipSuccess;
    const uint32_t cl = cfg.lanes < 1 ? 64u : (cfg.lanes > 64 ? 64u : (uint32_t)cfg.lanes);
    const int wpb = cfg.wg_threads / 64;
    const uint32_t waves = chain_waves_needed(n_units, cfg.quad ? 16u : cl);
    int grid = cfg.grid > 0 ? cfg.grid : (int)((waves + wpb - 1) / wpb);
    if (grid > n_cu && cfg.grid <= 0)
        grid = n_cu;
    // Fewer waves than compute units: one wave per workgroup spreads them out.
    int threads = cfg.wg_threads;
    if (cfg.grid <= 0 && waves < (uint32_t)n_cu * wpb) {
        const uint32_t per_cu = (waves + n_cu - 1) / n_cu;
        threads = 64 * (int)(per_cu < 1 ? 1 : per_cu);
        grid = (int)((waves + per_cu - 1) / per_cu);
    }
    hipLaunchKernelGGL(k_chains, dim3(grid < 1 ? 1 : grid), dim3(threads), 0,
                       (hipStream_t)stream, d_units, n_units, cfg.quad ? 0u : cl, d_sched, n_sched,
                       d_timg, d_in, d_out);
    return hipGetLastError();
}

int launch_mixed(const MixedArgs &a, int nb, int grid, void *stream) {
    if (!a.n_dec && !a.n_ctr && !a.n_chain)
        return hipSuccess;
    void (*k)(MixedArgs) = nullptr;
    if (nb == 1)
        k = a.chain_quad ? &k_mixed<1, true> : &k_mixed<1, false>;
    else if (nb == 2)
        k = a.chain_quad ? &k_mixed<2, true> : &k_mixed<2, false>;
    if (!k || grid < 1 || (a.n_dec && a.n_dec_wg < 1) ||
        ((a.n_ctr || a.n_chain) && (uint32_t)grid <= a.n_dec_wg) || a.chain_lanes < 1 ||
        a.chain_lanes > 64 || a.chain_quad > 1)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k, dim3(grid), dim3(1024), 0, (hipStream_t)stream, a);
    return hipGetLastError();
}

int launch_request(const aes_req_t &r, uint32_t tile, const aes_schedule_t *d_sched,
                   uint32_t n_sched, const uint32_t *d_timg, const uint8_t *d_in,
                   uint8_t *d_out, int n_cu, void *stream) {
    if (!r.length)
        return hipSuccess;
    // A request's tiles spread over as many compute units as it has tiles
    // (one single-wave workgroup per tile for small requests); larger
    // requests get up to 16 waves per workgroup and up to two workgroups per
    // compute unit in the grid.
    const uint32_t n_units = (uint32_t)((r.length + tile - 1) / tile);
    const uint32_t cus = (uint32_t)n_cu;
    uint32_t waves = (n_units + cus - 1) / cus;
    waves = waves < 1u ? 1u : (waves > 16u ? 16u : waves);
    uint32_t grid = (n_units + waves - 1) / waves;
    if (grid > 2u * cus)
        grid = 2u * cus;
    if (r.op == AES_OP_CBC_ENC) {
        grid = 1;
        waves = 1;
    }
    if (r.op == AES_OP_CBC_DEC || r.op == AES_OP_ECB_DEC)
        hipLaunchKernelGGL((k_request<true, 2>), dim3(grid), dim3(64 * waves), 0,
                           (hipStream_t)stream, r, tile, d_sched, n_sched, d_timg, d_in, d_out);
    else
        hipLaunchKernelGGL((k_request<false, 2>), dim3(grid), dim3(64 * waves), 0,
                           (hipStream_t)stream, r, tile, d_sched, n_sched, d_timg, d_in, d_out);
    return hipGetLastError();
}

int launch_snapshot_preds(const Unit *d_units, uint32_t n_units, const uint8_t *d_in,
                          void *d_preds, void *stream) {
    if (!n_units)
        return hipSuccess;
    hipLaunchKernelGGL(k_snapshot_preds, dim3((n_units + 255) / 256), dim3(256), 0,
                       (hipStream_t)stream, d_units, n_units, d_in, (uint4 *)d_preds);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_zero_words(uint32_t *p, uint32_t n) {
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i < n)
        p[i] = 0u;
}

int launch_zero_words(uint32_t *d_words, uint32_t n, void *stream) {
    if (!n)
        return hipSuccess;
    hipLaunchKernelGGL(k_zero_words, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream,
                       d_words, n);
    return hipGetLastError();
}

}  // namespace aesgpu
