// internal.h -- structures shared by the host planner and the HIP kernels.
#pragma once

#include <stdint.h>

#include "aesgpu.h"

namespace aesgpu {

// A work unit, 32 bytes, in device memory.  The planner cuts CTR and CBC
// decryption requests into tiles (many units per request, run in parallel)
// and gives each CBC encryption request one unit (a serial chain).
struct Unit {
    uint64_t off;     // byte offset of the unit's first byte (input and output)
    uint32_t nbytes;  // bytes in the unit
    uint32_t meta;    // bits 0..23 schedule index, bits 24..26 op, bits 27..31 flags
    uint32_t w[4];    // CTR: nonce words 0,1 then the 64-bit counter of the unit's
                      //      first block as an integer (w[2] low half, w[3] high half)
                      // CBC: the 16 bytes that precede the unit's first block in
                      //      the chain (the IV for a request's first unit)
};
static_assert(sizeof(Unit) == 32, "Unit is 32 bytes");

constexpr uint32_t META_KEY_MASK = 0x00FFFFFFu;
constexpr uint32_t META_OP_SHIFT = 24;
constexpr uint32_t META_OP_MASK = 7u;        // op in bits 24..26
constexpr uint32_t FLAG_PRED_IN = 1u << 27;  // CBC-dec: predecessor is in[off-16 .. off)

__host__ __device__ inline uint32_t unit_op(uint32_t meta) {
    return (meta >> META_OP_SHIFT) & META_OP_MASK;
}
constexpr uint32_t MAX_KEYS = 1u << 24;

// Table image in device memory (2304 words), written once per context:
//   [0, 1024)     Te0..Te3, 256 words each (encryption round tables)
//   [1024, 2048)  Td0..Td3 (equivalent inverse cipher round tables)
//   [2048, 2304)  Si4: the inverse S-box byte repeated in all four bytes
constexpr int TIMG_WORDS = 2304;

// Launch shape of the parallel-mode (tile) kernel.
struct TileLaunch {
    int nb = 2;             // 16-byte blocks per lane per step (1, 2 or 4)
    int wg_threads = 1024;  // threads per workgroup (multiple of 64, <= 1024)
    int grid = 0;           // workgroups; 0 = one per compute unit
};
bool tile_shape_supported(int nb, int wg_threads);

struct ChainLaunch {
    int wg_threads = 256;
    int lanes = 64;     // active lanes (chains) per wave, one lane per chain
    bool quad = false;  // instead: 16 chains per wave on four lanes each
    int grid = 0;       // 0 = as many as the chains need, at most one per compute unit
};

// Arguments of the fused mixed-batch kernel (one launch for all three ops).
struct MixedArgs {
    const Unit *dec;        // CBC-decrypt tiles
    const Unit *ctr;        // CTR tiles
    const Unit *chains;     // CBC-encrypt chains, longest first, ties by key
    const uint32_t *preds;  // NULL or 4 words per CBC-decrypt tile (in-place snapshots)
    const aes_schedule_t *sched;
    const uint32_t *timg;
    const uint8_t *in;
    uint8_t *out;
    uint32_t n_dec, n_ctr, n_chain;
    uint32_t n_sched;
    uint32_t n_dec_wg;      // workgroups [0, n_dec_wg) hold the decryption tables
    uint32_t chain_lanes;   // active lanes per chain wave (one lane per chain)
    uint32_t chain_quad;    // 1: 16 chains per wave on four lanes each
};

// Host-side launchers.  Each returns a hipError_t value.  Tile kernels:
// aes_tiles_ctr.hip and aes_tiles_dec.hip; the others: aes_kernels.hip.
// Tile launchers take d_ctrs: TILE_CTRS zeroed per-workgroup counters that
// every launch leaves zeroed (launches sharing them must not overlap).
constexpr uint32_t TILE_CTRS = 65536;
int launch_ctr_tiles(const Unit *d_units, uint32_t n_units, const aes_schedule_t *d_sched,
                     uint32_t n_sched, const uint32_t *d_timg, const uint8_t *d_in,
                     uint8_t *d_out, uint32_t *d_ctrs, const TileLaunch &cfg, int n_cu,
                     void *stream);
// Bitsliced CTR (aes_bitslice.hip): units in groups of 8 per wave, worked in
// 4 KiB chunks; a group whose units share a key makes one pass per chunk.
int launch_ctr_bitslice(const Unit *d_units, uint32_t n_units, const aes_schedule_t *d_sched,
                        uint32_t n_sched, const uint8_t *d_in, uint8_t *d_out, int n_cu,
                        void *stream);
// Bitsliced CBC and ECB decryption (aes_bitslice.hip): units in groups of 8
// per wave, worked in 4 KiB chunks; d_preds as for launch_cbcdec_tiles.
int launch_dec_bitslice(const Unit *d_units, uint32_t n_units, const aes_schedule_t *d_sched,
                        uint32_t n_sched, const void *d_preds, const uint8_t *d_in,
                        uint8_t *d_out, void *stream);
// d_preds: NULL, or one 16-byte predecessor per unit written by
// launch_snapshot_preds (used for FLAG_PRED_IN units instead of reading d_in).
int launch_cbcdec_tiles(const Unit *d_units, uint32_t n_units, const aes_schedule_t *d_sched,
                        uint32_t n_sched, const uint32_t *d_timg, const void *d_preds,
                        const uint8_t *d_in, uint8_t *d_out, uint32_t *d_ctrs,
                        const TileLaunch &cfg, int n_cu, void *stream);
int launch_cbcenc_chains(const Unit *d_units, uint32_t n_units, const aes_schedule_t *d_sched,
                         uint32_t n_sched, const uint32_t *d_timg, const uint8_t *d_in,
                         uint8_t *d_out, const ChainLaunch &cfg, int n_cu, void *stream);
// One launch over a mixed batch (nb = 1 or 2; 1024-thread workgroups).
int launch_mixed(const MixedArgs &a, int nb, int grid, void *stream);
// One request passed by value (the per-request launch form); tile = bytes per
// unit (the whole request length keeps an in-place CBC decryption in one wave).
int launch_request(const aes_req_t &r, uint32_t tile, const aes_schedule_t *d_sched,
                   uint32_t n_sched, const uint32_t *d_timg, const uint8_t *d_in,
                   uint8_t *d_out, int n_cu, void *stream);
// In-place CBC decryption: copies in[off-16, off) of every FLAG_PRED_IN unit u
// to d_preds[16u..16u+15] before the tile kernel overwrites those bytes.
int launch_snapshot_preds(const Unit *d_units, uint32_t n_units, const uint8_t *d_in,
                          void *d_preds, void *stream);
// Sets n words of device memory to zero with a kernel (a fill that stream
// capture records as a kernel node, not as a memset node).
int launch_zero_words(uint32_t *d_words, uint32_t n, void *stream);

// Records a failing hipError_t for aes_last_hip_error and returns
// AES_ERR_DEVICE (aes_abi.cpp).
int hip_fail_status(int hip_error);

// What the server needs to know about a context.
struct CtxInfo {
    int device;
    int n_cu;
    const uint32_t *d_timg;
};
int ctx_info(const aes_ctx_t *ctx, CtxInfo *out);

// Host table generation (tables.cpp).
void make_table_image(uint32_t img[TIMG_WORDS]);
int expand_key(const uint8_t *key, uint32_t key_bits, aes_schedule_t *out);

}  // namespace aesgpu
