/*
 * aesgpu.h -- C ABI of the MI355X (gfx950) batched AES library.
 *
 * The library runs the data-parallel service of "Augmenting Operating Systems
 * With the GPU" (Sun and Ricci): AES over many independent page-sized
 * buffers, offered by the GPU to an OS-kernel-like caller.  Section 3.3 of
 * the paper implements AES as a GPU service behind the kernel crypto layer;
 * section 3.2 defines how a caller uses such a service (a buffer in, a buffer
 * out, a service request, an optional completion callback, then block or
 * busy-wait); section 2 notes that one launch may carry either one large task
 * or many small tasks of different callers, and section 3.1 that batching
 * trades latency for throughput.  The cipher itself is FIPS-197 (AES-128,
 * -192, -256) in the CBC and CTR modes of NIST SP 800-38A.
 *
 * Conventions for every call:
 *   - Return value: AES_OK (0) or a negative AES_ERR_* code.  No call aborts
 *     or prints.  Arguments are validated on the host before any HIP call;
 *     on a validation error nothing is launched and no output byte changes.
 *   - "d_" pointers are device (HBM) addresses on the context's device; all
 *     other pointers are host addresses.  Host arrays may be freed as soon as
 *     the call returns.  Device buffers must stay valid until the work that
 *     uses them has completed on its stream.
 *   - hipStream_t arguments are passed as void*; NULL is the default stream.
 *     Calls that launch work are asynchronous with respect to the host.
 *   - One context must not be used by two host threads at once.
 */
#ifndef AESGPU_H
#define AESGPU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------- status codes */
enum {
    AES_OK = 0,
    AES_ERR_ARG = -1,      /* null pointer, bad enum, zero count where one is needed */
    AES_ERR_KEYSIZE = -2,  /* key_bits not 128, 192 or 256 */
    AES_ERR_LENGTH = -3,   /* CBC length not a multiple of 16, or a request >= 4 GiB */
    AES_ERR_RANGE = -4,    /* offset not a multiple of 16, or offset+length > buf_bytes,
                              or key index >= number of schedules */
    AES_ERR_OVERLAP = -5,  /* two requests write overlapping bytes, or in/out partly alias */
    AES_ERR_DEVICE = -6,   /* a HIP call failed (code in aes_last_hip_error), or the
                              context has no device */
    AES_ERR_NOMEM = -7,    /* host or device allocation failed */
    AES_ERR_AGAIN = -8,    /* serving: ring full or admission cap reached; retry */
    AES_ERR_TIMEOUT = -9,  /* serving: wait timed out */
    AES_ERR_STATE = -10    /* object used in a state that does not allow the call */
};

/* Static description of a status code (never NULL). */
const char *aes_strerror(int status);
/* The hipError_t of the last failing HIP call made by this host thread. */
int aes_last_hip_error(void);

/* ------------------------------------------------------------ key schedules */

/* Expanded key, 512 bytes, plain old data; made by aes_expand_key on the host
 * and copied by the caller to device memory as an array.
 *   ek[4*r + c]: round-key word c of round r (FIPS-197 5.2 w[4r+c]); the word's
 *                four bytes are stored in FIPS byte order, so a little-endian
 *                32-bit load of ek[i] has w[i]'s first byte in bits 0..7.
 *   dk[4*r + c]: round key of round r of the equivalent inverse cipher
 *                (FIPS-197 5.3.5): dk round 0 = w round Nr, dk round r =
 *                InvMixColumns(w round Nr-r) for 0 < r < Nr, dk round Nr =
 *                w round 0; same byte layout.
 * Words beyond round Nr are zero. */
typedef struct aes_schedule {
    uint32_t key_bits; /* 128, 192 or 256 */
    uint32_t nr;       /* 10, 12 or 14 rounds */
    uint32_t reserved0[2];
    uint32_t ek[60];
    uint32_t dk[60];
    uint32_t reserved1[4];
} aes_schedule_t;

/* FIPS-197 5.2 KeyExpansion of key (key_bits/8 bytes) into *out.  Pure host
 * function.  Errors: AES_ERR_ARG (null), AES_ERR_KEYSIZE. */
int aes_expand_key(const uint8_t *key, uint32_t key_bits, aes_schedule_t *out);

/* ------------------------------------------------------------------ context */

typedef struct aes_ctx aes_ctx_t;

/* AES_DEVICE_NONE makes a host-only context: every call validates and plans
 * as usual, and any call that would launch work returns AES_ERR_DEVICE. */
#define AES_DEVICE_NONE (-1)

/* Creates a context on HIP device hip_device (or AES_DEVICE_NONE).  The
 * context owns the cipher table images in device memory, pinned staging for
 * request metadata and the tuned launch configuration.
 * Errors: AES_ERR_ARG, AES_ERR_DEVICE, AES_ERR_NOMEM. */
int aes_ctx_create(int hip_device, aes_ctx_t **out);
/* Waits for the context's outstanding work, then frees it.  NULL is a no-op. */
void aes_ctx_destroy(aes_ctx_t *ctx);

/* ----------------------------------------------------------------- requests */

enum { AES_OP_CBC_ENC = 0, AES_OP_CBC_DEC = 1, AES_OP_CTR = 2, AES_OP_ECB_ENC = 3,
       AES_OP_ECB_DEC = 4 };

/* One service request (paper section 3.2: input buffer, output buffer and a
 * request naming the service).  Bytes [offset, offset+length) of the input
 * buffer are transformed into the same range of the output buffer.
 *   offset: multiple of 16.
 *   length: bytes, < 2^32; a multiple of 16 for CBC and ECB; any value for
 *           CTR (a final partial block uses the leading keystream bytes);
 *           0 = no-op.
 *   key_idx: index into the schedule array passed with the call.
 *   op:     AES_OP_CBC_ENC, AES_OP_CBC_DEC, AES_OP_CTR (CTR encrypts and
 *           decrypts alike), AES_OP_ECB_ENC or AES_OP_ECB_DEC (SP 800-38A 6.1:
 *           every block on its own -- the paper's service mode, section 3.3).
 *   iv:     CBC: the IV.  CTR: the initial counter block T1; bytes 0..7 are a
 *           nonce and bytes 8..15 a big-endian 64-bit counter that advances by
 *           one per block modulo 2^64 without carrying into the nonce.  ECB:
 *           unused.
 * Requests of one call must write pairwise disjoint byte ranges; the input
 * and output buffers are either the same buffer or do not overlap at all. */
typedef struct aes_req {
    uint64_t offset;
    uint64_t length;
    uint32_t key_idx;
    uint32_t op;
    uint8_t iv[16];
} aes_req_t;

/* Batched service call (paper sections 2 and 3.3: many independent buffers
 * in one GPU launch).  d_scheds: device array of n_scheds schedules.
 * d_in, d_out: device buffers of buf_bytes bytes.  reqs: host array of
 * n_reqs requests, validated and planned on the host, then copied to the
 * device through pinned staging before the call returns.  Work is launched on
 * stream; bytes of d_out outside every request are never written.
 * Errors: AES_ERR_ARG, AES_ERR_LENGTH, AES_ERR_RANGE, AES_ERR_OVERLAP,
 * AES_ERR_DEVICE, AES_ERR_NOMEM.  A schedule whose nr is not 10, 12 or 14
 * leaves its requests' output bytes unwritten. */
int aes_batch(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
              const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
              const aes_req_t *reqs, uint64_t n_reqs, void *stream);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): aes_batch with the
 * same arguments, rules, results and errors, that calls no allocation
 * routine.  The unit table (at most AES_NOALLOC_MAX_UNITS work units: one per
 * tile of the context's tile size for CTR, ECB and CBC-decrypt requests, one
 * per CBC-encrypt request), the in-place CBC-decrypt predecessor snapshots and
 * the tile counters live in one fixed device array per GPU (about 24.5 MiB,
 * held until the process ends); the requests are planned in fixed host
 * arrays and copied from there before the call returns.  Every call on one
 * GPU shares that GPU's array: calls whose work overlaps in time on one GPU
 * (launched on different streams without ordering, or from several host
 * threads) race on it and must be serialised by the caller; calls on one
 * stream are ordered.  Host work of concurrent calls is serialised inside.
 * CTR tiles stay in request order for both CTR variants.
 * Errors: those of aes_batch; AES_ERR_RANGE also when the batch needs more
 * than AES_NOALLOC_MAX_UNITS work units; AES_ERR_DEVICE also when the
 * context's device had no scratch address (device index 64 or above). */
#define AES_NOALLOC_MAX_UNITS (1u << 19)
int aes_batch_noalloc(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                      const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                      const aes_req_t *reqs, uint64_t n_reqs, void *stream);

/* Single-mode forms of aes_batch with the requests given as parallel host
 * arrays: offsets[i], lengths[i], key_idx[i] and ivs[16*i .. 16*i+15] form
 * request i; every request uses the mode the name says (SP 800-38A 6.2 CBC
 * encryption / decryption, 6.5 CTR, 6.1 ECB; the ECB forms take no IVs and
 * ignore ivs, which may be NULL).  Same errors as aes_batch. */
int aes_cbc_encrypt_batch(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                          const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                          const uint64_t *offsets, const uint64_t *lengths,
                          const uint32_t *key_idx, const uint8_t *ivs, uint64_t n,
                          void *stream);
int aes_cbc_decrypt_batch(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                          const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                          const uint64_t *offsets, const uint64_t *lengths,
                          const uint32_t *key_idx, const uint8_t *ivs, uint64_t n,
                          void *stream);
int aes_ctr_batch(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                  const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                  const uint64_t *offsets, const uint64_t *lengths,
                  const uint32_t *key_idx, const uint8_t *ivs, uint64_t n, void *stream);
int aes_ecb_encrypt_batch(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                          const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                          const uint64_t *offsets, const uint64_t *lengths,
                          const uint32_t *key_idx, const uint8_t *ivs, uint64_t n,
                          void *stream);
int aes_ecb_decrypt_batch(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                          const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                          const uint64_t *offsets, const uint64_t *lengths,
                          const uint32_t *key_idx, const uint8_t *ivs, uint64_t n,
                          void *stream);

/* -------------------------------------------------------------------- plans */

/* A plan is a validated request list cut into work units once and kept in
 * device memory, so that the same batch shape can be launched many times
 * (and captured in a HIP graph) with no host planning or metadata copy per
 * launch -- the "pre-loaded service" idea of paper section 3.1 applied to the
 * request metadata.  A plan must not be launched on two streams at once. */
typedef struct aes_plan aes_plan_t;

/* One work unit of a plan, 32 bytes (the device record the kernels read):
 *   offset, nbytes: the byte range the unit covers.
 *   meta: bits 0..23 schedule index, bits 24..26 op, bit 27 set when a CBC
 *         decryption unit takes its predecessor block from the 16 input bytes
 *         before offset (every tile of a request but the first).
 *   w: CTR -- nonce bytes 0..3 and 4..7 as little-endian words, then the
 *      64-bit counter of the unit's first block (w[2] low, w[3] high half);
 *      CBC -- the IV as four little-endian words (first unit of a request);
 *      ECB -- zero.
 * CTR, ECB and CBC-decryption requests become tiles of the context's tile
 * size (4096 bytes by default); each CBC-encryption request is one unit (a
 * serial chain), and chains are ordered longest first, chains of equal
 * length by key index. */
typedef struct aes_unit {
    uint64_t offset;
    uint32_t nbytes;
    uint32_t meta;
    uint32_t w[4];
} aes_unit_t;

typedef struct aes_plan_info {
    uint64_t n_units_cbc_dec;  /* decryption-table tiles: CBC and ECB decryption */
    uint64_t n_units_ctr;      /* encryption-table tiles: CTR, then ECB encryption */
    uint64_t n_chains_cbc_enc;
    uint64_t payload_bytes; /* sum of request lengths */
    uint64_t extent_bytes;  /* max(offset + length) */
    uint32_t tile_bytes;
    uint32_t reserved;
} aes_plan_info_t;

/* Validates reqs (same rules as aes_batch) for buffers of buf_bytes bytes and
 * n_scheds schedules, plans them and uploads the unit table (synchronously).
 * On a AES_DEVICE_NONE context the plan is host-only (inspectable, not
 * launchable).  Errors: as aes_batch. */
int aes_plan_create(aes_ctx_t *ctx, const aes_req_t *reqs, uint64_t n_reqs, uint32_t n_scheds,
                    uint64_t buf_bytes, aes_plan_t **out);
/* Launches a plan on stream over buffers of the plan's buf_bytes.  d_in may
 * equal d_out (in-place).  Launches of one plan (or replays of a graph made
 * from it) must not overlap in time: the tile kernels' work counters live in
 * the plan, so issue them on one stream or order them with events.  Errors:
 * AES_ERR_ARG, AES_ERR_OVERLAP, AES_ERR_DEVICE. */
int aes_plan_launch(aes_plan_t *plan, const aes_schedule_t *d_scheds, const uint8_t *d_in,
                    uint8_t *d_out, void *stream);
int aes_plan_info(const aes_plan_t *plan, aes_plan_info_t *info);
/* Copies up to max unit records (CBC- and ECB-decrypt tiles in request order,
 * then CTR tiles, then ECB-encrypt tiles, then chains longest first, those of
 * equal length by key index) to out and sets *n_out to the plan's total unit count.
 * CTR and ECB-encrypt tiles are in request order, or, when the context's CTR
 * variant was AES_CTR_BITSLICE at planning time, grouped by key with request
 * order kept within a key; decryption tiles likewise with AES_DEC_BITSLICE. */
int aes_plan_units(const aes_plan_t *plan, aes_unit_t *out, uint64_t max, uint64_t *n_out);
/* Waits for the device to be idle, then frees the plan.  NULL is a no-op. */
void aes_plan_destroy(aes_plan_t *plan);

/* ------------------------------------------------------- launch configuration */

/* Kernel shapes of a context; read at every launch (tile_bytes when a plan is
 * created).  Defaults: tile 4096, CTR tiles 2 blocks per lane x 1024 threads,
 * CBC-decrypt tiles 2 blocks per lane x 1024 threads, chains four lanes each
 * (chain_quad = 1; chain_lanes = 64 when it is 0) x 256 threads, fused kernel
 * 1 block per lane, fuse = 1, grid = 0 (one workgroup per compute unit),
 * ctr_variant = AES_CTR_TABLE. */
typedef struct aes_launch_config {
    uint32_t tile_bytes;  /* bytes per CTR / CBC-decrypt unit: multiple of 1024 */
    uint32_t ctr_nb;      /* CTR tile kernel: 16-byte blocks per lane per step (1, 2, 4) */
    uint32_t ctr_wg;      /* CTR tile kernel: threads per workgroup (256, 512, 1024) */
    uint32_t dec_nb;      /* CBC-decrypt tile kernel: as ctr_nb */
    uint32_t dec_wg;      /* CBC-decrypt tile kernel: as ctr_wg */
    uint32_t chain_lanes; /* CBC-encrypt: chains (active lanes) per wave, 1..64 */
    uint32_t chain_wg;    /* CBC-encrypt chain kernel: threads per workgroup */
    uint32_t mixed_nb;    /* fused mixed-batch kernel: blocks per lane (1, 2) */
    uint32_t fuse;        /* 1: a batch mixing CBC-encrypt chains with tiles runs as one launch
                             (batches without chains always run one launch per table set);
                             0: one launch per op */
    uint32_t grid;        /* workgroups of tile and fused kernels; 0 = one per compute unit */
    uint32_t ctr_variant; /* CTR units of batches and plans: AES_CTR_TABLE or AES_CTR_BITSLICE */
    uint32_t chain_quad;  /* CBC-encrypt chains: 0 = chain_lanes chains per wave, one lane each;
                             1 = 16 chains per wave, four lanes each (one state column per
                             lane: a quarter of the lookups per lane per round) */
    uint32_t dec_variant; /* CBC- and ECB-decrypt units of batches and plans: AES_DEC_TABLE or
                             AES_DEC_BITSLICE (not tuned: aes_tune and its cache keep it) */
    uint32_t reserved[3];
} aes_launch_config_t;

/* CTR kernel variants.  AES_CTR_TABLE: round tables in LDS, one block per
 * lane per step (paper section 3.2).  AES_CTR_BITSLICE: no tables; each lane
 * holds 32 counter blocks as 128 bit planes and computes SubBytes as a Boolean
 * circuit over the tower field GF((2^4)^2); the planner orders CTR tiles by
 * key so that the 8 tiles a wave works share one key schedule.  Per-request
 * launches and the serving engines always use the table kernels. */
#define AES_CTR_TABLE 0u
#define AES_CTR_BITSLICE 1u
/* Decryption kernel variants (CBC and ECB decryption; FIPS-197 5.3).
 * AES_DEC_TABLE: the equivalent inverse cipher with round tables in LDS.
 * AES_DEC_BITSLICE: the inverse cipher on 32 blocks per lane as bit planes,
 * the inverse S-box as a tower-field circuit; the planner orders decryption
 * tiles by key.  Per-request launches and the serving engines always use
 * the table kernels. */
#define AES_DEC_TABLE 0u
#define AES_DEC_BITSLICE 1u

int aes_ctx_get_config(const aes_ctx_t *ctx, aes_launch_config_t *cfg);
/* Errors: AES_ERR_ARG for an unsupported shape (nothing changes). */
int aes_ctx_set_config(aes_ctx_t *ctx, const aes_launch_config_t *cfg);

/* Autotuner: times plan launches of reqs on the caller's buffers (d_in must
 * differ from d_out; d_out is overwritten with the batch's result) by
 * coordinate descent from ctx's current configuration (each candidate: one
 * untimed launch, then the median of iters timed launches), one knob at a
 * time and only over knobs the batch's launch uses: the tile size (batches
 * with tiles), the fusion switch (chains mixed with tiles), the tile-kernel
 * shapes (unfused launches of table tiles), the fused kernel's blocks per
 * lane (fused launches), chain lanes or four-lane chains (batches with
 * CBC-encrypt chains) and the CTR variant (batches with CTR requests).  A
 * candidate replaces the best so far only when it is more than 2% faster,
 * so knobs that do not change the batch's time keep their starting values.  Leaves the chosen
 * configuration set in ctx and copies it to *best (may be NULL).  Plans
 * created afterwards use its tile size.
 *
 * Tune cache: when the environment variable AESGPU_TUNE_CACHE names a file,
 * the batch's signature (aes_tune_key) is looked up there first; a stored
 * configuration that the library supports is set and returned without any
 * launch (also on a host-only context).  Otherwise the tuner runs and stores
 * its result under the signature.  The file is text, one entry per line:
 * the signature, a TAB, and the twelve configuration fields tile_bytes ..
 * chain_quad as decimal numbers; '#' starts a comment line; lines that do
 * not parse are skipped; writes replace the signature's entry and go
 * through a temporary file renamed over the cache.  A file that cannot be
 * read counts as empty, one that cannot be written is left as it was.
 *
 * Errors: as aes_batch; AES_ERR_OVERLAP if d_in == d_out; AES_ERR_DEVICE
 * on a host-only context without a cached entry. */
int aes_tune(aes_ctx_t *ctx, const aes_req_t *reqs, uint64_t n_reqs, uint32_t n_scheds,
             uint64_t buf_bytes, const aes_schedule_t *d_scheds, const uint8_t *d_in,
             uint8_t *d_out, uint32_t iters, aes_launch_config_t *best);

/* The tune cache's signature of a batch (the batched service of paper
 * sections 2 and 3.3 is tuned per batch shape), as a NUL-terminated string in buf
 * (cap bytes): the device architecture and compute-unit count of ctx ("host"
 * and 0 for a host-only context), and size classes 2^k = floor(log2) ("-" for
 * zero) of the request count, of the requests per op (CBC-enc, CBC-dec,
 * CTR, ECB-enc, ECB-dec), of the total payload, of the shortest and longest
 * non-empty request, and of n_scheds.  *len_out (may be NULL) receives the
 * signature's length without the NUL.  Errors: AES_ERR_ARG for a NULL
 * argument or cap <= length (then *len_out still holds the length). */
int aes_tune_key(const aes_ctx_t *ctx, const aes_req_t *reqs, uint64_t n_reqs, uint32_t n_scheds,
                 char *buf, size_t cap, size_t *len_out);

/* ------------------------------------------------ per-request launches, graphs */

/* One request, one kernel launch, with the request passed by value (no unit
 * table, no copy): the plain per-call form that batching is compared with
 * (paper section 3.1: every GPU call pays a launch).  Same checks as
 * aes_batch for one request. */
int aes_request_launch(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                       const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                       const aes_req_t *req, void *stream);

/* aes_request_launch for each of n_reqs requests in turn (all validated
 * first, including disjointness), issued back to back on stream. */
int aes_request_launches(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                         const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                         const aes_req_t *reqs, uint64_t n_reqs, void *stream);

/* An instantiated HIP graph owned by the library. */
typedef struct aes_graph aes_graph_t;

/* Captures one launch of a plan (with these buffers) into a graph; its
 * replays count as launches of the plan (they must not overlap them). */
int aes_plan_graph(aes_plan_t *plan, const aes_schedule_t *d_scheds, const uint8_t *d_in,
                   uint8_t *d_out, aes_graph_t **out);
/* Captures n_reqs per-request launches (aes_request_launch) into one graph. */
int aes_requests_graph(aes_ctx_t *ctx, const aes_schedule_t *d_scheds, uint32_t n_scheds,
                       const uint8_t *d_in, uint8_t *d_out, uint64_t buf_bytes,
                       const aes_req_t *reqs, uint64_t n_reqs, aes_graph_t **out);
/* Launches a graph on stream.  Errors: AES_ERR_ARG, AES_ERR_DEVICE. */
int aes_graph_launch(aes_graph_t *graph, void *stream);
void aes_graph_destroy(aes_graph_t *graph);

/* ------------------------------------------------------------------ serving */

/* The serving form of paper sections 3.1-3.2: requests are posted one by one
 * while the GPU runs, each gets a ticket, and completions come back as they
 * finish (callback, poll, or blocking wait).  Two engines share this API:
 *   AES_SERVE_PERSISTENT: the paper's Non-Stop Kernel -- one kernel launched
 *     once (and again on demand after an idle exit) polls a ring of request
 *     descriptors in pinned host-mapped memory, keeps the cipher tables in
 *     LDS and the key schedules resident in HBM, splits each request into
 *     work units that idle waves claim (continuous batching: requests that
 *     arrive while others run are taken as soon as their descriptors land),
 *     and writes each completion into host-mapped memory.  Requests larger
 *     than max_request_bytes take a normal launch instead, as the paper's
 *     NSK does for services that need more threads.
 *   AES_SERVE_PER_LAUNCH: one kernel launch per request on a pool of
 *     streams (the baseline the paper compares the NSK with).
 * Payloads are buffers owned by the caller (d_src, d_dst: equal or
 * disjoint) that must stay valid until the request completes: device memory,
 * or pinned host memory from aes_server_host_alloc (either side, or both).
 * Host payloads (the paper's request path of section 3.2, with the pinned
 * region that section 4 proposes callers allocate in directly):
 *   persistent engine -- the kernel's waves load the input from and store
 *     the output to the pinned pages over the host link, so the copy-in,
 *     rounds and copy-out of different requests overlap with no copy
 *     commands and no staging;
 *   per-launch engine -- host_xfer = AES_XFER_COPY (default): each stream
 *     copies the input into its own HBM staging buffer, launches, and copies
 *     the output back (three commands in stream order, the traditional way
 *     the paper measures against); AES_XFER_DIRECT: the launched kernel
 *     reads and writes the pinned pages as the persistent engine does.
 *     Requests larger than max_request_bytes always go direct.
 * Admission: at most ring_slots requests and hbm_cap_bytes request bytes in
 * flight; beyond that aes_server_submit returns AES_ERR_AGAIN. */
typedef struct aes_server aes_server_t;

enum { AES_SERVE_PERSISTENT = 0, AES_SERVE_PER_LAUNCH = 1 };
enum { AES_XFER_COPY = 0, AES_XFER_DIRECT = 1 };

typedef struct aes_server_config {
    uint32_t mode;              /* AES_SERVE_PERSISTENT (default) or AES_SERVE_PER_LAUNCH */
    uint32_t ring_slots;        /* power of two, 64..65536 (default 4096) */
    uint32_t key_slots;         /* resident key schedules, 1..65536 (default 256) */
    uint32_t n_workgroups;      /* persistent grid of 512-thread workgroups, each holding a
                                   whole compute unit's LDS; 0 = seven eighths of the compute
                                   units (224 of 256); at most the workgroups the device holds
                                   at once (the compute units), else AES_ERR_ARG.  A grid that
                                   fills a shader engine (above 224 on a 256-CU device) holds
                                   back every kernel launched on the device beside it until
                                   the persistent kernel exits.  1 = one workgroup with the
                                   encryption tables only (CTR, ECB and CBC encryption in the
                                   kernel; decryption requests take a normal launch) */
    uint32_t dec_workgroups;    /* of those, workgroups holding decryption tables; 0 = half;
                                   1 .. n_workgroups - 1, and 0 when n_workgroups is 1 */
    uint32_t n_streams;         /* per-launch engine: stream pool (default 8) */
    uint32_t queue_units;       /* persistent engine: device queue capacity in work units per
                                   table set, power of two (default 65536) */
    uint32_t idle_timeout_ms;   /* persistent kernel exits after this long without requests
                                   (default 1000); the next submit launches it again */
    uint64_t hbm_cap_bytes;     /* admission cap on in-flight request bytes (default 256 MiB) */
    uint64_t max_request_bytes; /* larger requests take a normal launch (default 4 MiB) */
    uint32_t host_xfer;         /* per-launch engine, host payloads: AES_XFER_COPY (default,
                                   through n_streams HBM staging buffers of max_request_bytes)
                                   or AES_XFER_DIRECT */
    uint32_t reserved[7];
} aes_server_config_t;

/* One completion.  Times: host steady clock in ns (t_submit_ns when the
 * request was posted -- or its intended arrival time in aes_server_replay --
 * and t_done_ns when the host observed the completion); gpu_*_ticks are the
 * device's 100 MHz clock when the persistent kernel dispatched the request
 * and when its last unit finished (0 in the per-launch engine). */
typedef struct aes_done {
    uint64_t ticket;
    int32_t status; /* AES_OK, or the request's error */
    uint32_t units; /* work units the request was cut into (persistent engine) */
    uint64_t t_submit_ns;
    uint64_t t_done_ns;
    uint64_t gpu_dispatch_ticks;
    uint64_t gpu_done_ticks;
} aes_done_t;

/* Called on the library's completion thread; must not call back into the
 * same server except aes_server_submit. */
typedef void (*aes_done_cb)(const aes_done_t *done, void *user);

typedef struct aes_server_stats {
    uint64_t submitted, completed, rejected_again, fallbacks, kernel_launches;
    uint64_t in_flight, in_flight_bytes;
    uint64_t host_routed; /* requests run on the host route (size-based dispatch) */
} aes_server_stats_t;

/* cfg may be NULL (defaults).  The persistent kernel is launched by the first
 * submit, not here.  While it runs, its workgroups occupy n_workgroups compute
 * units; kernels of other calls on the device share the rest.
 * Errors: AES_ERR_ARG, AES_ERR_DEVICE, AES_ERR_NOMEM. */
int aes_server_create(aes_ctx_t *ctx, const aes_server_config_t *cfg, aes_server_t **out);
/* Copies a schedule into resident slot `slot` (synchronously).  Allowed while
 * nothing is in flight (else AES_ERR_STATE); a running persistent kernel is
 * stopped first (AES_ERR_TIMEOUT if it does not exit within 10 s) and
 * relaunched by the next submit.  The schedule's round count must match its
 * key size (10, 12, 14 for 128, 192, 256 bits), else AES_ERR_KEYSIZE: the
 * persistent engine takes the round count recorded here with each request. */
int aes_server_set_key(aes_server_t *srv, uint32_t slot, const aes_schedule_t *host_sched);
/* Posts one request (paper section 3.2: buffers, a service request, an
 * optional completion callback).  op and iv as in aes_req_t (iv may be NULL
 * for ECB); length > 0, < 2^32, a multiple of 16 for CBC and ECB.  Sets
 * *ticket.  Errors: AES_ERR_ARG, AES_ERR_LENGTH, AES_ERR_RANGE (key slot, or
 * a range that starts inside a buffer from aes_server_host_alloc and runs
 * past its end), AES_ERR_STATE (the key slot was never loaded with
 * aes_server_set_key), AES_ERR_OVERLAP, AES_ERR_AGAIN (admission),
 * AES_ERR_DEVICE. */
int aes_server_submit(aes_server_t *srv, uint32_t op, uint32_t key_slot, const uint8_t iv[16],
                      const uint8_t *d_src, uint8_t *d_dst, uint64_t length, aes_done_cb cb,
                      void *user, uint64_t *ticket);
/* Non-blocking: moves up to max finished completions (of requests posted
 * without a callback) to out, oldest first. */
int aes_server_poll(aes_server_t *srv, aes_done_t *out, uint32_t max, uint32_t *n_out);
/* Blocks until `ticket` (posted without a callback) completes, then moves its
 * completion to *out (may be NULL).  The calling thread spins for up to
 * 200 us (or timeout_ns, if shorter) before it sleeps, so a short request
 * does not pay an operating-system wake-up; the server's completion thread
 * likewise spins for 200 us after its last request before it sleeps.
 * Errors: AES_ERR_TIMEOUT, AES_ERR_ARG (unknown ticket). */
int aes_server_wait(aes_server_t *srv, uint64_t ticket, uint64_t timeout_ns, aes_done_t *out);
/* Open-loop replay of a request trace: request i (offset into both bases,
 * length, key slot in key_idx, op, iv) is posted at arrival_s[i] seconds
 * after the call starts, retried while admission says AES_ERR_AGAIN; the call
 * returns when all have completed, with out[i] its completion (t_submit_ns =
 * the arrival time, so latency includes any admission wait). */
int aes_server_replay(aes_server_t *srv, const aes_req_t *reqs, const double *arrival_s,
                      uint64_t n, const uint8_t *d_src_base, uint8_t *d_dst_base,
                      aes_done_t *out);
int aes_server_stats(aes_server_t *srv, aes_server_stats_t *out);
/* Allocates `bytes` (> 0) of pinned host memory mapped into the server's
 * device, for request payloads (paper section 4: callers allocate in the
 * pinned region and save a copy).  *host_ptr is an ordinary host pointer;
 * pass pointers into the buffer to aes_server_submit or aes_server_replay
 * (a request's range must lie inside one buffer).  The buffer is owned by
 * the server: freed by aes_server_host_free or aes_server_destroy.
 * Errors: AES_ERR_ARG, AES_ERR_NOMEM, AES_ERR_DEVICE. */
int aes_server_host_alloc(aes_server_t *srv, uint64_t bytes, void **host_ptr);
/* Frees a buffer from aes_server_host_alloc.  Allowed while nothing is in
 * flight (else AES_ERR_STATE); AES_ERR_ARG if host_ptr is not such a
 * buffer's start. */
int aes_server_host_free(aes_server_t *srv, void *host_ptr);

/* Size-based CPU/GPU dispatch (paper section 4: calling the GPU has a fixed
 * cost, so small tasks can finish sooner on the CPU; the crossover depends on
 * the task and the machine and is best measured at start-up).  With a
 * crossover set for op, aes_server_submit and aes_server_replay run a request
 * of that op on the host route -- AES-NI on the submitting thread,
 * aes_host_route_crypt -- when its length is below the crossover, its key
 * slot has been set, and both its source and destination lie in buffers from
 * aes_server_host_alloc.  Such a request completes before submit returns
 * (its callback, if any, runs on the submitting thread).  Every other request
 * goes to the GPU engine.  Off by default: every crossover is 0.
 * Errors: AES_ERR_ARG (null server or pointer, op > AES_OP_ECB_DEC). */
int aes_server_set_crossover(aes_server_t *srv, uint32_t op, uint64_t bytes);
int aes_server_get_crossover(aes_server_t *srv, uint32_t op, uint64_t *bytes);
/* Measures the crossovers on this machine and sets them.  For CTR, CBC
 * decryption and CBC encryption (ECB encryption takes CTR's value, ECB
 * decryption CBC decryption's): one request at a time at 4 KiB, 8 KiB, ...
 * up to min(max_request_bytes, 4 MiB) -- 256 KiB for CBC encryption, whose
 * chain is serial on both sides -- timing the median of 5 round trips
 * (submit to observed completion) through this server's GPU engine against
 * the median of 5 host-route runs, with payloads in pinned host buffers and
 * schedule key_slot (set beforehand).  A crossover is the smallest tested
 * size from which the GPU engine is faster at every larger tested size, or
 * UINT64_MAX when it is faster at none (every such request then runs on the
 * host).  out (may be NULL) receives the five values, indexed by op.  Allowed
 * while nothing is in flight (else AES_ERR_STATE).  Errors: AES_ERR_ARG,
 * AES_ERR_RANGE (key slot out of range or never set), AES_ERR_DEVICE (no AES
 * instructions on the host, or a GPU error), AES_ERR_NOMEM. */
int aes_server_calibrate(aes_server_t *srv, uint32_t key_slot, uint64_t out[5]);

/* The host route on its own: one request (op and iv as in aes_req_t; iv may
 * be NULL for ECB) with a host-memory schedule and host-memory payloads
 * (src == dst, or disjoint), on the calling thread with the CPU's AES
 * instructions.  Pure host function.  Errors: AES_ERR_ARG, AES_ERR_KEYSIZE
 * (nr and key_bits not one of 10/128, 12/192, 14/256), AES_ERR_LENGTH,
 * AES_ERR_OVERLAP, AES_ERR_DEVICE (the CPU has no AES instructions). */
int aes_host_route_crypt(const aes_schedule_t *sched, uint32_t op, const uint8_t *iv,
                         const uint8_t *src, uint8_t *dst, uint64_t length);

/* A whole batch on the host route (paper section 3.3 sets the GPU service
 * against AES on the CPU; section 4 proposes running work the GPU would do
 * no faster on the CPU): the requests, buffer rules and results of
 * aes_batch, with host-memory schedules (n_scheds records) and host-memory
 * in/out buffers of buf_bytes each (in == out, or disjoint), run by
 * n_threads host threads (0 = as many as the CPUs this process may run on;
 * the calling thread is one of them), each taking the next request.  A CPU baseline for the GPU
 * forms and a CPU path for callers without a GPU; not the oracle.  Returns
 * when every request is done.  Errors: those of aes_batch's validation
 * (nothing runs), AES_ERR_ARG for n_threads > 1024; then, if requests failed
 * on the host route (a schedule whose round count does not match its key
 * size: that request's bytes stay untouched; AES_ERR_DEVICE without AES
 * instructions), the error of the lowest-numbered failed request after the
 * others have run. */
int aes_host_batch(const aes_schedule_t *scheds, uint32_t n_scheds, const uint8_t *in,
                   uint8_t *out, uint64_t buf_bytes, const aes_req_t *reqs, uint64_t n_reqs,
                   uint32_t n_threads);
/* Waits (up to 10 s) for in-flight requests, stops the persistent kernel
 * (waiting up to 10 s for it to exit) and frees the server; the handle is
 * invalid afterwards in every case.  Returns AES_ERR_TIMEOUT if requests were
 * still in flight or the kernel did not exit; in the second case the memory
 * and stream that kernel may still use are left allocated (leaked), not freed
 * under it. */
int aes_server_destroy(aes_server_t *srv);

#ifdef __cplusplus
}
#endif

#endif /* AESGPU_H */
