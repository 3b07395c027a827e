/*
 * aes_oracle.c -- plain, slow, obviously correct CPU AES.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity authority for the GPU
 * library: only the test suite, the package's smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, table or header with the
 * GPU path.
 *
 * What it follows (the paper, section 3.3, offers AES as a GPU service for
 * the kernel's crypto layer but fixes no key size or mode beyond ECB, so the
 * arithmetic below is the standards' definitions written out):
 *   - FIPS-197 section 4.2 (GF(2^8) multiplication, xtime),
 *     section 5.1.1 (S-box = affine map of the multiplicative inverse),
 *     section 5.1 (Cipher), section 5.2 (KeyExpansion),
 *     section 5.3 (InvCipher, the straightforward form -- not the equivalent
 *     inverse cipher the GPU kernels use).
 *   - NIST SP 800-38A section 6.1 (ECB), section 6.2 (CBC) and section 6.5
 *     with appendix B.1
 *     (CTR, counter incremented on the low m = 64 bits, big-endian, mod 2^64,
 *     no carry into the high 64 bits; a final partial block uses the leading
 *     bytes of the last keystream block).
 *
 * Nothing is tabulated by hand: the S-box is built at first use from its
 * definition, with each inverse found by brute force over all 255 candidates.
 * The state is a 4x4 byte array s[r][c] = in[r + 4c] exactly as FIPS-197 lays
 * it out; every step loops over rows and columns.  It is meant to be read
 * against the standard, not to be fast.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <pthread.h>
#include <unistd.h>

#define ORACLE_OK 0
#define ORACLE_ERR_ARG (-1)
#define ORACLE_ERR_KEYSIZE (-2)
#define ORACLE_ERR_LENGTH (-3)
#define ORACLE_ERR_RANGE (-4)

#define OP_CBC_ENC 0
#define OP_CBC_DEC 1
#define OP_CTR 2
#define OP_ECB_ENC 3
#define OP_ECB_DEC 4

/* One request of a batch: bytes [offset, offset+length) of the input buffer
 * are transformed into the same byte range of the output buffer. */
typedef struct {
    uint64_t offset;
    uint64_t length;
    uint32_t key_idx;
    uint32_t op;
    uint8_t iv[16];
} oracle_req_t;

static uint8_t SBOX[256];
static uint8_t INV_SBOX[256];
static pthread_once_t sbox_once = PTHREAD_ONCE_INIT;

/* FIPS-197 4.2.1: multiplication by x modulo m(x) = x^8 + x^4 + x^3 + x + 1. */
static uint8_t xtime(uint8_t b)
{
    return (uint8_t)((b << 1) ^ ((b & 0x80) ? 0x1b : 0x00));
}

/* FIPS-197 4.2: product in GF(2^8) by repeated xtime and addition (XOR). */
static uint8_t gmul(uint8_t a, uint8_t b)
{
    uint8_t p = 0;
    while (b) {
        if (b & 1)
            p ^= a;
        a = xtime(a);
        b >>= 1;
    }
    return p;
}

/* FIPS-197 5.1.1: S(a) = affine(inverse(a)), inverse(0) = 0, constant c = 0x63,
 * b'_i = b_i ^ b_(i+4) ^ b_(i+5) ^ b_(i+6) ^ b_(i+7) ^ c_i (indices mod 8). */
static void build_sbox(void)
{
    for (int a = 0; a < 256; a++) {
        int inv = 0;
        if (a != 0) {
            for (int cand = 1; cand < 256; cand++) {
                if (gmul((uint8_t)a, (uint8_t)cand) == 1) {
                    inv = cand;
                    break;
                }
            }
        }
        int s = 0;
        for (int i = 0; i < 8; i++) {
            int bit = ((inv >> i) ^ (inv >> ((i + 4) % 8)) ^ (inv >> ((i + 5) % 8)) ^
                       (inv >> ((i + 6) % 8)) ^ (inv >> ((i + 7) % 8)) ^ (0x63 >> i)) & 1;
            s |= bit << i;
        }
        SBOX[a] = (uint8_t)s;
    }
    for (int a = 0; a < 256; a++)
        INV_SBOX[SBOX[a]] = (uint8_t)a;
}

static void init(void) { pthread_once(&sbox_once, build_sbox); }

static int rounds_for(uint32_t key_bits)
{
    switch (key_bits) {
    case 128: return 10;
    case 192: return 12;
    case 256: return 14;
    default: return -1;
    }
}

/* FIPS-197 5.2 KeyExpansion.  w holds 4*(Nr+1) words, each word as its four
 * bytes in order (w[i][0] is the first byte).  Returns Nr or -1. */
static int key_expansion(const uint8_t *key, uint32_t key_bits, uint8_t w[60][4])
{
    int nr = rounds_for(key_bits);
    if (nr < 0)
        return -1;
    int nk = (int)key_bits / 32;
    int total = 4 * (nr + 1);
    for (int i = 0; i < nk; i++)
        for (int j = 0; j < 4; j++)
            w[i][j] = key[4 * i + j];
    uint8_t rcon = 0x01; /* Rcon[i/Nk] = (x^(i/Nk - 1), 0, 0, 0) */
    for (int i = nk; i < total; i++) {
        uint8_t temp[4];
        memcpy(temp, w[i - 1], 4);
        if (i % nk == 0) {
            uint8_t t0 = temp[0]; /* RotWord */
            temp[0] = temp[1];
            temp[1] = temp[2];
            temp[2] = temp[3];
            temp[3] = t0;
            for (int j = 0; j < 4; j++) /* SubWord */
                temp[j] = SBOX[temp[j]];
            temp[0] ^= rcon;
            rcon = xtime(rcon);
        } else if (nk > 6 && i % nk == 4) {
            for (int j = 0; j < 4; j++)
                temp[j] = SBOX[temp[j]];
        }
        for (int j = 0; j < 4; j++)
            w[i][j] = w[i - nk][j] ^ temp[j];
    }
    return nr;
}

/* FIPS-197 5.1.4 AddRoundKey: column c of the state is XORed with word
 * w[round*4 + c]. */
static void add_round_key(uint8_t s[4][4], uint8_t w[60][4], int round)
{
    for (int c = 0; c < 4; c++)
        for (int r = 0; r < 4; r++)
            s[r][c] ^= w[round * 4 + c][r];
}

/* FIPS-197 5.1.1 SubBytes / 5.3.2 InvSubBytes. */
static void sub_bytes(uint8_t s[4][4], const uint8_t box[256])
{
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            s[r][c] = box[s[r][c]];
}

/* FIPS-197 5.1.2 ShiftRows: row r is rotated left by r positions,
 * s'[r][c] = s[r][(c + r) mod 4]. */
static void shift_rows(uint8_t s[4][4])
{
    for (int r = 1; r < 4; r++) {
        uint8_t t[4];
        for (int c = 0; c < 4; c++)
            t[c] = s[r][(c + r) % 4];
        for (int c = 0; c < 4; c++)
            s[r][c] = t[c];
    }
}

/* FIPS-197 5.3.1 InvShiftRows: s'[r][(c + r) mod 4] = s[r][c]. */
static void inv_shift_rows(uint8_t s[4][4])
{
    for (int r = 1; r < 4; r++) {
        uint8_t t[4];
        for (int c = 0; c < 4; c++)
            t[(c + r) % 4] = s[r][c];
        for (int c = 0; c < 4; c++)
            s[r][c] = t[c];
    }
}

/* FIPS-197 5.1.3 MixColumns: each column times the circulant (02 03 01 01). */
static void mix_columns(uint8_t s[4][4])
{
    for (int c = 0; c < 4; c++) {
        uint8_t a0 = s[0][c], a1 = s[1][c], a2 = s[2][c], a3 = s[3][c];
        s[0][c] = gmul(a0, 2) ^ gmul(a1, 3) ^ a2 ^ a3;
        s[1][c] = a0 ^ gmul(a1, 2) ^ gmul(a2, 3) ^ a3;
        s[2][c] = a0 ^ a1 ^ gmul(a2, 2) ^ gmul(a3, 3);
        s[3][c] = gmul(a0, 3) ^ a1 ^ a2 ^ gmul(a3, 2);
    }
}

/* FIPS-197 5.3.3 InvMixColumns: each column times the circulant (0e 0b 0d 09). */
static void inv_mix_columns(uint8_t s[4][4])
{
    for (int c = 0; c < 4; c++) {
        uint8_t a0 = s[0][c], a1 = s[1][c], a2 = s[2][c], a3 = s[3][c];
        s[0][c] = gmul(a0, 0x0e) ^ gmul(a1, 0x0b) ^ gmul(a2, 0x0d) ^ gmul(a3, 0x09);
        s[1][c] = gmul(a0, 0x09) ^ gmul(a1, 0x0e) ^ gmul(a2, 0x0b) ^ gmul(a3, 0x0d);
        s[2][c] = gmul(a0, 0x0d) ^ gmul(a1, 0x09) ^ gmul(a2, 0x0e) ^ gmul(a3, 0x0b);
        s[3][c] = gmul(a0, 0x0b) ^ gmul(a1, 0x0d) ^ gmul(a2, 0x09) ^ gmul(a3, 0x0e);
    }
}

/* FIPS-197 5.1 Cipher. */
static void cipher(const uint8_t in[16], uint8_t out[16], uint8_t w[60][4], int nr)
{
    uint8_t s[4][4];
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            s[r][c] = in[r + 4 * c];
    add_round_key(s, w, 0);
    for (int round = 1; round < nr; round++) {
        sub_bytes(s, SBOX);
        shift_rows(s);
        mix_columns(s);
        add_round_key(s, w, round);
    }
    sub_bytes(s, SBOX);
    shift_rows(s);
    add_round_key(s, w, nr);
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            out[r + 4 * c] = s[r][c];
}

/* FIPS-197 5.3 InvCipher (straightforward order). */
static void inv_cipher(const uint8_t in[16], uint8_t out[16], uint8_t w[60][4], int nr)
{
    uint8_t s[4][4];
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            s[r][c] = in[r + 4 * c];
    add_round_key(s, w, nr);
    for (int round = nr - 1; round >= 1; round--) {
        inv_shift_rows(s);
        sub_bytes(s, INV_SBOX);
        add_round_key(s, w, round);
        inv_mix_columns(s);
    }
    inv_shift_rows(s);
    sub_bytes(s, INV_SBOX);
    add_round_key(s, w, 0);
    for (int r = 0; r < 4; r++)
        for (int c = 0; c < 4; c++)
            out[r + 4 * c] = s[r][c];
}

/* SP 800-38A 6.2: C_1 = E(P_1 ^ IV), C_j = E(P_j ^ C_(j-1)).  len % 16 == 0. */
static void cbc_encrypt(const uint8_t *in, uint8_t *out, uint64_t len, const uint8_t iv[16],
                        uint8_t w[60][4], int nr)
{
    uint8_t prev[16], x[16];
    memcpy(prev, iv, 16);
    for (uint64_t j = 0; j < len; j += 16) {
        for (int b = 0; b < 16; b++)
            x[b] = in[j + b] ^ prev[b];
        cipher(x, prev, w, nr);
        memcpy(out + j, prev, 16);
    }
}

/* SP 800-38A 6.2: P_j = D(C_j) ^ C_(j-1), C_0 = IV.  Safe when in == out
 * because C_j is copied before P_j is written. */
static void cbc_decrypt(const uint8_t *in, uint8_t *out, uint64_t len, const uint8_t iv[16],
                        uint8_t w[60][4], int nr)
{
    uint8_t prev[16], cur[16], x[16];
    memcpy(prev, iv, 16);
    for (uint64_t j = 0; j < len; j += 16) {
        memcpy(cur, in + j, 16);
        inv_cipher(cur, x, w, nr);
        for (int b = 0; b < 16; b++)
            out[j + b] = x[b] ^ prev[b];
        memcpy(prev, cur, 16);
    }
}

/* SP 800-38A 6.5 CTR with the standard incrementing function of appendix B.1
 * applied to the low m = 64 bits: T_j = nonce || ((low(T_1) + j - 1) mod 2^64),
 * the low half read and written big-endian.  O_j = E(T_j), C_j = P_j ^ O_j; a
 * final partial block of u bytes uses the first u bytes of O_n.  Decryption
 * is the same operation. */
static void ctr_xcrypt(const uint8_t *in, uint8_t *out, uint64_t len, const uint8_t t1[16],
                       uint8_t w[60][4], int nr)
{
    uint64_t low = 0;
    for (int b = 8; b < 16; b++)
        low = (low << 8) | t1[b];
    uint8_t t[16], o[16];
    memcpy(t, t1, 8);
    for (uint64_t j = 0; j < len; j += 16) {
        uint64_t ctr = low + j / 16; /* wraps mod 2^64; the nonce half is untouched */
        for (int b = 0; b < 8; b++)
            t[15 - b] = (uint8_t)(ctr >> (8 * b));
        cipher(t, o, w, nr);
        uint64_t n = len - j < 16 ? len - j : 16;
        for (uint64_t b = 0; b < n; b++)
            out[j + b] = in[j + b] ^ o[b];
    }
}

/* ---------------------------------------------------------------- exports */

/* Writes the S-box and its inverse. */
void oracle_sbox(uint8_t sbox[256], uint8_t inv_sbox[256])
{
    init();
    memcpy(sbox, SBOX, 256);
    memcpy(inv_sbox, INV_SBOX, 256);
}

/* Writes the 4*(Nr+1) expanded-key words as bytes (16*(Nr+1) bytes, word i
 * at w_bytes[4i..4i+3]) and returns Nr, or ORACLE_ERR_KEYSIZE. */
int oracle_expand_key(const uint8_t *key, uint32_t key_bits, uint8_t *w_bytes)
{
    init();
    uint8_t w[60][4];
    int nr = key_expansion(key, key_bits, w);
    if (nr < 0)
        return ORACLE_ERR_KEYSIZE;
    memcpy(w_bytes, w, (size_t)16 * (nr + 1));
    return nr;
}

/* ECB over n whole blocks; decrypt selects InvCipher.  Blocks are processed
 * one at a time, so in == out is allowed. */
int oracle_ecb(const uint8_t *key, uint32_t key_bits, int decrypt, const uint8_t *in,
               uint8_t *out, uint64_t n_blocks)
{
    init();
    uint8_t w[60][4];
    int nr = key_expansion(key, key_bits, w);
    if (nr < 0)
        return ORACLE_ERR_KEYSIZE;
    for (uint64_t i = 0; i < n_blocks; i++) {
        uint8_t x[16];
        if (decrypt)
            inv_cipher(in + 16 * i, x, w, nr);
        else
            cipher(in + 16 * i, x, w, nr);
        memcpy(out + 16 * i, x, 16);
    }
    return ORACLE_OK;
}

/* One request of one mode on one contiguous buffer. */
int oracle_mode(uint32_t op, const uint8_t *key, uint32_t key_bits, const uint8_t iv[16],
                const uint8_t *in, uint8_t *out, uint64_t len)
{
    init();
    uint8_t w[60][4];
    int nr = key_expansion(key, key_bits, w);
    if (nr < 0)
        return ORACLE_ERR_KEYSIZE;
    switch (op) {
    case OP_CBC_ENC:
        if (len % 16)
            return ORACLE_ERR_LENGTH;
        cbc_encrypt(in, out, len, iv, w, nr);
        return ORACLE_OK;
    case OP_CBC_DEC:
        if (len % 16)
            return ORACLE_ERR_LENGTH;
        cbc_decrypt(in, out, len, iv, w, nr);
        return ORACLE_OK;
    case OP_CTR:
        ctr_xcrypt(in, out, len, iv, w, nr);
        return ORACLE_OK;
    case OP_ECB_ENC:
    case OP_ECB_DEC:
        /* SP 800-38A 6.1: every block on its own, no IV */
        if (len % 16)
            return ORACLE_ERR_LENGTH;
        for (uint64_t j = 0; j < len; j += 16) {
            uint8_t x[16];
            if (op == OP_ECB_DEC)
                inv_cipher(in + j, x, w, nr);
            else
                cipher(in + j, x, w, nr);
            memcpy(out + j, x, 16);
        }
        return ORACLE_OK;
    default:
        return ORACLE_ERR_ARG;
    }
}

/* ------------------------------------------------------------ batch driver */

typedef struct {
    const uint8_t *in;
    uint8_t *out;
    const oracle_req_t *reqs;
    uint64_t n_reqs;
    const uint8_t *keys;      /* key k at keys + 32*k (first key_bits/8 bytes used) */
    const uint32_t *key_bits; /* per key */
    uint64_t next;            /* next request to take */
    pthread_mutex_t lock;
    int status;
} batch_job_t;

static void *batch_worker(void *arg)
{
    batch_job_t *job = (batch_job_t *)arg;
    for (;;) {
        pthread_mutex_lock(&job->lock);
        uint64_t i = job->next++;
        pthread_mutex_unlock(&job->lock);
        if (i >= job->n_reqs)
            break;
        const oracle_req_t *r = &job->reqs[i];
        int st = oracle_mode(r->op, job->keys + 32 * (uint64_t)r->key_idx,
                             job->key_bits[r->key_idx], r->iv, job->in + r->offset,
                             job->out + r->offset, r->length);
        if (st != ORACLE_OK) {
            pthread_mutex_lock(&job->lock);
            job->status = st;
            pthread_mutex_unlock(&job->lock);
        }
    }
    return NULL;
}

/* Applies every request: out[off, off+len) = op(in[off, off+len)).  Bytes of
 * out outside every request are not touched.  Requests are checked first
 * (key index, key size, range, CBC length); nothing is written on error.
 * n_threads <= 0 means one thread per online CPU.  Returns the number of
 * threads used (>= 1) or a negative error. */
int oracle_batch(const uint8_t *in, uint8_t *out, uint64_t buf_bytes, const oracle_req_t *reqs,
                 uint64_t n_reqs, const uint8_t *keys, const uint32_t *key_bits, uint32_t n_keys,
                 int n_threads)
{
    init();
    for (uint64_t i = 0; i < n_reqs; i++) {
        const oracle_req_t *r = &reqs[i];
        if (r->key_idx >= n_keys || r->op > OP_ECB_DEC)
            return ORACLE_ERR_ARG;
        if (rounds_for(key_bits[r->key_idx]) < 0)
            return ORACLE_ERR_KEYSIZE;
        if (r->offset > buf_bytes || r->length > buf_bytes - r->offset)
            return ORACLE_ERR_RANGE;
        if (r->op != OP_CTR && r->length % 16)
            return ORACLE_ERR_LENGTH;
    }
    if (n_threads <= 0) {
        long n = sysconf(_SC_NPROCESSORS_ONLN);
        n_threads = n > 0 ? (int)n : 1;
    }
    if ((uint64_t)n_threads > n_reqs)
        n_threads = n_reqs ? (int)n_reqs : 1;
    if (n_threads > 512)
        n_threads = 512;
    batch_job_t job;
    job.in = in;
    job.out = out;
    job.reqs = reqs;
    job.n_reqs = n_reqs;
    job.keys = keys;
    job.key_bits = key_bits;
    job.next = 0;
    job.status = ORACLE_OK;
    pthread_mutex_init(&job.lock, NULL);
    pthread_t th[512];
    int started = 0;
    for (int t = 1; t < n_threads; t++) {
        if (pthread_create(&th[t], NULL, batch_worker, &job) != 0)
            break;
        started++;
    }
    batch_worker(&job);
    for (int t = 1; t <= started; t++)
        pthread_join(th[t], NULL);
    pthread_mutex_destroy(&job.lock);
    return job.status != ORACLE_OK ? job.status : started + 1;
}
