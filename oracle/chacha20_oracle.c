/*
 * Plain CPU oracle for MemShield's page cipher.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: it exists so that tests, the smoke check and the CPU
 * baseline leg of the benchmark can compare the GPU engine against an
 * obviously correct, slow implementation.  It shares no code, header,
 * constant table or helper with the HIP engine.
 *
 * What it computes (MemShield paper, section 4.4 "GPU encryption"):
 *   - a page is 4096 bytes and is processed as a whole;
 *   - the cipher is ChaCha with 20 rounds (the paper's "strongest variant");
 *   - one keystream block is 512 bits, made from a 384-bit seed: a 256-bit
 *     key plus a 128-bit value that holds the per-page nonce and a block
 *     counter running 0..63, the index of the 64-byte block inside the page;
 *   - the page is XORed with its 64 keystream blocks; encryption and
 *     decryption are the same operation.
 * The round function and the state layout are those of ChaCha as published
 * by Bernstein (2008) and fixed for the 96-bit-nonce form in RFC 8439,
 * sections 2.1-2.3, which the paper cites but does not restate:
 *   state = [ "expand 32-byte k" as 4 little-endian words,
 *             key as 8 little-endian words,
 *             block counter,
 *             nonce as 3 little-endian words ]
 *   a column round on (0,4,8,12) (1,5,9,13) (2,6,10,14) (3,7,11,15),
 *   a diagonal round on (0,5,10,15) (1,6,11,12) (2,7,8,13) (3,4,9,14),
 *   rounds/2 such double rounds, then the input state is added word-wise
 *   and the 16 words are written out little-endian.
 * The reading of the paper's 128-bit value is: word 12 = block counter j,
 * words 13..15 = the 96-bit page nonce.
 *
 * The engine's second cipher, Salsa20, follows further below with its own
 * block function and page loop.
 *
 * Deliberately scalar and unoptimised: byte-wise little-endian loads and
 * stores, one block at a time, no intrinsics.
 */
#include <stddef.h>
#include <stdint.h>
#include <string.h>
#include <pthread.h>

#define ORACLE_PAGE_BYTES 4096u
#define ORACLE_BLOCK_BYTES 64u
#define ORACLE_BLOCKS_PER_PAGE (ORACLE_PAGE_BYTES / ORACLE_BLOCK_BYTES)

static uint32_t read_le32(const uint8_t *p)
{
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) |
           ((uint32_t)p[3] << 24);
}

static void write_le32(uint8_t *p, uint32_t v)
{
    p[0] = (uint8_t)(v & 0xffu);
    p[1] = (uint8_t)((v >> 8) & 0xffu);
    p[2] = (uint8_t)((v >> 16) & 0xffu);
    p[3] = (uint8_t)((v >> 24) & 0xffu);
}

static uint32_t rotate_left(uint32_t v, unsigned n)
{
    return (v << n) | (v >> (32u - n));
}

/* The quarter round: add, xor, rotate by 16, 12, 8 and 7. */
static void quarter_round(uint32_t x[16], int a, int b, int c, int d)
{
    x[a] = x[a] + x[b];
    x[d] = rotate_left(x[d] ^ x[a], 16);
    x[c] = x[c] + x[d];
    x[b] = rotate_left(x[b] ^ x[c], 12);
    x[a] = x[a] + x[b];
    x[d] = rotate_left(x[d] ^ x[a], 8);
    x[c] = x[c] + x[d];
    x[b] = rotate_left(x[b] ^ x[c], 7);
}

/*
 * One 64-byte keystream block for (key, counter, nonce) after `rounds`
 * rounds (20 for ChaCha20).  `rounds` must be even and positive.
 */
void oracle_chacha_block(const uint8_t key[32], uint32_t counter,
                         const uint8_t nonce[12], int rounds, uint8_t out[64])
{
    static const char sigma[] = "expand 32-byte k";
    uint32_t input[16];
    uint32_t work[16];
    int i;

    for (i = 0; i < 4; i++)
        input[i] = read_le32((const uint8_t *)sigma + 4 * i);
    for (i = 0; i < 8; i++)
        input[4 + i] = read_le32(key + 4 * i);
    input[12] = counter;
    for (i = 0; i < 3; i++)
        input[13 + i] = read_le32(nonce + 4 * i);

    memcpy(work, input, sizeof(work));
    for (i = 0; i < rounds; i += 2) {
        /* column round */
        quarter_round(work, 0, 4, 8, 12);
        quarter_round(work, 1, 5, 9, 13);
        quarter_round(work, 2, 6, 10, 14);
        quarter_round(work, 3, 7, 11, 15);
        /* diagonal round */
        quarter_round(work, 0, 5, 10, 15);
        quarter_round(work, 1, 6, 11, 12);
        quarter_round(work, 2, 7, 8, 13);
        quarter_round(work, 3, 4, 9, 14);
    }
    for (i = 0; i < 16; i++)
        write_le32(out + 4 * i, work[i] + input[i]);
}

/* XOR one 4096-byte page with its 64 keystream blocks, counters 0..63. */
void oracle_cipher_page(const uint8_t key[32], const uint8_t nonce[12],
                        int rounds, const uint8_t *in, uint8_t *out)
{
    uint8_t ks[ORACLE_BLOCK_BYTES];
    uint32_t j, i;

    for (j = 0; j < ORACLE_BLOCKS_PER_PAGE; j++) {
        oracle_chacha_block(key, j, nonce, rounds, ks);
        for (i = 0; i < ORACLE_BLOCK_BYTES; i++)
            out[j * ORACLE_BLOCK_BYTES + i] =
                (uint8_t)(in[j * ORACLE_BLOCK_BYTES + i] ^ ks[i]);
    }
}

/*
 * n_pages pages, page p using nonces[12*p .. 12*p+11].  `in` and `out` may
 * be the same buffer.
 */
void oracle_cipher_pages(const uint8_t key[32], const uint8_t *nonces,
                         int rounds, const uint8_t *in, uint8_t *out,
                         uint64_t n_pages)
{
    uint64_t p;

    for (p = 0; p < n_pages; p++)
        oracle_cipher_page(key, nonces + 12 * p, rounds,
                           in + p * ORACLE_PAGE_BYTES,
                           out + p * ORACLE_PAGE_BYTES);
}

/* ------------------------------------------------------------------------
 * Salsa20, the engine's second cipher (the paper's modular cipher: its
 * section 1 lists modular cryptographic components among the contributions,
 * and its section 6 expects the GPU kernel to be replaceable by another
 * cipher).  Salsa20 is Bernstein's predecessor of ChaCha ("The Salsa20
 * family of stream ciphers", 2008): the same 512-bit block from a 256-bit
 * key and a 128-bit value, a different state layout and round function:
 *   state = [ c0 k0 k1 k2 | k3 c1 v0 v1 | t0 t1 c2 k4 | k5 k6 k7 c3 ]
 *   (c = "expand 32-byte k" as 4 little-endian words, k = key words,
 *    v = the 64-bit nonce, t = the 64-bit block counter, low word first);
 *   quarter round on (a, b, c, d):
 *     b ^= (a + d) <<< 7;  c ^= (b + a) <<< 9;
 *     d ^= (c + b) <<< 13; a ^= (d + c) <<< 18;
 *   a column round on (0,4,8,12) (5,9,13,1) (10,14,2,6) (15,3,7,11),
 *   a row round on (0,1,2,3) (5,6,7,4) (10,11,8,9) (15,12,13,14),
 *   rounds/2 such double rounds, then the input state is added word-wise.
 * Reading of the page's 128-bit value for this cipher: the nonce words
 * v0, v1 are the page nonce's first two words, the counter's low word t0
 * is the block index j (0..63) and its high word t1 is the page nonce's
 * third word.  As j < 64 never carries, a page is exactly Salsa20 with the
 * 8-byte nonce = page nonce bytes 0..7 and the initial block counter =
 * (page nonce word 2) * 2^32, run over 4096 bytes.
 * ------------------------------------------------------------------------ */

/* The Salsa20 quarter round on positions a, b, c, d. */
static void salsa_quarter(uint32_t x[16], int a, int b, int c, int d)
{
    x[b] ^= rotate_left(x[a] + x[d], 7);
    x[c] ^= rotate_left(x[b] + x[a], 9);
    x[d] ^= rotate_left(x[c] + x[b], 13);
    x[a] ^= rotate_left(x[d] + x[c], 18);
}

/*
 * One 64-byte Salsa20 keystream block for (key, 64-bit nonce, 64-bit
 * counter) after `rounds` rounds.  `rounds` must be even and positive.
 */
void oracle_salsa_block(const uint8_t key[32], const uint8_t nonce8[8],
                        uint64_t counter, int rounds, uint8_t out[64])
{
    static const char sigma[] = "expand 32-byte k";
    uint32_t input[16];
    uint32_t work[16];
    int i;

    input[0] = read_le32((const uint8_t *)sigma + 0);
    input[5] = read_le32((const uint8_t *)sigma + 4);
    input[10] = read_le32((const uint8_t *)sigma + 8);
    input[15] = read_le32((const uint8_t *)sigma + 12);
    for (i = 0; i < 4; i++) {
        input[1 + i] = read_le32(key + 4 * i);
        input[11 + i] = read_le32(key + 16 + 4 * i);
    }
    input[6] = read_le32(nonce8);
    input[7] = read_le32(nonce8 + 4);
    input[8] = (uint32_t)(counter & 0xffffffffu);
    input[9] = (uint32_t)(counter >> 32);

    memcpy(work, input, sizeof(work));
    for (i = 0; i < rounds; i += 2) {
        /* column round */
        salsa_quarter(work, 0, 4, 8, 12);
        salsa_quarter(work, 5, 9, 13, 1);
        salsa_quarter(work, 10, 14, 2, 6);
        salsa_quarter(work, 15, 3, 7, 11);
        /* row round */
        salsa_quarter(work, 0, 1, 2, 3);
        salsa_quarter(work, 5, 6, 7, 4);
        salsa_quarter(work, 10, 11, 8, 9);
        salsa_quarter(work, 15, 12, 13, 14);
    }
    for (i = 0; i < 16; i++)
        write_le32(out + 4 * i, work[i] + input[i]);
}

/* One page with Salsa20: block j uses counter (page nonce word 2) * 2^32 + j. */
void oracle_salsa_cipher_page(const uint8_t key[32], const uint8_t nonce[12],
                              int rounds, const uint8_t *in, uint8_t *out)
{
    uint8_t ks[ORACLE_BLOCK_BYTES];
    const uint64_t high = (uint64_t)read_le32(nonce + 8) << 32;
    uint32_t j, i;

    for (j = 0; j < ORACLE_BLOCKS_PER_PAGE; j++) {
        oracle_salsa_block(key, nonce, high + j, rounds, ks);
        for (i = 0; i < ORACLE_BLOCK_BYTES; i++)
            out[j * ORACLE_BLOCK_BYTES + i] =
                (uint8_t)(in[j * ORACLE_BLOCK_BYTES + i] ^ ks[i]);
    }
}

/* Cipher selector of the page loops below. */
#define ORACLE_CHACHA 0
#define ORACLE_SALSA 1

void oracle_cipher_pages_with(int cipher, const uint8_t key[32],
                              const uint8_t *nonces, int rounds,
                              const uint8_t *in, uint8_t *out,
                              uint64_t n_pages)
{
    uint64_t p;

    for (p = 0; p < n_pages; p++) {
        if (cipher == ORACLE_SALSA)
            oracle_salsa_cipher_page(key, nonces + 12 * p, rounds,
                                     in + p * ORACLE_PAGE_BYTES,
                                     out + p * ORACLE_PAGE_BYTES);
        else
            oracle_cipher_page(key, nonces + 12 * p, rounds,
                               in + p * ORACLE_PAGE_BYTES,
                               out + p * ORACLE_PAGE_BYTES);
    }
}

/* --- the same loop spread over host threads, for the CPU baseline --- */

struct oracle_slice {
    int cipher;
    const uint8_t *key;
    const uint8_t *nonces;
    int rounds;
    const uint8_t *in;
    uint8_t *out;
    uint64_t first;
    uint64_t count;
};

static void *oracle_slice_main(void *arg)
{
    struct oracle_slice *s = (struct oracle_slice *)arg;

    oracle_cipher_pages_with(s->cipher, s->key, s->nonces + 12 * s->first,
                             s->rounds, s->in + s->first * ORACLE_PAGE_BYTES,
                             s->out + s->first * ORACLE_PAGE_BYTES, s->count);
    return NULL;
}

/* Returns the number of threads actually used (>= 1). */
int oracle_cipher_pages_mt_with(int cipher, const uint8_t key[32],
                                const uint8_t *nonces, int rounds,
                                const uint8_t *in, uint8_t *out,
                                uint64_t n_pages, int threads)
{
    pthread_t tid[256];
    struct oracle_slice slice[256];
    uint64_t per, extra, next = 0;
    int t, used;

    if (threads < 1)
        threads = 1;
    if (threads > 256)
        threads = 256;
    if ((uint64_t)threads > n_pages)
        threads = n_pages ? (int)n_pages : 1;
    per = n_pages / (uint64_t)threads;
    extra = n_pages % (uint64_t)threads;
    for (t = 0; t < threads; t++) {
        slice[t].cipher = cipher;
        slice[t].key = key;
        slice[t].nonces = nonces;
        slice[t].rounds = rounds;
        slice[t].in = in;
        slice[t].out = out;
        slice[t].first = next;
        slice[t].count = per + ((uint64_t)t < extra ? 1u : 0u);
        next += slice[t].count;
    }
    used = 0;
    for (t = 1; t < threads; t++) {
        if (pthread_create(&tid[t], NULL, oracle_slice_main, &slice[t]) != 0)
            break;
        used = t;
    }
    oracle_slice_main(&slice[0]);
    for (t = 1; t <= used; t++)
        pthread_join(tid[t], NULL);
    if (used + 1 < threads) {
        /* thread creation failed part way: finish the rest here */
        for (t = used + 1; t < threads; t++)
            oracle_slice_main(&slice[t]);
    }
    return used + 1;
}

int oracle_cipher_pages_mt(const uint8_t key[32], const uint8_t *nonces,
                           int rounds, const uint8_t *in, uint8_t *out,
                           uint64_t n_pages, int threads)
{
    return oracle_cipher_pages_mt_with(ORACLE_CHACHA, key, nonces, rounds, in,
                                       out, n_pages, threads);
}
