/*
 * Oracle for the secure k-NN homomorphic distance stage -- TEST INFRASTRUCTURE.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load this file's library.  It shares no code with the HIP path: every loop
 * below is the textbook definition of what the method computes, written for a
 * reader to check by eye, in exact integer arithmetic (unsigned/signed
 * __int128 accumulators, one reduction at the end).
 *
 * What is computed, and where the paper defines it:
 *   - negacyclic products in R_q = Z_q[x]/(x^N + 1): the BFV ring the paper's
 *     additive HE scheme works in (Section 2.3; Section 4.2, "Distance
 *     Computation via AHE");
 *   - the server's inner product  sum_i c_i * g_i  (Section 4.2, the identity
 *     sum_i f_i g_i = sum_j <q, p_j> x^(j-1); linear-scan protocol, step 3);
 *   - the server's uniform mask r in Z_t (linear-scan protocol, step 3), drawn
 *     from the ChaCha20 block function of RFC 8439, Section 2.3.
 */
#include <stdint.h>
#include <stddef.h>
#include <string.h>
#include <omp.h>

/* Threads of the OpenMP loops below (the benchmark times the oracle on one
 * thread and on every core the process may use). */
void oracle_set_threads(int n) { omp_set_num_threads(n); }
int oracle_max_threads(void) { return omp_get_max_threads(); }

typedef unsigned __int128 u128;
typedef __int128 i128;

static uint64_t mod_i128(i128 x, uint64_t q)
{
    i128 r = x % (i128)q;
    if (r < 0) r += q;
    return (uint64_t)r;
}

/* c = a * b in Z_q[x]/(x^N+1); a, b given as residues in [0, q).
 * Schoolbook: c_j = sum_{u+v=j} a_u b_v - sum_{u+v=j+N} a_u b_v. */
void oracle_negacyclic_mul(const uint64_t *a, const uint64_t *b, int N,
                           uint64_t q, uint64_t *c)
{
    for (int j = 0; j < N; j++) {
        u128 pos = 0, neg = 0;
        for (int u = 0; u < N; u++) {
            int v = j - u;
            if (v >= 0)
                pos += ((u128)a[u] * b[v]) % q;
            else
                neg += ((u128)a[u] * b[v + N]) % q;
        }
        uint64_t p = (uint64_t)(pos % q), n = (uint64_t)(neg % q);
        c[j] = p >= n ? p - n : p + q - n;
    }
}

/* One coefficient j of  sum_{i<d} a_i * g_i  in Z_q[x]/(x^N+1), where a_i are
 * residues in [0, q) (row stride sa) and g_i are small signed integers (row
 * stride sg), i.e. the plaintext polynomial taken as an integer polynomial. */
uint64_t oracle_inner_coeff(const uint64_t *a, int64_t sa, const int64_t *g,
                            int64_t sg, int d, int N, uint64_t q, int j)
{
    i128 acc = 0;
    for (int i = 0; i < d; i++) {
        const uint64_t *ai = a + (int64_t)i * sa;
        const int64_t *gi = g + (int64_t)i * sg;
        for (int u = 0; u < N; u++) {
            int v = j - u;
            i128 prod = v >= 0 ? (i128)ai[u] * gi[v] : -((i128)ai[u] * gi[v + N]);
            acc += prod;
        }
    }
    return mod_i128(acc, q);
}

/* All N coefficients of sum_i a_i * g_i (threads over output coefficients). */
void oracle_inner_all(const uint64_t *a, int64_t sa, const int64_t *g,
                      int64_t sg, int d, int N, uint64_t q, uint64_t *out)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int j = 0; j < N; j++)
        out[j] = oracle_inner_coeff(a, sa, g, sg, d, N, q, j);
}

/* c = a * s with s a small signed polynomial (the secret key, or an error),
 * all coefficients (threads over output coefficients). */
void oracle_mul_small(const uint64_t *a, const int64_t *s, int N, uint64_t q,
                      uint64_t *out)
{
    oracle_inner_all(a, 0, s, 0, 1, N, q, out);
}

/* ---------------- ChaCha20 (RFC 8439, Section 2.3) ---------------------- */

static uint32_t rotl32(uint32_t x, int n) { return (x << n) | (x >> (32 - n)); }

static void quarter_round(uint32_t *s, int a, int b, int c, int d)
{
    s[a] += s[b]; s[d] ^= s[a]; s[d] = rotl32(s[d], 16);
    s[c] += s[d]; s[b] ^= s[c]; s[b] = rotl32(s[b], 12);
    s[a] += s[b]; s[d] ^= s[a]; s[d] = rotl32(s[d], 8);
    s[c] += s[d]; s[b] ^= s[c]; s[b] = rotl32(s[b], 7);
}

/* The 16 output words of the ChaCha20 block function for (key, counter, nonce):
 * state = constants | key | counter | nonce, 10 double rounds, then the
 * original state added word by word. */
void oracle_chacha20_block(const uint32_t key[8], uint32_t counter,
                           const uint32_t nonce[3], uint32_t out[16])
{
    uint32_t init[16] = {0x61707865u, 0x3320646eu, 0x79622d32u, 0x6b206574u};
    for (int i = 0; i < 8; i++) init[4 + i] = key[i];
    init[12] = counter;
    init[13] = nonce[0]; init[14] = nonce[1]; init[15] = nonce[2];
    uint32_t s[16];
    memcpy(s, init, sizeof s);
    for (int r = 0; r < 10; r++) {
        quarter_round(s, 0, 4, 8, 12);
        quarter_round(s, 1, 5, 9, 13);
        quarter_round(s, 2, 6, 10, 14);
        quarter_round(s, 3, 7, 11, 15);
        quarter_round(s, 0, 5, 10, 15);
        quarter_round(s, 1, 6, 11, 12);
        quarter_round(s, 2, 7, 8, 13);
        quarter_round(s, 3, 4, 9, 14);
    }
    for (int i = 0; i < 16; i++) out[i] = s[i] + init[i];
}

/* Server masks r_j, j in [j0, j0+cnt), of one (query id, chunk) pair.
 * Stream: key = the 32 key bytes read as 8 little-endian words; nonce =
 * (query_id low word, query_id high word, chunk); block counter = j / 4.
 * Slot j takes the 128-bit little-endian integer X formed by words
 * 4(j%4) .. 4(j%4)+3 of that block, and r_j = X mod t. */
void oracle_masks(const uint8_t key_bytes[32], uint64_t query_id,
                  uint32_t chunk, uint64_t t, int j0, int cnt, uint32_t *out)
{
    uint32_t key[8], nonce[3] = {(uint32_t)query_id, (uint32_t)(query_id >> 32),
                                 chunk};
    for (int i = 0; i < 8; i++)
        key[i] = (uint32_t)key_bytes[4 * i] | (uint32_t)key_bytes[4 * i + 1] << 8 |
                 (uint32_t)key_bytes[4 * i + 2] << 16 |
                 (uint32_t)key_bytes[4 * i + 3] << 24;
    for (int n = 0; n < cnt; n++) {
        int j = j0 + n;
        uint32_t blk[16];
        oracle_chacha20_block(key, (uint32_t)(j / 4), nonce, blk);
        const uint32_t *w = blk + 4 * (j % 4);
        u128 X = (u128)w[0] | (u128)w[1] << 32 | (u128)w[2] << 64 |
                 (u128)w[3] << 96;
        out[n] = (uint32_t)(X % t);
    }
}

/* The client's randomness when it is drawn from a seed (key generation and
 * encryption; the private-key AHE of Section 2.3): ChaCha20 with
 * key = (seed low word, seed high word, purpose, 0, 0, 0, 0, 0), purpose
 * 1 = secret key, 2 = uniform component a, 3 = error e, 4 and 5 = the same
 * for the public key. */
static void client_key(uint64_t seed, uint32_t purpose, uint32_t key[8])
{
    memset(key, 0, 8 * sizeof key[0]);
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    key[2] = purpose;
}

/* 64-bit word n (n in [0, 8)) of a block: words 2n (low) and 2n + 1. */
static uint64_t word64(const uint32_t blk[16], int n)
{
    return (uint64_t)blk[2 * n] | (uint64_t)blk[2 * n + 1] << 32;
}

/* Ternary secret s_j = (x_j mod 3) - 1, x_j the 64-bit word j % 8 of block
 * j / 8, nonce (0, 0, 0). */
void oracle_sample_ternary(uint64_t seed, int N, int8_t *out)
{
    uint32_t key[8], nonce[3] = {0, 0, 0}, blk[16];
    client_key(seed, 1, key);
    for (int j = 0; j < N; j++) {
        oracle_chacha20_block(key, (uint32_t)(j / 8), nonce, blk);
        out[j] = (int8_t)((int)(word64(blk, j % 8) % 3) - 1);
    }
}

/* Uniform residue a_j in [0, q) of (query qi, coordinate i, limb l): the
 * 128-bit little-endian integer of words 4(j%4) .. 4(j%4)+3 of block j / 4,
 * nonce (qi, i, l), reduced mod q.  Purpose 2 for encryptions, 4 for the
 * public key. */
void oracle_sample_uniform(uint64_t seed, uint32_t purpose, uint32_t qi, uint32_t i,
                           uint32_t l, uint64_t q, int N, uint64_t *out)
{
    uint32_t key[8], nonce[3] = {qi, i, l}, blk[16];
    client_key(seed, purpose, key);
    for (int j = 0; j < N; j++) {
        oracle_chacha20_block(key, (uint32_t)(j / 4), nonce, blk);
        const uint32_t *w = blk + 4 * (j % 4);
        u128 X = (u128)w[0] | (u128)w[1] << 32 | (u128)w[2] << 64 | (u128)w[3] << 96;
        out[j] = (uint64_t)(X % q);
    }
}

/* Centred binomial error with eta = 21 of (query qi, coordinate i):
 * e_j = popcount(bits 0..20 of x_j) - popcount(bits 21..41 of x_j), x_j the
 * 64-bit word j % 8 of block j / 8, nonce (qi, i, 0).  Purpose 3 for
 * encryptions, 5 for the public key. */
void oracle_sample_cbd21(uint64_t seed, uint32_t purpose, uint32_t qi, uint32_t i, int N,
                         int16_t *out)
{
    uint32_t key[8], nonce[3] = {qi, i, 0}, blk[16];
    client_key(seed, purpose, key);
    for (int j = 0; j < N; j++) {
        oracle_chacha20_block(key, (uint32_t)(j / 8), nonce, blk);
        const uint64_t x = word64(blk, j % 8);
        int pa = 0, pb = 0;
        for (int b = 0; b < 21; b++) {
            pa += (int)((x >> b) & 1);
            pb += (int)((x >> (21 + b)) & 1);
        }
        out[j] = (int16_t)(pa - pb);
    }
}

/* The server's re-randomisation and flooding randomness of one output (query
 * id, chunk), for circuit privacy (Section 2.3; Section 5 "Parameters"):
 * ChaCha20 under the server's mask key and the mask stream's nonce (query id
 * low word, high word, chunk), with the block counter of stream s starting at
 * s * 2^24 (s = 0 is the mask stream itself):
 *   s = 1  u_j  = (x_j mod 3) - 1,
 *   s = 2  e1_j = popcount(bits 0..20 of x_j) - popcount(bits 21..41 of x_j),
 *   s = 3  e2_j likewise,
 *   with x_j the 64-bit word (2n, 2n+1), n = j % 8, of block j / 8;
 *   s = 4  the eight words 8(j%2) .. 8(j%2)+7 of block j / 2 (a 256-bit
 *          little-endian integer; the caller keeps its low bits). */
void oracle_cp_streams(const uint8_t key_bytes[32], uint64_t query_id,
                       uint32_t chunk, int N, int8_t *u, int16_t *e1,
                       int16_t *e2, uint32_t *flood_words)
{
    uint32_t key[8], nonce[3] = {(uint32_t)query_id, (uint32_t)(query_id >> 32),
                                 chunk}, blk[16];
    for (int i = 0; i < 8; i++)
        key[i] = (uint32_t)key_bytes[4 * i] | (uint32_t)key_bytes[4 * i + 1] << 8 |
                 (uint32_t)key_bytes[4 * i + 2] << 16 |
                 (uint32_t)key_bytes[4 * i + 3] << 24;
    for (int j = 0; j < N; j++) {
        oracle_chacha20_block(key, (1u << 24) + (uint32_t)(j / 8), nonce, blk);
        u[j] = (int8_t)((int)(word64(blk, j % 8) % 3) - 1);
        for (int s = 0; s < 2; s++) {
            oracle_chacha20_block(key, ((uint32_t)(2 + s) << 24) + (uint32_t)(j / 8),
                                  nonce, blk);
            const uint64_t x = word64(blk, j % 8);
            int pa = 0, pb = 0;
            for (int b = 0; b < 21; b++) {
                pa += (int)((x >> b) & 1);
                pb += (int)((x >> (21 + b)) & 1);
            }
            (s == 0 ? e1 : e2)[j] = (int16_t)(pa - pb);
        }
        oracle_chacha20_block(key, (4u << 24) + (uint32_t)(j / 2), nonce, blk);
        memcpy(flood_words + 8 * (size_t)j, blk + 8 * (j % 2), 8 * sizeof(uint32_t));
    }
}

/* Squared Euclidean distances from one query to n points (exact int64). */
void oracle_sqdist(const int32_t *qv, const int32_t *pts, int64_t n, int d,
                   int64_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < n; p++) {
        int64_t acc = 0;
        for (int i = 0; i < d; i++) {
            int64_t diff = (int64_t)qv[i] - pts[p * d + i];
            acc += diff * diff;
        }
        out[p] = acc;
    }
}
