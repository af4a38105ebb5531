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
