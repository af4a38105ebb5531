/*
 * sanns.h -- C ABI of the MI355X homomorphic distance stage of secure
 * approximate k-NN search (SANNS, Chen et al.).
 *
 * The stage (Section 4.2 "Distance Computation via AHE"; linear-scan protocol,
 * steps 2-4): the client sends d BFV ciphertexts c_i, each encrypting the
 * constant polynomial q'[i] over R_q = Z_q[x]/(x^N + 1), q = q_0 ... q_{L-1}
 * (RNS primes).  The server holds its n points packed N per chunk, coordinate
 * i of chunk k as the plaintext polynomial g_{i,k}, and returns for every
 * chunk
 *         f_k = sum_i c_i * g_{i,k}  +  Delta [ ||p||^2 - r ]_t
 * with r uniform in Z_t.  Decrypting f_k gives the client
 * [-2 <q,p> + ||p||^2 - r]_t per slot, so client share [Dec + ||q||^2]_t and
 * server share r add up to ||q - p||^2 mod t (Section 2.1 arithmetic shares).
 *
 * Conventions (all entry points):
 *   - Every call returns sanns_status; SANNS_OK is 0, errors are negative and
 *     sanns_last_error() returns a message for the calling thread.
 *   - Argument errors found on the host return before anything is enqueued.
 *   - "dev" pointers are HIP device memory owned by the caller; the library
 *     never frees caller memory.  "host" pointers are read before return.
 *   - All device work is enqueued on the caller's stream (hipStream_t passed
 *     as void*; NULL is the null stream).  Inputs must stay alive and
 *     unmodified until the stream reaches the end of the call's work.
 *   - Ciphertexts cross the boundary in coefficient form with every residue
 *     in [0, q_l).  Layout of one ciphertext: [2][L][N] uint64 (component,
 *     limb, coefficient).  The NTT form is internal.
 *   - Shares are uint32 in [0, t).
 *   - A context may be used from several host threads only with distinct
 *     streams and distinct output and workspace buffers.
 */
#ifndef SANNS_H
#define SANNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SANNS_OK = 0,
    SANNS_E_INVALID = -1,   /* null pointer, zero or oversized dimension     */
    SANNS_E_PARAMS = -2,    /* parameter set rejected (see sanns_ctx_create)  */
    SANNS_E_RANGE = -3,     /* input value outside its documented range       */
    SANNS_E_WORKSPACE = -4, /* caller's buffer smaller than the size queried  */
    SANNS_E_DEVICE = -5,    /* HIP runtime error (message has the HIP text)   */
    SANNS_E_NOMEM = -6      /* device allocation for internal tables failed   */
} sanns_status;

#define SANNS_MAX_LIMBS 4
#define SANNS_MAX_D 4096

/* Parameter flags. */
#define SANNS_FLAG_INSECURE_TEST 1u /* allow N < 1024 or log2 q above the
                                       128-bit cap (tests only)            */
#define SANNS_FLAG_DIGIT_DB 2u      /* databases of dimension d <= 128 (and
                                       N >= 64) also hold their int8 digit
                                       form, which the matrix-core schedule
                                       SANNS_SCHEDULE_MFMA reads; by default
                                       all-pairs batches use it when a cost
                                       model of the two schedules predicts
                                       it faster (many queries and chunks) */

/* BFV parameters (Section 2.3; Section 5 "Parameters").
 *   N    ring degree, power of two, 16 <= N <= 16384
 *   L    number of RNS primes, 1 <= L <= SANNS_MAX_LIMBS
 *   q    distinct primes, q_l < 2^54, q_l = 1 mod 2N
 *   t    plaintext modulus, 2 <= t < 2^31, coprime to every q_l
 *   flags SANNS_FLAG_* */
typedef struct {
    uint32_t N;
    uint32_t L;
    uint64_t q[SANNS_MAX_LIMBS];
    uint64_t t;
    uint32_t flags;
} sanns_params;

/* Point coordinate types accepted by sanns_encode_db (and by
 * sanns_distances_gathered, which also takes SANNS_SHARE32). */
#define SANNS_U8 0
#define SANNS_I8 1
#define SANNS_SHARE32 2 /* uint32 additive shares in [0, t) of secret-shared
                           points (sanns_distances_gathered only)           */

/* Execution forms of sanns_distances. */
#define SANNS_MODE_PLAIN 0   /* one kernel launch per ciphertext operation    */
#define SANNS_MODE_FUSED 1   /* fused NTT / multiply-accumulate / INTT+mask   */
#define SANNS_MODE_BATCHED 2 /* fused kernels replayed from a cached hipGraph */
#define SANNS_MODE_PERSISTENT 3 /* one persistent work-queue launch of all phases,
                                   replayed from a cached hipGraph              */

typedef struct sanns_ctx sanns_ctx;

/* Resident database descriptor (non-owning).  The buffer `mem` holds, in
 * this order:
 *   residues [L][n_chunks][d][N] of 8 bytes: the NTT form of g_{i,k} mod q_l,
 *            stored as two 27-bit halves (low half in the first 32-bit word);
 *   norms    [n_chunks][N] uint32: ||p||^2 of the point in each slot (0 for
 *            padding slots);
 *   digits   (contexts created with SANNS_FLAG_DIGIT_DB, d <= 128 only)
 *            [L][N][n_chunks][7 Dp + 16] int8, Dp = d rounded up to 32: the
 *            same residues x as seven signed base-256 digits x_a in
 *            [-128, 127] (x = sum_a x_a 256^a), digit rows of Dp bytes
 *            indexed by coordinate, zero past d, then 16 padding bytes;
 *            followed by 64 KiB of slack the kernels may read.
 * Size: sanns_db_bytes(). */
typedef struct {
    void *mem;
    size_t bytes;
    uint32_t n_chunks;
    uint32_t d;
} sanns_db;

/* ------------------------------------------------------------------------
 * Context and parameters
 * ---------------------------------------------------------------------- */

/* Derive the default parameter set for ring degree N (Section 5
 * "Parameters"; the workloads fix N, L and the width of t):
 *   q_l  = the L largest primes below 2^54 with q_l = 1 mod 2N, descending;
 *   t    = the smallest prime >= 2^(t_bits-1) with t = 1 mod 2N.
 * out: host.  Errors: SANNS_E_INVALID (null, N not a power of two in
 * [16, 16384], L outside [1, SANNS_MAX_LIMBS], t_bits outside [2, 31]). */
sanns_status sanns_params_derive(uint32_t N, uint32_t L, uint32_t t_bits,
                                 sanns_params *out);

/* Create a context on HIP device `device`: checks the parameters (primality,
 * q_l = 1 mod 2N, t coprime to q, log2 q at most the 128-bit-security cap
 * 27/54/109/218/438 bits for N = 1024..16384 unless SANNS_FLAG_INSECURE_TEST)
 * and uploads the twiddle tables and constants.  *out receives the context.
 * Errors: SANNS_E_INVALID, SANNS_E_PARAMS, SANNS_E_DEVICE, SANNS_E_NOMEM. */
sanns_status sanns_ctx_create(const sanns_params *p, int device,
                              sanns_ctx **out);

/* Release the context's device tables and cached graphs.  NULL is a no-op.
 * The caller must have synchronised every stream the context was used on. */
void sanns_ctx_destroy(sanns_ctx *ctx);

/* Message of the last failing call on this thread ("" if none). */
const char *sanns_last_error(void);

/* Copy the context's parameters to *out (host). */
sanns_status sanns_ctx_params(const sanns_ctx *ctx, sanns_params *out);

/* ------------------------------------------------------------------------
 * Server: database encoding (linear-scan protocol steps 1 and 3)
 * ---------------------------------------------------------------------- */

/* Bytes of a resident database with n_chunks chunks of dimension d. */
size_t sanns_db_bytes(const sanns_ctx *ctx, uint32_t n_chunks, uint32_t d);

/* Encode the server's points (Section 4.2; linear-scan protocol, steps 1
 * and 3): slot j of chunk k holds point slot_point[kN + j] (the server's
 * random permutation, or a cluster layout), -1 marking a padding slot.  For
 * every (limb l, chunk k, coordinate i) the plaintext g_{i,k}[j] = -2 p[i] of
 * the slot's point (0 for padding), taken as a signed integer, is lifted mod
 * q_l and transformed to NTT form; norms[k][j] = ||p||^2.
 *   points      dev [n][d], uint8 (SANNS_U8) or int8 (SANNS_I8), row-major
 *   slot_point  dev [n_chunks * N] int64, each -1 or in [0, n)
 *   db          descriptor: mem (dev) of at least sanns_db_bytes(), n_chunks
 *               and d filled in by the caller
 * A slot index outside [-1, n) is encoded as padding and sets the device
 * error word (sanns_device_status).  Errors: SANNS_E_INVALID (null, d = 0 or > SANNS_MAX_D,
 * n_chunks = 0), SANNS_E_WORKSPACE (db->bytes too small), SANNS_E_RANGE
 * (d * max|coordinate difference|^2 >= t), SANNS_E_DEVICE. */
sanns_status sanns_encode_db(sanns_ctx *ctx, const void *points, int dtype,
                             uint64_t n, const int64_t *slot_point,
                             const sanns_db *db, void *stream);

/* ------------------------------------------------------------------------
 * Client (test helpers): encryption and decryption
 * ---------------------------------------------------------------------- */

/* Symmetric BFV encryption of constants (Section 2.3 private-key AHE;
 * linear-scan protocol step 2): for each query qi < Q and coordinate i < d,
 *   c1 = a,   c0 = -a*s + e + Delta [msg]_t  (Delta = floor(q/t); the
 *   constant sits in coefficient 0), every limb l reduced mod q_l.
 *   sk      dev [N] int8 in {-1, 0, 1}
 *   msgs    dev [Q][d] int32 (any sign; reduced mod t)
 *   a       dev [Q][d][L][N] uint64, a[..][l][..] in [0, q_l)
 *   e       dev [Q][d][N] int16
 *   ct_out  dev [Q][d][2][L][N] uint64, coefficient form
 * The randomness (sk, a, e) is an input: the caller draws it.  Errors:
 * SANNS_E_INVALID, SANNS_E_DEVICE. */
sanns_status sanns_encrypt_query(sanns_ctx *ctx, const int8_t *sk,
                                 const int32_t *msgs, uint32_t Q, uint32_t d,
                                 const uint64_t *a, const int16_t *e,
                                 uint64_t *ct_out, void *stream);

/* Client randomness drawn from a seed, for tests and examples (the same
 * definitions are implemented independently by the CPU oracle).  Both draw
 * from ChaCha20 (RFC 8439 block function) with the 32-byte key
 * (seed low 32 bits, seed high 32 bits, purpose, 0, 0, 0, 0, 0) as eight
 * little-endian words; x_j below is the 64-bit word (2n, 2n+1), n = j % 8, of
 * block j / 8, and X_j the 128-bit integer of words 4(j%4) .. 4(j%4)+3 of
 * block j / 4.
 *
 * Key generation (Section 2.3, private-key AHE; linear-scan protocol step 1,
 * the client's key): purpose 1, nonce (0, 0, 0); s_j = (x_j mod 3) - 1.
 *   sk  dev [N] int8 out, in {-1, 0, 1}
 * Errors: SANNS_E_INVALID, SANNS_E_DEVICE. */
sanns_status sanns_keygen(sanns_ctx *ctx, uint64_t seed, int8_t *sk, void *stream);

/* Encryption with its randomness drawn from enc_seed (linear-scan protocol
 * step 2): sanns_encrypt_query with, for query qi and coordinate i,
 *   a[qi][i][l][j] = X_j mod q_l  (purpose 2, nonce (qi, i, l)),
 *   e[qi][i][j]    = popcount(bits 0..20 of x_j) - popcount(bits 21..41 of
 *                    x_j), a centred binomial with eta = 21 (purpose 3,
 *                    nonce (qi, i, 0)).
 * A seed must not be reused for two encryptions under one key.  Temporary
 * device memory for a and e (Q d (8 L + 2) N bytes) is taken from the
 * stream-ordered allocator.  Arguments as sanns_encrypt_query.  Errors:
 * SANNS_E_INVALID, SANNS_E_DEVICE. */
sanns_status sanns_encrypt_query_seeded(sanns_ctx *ctx, const int8_t *sk,
                                        const int32_t *msgs, uint32_t Q, uint32_t d,
                                        uint64_t enc_seed, uint64_t *ct_out,
                                        void *stream);

/* The client's public key for the circuit-private form (Section 2.3): an
 * encryption of zero pk = (p0, p1) = (-a s + e, a) mod q_l, with a and e drawn
 * from `seed` as in sanns_encrypt_query_seeded but with purposes 4 and 5
 * (a: nonce (0, 0, l); e: nonce (0, 0, 0)).
 *   sk  dev [N] int8
 *   pk  dev [2][L][N] uint64 out, coefficient form
 * Errors: SANNS_E_INVALID, SANNS_E_DEVICE. */
sanns_status sanns_public_key(sanns_ctx *ctx, const int8_t *sk, uint64_t seed,
                              uint64_t *pk, void *stream);

/* Client decryption to shares (linear-scan protocol steps 4-5): for each of
 * the M ciphertexts, x = c0 + c1*s mod q (exact CRT over the limbs),
 * m = floor((t x + floor(q/2)) / q) mod t, and
 *   client_share[m][j] = [m_j + qnorm2[m]]_t.
 *   sk            dev [N] int8
 *   ct            dev [M][2][L][N] uint64, residues in [0, q_l)
 *   qnorm2        dev [M] uint32 = [||q||^2]_t of each ciphertext's query, or
 *                 NULL to return the decrypted message m itself
 *   client_share  dev [M][N] uint32
 * Errors: SANNS_E_INVALID, SANNS_E_DEVICE. */
sanns_status sanns_decrypt_shares(sanns_ctx *ctx, const int8_t *sk,
                                  const uint64_t *ct, uint32_t M,
                                  const uint32_t *qnorm2,
                                  uint32_t *client_share, void *stream);

/* ------------------------------------------------------------------------
 * Server hot path: distances to secret shares
 * ---------------------------------------------------------------------- */

/* Work description: output m < M is the pair (query work[2m], chunk
 * work[2m+1]), work a host array [M][2] uint32 read before the call
 * returns.  work == NULL means every chunk for every query in query-major
 * order (M = Q * n_chunks, m = q * n_chunks + k). */

/* Bytes of device workspace sanns_distances needs for Q queries and M
 * outputs in the given mode, under the context's current schedule (a call
 * that will run the matrix-core schedule, SANNS_SCHEDULE_MFMA, needs more;
 * query the size again after sanns_set_schedule).  M = Q * n_chunks is
 * sized for an all-pairs call. */
size_t sanns_distances_workspace(const sanns_ctx *ctx, const sanns_db *db,
                                 uint32_t Q, uint32_t M, int mode);

/* The server's distance stage (Section 4.2; linear-scan protocol step 3,
 * with the norm and mask folded into the ciphertext): for each output m with
 * (query qi, chunk k),
 *   ct_out[m]       = sum_i c_{qi,i} * g_{i,k}  +  Delta [ ||p||^2 - r ]_t
 *   server_share[m] = r
 * where r[j] is the ChaCha20 mask of slot j: key = mask_key (32 bytes read as
 * 8 little-endian words), nonce = (query_ids[qi] low word, high word, k),
 * block counter j/4, and r[j] = (128-bit little-endian integer of block words
 * 4(j%4)..4(j%4)+3) mod t.  A (mask_key, query id) pair must never be reused
 * for different queries.
 *   ct_in         dev [Q][d][2][L][N] uint64, coefficient form, residues
 *                 < q_l (checked on the device; a violation sets the error
 *                 word read by sanns_device_status and the outputs are
 *                 undefined)
 *   mask_key      host [32]
 *   query_ids     dev [Q] uint64
 *   work          host [M][2] uint32 or NULL (see above); entries outside
 *                 Q x n_chunks are rejected with SANNS_E_RANGE
 *   mode          SANNS_MODE_PLAIN, SANNS_MODE_FUSED, SANNS_MODE_BATCHED or
 *                 SANNS_MODE_PERSISTENT (2048 <= N <= 16384, d <= 252); all
 *                 give bit-identical outputs
 *   ct_out        dev [M][2][L][N] uint64, coefficient form
 *   server_share  dev [M][N] uint32
 *   workspace     dev, at least sanns_distances_workspace() bytes
 * SANNS_MODE_BATCHED captures the launches into a hipGraph cached in the
 * context under the call's pointers and sizes and replays it on later calls
 * with the same ones (new contents of every device buffer, query_ids
 * included, are picked up; the mask_key bytes are part of the cache key).
 * A context caches at most 32 such graphs; beyond that the least recently
 * launched one is destroyed once its last launch has completed.
 * SANNS_MODE_PERSISTENT runs the whole call as one launch of a work-queue
 * kernel (after a reset of its control words in the workspace): query NTTs
 * and mask rows first, then the multiply-accumulate tiles, then INTT + mask,
 * each phase entered once the items it reads are published device-wide; it
 * is captured and replayed the same way.  Calls that share a workspace must
 * not overlap.  Errors: SANNS_E_INVALID, SANNS_E_WORKSPACE, SANNS_E_DEVICE. */
sanns_status sanns_distances(sanns_ctx *ctx, const sanns_db *db,
                             const uint64_t *ct_in, uint32_t Q,
                             const uint8_t *mask_key,
                             const uint64_t *query_ids,
                             const uint32_t *work, uint32_t M, int mode,
                             uint64_t *ct_out, uint32_t *server_share,
                             void *workspace, size_t ws_bytes, void *stream);

/* The distance stage on chunks gathered for this call instead of a resident
 * database (clustering-based protocol, steps 6-7: the points of each query's
 * retrieved clusters; Section 4.2, last paragraph: when the points are
 * secret-shared between client and server, the server's plaintexts are its
 * shares).  Chunk m of the call holds in slot j the point
 * slot_point[m N + j] (-1: padding) and belongs to query row_query[m]; it is
 * encoded on the fly (as sanns_encode_db would, into the workspace) and
 *   ct_out[m]       = sum_i c_{q,i} * g_{i,m}  +  Delta [ P_m - r ]_t
 *   server_share[m] = r,   r drawn as in sanns_distances with chunk = m,
 * q = row_query[m].  Plaintexts by dtype:
 *   SANNS_U8, SANNS_I8  points dev [n][d]: g = -2 p (signed), P = ||p||^2;
 *   SANNS_SHARE32       points dev [n][d] uint32, the server's shares p_s in
 *                       [0, t) of points p = p_c + p_s mod t: g = the centred
 *                       representative of -2 p_s mod t; norm_shares dev [n]
 *                       uint32, its shares of ||p||^2: P = norm share.  The
 *                       client's share is then [Dec + ||q||^2 - 2 <q, p_c> +
 *                       ||p||^2_c]_t (its own cleartext terms).
 *   row_query  host [M] uint32 < Q;
 *   tail       optional resident database of dimension d (NULL for none),
 *              scanned by every query after the gathered chunks (the stash
 *              of the clustering-based form): rows M + q Ct + k, q < Q,
 *              k < Ct = tail->n_chunks, are (query q, tail chunk k);
 *   ct_in, query_ids, mask_key as sanns_distances;
 *   ct_out     dev [M + Q Ct][2][L][N], server_share dev [M + Q Ct][N];
 *   workspace  dev, sanns_distances_gathered_workspace(ctx, d, Q, M, tail)
 *              bytes (the tail's residues are copied into it).
 * The chunk word of the mask nonce is m for gathered chunk m and M + k for
 * tail chunk k, so a (mask_key, query id) pair must not be reused across
 * calls.  A slot index outside [-1, n) is taken as padding and a share (or
 * norm share) >= t as 0; both set the device error word.  Errors:
 * SANNS_E_INVALID, SANNS_E_RANGE (row_query entry >= Q, d 255^2 >= t for
 * points), SANNS_E_WORKSPACE, SANNS_E_DEVICE. */
sanns_status sanns_distances_gathered(sanns_ctx *ctx, const void *points, int dtype,
                                      uint64_t n, uint32_t d,
                                      const uint32_t *norm_shares,
                                      const int64_t *slot_point,
                                      const uint32_t *row_query, uint32_t M,
                                      const sanns_db *tail, const uint64_t *ct_in,
                                      uint32_t Q, const uint8_t *mask_key,
                                      const uint64_t *query_ids, uint64_t *ct_out,
                                      uint32_t *server_share, void *workspace,
                                      size_t ws_bytes, void *stream);
size_t sanns_distances_gathered_workspace(const sanns_ctx *ctx, uint32_t d, uint32_t Q,
                                          uint32_t M, const sanns_db *tail);

/* Slot map of gathered chunks built on the device from point ranges (the
 * points of retrieved clusters are contiguous runs of the point array):
 * slot_point[0 .. total) = -1, then slot_point[off[r] + i] = start[r] + i
 * for i < len[r], r < R (start, len, off dev [R] int64; writes outside
 * [0, total) are dropped).  Errors: SANNS_E_INVALID, SANNS_E_DEVICE. */
sanns_status sanns_slot_ranges(const int64_t *start, const int64_t *len, const int64_t *off,
                               uint32_t R, int64_t *slot_point, uint64_t total, void *stream);

/* ------------------------------------------------------------------------
 * Server preprocessing: k-means of the balanced clustering (Section 3.3
 * "Balanced Clustering and Stash"; Lloyd's k-means, Section 2).  Exact
 * integer arithmetic: points int8 [n][d] (d <= 256; uint8 data shifted by
 * -128 first, which moves no point relative to another), centres int32
 * [k][d] on a grid of 2^-8 (the value 256 stands for 1).  These calls need no
 * context; they run on the current device and the caller's stream.
 * ---------------------------------------------------------------------- */

/* Workspace bytes of sanns_kmeans_assign / sanns_kmeans_update (0 for a bad
 * shape). */
size_t sanns_kmeans_workspace(uint32_t k, uint32_t d);

/* Initial centres C_j = 256 x_{idx[j]} (idx dev [k] int64, the caller's
 * random choice of k points).  An index outside [0, n) takes point 0 and sets
 * *bad (dev uint32) to 1.  Errors: SANNS_E_INVALID, SANNS_E_DEVICE. */
sanns_status sanns_kmeans_init(const int8_t *points, uint64_t n, uint32_t d,
                               const int64_t *idx, uint32_t k, int32_t *centers,
                               uint32_t *bad, void *stream);

/* Assignment step: assign[p] = argmin_j ||256 x_p - C_j||^2 over the k
 * centres (dev int32 [k][d]), ties to the lower index, into assign (dev int32
 * [n]).  With prev (dev int32 [n], may be NULL) and changed (dev uint32, may
 * be NULL), *changed is incremented by the number of points whose centre
 * differs from prev.  Errors: SANNS_E_INVALID, SANNS_E_WORKSPACE,
 * SANNS_E_DEVICE. */
sanns_status sanns_kmeans_assign(const int8_t *points, uint64_t n, uint32_t d,
                                 const int32_t *centers, uint32_t k,
                                 const int32_t *prev, int32_t *assign,
                                 uint32_t *changed, void *workspace,
                                 size_t ws_bytes, void *stream);

/* Update step: every centre with n_j > 0 points becomes
 * floor(256 S_j / n_j + 1/2) (S_j the exact coordinate sums); a centre with
 * no point keeps its value.  counts (dev int64 [k], may be NULL) receives
 * n_j.  Assignments outside [0, k) are ignored.  Errors: as
 * sanns_kmeans_assign. */
sanns_status sanns_kmeans_update(const int8_t *points, uint64_t n, uint32_t d,
                                 const int32_t *assign, uint32_t k, int32_t *centers,
                                 int64_t *counts, void *workspace, size_t ws_bytes,
                                 void *stream);

/* Circuit-private form of sanns_distances (Section 2.3: the server's result
 * must reveal nothing beyond its plaintext, by noise flooding; Section 5
 * "Parameters", statistical circuit privacy).  Every output ciphertext f of
 * query qi, chunk k additionally receives a fresh encryption of zero under
 * that query's public key pk = (p0, p1), and c0 a flood:
 *   ct_out[m] = f + (p0 u + e1 + F, p1 u + e2)
 * with u ternary, e1, e2 centred binomial (eta = 21) and F uniform in
 * [-2^b, 2^b), drawn from ChaCha20 under mask_key with the mask stream's nonce
 * (query id low word, high word, k) and block counter s 2^24 + block for
 * stream s: 1 u_j = (x_j mod 3) - 1, 2 e1_j and 3 e2_j = popcount(bits 0..20
 * of x_j) - popcount(bits 21..41 of x_j), x_j the 64-bit word (2n, 2n+1),
 * n = j % 8, of block j / 8; 4 F_j = (Y_j mod 2^(b+1)) - 2^b, Y_j the 256-bit
 * integer of words 8(j%2) .. 8(j%2)+7 of block j / 2.  The re-randomisation
 * replaces c1 = sum_i a_i g_i (which the client could relate to the points)
 * by a fresh RLWE sample; the flood hides the product's noise.  Decryption is
 * unchanged while |noise| + 2^b stays below Delta / 2 - t.
 *   pk          dev [Q][2][L][N] uint64, coefficient form, residues < q_l
 *               (checked on the device like ct_in)
 *   flood_bits  b, at most sanns_flood_bits(ctx); 0 selects that maximum
 *   other arguments as sanns_distances; mode SANNS_MODE_FUSED or
 *   SANNS_MODE_BATCHED; the workspace from sanns_distances_cp_workspace.
 * The server shares are those of sanns_distances.  Errors: those of
 * sanns_distances; SANNS_E_RANGE for flood_bits above the maximum;
 * SANNS_E_INVALID for another mode. */
sanns_status sanns_distances_cp(sanns_ctx *ctx, const sanns_db *db,
                                const uint64_t *ct_in, uint32_t Q,
                                const uint8_t *mask_key,
                                const uint64_t *query_ids, const uint64_t *pk,
                                uint32_t flood_bits, const uint32_t *work,
                                uint32_t M, int mode, uint64_t *ct_out,
                                uint32_t *server_share, void *workspace,
                                size_t ws_bytes, void *stream);

/* Workspace bytes of sanns_distances_cp (that of sanns_distances plus the
 * public keys' NTT form, Q 2 L N 8 bytes, and the noise of the outputs,
 * M (8 L + 2) N bytes). */
size_t sanns_distances_cp_workspace(const sanns_ctx *ctx, const sanns_db *db,
                                    uint32_t Q, uint32_t M, int mode);

/* Largest flood width b of the context: the largest b with 2^b <= Delta / 4,
 * Delta = floor(q / t) (0 for a null context). */
uint32_t sanns_flood_bits(const sanns_ctx *ctx);

/* For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation: the fused
 * form of sanns_distances for Q queries against every chunk of `db`
 * (work == NULL, M = Q * n_chunks), with the workspace taken from a scratch
 * array the library holds on each GPU (SANNS_NOALLOC_SCRATCH_BYTES, 64 MiB,
 * kept until the process ends; its device address is looked up when a
 * context is created on that GPU).  Arguments and outputs are those of
 * sanns_distances; the outputs are bit-identical to it.  The call allocates
 * nothing (no device or pinned memory, no graph, no profiler events; the
 * per-phase profiler does not record it).  A call whose workspace would
 * exceed the scratch array is rejected with SANNS_E_WORKSPACE: at N = 8192,
 * L = 3 against a 123-chunk (1M-point) database that admits one query of up
 * to 169 coordinates (the 1M x 128 scan of one query needs 48.4 MiB).  All calls on one GPU share its scratch array and every
 * call leaves its contents behind: calls that overlap on one GPU (different
 * streams or host threads) race and give undefined outputs; calls on one
 * stream are ordered and safe.  Errors: those of sanns_distances. */
#define SANNS_NOALLOC_SCRATCH_BYTES (64u << 20)
sanns_status sanns_distances_noalloc(sanns_ctx *ctx, const sanns_db *db,
                                     const uint64_t *ct_in, uint32_t Q,
                                     const uint8_t *mask_key,
                                     const uint64_t *query_ids,
                                     uint64_t *ct_out, uint32_t *server_share,
                                     void *stream);

/* Synchronise `stream` and return (and clear) the context's device error
 * word: SANNS_E_RANGE if, since the last call, an input residue was >= q_l
 * or a slot index of sanns_encode_db was outside [-1, n) (such a slot is
 * encoded as padding); SANNS_E_DEVICE if a persistent launch gave up waiting
 * for a phase (its bounded wait expired; outputs are undefined); SANNS_E_RANGE
 * also when a share given to sanns_distances_gathered was >= t. */
sanns_status sanns_device_status(sanns_ctx *ctx, void *stream);

/* Fix the multiply-accumulate schedule (used by the autotuner):
 *   lds_variant  LDS-staged kernel used for batches of >= 2 queries against
 *                every chunk (work == NULL): 1..11 (register-staged) or 21..27
 *                (direct-to-LDS staged), SANNS_SCHEDULE_MFMA (int8 matrix
 *                cores on the digit form; the context needs
 *                SANNS_FLAG_DIGIT_DB and sanns_distances then needs d <= 128),
 *                or 0 for the default; or the tile shape of
 *                SANNS_MODE_PERSISTENT: 41..44 (N = 8192), 51..52 (N = 4096),
 *                61 (N = 2048), 71 (N = 16384);
 *   qt x ct      register tile (queries x chunks per thread) used for every
 *                other call: 1x1, 1x2, 1x4, 1x8, 2x2, 2x4, 4x2, 2x3, 3x2, or
 *                0x0 for the automatic choice.
 * Outputs do not depend on the schedule.  Errors: SANNS_E_INVALID for a
 * variant or shape that is not built. */
#define SANNS_SCHEDULE_MFMA 81
sanns_status sanns_set_schedule(sanns_ctx *ctx, int lds_variant, int qt, int ct);

/* Phases timed by the profiler, in launch order. */
#define SANNS_PHASE_QUERY_NTT 0 /* forward NTT of the query ciphertexts     */
#define SANNS_PHASE_MASKS 1     /* ChaCha20 masks -> server shares (drawn
                                   inside SANNS_PHASE_SUMS by the matrix-core
                                   schedule: 0 there)                       */
#define SANNS_PHASE_MAC 2       /* multiply-accumulate over the database    */
#define SANNS_PHASE_INTT_MASK 3 /* INTT + Delta [||p||^2 - r]_t             */
#define SANNS_PHASE_DIGITS 4    /* SANNS_SCHEDULE_MFMA: query NTT form ->
                                   signed digits (0 for other schedules)    */
#define SANNS_PHASE_SUMS 5      /* SANNS_SCHEDULE_MFMA: slot-major sums ->
                                   NTT-form outputs, and the masks (0 for
                                   other schedules)                         */
#define SANNS_PHASE_RERAND 6    /* sanns_distances_cp: public keys' NTT and
                                   u pk added to the NTT-form outputs       */
#define SANNS_N_PHASES 7

/* Per-phase timing of the fused form (tracing aid).  While enabled,
 * sanns_distances in SANNS_MODE_FUSED or SANNS_MODE_BATCHED records a HIP
 * event pair around each phase's launch on the caller's stream (batched
 * calls then launch the kernels directly instead of replaying the graph).
 * SANNS_MODE_PERSISTENT calls are not timed per phase.
 * Enabling resets the accumulated times. */
sanns_status sanns_profile_enable(sanns_ctx *ctx, int on);

/* Synchronise on the recorded events and write, for each phase, the mean
 * duration in milliseconds over the calls since enabling (ms_out[SANNS_N_PHASES], host)
 * and the number of calls (*calls, host, may be NULL). */
sanns_status sanns_profile_read(sanns_ctx *ctx, double *ms_out, int *calls);

#ifdef __cplusplus
}
#endif

#endif /* SANNS_H */
