/*
 * fhe_spmspm.h - C-ABI of the MI355X (gfx950) library for sparse x sparse
 * matrix multiplication on RNS-CKKS ciphertexts.
 *
 * The operation is the paper's CSR x CSC method: the left operand's values
 * are packed row-major (CSR order) into ciphertext slots, the right
 * operand's values column-major (CSC order); the sparsity pattern is public
 * and only the values are encrypted (Section 3.2.1). Every matched pair of
 * non-zeros found by the merge of Algorithm 1 is aligned by one rotation,
 * multiplied, relinearised and rescaled, isolated with a one-hot plaintext
 * mask, rescaled again, rotated to its row-major target slot and added to
 * the result (Algorithm 2, Section 3.1).
 *
 * Conventions for every entry point
 *   - Return value: FHE_OK (0) or a negative FHE_E* code; fhe_last_error()
 *     then returns a message describing the failure (thread-local, valid
 *     until the next call on the same thread).
 *   - Host arrays passed in are read during the call only and stay owned by
 *     the caller. Handles returned through out-pointers are owned by the
 *     caller and released with the matching *_free call (NULL is accepted).
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Device work is enqueued on it; functions that return host data
 *     synchronise that stream before returning.
 *   - Device memory comes from the allocator registered with
 *     fhe_set_allocator (default: hipMalloc / hipFree).
 *   - Rotation by r is a LEFT rotation: slot t of the output holds slot
 *     t + r (mod S) of the input, S = N/2 slots. It is applied as at most
 *     rot_digits key-switched steps of the form r_t * 2^(b t), b =
 *     ceil(log2 S / rot_digits) (a rotation by 0 is the identity).
 *   - Coefficient-domain exports hold residues in [0, q_i), layout
 *     [component][limb][coefficient], limb i modulo the i-th Q prime.
 */
#ifndef FHE_SPMSPM_H
#define FHE_SPMSPM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FHE_OK 0
#define FHE_EINVAL (-1)  /* malformed argument (bad CSR/CSC, NULL, out-of-range value) */
#define FHE_ESHAPE (-2)  /* incompatible shapes (A.cols != B.rows, buffer too small, level mismatch) */
#define FHE_ELEVEL (-3)  /* not enough Q primes left for the operation (the method needs >= 3) */
#define FHE_EKEY (-4)    /* a rotation key needed by the operation was not generated */
#define FHE_ENOMEM (-5)  /* device allocation failed */
#define FHE_EAGAIN (-6)  /* resource temporarily unavailable */
#define FHE_EDEVICE (-7) /* HIP runtime error */
#define FHE_ECANCELED (-8) /* the request was cancelled (server closed before admitting it) */

typedef struct fhe_ctx fhe_ctx; /* parameters, device tables and evaluation keys (server side) */
typedef struct fhe_sk fhe_sk;   /* secret key (client side) */
typedef struct fhe_mat fhe_mat; /* encrypted matrix: public shape/pattern + ciphertext chunks */
typedef struct fhe_ct fhe_ct;   /* a single ciphertext (operation-level interface) */

/* RNS-CKKS parameter set (Section 2.1 describes CKKS; the paper fixes no values).
 * Q primes: the n_q largest primes q < 2^q_bits with q = 1 (mod 2N), descending (q_0 > q_1 > ...).
 * P primes: the n_p largest primes p < 2^p_bits with p = 1 (mod 2N), descending.
 * Key switching is hybrid with `alpha` Q primes per digit. Scales: the CSR operand is encoded at
 * 2^log_delta, the CSC operand at exactly q_(n_q-1), the one-hot mask at 2^mask_bits * q_(n_q-2);
 * products of the method therefore end at scale exactly 2^(log_delta + mask_bits). */
typedef struct fhe_params_desc {
  int32_t log_n;      /* N = 2^log_n, 12 <= log_n <= 17 */
  int32_t n_q;        /* number of Q primes, 3 <= n_q <= 64 */
  int32_t q_bits;     /* bits of the Q primes, 30 <= q_bits <= 50 */
  int32_t n_p;        /* number of special primes K, 1 <= n_p <= 8 */
  int32_t p_bits;     /* bits of the special primes, q_bits < p_bits <= 61 */
  int32_t alpha;      /* Q primes per key-switching digit, 1 <= alpha <= n_q */
  int32_t rot_digits; /* D: key-switched steps per rotation, 1 <= D <= log2(N/2) */
  int32_t log_delta;  /* scale of the CSR operand, 2^log_delta */
  int32_t mask_bits;  /* s: mask scale 2^s * q_(n_q-2) */
  int32_t device;     /* HIP device ordinal */
} fhe_params_desc;

/* Device allocator hooks: alloc(size, stream, user) returns device memory or NULL;
 * free_(ptr, stream, user). Passing NULL for both restores hipMalloc/hipFree. Must be set before
 * fhe_params_create; objects keep the hooks that were current when they were created. */
typedef void* (*fhe_alloc_fn)(size_t size, void* stream, void* user);
typedef void (*fhe_free_fn)(void* ptr, void* stream, void* user);
int fhe_set_allocator(fhe_alloc_fn alloc, fhe_free_fn free_, void* user);

/* Creates a context: prime chain, NTT tables, base-conversion and rescale constants and the
 * transformed base mask, all resident on `desc->device`. Its schedule (same results either way)
 * starts from the NTT split k1 = log_n - 9 for log_n >= 15, else log_n / 2 (environment
 * FHE_NTT_K1 overrides it) and row-phase workgroups of 512 threads (FHE_ROWS_NT=256 for 256);
 * fhe_autotune may change both. Errors: FHE_EINVAL (desc out of range, not enough primes),
 * FHE_ELEVEL (n_q < 3), FHE_ENOMEM, FHE_EDEVICE. */
int fhe_params_create(const fhe_params_desc* desc, fhe_ctx** out);
void fhe_ctx_free(fhe_ctx* ctx);

/* Copies the moduli q_0..q_(n_q-1), p_0..p_(n_p-1) into out[cap]; returns their count (or < 0). */
int fhe_ctx_primes(const fhe_ctx* ctx, uint64_t* out, size_t cap);

/* Key generation (the paper's client holds the secret, Figure 1). Samples the ternary secret from
 * `seed` and installs the relinearisation key (target s^2) into ctx. With rot_digits >= 2 it also
 * installs every digit rotation key r_t * 2^(b t) (r_t in [1, 2^b)); with rot_digits == 1 rotation
 * keys are generated on demand by fhe_keygen_rotations. Keys stay resident on the device
 * (Section 3: ciphertexts and keys are uploaded once). Randomness: SplitMix64 streams keyed by
 * (seed, object tag); this generator is reproducible, not cryptographically secure. */
int fhe_keygen(fhe_ctx* ctx, uint64_t seed, void* stream, fhe_sk** sk_out);
void fhe_sk_free(fhe_sk* sk);

/* Installs the rotation keys needed to rotate left by each of amounts[0..n) (amounts are taken
 * mod S; keys already present are skipped). Errors: FHE_EINVAL. */
int fhe_keygen_rotations(fhe_ctx* ctx, const fhe_sk* sk, const int32_t* amounts, size_t n, void* stream);

/* Encrypts a CSR matrix (left operand, Algorithm 1): indptr[rows+1], indices[nnz] (column ids,
 * strictly ascending per row), values[nnz]. Values are packed in CSR order, S per ciphertext chunk,
 * encoded at 2^log_delta and encrypted under the secret key at the top level with the SplitMix64
 * stream `seed`. The pattern is kept in the handle as public metadata (Section 3.2.1).
 * Errors: FHE_EINVAL (pattern malformed: indptr not non-decreasing from 0 to nnz, index out of
 * range or not strictly ascending). */
int fhe_encrypt_csr(fhe_ctx* ctx, const fhe_sk* sk, int32_t rows, int32_t cols, const int32_t* indptr,
                    const int32_t* indices, const double* values, uint64_t seed, void* stream, fhe_mat** out);

/* Encrypts a CSC matrix (right operand): indptr[cols+1], indices[nnz] (row ids, strictly ascending
 * per column), values[nnz] in CSC order, encoded at exactly q_(n_q-1). Same errors as above. */
int fhe_encrypt_csc(fhe_ctx* ctx, const fhe_sk* sk, int32_t rows, int32_t cols, const int32_t* indptr,
                    const int32_t* indices, const double* values, uint64_t seed, void* stream, fhe_mat** out);

/* C = A B (Algorithms 1 and 2). A: CSR handle (rows m, cols k); B: CSC handle (rows k, cols n).
 * C is a dense encrypted m x n matrix packed row-major, S slots per chunk, two levels below the
 * top, at scale 2^(log_delta + mask_bits). Its ciphertext limbs are bit-identical to performing
 * every matched pair's operation sequence one by one, in any order. Errors: FHE_EINVAL (wrong
 * handle kinds), FHE_ESHAPE (A.cols != B.rows), FHE_EKEY (a rotation key is missing). */
int fhe_spmspm(fhe_ctx* ctx, const fhe_mat* A, const fhe_mat* B, void* stream, fhe_mat** C_out);

/* As fhe_spmspm, restricted to the matched pairs with index in [pair_begin, pair_end) of
 * Algorithm 1's traversal order (i-major, then j, then the merge). Used to check sampled
 * contributions at full size. */
int fhe_spmspm_pairs(fhe_ctx* ctx, const fhe_mat* A, const fhe_mat* B, int64_t pair_begin, int64_t pair_end,
                     void* stream, fhe_mat** C_out);

/* Batched form: C_out[i] = A[i] B[i] for i < cnt, run as one stream of batched launches. The plans
 * of all matmuls are merged (products and matched pairs of every matmul share the same launches, and
 * pairs that use the same rotation keys are processed together), so many small or uneven matmuls
 * fill the GPU where one at a time would not. Each result is bit-identical to fhe_spmspm on the same
 * operands. On error no result handle is returned (all C_out[i] are NULL). */
int fhe_spmspm_batch(fhe_ctx* ctx, size_t cnt, const fhe_mat* const* A, const fhe_mat* const* B, void* stream,
                     fhe_mat** C_out);

/* Batched form restricted per matmul to the matched pairs with traversal index in
 * [pair_begin[i], pair_end[i]) (as fhe_spmspm_pairs); both arrays are host arrays of cnt entries,
 * or both NULL for the full matmuls. Used to measure a bounded prefix of very large batches. */
int fhe_spmspm_batch_pairs(fhe_ctx* ctx, size_t cnt, const fhe_mat* const* A, const fhe_mat* const* B,
                           const int64_t* pair_begin, const int64_t* pair_end, void* stream, fhe_mat** C_out);

/* Plan modes of fhe_spmspm_plan. */
#define FHE_PLAN_PER_PAIR 0 /* Algorithm 2 per matched pair (the form of fhe_spmspm) */
#define FHE_PLAN_GROUPED 1  /* grouped target rotations, see fhe_spmspm_plan */
#define FHE_PLAN_TREE 2     /* grouped, with the target rotations shared digit by digit */
#define FHE_PLAN_GRAPH 256  /* flag: record the launch stream as a HIP graph and replay it, see below */
#define FHE_PLAN_HOIST 512  /* flag: hoisted alignment rotations, see below */

/* General form of the matmul calls: C_out[i] = A[i] B[i] for i < cnt as one merged launch stream,
 * each restricted to the matched pairs with traversal index in [pair_begin[i], pair_end[i]) (both
 * NULL: all pairs), in plan mode `mode`. FHE_PLAN_PER_PAIR gives exactly fhe_spmspm_batch_pairs.
 * FHE_PLAN_GROUPED follows the paper's aim of issuing as few rotations as possible (Section 3.2):
 * after its one-hot mask every matched pair's product occupies one slot, so the masked products
 * of a matmul's pairs that share (result chunk, target rotation) are added (exactly, mod q) and go
 * through one second rescale and one target rotation. The groups are formed over the pairs of the
 * call's range. Decrypted results equal the per-pair form's up to noise (lower: fewer roundings
 * and key switches); the ciphertext limbs are those of that grouped sequence, not the per-pair
 * ones. The grouped form keeps the products (2 (n_q - 1) N words each) its groups use resident in
 * device memory, up to FHE_GROUP_MB (environment, default 49152 MiB, raised to the largest group's
 * products if needed); beyond that it runs the groups in passes and each pass recomputes the
 * products its pairs use. The context keeps that store between calls and grows it on demand (like
 * the executor scratch); fhe_server_create releases it. Errors as fhe_spmspm_batch_pairs, FHE_EINVAL for
 * an unknown mode; on error all C_out[i] are NULL.
 * FHE_PLAN_TREE is the grouped plan with its target rotations shared further: a rotation by
 * r = sum_t r_t 2^(b t) is the composition of its digit steps, so each group is rotated by its low
 * digit only and added to the partial sum of its (result chunk, higher digits); each partial sum is
 * then rotated by its next digit and added into the next level's, and so on. One key switch per
 * group with a nonzero low digit plus one per distinct nonzero higher-digit key. Same decryption up
 * to noise; the limbs are those of that sequence. Its partial sums (one ciphertext per distinct key
 * per level) are kept in device memory besides the resident products.
 * With FHE_PLAN_GRAPH or-ed into mode, the first call records the call's whole launch stream as one
 * HIP graph (on a stream of the context's own) and keeps it on the context, together with the pointer
 * tables and scratch its kernels read; later calls with the same operand handles, ranges, plan mode
 * and NTT split replay it with a single launch on `stream`. Results are bit-identical to the eager
 * form. A context keeps at most two graphs (the oldest is dropped) and drops them all when its
 * scratch has to grow. Graph calls are not timed per kernel by fhe_profile_* (one "graph_replay"
 * record per call).
 * With FHE_PLAN_HOIST or-ed into mode, every alignment rotation step (Algorithm 1) is hoisted: the
 * key switch uses the automorphism of the ModUp digits of its input, tau(ModUp(c1)), rather than
 * ModUp(tau(c1)); both are congruent modulo every digit modulus, so the rotation decrypts the same up
 * to noise, while one ModUp (and one transform of its digits) serves every rotation of the same
 * ciphertext in a batch. The limbs are those of that sequence (any plan mode). */
int fhe_spmspm_plan(fhe_ctx* ctx, size_t cnt, const fhe_mat* const* A, const fhe_mat* const* B,
                    const int64_t* pair_begin, const int64_t* pair_end, int32_t mode, void* stream, fhe_mat** C_out);

/* The naive sparse method of the paper's evaluation (Section 4, method (ii)), on the same executor: the
 * multiplication stays element-wise, and a product is skipped only where both of its entries are
 * zero. A and B store every entry they may multiply (typically all m k and k n entries, zeros
 * included, as CSR / CSC patterns); nonzero_a[A.nnz] and nonzero_b[B.nnz] (host arrays, one byte per
 * stored entry in packing order: 1 = nonzero, 0 = zero) give the public zero pattern. Every matched
 * pair of Algorithm 1's traversal whose two entries are not both zero runs Algorithm 2 exactly as in
 * fhe_spmspm, so C's limbs are those of that per-pair sequence over the kept pairs (with every flag 1
 * this is fhe_spmspm, the naive dense method when every entry is stored). Errors as fhe_spmspm,
 * FHE_EINVAL for a NULL flag array of a non-empty operand. */
int fhe_spmspm_naive_sparse(fhe_ctx* ctx, const fhe_mat* A, const fhe_mat* B, const uint8_t* nonzero_a,
                            const uint8_t* nonzero_b, void* stream, fhe_mat** C_out);

/* Plan statistics of fhe_spmspm_naive_sparse (as fhe_plan_stats, over the kept pairs). */
int fhe_plan_stats_naive_sparse(fhe_ctx* ctx, const fhe_mat* A, const fhe_mat* B, const uint8_t* nonzero_a,
                                const uint8_t* nonzero_b, int64_t counts[6]);

/* Autotuner (batch scheduler): picks, for ctx, the NTT split 2^k1 x 2^(log_n - k1) (every k1 in
 * [max(1, log_n - 9), min(9, log_n - 1)]) and the row-phase workgroup shape (512 threads x 8
 * elements or 256 x 16) by timing every combination; keeps the current choice unless another is at
 * least 2% faster. Every choice computes the same transform, so results are unchanged; only the
 * kernel schedule (LDS rounds, fused column kernels, row segment width, registers per thread)
 * differs. With A and B (a CSR and a CSC operand of ctx): times the first `pairs` matched pairs of
 * A B, each with its full sequence (median of 3). With A = B = NULL: times `batch` synthetic key
 * switches at the top level and two levels below (median of 5; needs fhe_keygen first, FHE_EKEY;
 * batch in [1, 4096], FHE_EINVAL). Reports the chosen k1, row-phase threads and time (ms); if
 * cap > 0, the first cap candidates tried (k1_tried[i], rows_tried[i], ms_tried[i]) and their
 * count (n_tried). Allocates device memory for its runs. Must not overlap other calls on ctx. */
int fhe_autotune(fhe_ctx* ctx, void* stream, const fhe_mat* A, const fhe_mat* B, int64_t pairs, int32_t batch,
                 int32_t* k1_out, int32_t* rows_out, double* ms_out, int32_t* n_tried, int32_t* k1_tried,
                 int32_t* rows_tried, double* ms_tried, int32_t cap);

/* Plan statistics of A B without running it: counts[0] = matched pairs F, [1] = distinct products,
 * [2] = alignment key switches, [3] = product relinearisations, [4] = target-rotation key switches,
 * [5] = result chunks. Errors as fhe_spmspm. */
int fhe_plan_stats(fhe_ctx* ctx, const fhe_mat* A, const fhe_mat* B, int64_t counts[6]);

/* Grouped-plan statistics of A B: counts[0] = groups (distinct result chunk and target rotation),
 * counts[1] = their target-rotation key switches, counts[2] = the target-rotation key switches of
 * the digit tree (FHE_PLAN_TREE); the other counts are those of fhe_plan_stats. Errors as fhe_spmspm. */
int fhe_plan_groups(fhe_ctx* ctx, const fhe_mat* A, const fhe_mat* B, int64_t counts[3]);

/* Host-only planning from the public patterns (no context, no device): the same counts as
 * fhe_plan_stats for A (m x k, CSR pattern) times B (k x n, CSC pattern) at ring dimension 2^log_n
 * with rot_digits rotation steps. Errors: FHE_EINVAL (malformed pattern or parameters). */
int fhe_plan_pattern(int32_t log_n, int32_t rot_digits, int32_t m, int32_t k, int32_t n, const int32_t* indptr_a,
                     const int32_t* indices_a, const int32_t* indptr_b, const int32_t* indices_b, int64_t counts[6]);

/* The distinct rotation step amounts the plan for A B uses (each < S); writes up to cap of them into
 * out and the total into *n_out. Feed them to fhe_keygen_rotations when rot_digits == 1. */
int fhe_plan_rotations(fhe_ctx* ctx, const fhe_mat* A, const fhe_mat* B, int32_t* out, size_t cap, size_t* n_out);

/* Decrypts and decodes a matrix handle into out[rows * cols] (row-major; for an encrypted CSR/CSC
 * operand, out receives its values array in packing order instead, length nnz): the client-side
 * step after the server's result comes back (Figure 1). Decryption uses the exact CRT of limbs
 * q_0, q_1; decoding divides by the handle's scale. Errors: FHE_ESHAPE if cap is too small,
 * FHE_EINVAL for NULL arguments. */
int fhe_decrypt_decode(fhe_ctx* ctx, const fhe_sk* sk, const fhe_mat* M, void* stream, double* out, size_t cap);

/* Shape of a matrix handle: kind (0 = CSR operand, 1 = CSC operand, 2 = dense result), rows, cols,
 * number of ciphertext chunks, active Q limbs per chunk, scale. Any out-pointer may be NULL. */
int fhe_mat_info(const fhe_mat* M, int32_t* kind, int32_t* rows, int32_t* cols, int32_t* chunks, int32_t* limbs,
                 double* scale);

/* Exports ciphertext chunk `chunk` of M in the coefficient domain into out[cap] (uint64,
 * [2][limbs][N]). Errors: FHE_ESHAPE if cap is too small, FHE_EINVAL for a bad chunk index. */
int fhe_mat_export(fhe_ctx* ctx, const fhe_mat* M, int32_t chunk, uint64_t* out, size_t cap, void* stream);
/* Releases M. The device block of a matmul result goes back to its context (while the context
 * lives), which hands it to its next result of the same size, up to FHE_RESULT_POOL_MB (environment,
 * default 4096 MiB; 0 keeps none) of kept blocks per context; a context under fhe_server_create keeps
 * none. Free a matrix only when no call that uses it is running. */
void fhe_mat_free(fhe_mat* M);

/* ---- Operation-level interface on single ciphertexts (the operations Algorithm 2 issues). ---- */

/* Imports a ciphertext given in the coefficient domain: coeffs[ncomp][limbs][N], residues < q_i,
 * ncomp in {2, 3}, 1 <= limbs <= n_q. */
int fhe_ct_import(fhe_ctx* ctx, const uint64_t* coeffs, int32_t ncomp, int32_t limbs, double scale, void* stream,
                  fhe_ct** out);
/* Exports in the coefficient domain into out[cap] ([ncomp][limbs][N]). */
int fhe_ct_export(fhe_ctx* ctx, const fhe_ct* ct, uint64_t* out, size_t cap, void* stream);
int fhe_ct_info(const fhe_ct* ct, int32_t* ncomp, int32_t* limbs, double* scale);
/* EvalRotate: left rotation by r (automorphism tau_(5^step) + hybrid key switch per step). */
int fhe_ct_rotate(fhe_ctx* ctx, const fhe_ct* ct, int32_t r, void* stream, fhe_ct** out);
/* EvalMult + Relinearize of two 2-component ciphertexts at the same level (scale multiplies). */
int fhe_ct_mult_relin(fhe_ctx* ctx, const fhe_ct* a, const fhe_ct* b, void* stream, fhe_ct** out);
/* Rescale: drops the last limb with nearest rounding (scale /= dropped prime). Needs >= 2 limbs. */
int fhe_ct_rescale(fhe_ctx* ctx, const fhe_ct* ct, void* stream, fhe_ct** out);
/* Plaintext multiply by the one-hot mask at `slot` (scale *= 2^mask_bits * q_(n_q-2)). */
int fhe_ct_mask(fhe_ctx* ctx, const fhe_ct* ct, int32_t slot, void* stream, fhe_ct** out);
/* EvalAdd of two ciphertexts of equal shape. */
int fhe_ct_add(fhe_ctx* ctx, const fhe_ct* a, const fhe_ct* b, void* stream, fhe_ct** out);
void fhe_ct_free(fhe_ct* ct);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops and
 * harnesses that forbid hipMalloc): fhe_ct_rotate into an existing caller-owned ciphertext `out`
 * (2 components, the limb count of `ct`; it may be `ct` itself), with the same result bit for bit.
 * Nothing is allocated on the device: the automorphism's copy of the input, the key-switch workspace
 * and the launch argument words live in one static device array of FHE_NOALLOC_SCRATCH_BYTES per
 * GPU, which the library holds until the process ends. A rotation needing more (4 KiB + 8 bytes x
 * (2 limbs N + the key-switch workspace words)) fails with FHE_ENOMEM before any work is enqueued;
 * every level fits at N <= 2^15 and at N = 2^16 with up to 24 Q + 3 special primes (alpha = 3).
 * All calls on one GPU share its array and nothing in it needs clearing: calls that overlap on one
 * GPU (other host threads or streams) race and must be serialised by the caller. Returns once
 * `stream` has finished the rotation; out's scale becomes ct's. Errors: FHE_EINVAL (NULL),
 * FHE_ESHAPE (a 3-component ct or out, or out's limb count differs), FHE_ENOMEM (scratch too
 * small), FHE_EKEY (a rotation key is missing), FHE_EDEVICE. */
#define FHE_NOALLOC_SCRATCH_BYTES ((size_t)192 << 20)
int fhe_ct_rotate_into(fhe_ctx* ctx, const fhe_ct* ct, int32_t r, fhe_ct* out, void* stream);


/* ---- Request loop with continuous batching (Section 3: ciphertexts and keys stay on the GPU). ---- */

typedef struct fhe_server fhe_server;

/* Starts a serving loop over nctx contexts (parameter sets with their evaluation keys resident, all on
 * one GPU): a worker thread with its own HIP stream serves the requests of every context. Requests
 * wait in one arrival-order queue (at most max_queue) and are admitted while fewer than max_inflight
 * run and the server's memory stays within hbm_budget bytes, one budget shared by all contexts:
 *   - charged once, at creation: each context's constant tables and evaluation keys, and each
 *     context's executor scratch, capped at workspace_bytes per context (0: automatic, a quarter of
 *     what the budget leaves after the keys divided among the contexts, at most FHE_WORKSPACE_MB);
 *     the requests of one context share that scratch within a step. A larger scratch left on a
 *     context by earlier calls is released. Grouped plans (fhe_server_set_plan) add the tail's
 *     second ping-pong buffers to this part;
 *   - charged per request from admission to completion: its result chunks (2 (n_q - 2) N words each)
 *     and, for grouped plans, its products kept resident (2 (n_q - 1) N words each) and, for the
 *     digit tree, its partial sums.
 * Each scheduling step runs, per context, the next slice_products products (with all their matched
 * pairs) of every admitted request of that context as one merged launch stream, so a request that
 * arrives while others run joins the next step. Errors: FHE_EINVAL (NULL or out-of-range arguments,
 * contexts on different devices), FHE_ENOMEM (the fixed part exceeds hbm_budget), FHE_EDEVICE. */
int fhe_server_create(fhe_ctx* const* ctxs, size_t nctx, size_t hbm_budget, size_t workspace_bytes,
                      int32_t max_inflight, int32_t slice_products, int32_t max_queue, fhe_server** out);

/* Plan mode of the server's requests (FHE_PLAN_PER_PAIR, FHE_PLAN_GROUPED or FHE_PLAN_TREE, optionally
 * or-ed with FHE_PLAN_HOIST; not FHE_PLAN_GRAPH). Grouped and tree plans run every request as one
 * slice (all of its products in one step, merged with the other requests of that context in that step);
 * each result is bit-identical to fhe_spmspm_plan in the same mode. Only before the first submission:
 * FHE_EAGAIN afterwards; FHE_EINVAL for an unknown mode; FHE_ENOMEM if the grouped tail buffers do
 * not fit the budget. */
int fhe_server_set_plan(fhe_server* s, int32_t mode);

/* Queues C = A B on context ctxs[ctx_id] (A: CSR handle, B: CSC handle of that context; both must stay
 * alive until the request is polled). Returns a ticket. In the per-pair plan the request's plan
 * (Algorithm 1's merge) is built by the worker at admission, so submission costs O(1); grouped plans
 * build it here, since their charge depends on it. Errors: FHE_EAGAIN (queue full), FHE_ENOMEM
 * (the request's own charge does not fit the budget even with nothing else in flight), FHE_EINVAL
 * (bad handle kinds or ctx_id), FHE_ESHAPE (A.cols != B.rows). */
int fhe_server_submit(fhe_server* s, int32_t ctx_id, const fhe_mat* A, const fhe_mat* B, uint64_t* ticket);

/* Waits up to wait_ms for the ticket. FHE_OK: *C_out receives the result (bit-identical to
 * fhe_spmspm, or to fhe_spmspm_plan in the server's plan mode, on the same operands) and *latency_s
 * the submit-to-completion time; the ticket is retired. FHE_EAGAIN: not finished yet. FHE_ECANCELED:
 * the server was closed before the request was admitted; the ticket is retired. Other codes: the
 * request failed (for instance FHE_EKEY for a missing rotation key) and the ticket is retired. */
int fhe_server_poll(fhe_server* s, uint64_t ticket, int32_t wait_ms, fhe_mat** C_out, double* latency_s);

/* Cancels a request: one still waiting for admission at once, one in flight at the next step
 * boundary (its partial result is dropped and its memory released); its poll then returns
 * FHE_ECANCELED. A request already finished keeps its outcome. Errors: FHE_EINVAL (unknown ticket). */
int fhe_server_cancel(fhe_server* s, uint64_t ticket);

typedef struct fhe_server_info {
  double p50_s, p99_s;        /* latency percentiles over completed requests (0 if none) */
  int64_t completed, failed, cancelled, inflight, queued;
  int64_t steps;              /* scheduling steps that ran work */
  int64_t max_merged;         /* most requests of one context merged into one launch stream */
  int64_t max_step_requests;  /* most requests (all contexts) served by one step */
  size_t budget_bytes, fixed_bytes, inflight_bytes; /* the budget, its fixed part, the admitted requests' charges */
} fhe_server_info;

/* Snapshot of the server's counters. Errors: FHE_EINVAL. */
int fhe_server_stats(fhe_server* s, fhe_server_info* out);

/* Cancels the requests still waiting for admission (their polls return FHE_ECANCELED), lets the
 * admitted ones run to the end, stops the worker, wakes the threads waiting in fhe_server_poll and
 * waits for them to return, then frees the server (result handles not yet polled are released with
 * it). No call on s may start once fhe_server_free has been called. */
void fhe_server_free(fhe_server* s);

/* ---- Measurement hooks (not part of the method). ---- */

/* Per-kernel device timing. fhe_profile_enable(1) clears earlier records and starts bracketing every
 * kernel launch of this library with two HIP events on the launch stream; fhe_profile_enable(0) stops
 * recording (records are kept until the next enable). Process-wide. */
int fhe_profile_enable(int on);

typedef struct fhe_kernel_stat {
  char name[32];        /* kernel name, e.g. "ks_inner", "ntt_fwd_p1" */
  int64_t launches;     /* recorded launches */
  double total_ms;      /* sum of event-measured durations */
  double bytes;         /* sum of the launches' algorithmic HBM bytes (reads + writes the kernel must do) */
  double mulmods;       /* sum of the launches' modular products (NTT butterflies, pointwise and
                           base-conversion products; 0 for kernels that are not counted) */
} fhe_kernel_stat;

/* Aggregates the records per kernel name into out[cap] (synchronises on the recorded events);
 * returns the number of distinct kernels (entries beyond cap are not written). */
int fhe_profile_read(fhe_kernel_stat* out, size_t cap);

/* Throughput probe of the modular products the kernels use, for stating ALU bounds: runs 8
 * independent chains of `iters` dependent products per thread over a full grid on `device` and
 * writes the products per second of the second of two launches into *per_s. kind 0: the FP64 product
 * of the Q primes (q < 2^50: quotient estimate from a precomputed w/q, remainder recovered exactly by
 * two FMAs), 1: the lazy Shoup product of the special primes (p < 2^61), 2: the Montgomery product
 * (R = 2^64) of the special primes' key words. Allocates device memory. Errors: FHE_EINVAL,
 * FHE_EDEVICE. */
int fhe_bench_mulmod(int32_t device, int32_t kind, int32_t iters, void* stream, double* per_s);

/* Message of the last failing call on this thread ("" if none). */
const char* fhe_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FHE_SPMSPM_H */
