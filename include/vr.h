/*
 * vr.h -- C ABI of the MI355X (gfx950) library for the column-wise encrypted
 * inference path of "Volley Revolver: A Novel Matrix-Encoding Method for
 * Privacy-Preserving Deep Learning (Inference++)".
 *
 * Scheme: RNS-CKKS.  The paper's HE interface is KeyGen, Enc_pk, Dec_sk, Add,
 * Mul, cMul and Rot (left rotation), with rescaling treated as automatic
 * (Preliminaries, "Fully Homomorphic Encryption").  The usage model ("Secure
 * Inference", Usage Model) splits the roles: the data owner and model provider
 * hold the secret key and call the client functions; the cloud calls the
 * server functions, which never see a secret key.
 *
 * Conventions for every function:
 *  - Returns vr_status; VR_OK is 0, errors are negative.  On error every
 *    output handle is set to NULL, no partial result exists, and
 *    vr_last_error() (thread-local) describes the failure.  No C++ exception
 *    crosses this boundary.
 *  - Handles are opaque and owned by the caller.  Every handle a function
 *    returns is new and must be released with the matching vr_free_*.
 *    Inputs are never modified.
 *  - Host pointers (double*, uint64_t*, int32_t*) are read or written before
 *    the call returns.  Device memory behind handles comes from the
 *    context's caching allocator (stream-ordered) unless a hook is set.
 *  - `stream` is a hipStream_t; NULL means the context's stream (the null
 *    stream unless vr_context_set_stream was called).  Server calls only
 *    enqueue work; vr_ct_export, vr_pt_export, vr_decode and the serving poll
 *    synchronise.
 *  - Polynomials are stored on the device in the evaluation (NTT) domain;
 *    every export is in the coefficient domain, uint64 [component][limb][t],
 *    limbs q_0..q_level, values in [0, q).
 *  - The product path runs on the GPU only.  Without a usable gfx950 device,
 *    vr_context_create fails with VR_EDEVICE.
 */
#ifndef VR_H
#define VR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VR_OK = 0,
    VR_EINVAL = -1,     /* bad argument or shape                                  */
    VR_ESECURITY = -2,  /* parameters above the 128-bit bound, allow_insecure = 0 */
    VR_ELEVEL = -3,     /* operand levels differ / no level left                  */
    VR_ESCALE = -4,     /* operand scales are not bitwise-equal doubles           */
    VR_ENOKEY = -5,     /* missing rotation key                                   */
    VR_ENOMEM = -6,     /* device allocation failed                               */
    VR_EDEVICE = -7,    /* HIP runtime error or no gfx950 device                  */
    VR_EBUSY = -8,      /* serving: request can never fit the memory budget       */
    VR_ECANCELED = -9   /* serving: request cancelled (deadline)                  */
} vr_status;

typedef struct vr_context vr_context;
typedef struct vr_ciphertext vr_ciphertext;
typedef struct vr_plaintext vr_plaintext;
typedef struct vr_secret_key vr_secret_key;
typedef struct vr_eval_keys vr_eval_keys;
typedef struct vr_server vr_server;

/* RNS-CKKS parameters.  Primes: for each bit size in order (q_bits then
 * p_bits), the largest prime q < 2^b with q = 1 mod 2N not taken yet.
 * alpha = ceil(n_q / dnum) Q primes per key-switching digit.  sigma must be
 * 3.2 (the error table is built for it). */
typedef struct {
    uint32_t log_n;          /* N = 2^log_n, 3 <= log_n <= 16           */
    uint32_t n_q;            /* Q chain length L+1                      */
    uint32_t n_p;            /* special primes K >= 1                   */
    uint32_t dnum;           /* key-switching digits                    */
    const uint32_t *q_bits;  /* [n_q], each in [20, 60]                 */
    const uint32_t *p_bits;  /* [n_p]                                   */
    double log2_scale;       /* default encoding scale 2^log2_scale     */
    double sigma;            /* error standard deviation (3.2)          */
    uint32_t allow_insecure; /* 1: skip the 128-bit bound (labelled)    */
} vr_params;

/* ---------------------------------------------------------------- context */

/* Creates a context on `device`: primes, roots, twiddles and base-conversion
 * constants go to device memory.  Checks the 128-bit bound (total prime bits
 * <= 218 / 438 / 881 / 1740 for N = 2^13 / 2^14 / 2^15 / 2^16, HE standard
 * 2018, 2^16 extrapolated conservatively): VR_ESECURITY unless allow_insecure. */
vr_status vr_context_create(const vr_params *params, int device, vr_context **out);
void vr_context_destroy(vr_context *ctx);  /* NULL-safe; frees device tables */

/* moduli[0..n_q+n_p) = q_0..q_L, p_0..p_{K-1}; cap = capacity of moduli. */
vr_status vr_context_moduli(const vr_context *ctx, uint64_t *moduli, size_t cap);
/* info[0..8) = log_n, slots, n_q, n_p, dnum, alpha, secure, total_bits */
vr_status vr_context_info(const vr_context *ctx, uint32_t *info8, double *default_scale);
/* Stream used when a call passes stream = NULL. */
vr_status vr_context_set_stream(vr_context *ctx, void *stream);
/* Optional device allocator (e.g. a framework's caching allocator).  Both
 * functions receive the stream the memory is used on and `user`.  NULL
 * restores the built-in caching allocator: blocks from hipMalloc are kept
 * after their handles are freed and reused, stream-ordered, by later calls;
 * they return to the runtime on vr_context_trim, on a failed hipMalloc, and
 * when the context and every handle from it are gone.  A handle must be
 * freed before the stream it was produced on is destroyed. */
vr_status vr_context_set_allocator(vr_context *ctx,
                                   void *(*alloc_fn)(size_t bytes, void *stream, void *user),
                                   void (*free_fn)(void *ptr, void *stream, void *user),
                                   void *user);
/* Built-in allocator: bytes held from the runtime and bytes behind live
 * handles and in-flight work. */
vr_status vr_context_mem_info(vr_context *ctx, size_t *reserved, size_t *in_use);
/* Synchronises the device and returns the built-in allocator's cached free
 * blocks to the runtime. */
vr_status vr_context_trim(vr_context *ctx);
/* Kernel choices.  Knob "base_convert": "auto" (default: each base-conversion
 * table times the 128-bit vector-ALU kernel, the exact FP64 kernel and the
 * INT8-split MFMA kernel, twice each on its first call, and keeps the
 * fastest; all give identical words), "alu", "fp64", "mfma" or "split" (for
 * tables whose only target of 2^51 or more is the first, the FP64 kernel on
 * the other targets with the ALU kernel on that one; elsewhere FP64 where
 * that applies, else the ALU kernel).  Knob
 * "ntt": "auto" (default: the first transform in each direction times the
 * candidate pass plans -- one LDS-resident pass, two passes with every split
 * of log N and 8..128 groups per workgroup, and at N = 2^15, 2^16 the
 * compile-time two-pass kernels -- on 256 scratch limbs and keeps the
 * fastest), "fixed" (the built-in plan) or "cand:<i>" (candidate i,
 * for tests; VR_EINVAL at the next transform if there is none).  Knob
 * "switch_chunk": "<k>" key-switches at most k ciphertexts per launch in the
 * layer calls ("0": as many as 16 GiB of scratch allows, the default).  Knob
 * "conv_prune": "on" (default) or "off": in the network call, when the FC
 * reads the conv's output only on limbs q_0..q_f (the unrelinearised x^2
 * into an FC at level f), the conv's rotations, sums and ModDown by P q_l
 * produce only those limbs; "off" computes every limb and drops them after
 * (identical words).  Knob "fc_compact": "on" (default) or "off": FC weights
 * from vr_encode_fc_weights lie in the subring Z[X^r], r = N / (2 block), so
 * each limb in the evaluation domain repeats in runs of r words; the FC reads
 * a copy that keeps each run once (N / r words per limb) instead of the full
 * limbs ("off"; identical words).  Knob "lincomb_wide": "on" (default) or
 * "off": the conv's weighted sums on moduli of 2^51 or more (the 60-bit
 * q_0) as exact FP64 sums of 21-bit pieces, or ("off") as 64-bit integer
 * products (identical words).
 * Tuning synchronises
 * once; the transform is the same exact map under every plan. */
vr_status vr_context_set_tuning(vr_context *ctx, const char *knob, const char *value);
/* One line per base-conversion table built so far (shape, kernel chosen) and
 * per tuned NTT direction (passes as {first stage, stages, log groups}). */
vr_status vr_context_tuning_report(vr_context *ctx, char *buf, size_t cap);
const char *vr_last_error(void);

/* ------------------------------------------------------------ client side */

/* Randomness.  Every `seed` below is a 256-bit ChaCha20 key given as four
 * host words (seed[0] holds key bytes 0..7, little-endian; seed[3] bytes
 * 24..31); a NULL seed is VR_EINVAL.  The security level the context reports
 * holds only for a seed drawn uniformly at random and kept secret: a seed
 * with a small range (for instance a 64-bit value in seed[0] and zeros
 * elsewhere, as the tests use) lets anyone holding the public key search the
 * range and recover the secret key.  Encryption randomness is a function of
 * (seed, ct_id) only: under one public key a (seed, ct_id) pair must never be
 * used twice, since two encryptions with the same pair share their mask and
 * their difference reveals the difference of the messages. */

/* Secret key s (ternary), public key, relinearisation key and one rotation
 * key per distinct Galois element 5^(step mod S) in rot_steps (hybrid key
 * switching, dnum digits, special primes P).  All randomness is the ChaCha20
 * stream keyed by `seed` (purpose/object nonce per key part), so the keys are
 * a deterministic function of (params, seed, steps). */
vr_status vr_keygen(vr_context *ctx, const uint64_t seed[4], const int32_t *rot_steps, size_t n_steps,
                    vr_secret_key **sk, vr_eval_keys **ek);
/* Adds rotation keys (same seed as the original keygen keeps them canonical). */
vr_status vr_keys_add_rotations(vr_context *ctx, const vr_secret_key *sk, vr_eval_keys *ek,
                                const uint64_t seed[4], const int32_t *rot_steps, size_t n_steps);
/* Canonical embedding: slot j of x (j < n <= S, rest zero) is the value at
 * the root psi^(5^j); coefficients m_t = round-half-away((2 scale / N) Re
 * sum_j x_j exp(-i pi 5^j t / N)), |m_t| < 2^62, reduced into q_0..q_level. */
vr_status vr_encode(vr_context *ctx, const double *x, size_t n, uint32_t level, double scale,
                    vr_plaintext **out);
/* Public-key encryption (v b + e0 + m, v a + e1) with v, e0, e1 drawn from
 * the stream of (seed, ct_id); the pair must be unique under one public key. */
vr_status vr_encrypt(vr_context *ctx, const vr_eval_keys *ek, const vr_plaintext *pt,
                     const uint64_t seed[4], uint64_t ct_id, vr_ciphertext **out);
/* Column-wise image encoding (abstract and contributions: an h x w image is
 * w ciphertexts of h slots).  x is [B][C][h][w] row-major FP64.  Block height
 * H' = pow2(h + 2 pad); image b occupies slots b H' .. b H' + H' - 1 of every
 * column ciphertext (virtual ciphertexts), row i at b H' + pad + i.  Requires
 * B H' <= S.  cols receives C*w handles, column (c, j) at index c*w + j,
 * encrypted with ct_id = first_ct_id + c*w + j (the caller keeps the ranges
 * of different calls under one seed and public key disjoint). */
vr_status vr_encrypt_columns(vr_context *ctx, const vr_eval_keys *ek, const double *x,
                             uint32_t B, uint32_t C, uint32_t h, uint32_t w, uint32_t pad,
                             uint32_t level, const uint64_t seed[4], uint64_t first_ct_id,
                             vr_ciphertext **cols);
/* Matrix operand as n column ciphertexts (abstract: A (m x n) and B (n x p)
 * as n ciphertexts each).  role 0: M is A (rows x cols = m x n), ciphertext k
 * holds slot s -> A[s mod M'][k] (column k of the tau_a encoding, period
 * M' = pow2(m)).  role 1: M is B (n x p), ciphertext k holds slot s ->
 * B[k][s mod P'] (column k of the tau_b encoding, period P' = pow2(p)).
 * Zeros past m rows / p columns.  out receives n handles.  Outer-product
 * operands (vr_matmul_outer): role 2: M is A (m x n), T n ciphertexts
 * A'_{t,k} at index t n + k (T = ceil(m / R), R = S / P'), slot r P' + j ->
 * A[t R + r][k] for j < p and t R + r < m; role 3: M is B (n x p), n
 * ciphertexts B'_k, slot r P' + j -> B[k][j] for j < p and every r < R.
 * Column-block operands (vr_matmul_block; blocks of Mb = P' ceil((m + P' -
 * 1) / P') slots, c columns per ciphertext, nb = ceil(n / c) ciphertexts,
 * see vr_matmul_plan): role 4: M is A (m x n), block j of ciphertext K holds
 * column K c + j of A in its first m slots; role 5: M is B (n x p), block j
 * holds row K c + j of B, entry r mod P' in slot r of the block (r mod P' <
 * p).  out receives nb handles for roles 4 and 5.
 * Ciphertext i is encrypted with ct_id = first_ct_id + i (ranges of
 * different calls under one seed and public key must not overlap). */
vr_status vr_encrypt_matrix_columns(vr_context *ctx, const vr_eval_keys *ek, const double *M,
                                    uint32_t rows, uint32_t cols, uint32_t role, uint32_t m,
                                    uint32_t p, uint32_t level, const uint64_t seed[4],
                                    uint64_t first_ct_id, vr_ciphertext **out);
/* m' = c0 + c1 s (+ c2 s^2): plaintext at the ciphertext's level and scale. */
vr_status vr_decrypt(vr_context *ctx, const vr_secret_key *sk, const vr_ciphertext *ct,
                     vr_plaintext **out);
/* Slots 0..n-1 from limb q_0 (centred): valid while |coefficients| < q_0/2. */
vr_status vr_decode(vr_context *ctx, const vr_plaintext *pt, double *out, size_t n);

/* ------------------------------------------------------------ server side */

/* Add / Sub: levels equal (VR_ELEVEL) and scales bitwise equal (VR_ESCALE). */
vr_status vr_add(vr_context *ctx, const vr_ciphertext *a, const vr_ciphertext *b,
                 vr_ciphertext **out, void *stream);
vr_status vr_sub(vr_context *ctx, const vr_ciphertext *a, const vr_ciphertext *b,
                 vr_ciphertext **out, void *stream);
/* cMul by a scalar: C = round-half-away(c * c_scale) as an exact integer,
 * every limb times [C]_q; scale *= c_scale. */
vr_status vr_mul_const(vr_context *ctx, const vr_ciphertext *a, double c, double c_scale,
                       vr_ciphertext **out, void *stream);
/* Adds [round-half-away(c * scale)]_q to the constant coefficient of c0. */
vr_status vr_add_const(vr_context *ctx, const vr_ciphertext *a, double c, vr_ciphertext **out,
                       void *stream);
/* cMul by an encoded plaintext (limb-wise product); scale *= pt scale.  The
 * plaintext level must be >= the ciphertext level. */
vr_status vr_mul_plain(vr_context *ctx, const vr_ciphertext *a, const vr_plaintext *pt,
                       vr_ciphertext **out, void *stream);
/* (a0 b0, a0 b1 + a1 b0, a1 b1): a 3-component ciphertext. */
vr_status vr_tensor(vr_context *ctx, const vr_ciphertext *a, const vr_ciphertext *b,
                    vr_ciphertext **out, void *stream);
/* Key-switches the s^2 component back to s (hybrid key switching). */
vr_status vr_relinearize(vr_context *ctx, const vr_eval_keys *ek, const vr_ciphertext *a,
                         vr_ciphertext **out, void *stream);
/* Mul of the paper: tensor then relinearise (no rescale). */
vr_status vr_mul(vr_context *ctx, const vr_eval_keys *ek, const vr_ciphertext *a,
                 const vr_ciphertext *b, vr_ciphertext **out, void *stream);
/* Divide by q_level with a centred last limb; level - 1; scale /= q_level. */
vr_status vr_rescale(vr_context *ctx, const vr_ciphertext *a, vr_ciphertext **out, void *stream);
/* Relinearisation and the rescale that follows it (every ciphertext product of
 * "Homomorphic Matrix Multiplication" and of the layers in "Secure Inference"
 * is a Mul followed by a Rescale) as one ModDown by P q_level: with
 * (u0, u1) the key-switch sums of the s^2 component over q_0..q_level and the
 * special primes, out_j = round((u_j + P c_j) / (P q_level)) on q_0..q_{level-1}
 * (the centred fast conversion of ModDown, now from {q_level, p_0..p_{K-1}}).
 * `a` must have 3 components and level >= 1 (VR_ELEVEL otherwise); output at
 * level - 1 with scale / q_level.  Equal to vr_rescale(vr_relinearize(a)) up
 * to one rounding (a few units in the last place of the coefficients), not
 * word for word.  *out is a new ciphertext owned by the caller.  The layer
 * calls below write this operation RelinRescale(.) and use it for every
 * product they relinearise. */
vr_status vr_relin_rescale(vr_context *ctx, const vr_eval_keys *ek, const vr_ciphertext *a,
                           vr_ciphertext **out, void *stream);
/* vr_tensor then vr_relin_rescale. */
vr_status vr_mul_rescale(vr_context *ctx, const vr_eval_keys *ek, const vr_ciphertext *a,
                         const vr_ciphertext *b, vr_ciphertext **out, void *stream);
/* Drop limbs above `level` (scale unchanged). */
vr_status vr_mod_drop(vr_context *ctx, const vr_ciphertext *a, uint32_t level,
                      vr_ciphertext **out, void *stream);
/* Rot(ct, step): slots rotated left by step (Galois element 5^step). */
vr_status vr_rotate(vr_context *ctx, const vr_eval_keys *ek, const vr_ciphertext *a,
                    int32_t step, vr_ciphertext **out, void *stream);
/* k rotations sharing one ModUp (hoisted); bit-identical to k vr_rotate calls. */
vr_status vr_rotate_many(vr_context *ctx, const vr_eval_keys *ek, const vr_ciphertext *a,
                         const int32_t *steps, size_t k, vr_ciphertext **outs, void *stream);

/* n ciphertexts (same level and scale) each rotated by the same step, in one
 * batched key switch: the rotation key streams from HBM once for all of them.
 * Bit-identical to n vr_rotate calls.  outs receives n handles. */
vr_status vr_rotate_batch(vr_context *ctx, const vr_eval_keys *ek, const vr_ciphertext *const *in,
                          size_t n, int32_t step, vr_ciphertext **outs, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * rotation of vr_rotate, bit-identical to it, on a ciphertext given as device
 * limbs.  in: device pointer to [2][level+1][N] uint64, c0 then c1, each limb
 * i in the evaluation domain modulo q_i (the form ciphertext handles hold on
 * the device: vr_ntt forward of the coefficient limbs vr_ct_export returns);
 * out: device pointer to caller-owned memory of the same size and form, not
 * overlapping in; the scale is the input's.  Every
 * key-switching intermediate lives in one fixed device array of the library,
 * VR_NOALLOC_SCRATCH_BYTES per GPU (held from the first context on that GPU
 * to process exit); a level whose key switch needs more returns VR_EINVAL
 * (the limit admits every level at N <= 2^14 and, at N = 2^16 with nine
 * special primes and dnum 3, the whole L = 24 chain).  The call allocates
 * nothing: the NTT plans and this level's base-conversion tables must exist
 * already (else VR_EINVAL; one vr_rotate at the level builds them), and a
 * missing rotation key is VR_ENOKEY.  Calls on one GPU share the array: calls
 * that overlap in time on one GPU (different streams or threads) race; calls
 * on one stream are ordered and safe.  Enqueued on `stream` (NULL = the
 * context's) and returns without synchronising. */
#define VR_NOALLOC_SCRATCH_BYTES (144ull << 20)
vr_status vr_rotate_noalloc(vr_context *ctx, const vr_eval_keys *ek, const uint64_t *in, uint32_t level,
                            int32_t step, uint64_t *out, void *stream);

/* Column-split matrix product (abstract and contributions; "Homomorphic
 * Matrix Multiplication" with RowShifter reduced to one rotation and the
 * ciphertext-pair split of "Parallelized Matrix Multiplication"): from A_k,
 * Bbar_k (k < n, from vr_encrypt_matrix_columns), for idx < P',
 *   C[idx] = RelinRescale(sum_k A_k * Rot(Bbar_k, idx)),
 * slot i < m of C[idx] holding (A B)[i][(i + idx) mod P'].  Rotation keys
 * for steps 1..P'-1; C receives P' handles.  For m < p the product is the
 * paper's transposed one, C^T = B^T A^T, on the same ciphertexts with their
 * roles swapped: M' = pow2(m) outputs, slot i < p of C[idx] holding
 * (A B)[(i + idx) mod M'][i], rotation keys for steps 1..M'-1. */
vr_status vr_matmul(vr_context *ctx, const vr_eval_keys *ek, const vr_ciphertext *const *A,
                    const vr_ciphertext *const *Bbar, uint32_t m, uint32_t n, uint32_t p,
                    vr_ciphertext **C, void *stream);

/* Outer-product matrix product, the rotation-free form of the split product
 * (split operands are multiplied pair-wise and summed by linearity: "Secure
 * Inference"): C is tiled by R = S / P' rows per ciphertext (P' = pow2(p),
 * S slots), T = ceil(m / R) tiles.  A holds T n ciphertexts A'_{t,k} (index
 * t n + k; vr_encrypt_matrix_columns role 2): slot r P' + j = A[t R + r][k]
 * for j < p; B holds n ciphertexts B'_k (role 3): slot r P' + j = B[k][j].
 *   C[t] = RelinRescale(sum_k A'_{t,k} * B'_k),
 * slot r P' + j of C[t] holding (A B)[t R + r][j].  No rotation and no
 * rotation key; any m, n and p with P' <= S.  C receives T handles.
 * VR_EINVAL for empty shapes or p above S; VR_ELEVEL / VR_ESCALE when the
 * inputs differ in level or scale. */
vr_status vr_matmul_outer(vr_context *ctx, const vr_eval_keys *ek, const vr_ciphertext *const *A,
                          const vr_ciphertext *const *B, uint32_t m, uint32_t n, uint32_t p,
                          vr_ciphertext **C, void *stream);

/* Column-block form of the column-split product: c columns per ciphertext
 * (roles 4 / 5 of vr_encrypt_matrix_columns), each in a block padded by P' -
 * 1 slots past m so that every rotated read of Bbar stays in its own block
 * wherever A is non-zero (no RowShifter fix-up):
 *   D[idx] = RelinRescale(sum_K A_K * Rot(Bbar_K, idx)), idx < P',
 * then the c blocks folded into block 0, D += Rot(D, Mb 2^t) for t <
 * log2 c.  Slot i < m of C[idx] holds (A B)[i][(i + idx) mod P'].  Needs
 * m >= p; rotation keys for steps 1..P'-1 and Mb 2^t.  nb (P' - 1) + P'
 * log2 c rotations against n (P' - 1) for the column-split form.  C
 * receives P' handles. */
vr_status vr_matmul_block(vr_context *ctx, const vr_eval_keys *ek, const vr_ciphertext *const *A,
                          const vr_ciphertext *const *Bbar, uint32_t m, uint32_t n, uint32_t p,
                          vr_ciphertext **C, void *stream);

/* Cost-model planner for one product A (m x n) B (n x p) at `level`: fills
 * costs[form] for the column-split (vr_matmul), column-block
 * (vr_matmul_block) and outer-product (vr_matmul_outer) forms -- the client's
 * ciphertext count (its upload), key switches (rotations and
 * relinearisations), tensors, and an estimated device time from the limb
 * passes each form streams (at 5 TB/s effective) -- and picks the cheapest
 * feasible form whose client ciphertexts fit max_client_cts (0: no limit).
 * For m < p the column forms multiply the transposes (transposed = 1: the
 * client encodes B^T as A and A^T as B).  VR_EINVAL when no form fits. */
enum { VR_MATMUL_COLUMN_SPLIT = 0, VR_MATMUL_COLUMN_BLOCK = 1, VR_MATMUL_OUTER = 2, VR_MATMUL_NONE = 0xffffffffu };
typedef struct {
    uint32_t feasible, transposed;
    uint64_t client_cts, key_switches, tensors;
    double est_us;
} vr_matmul_cost;
vr_status vr_matmul_plan(vr_context *ctx, uint32_t m, uint32_t n, uint32_t p, uint32_t level,
                         uint64_t max_client_cts, vr_matmul_cost costs[3], uint32_t *chosen);
/* Column convolution (conv layer of "Convolutional Neural Networks", with
 * per-channel accumulation of "Parallelized Convolution Operation"): inputs
 * in[c*w + j] from vr_encrypt_columns; K is [C_out][C_in][k][k], bias
 * [C_out] (FP64).  Output column (c', j') at index c'*w_out + j':
 *   Rescale(sum_{c,u,v} MulConst(Rot(in[c][s j'+v-pad], u), K[c'][c][u][v],
 *           q_level) + AddConst(bias[c'])),
 * slot b H' + s i' holding output row i' of image b.  Needs rotation keys for
 * steps 1..k-1.  When k > 1 and the special primes number at most level + 1,
 * the rotations keep their key-switch sums in the extended basis (P times the
 * rotated ciphertext over q_0..q_level and the special primes), the sum is
 * taken there and one ModDown by P q_level per output both finishes the key
 * switches and rescales (one rounding per output instead of one per
 * rotation; the same message). */
vr_status vr_conv2d(vr_context *ctx, const vr_eval_keys *ek, const vr_ciphertext *const *in,
                    uint32_t C_in, uint32_t h, uint32_t w, uint32_t pad, const double *K,
                    const double *bias, uint32_t C_out, uint32_t k, uint32_t stride,
                    vr_ciphertext **out, void *stream);
/* The same layer on n_sets independent image sets (mini-batches of the
 * paper's "Secure Inference" section, each its own C_in*w column set) in one
 * batched evaluation: in[s*C_in*w + c*w + j], out[s*C_out*w_out + c'*w_out + j'].
 * Identical limbs to n_sets vr_conv2d calls. */
vr_status vr_conv2d_sets(vr_context *ctx, const vr_eval_keys *ek, const vr_ciphertext *const *in,
                         uint32_t n_sets, uint32_t C_in, uint32_t h, uint32_t w, uint32_t pad,
                         const double *K, const double *bias, uint32_t C_out, uint32_t k,
                         uint32_t stride, vr_ciphertext **out, void *stream);
/* x^2 activation on n ciphertexts: RelinRescale(Tensor(y, y)). */
vr_status vr_square(vr_context *ctx, const vr_eval_keys *ek, const vr_ciphertext *const *in,
                    size_t n, vr_ciphertext **out, void *stream);
/* Encrypted-weight mode (the paper's usage model, "Homomorphic CNN
 * Evaluation": the model provider encrypts the weights, the cloud sees none
 * in the clear).  The conv of vr_conv2d with K_ct[((c' C_in + c) k + u) k + v]
 * encrypting K[c'][c][u][v] in every slot at scale q_l (same level as the
 * inputs) and bias_ct[c'] encrypting the bias in every slot one level lower
 * at the rescaled products' scale ((input scale q_l) / q_l as a double):
 *   Y(c', j') = RelinRescale(sum_{c,u,v} Tensor(Rot(col(c, s j'+v-pi), u),
 *               K_ct[c', c, u, v])) + bias_ct[c']
 * (one lazy relinearisation per output).  VR_ESCALE / VR_ELEVEL when the
 * bias ciphertexts do not match.  out receives C_out * w_out handles. */
vr_status vr_conv2d_encw(vr_context *ctx, const vr_eval_keys *ek, const vr_ciphertext *const *in, uint32_t C_in,
                         uint32_t h, uint32_t w, uint32_t pad, const vr_ciphertext *const *K_ct,
                         const vr_ciphertext *const *bias_ct, uint32_t C_out, uint32_t k, uint32_t stride,
                         vr_ciphertext **out, void *stream);
/* The FC of vr_fc with encrypted weights: W_ct[o n_in + i] encrypts the
 * weight pattern vr_encode_fc_weights encodes (scale q_l, the inputs'
 * level), bias_ct[o] the bias in every slot one level lower at the rescaled
 * scale:  Z_o = RotSum_block(RelinRescale(sum_i Tensor(Y_i, W_ct[o][i]))) +
 * bias_ct[o]. */
vr_status vr_fc_encw(vr_context *ctx, const vr_eval_keys *ek, const vr_ciphertext *const *Y, uint32_t n_in,
                     const vr_ciphertext *const *W_ct, const vr_ciphertext *const *bias_ct, uint32_t n_out,
                     uint32_t block, vr_ciphertext **out, void *stream);
/* Polynomial activation sum_i coeffs[i] x^i (degree >= 1; the cubic
 * activations of the paper's CNN, "Neural Network Architecture", Table 1) on
 * n ciphertexts of one level and scale, by Horner's rule: t =
 * Rescale(MulConst(x, coeffs[d]) at constant scale q_l + coeffs[d-1]), then
 * t = RelinRescale(Tensor(t, x dropped to t's level)) + coeffs[i] for
 * i = d-2 .. 0.  Depth d (VR_ELEVEL below it); out receives n handles. */
vr_status vr_poly_eval(vr_context *ctx, const vr_eval_keys *ek, const vr_ciphertext *const *in, size_t n,
                       const double *coeffs, uint32_t degree, vr_ciphertext **out, void *stream);
/* Dense layer on neuron ciphertexts (the last FC of the paper's CNN, Table 1:
 * each input holds one neuron's value at the same slots):
 *   out_o = Rescale(sum_j MulConst(in_j, W[o][j]) + AddConst(bias[o])),
 * W row-major [n_out][n_in] FP64, constants at scale q_l.  One level. */
vr_status vr_dense(vr_context *ctx, const vr_ciphertext *const *in, uint32_t n_in, const double *W,
                   const double *bias, uint32_t n_out, vr_ciphertext **out, void *stream);
/* Fully connected layer on conv outputs Y[c*w_out + j'] (C channels):
 *   Z_o = Rescale(sum_{c,j'} MulPlain(Y, W_pt[o][c*w_out + j'])), then
 *   Z_o += Rot(Z_o, 2^t) for 2^t < block, then AddConst(bias[o]).
 * W_pt from vr_encode_fc_weights; slot b*block holds logit o of image b.
 * Needs rotation keys for steps 1, 2, 4, ..., block/2. */
vr_status vr_fc(vr_context *ctx, const vr_eval_keys *ek, const vr_ciphertext *const *Y,
                uint32_t C, uint32_t w_out, const vr_plaintext *const *W_pt, const double *bias,
                uint32_t n_out, uint32_t block, vr_ciphertext **out, void *stream);
/* Model-provider side of the FC layer: W is [n_out][C][h_out][w_out];
 * plaintext (o, c, j') has slot b*block + stride*i' -> W[o][c][i'][j'] for
 * i' < h_out in every block b, encoded at scale (double) q_level.  The slot
 * vector repeats with period `block`, so its exact encoding lies in Z[X^r],
 * r = N / (2 block): coefficients off that subring are set to zero rather
 * than rounded, and each plaintext also keeps a compact evaluation-domain
 * copy (each limb's runs of r equal words kept once) that vr_fc and the
 * network call read.  W_pt receives n_out*C*w_out handles, index
 * (o*C + c)*w_out + j'. */
vr_status vr_encode_fc_weights(vr_context *ctx, const double *W, uint32_t n_out, uint32_t C,
                               uint32_t h_out, uint32_t w_out, uint32_t stride, uint32_t block,
                               uint32_t level, vr_plaintext **W_pt);

/* ---------------------------------------------------- parity and lifetime */

/* Coefficient-domain export, uint64 [ncomp][level+1][N]; cap_words must hold
 * it.  Synchronises the context stream. */
vr_status vr_ct_export(vr_context *ctx, const vr_ciphertext *ct, uint64_t *host, size_t cap_words,
                       uint32_t *ncomp, uint32_t *level, double *scale);
vr_status vr_ct_import(vr_context *ctx, const uint64_t *host, uint32_t ncomp, uint32_t level,
                       double scale, vr_ciphertext **out);
vr_status vr_pt_export(vr_context *ctx, const vr_plaintext *pt, uint64_t *host, size_t cap_words,
                       uint32_t *level, double *scale);
vr_status vr_pt_import(vr_context *ctx, const uint64_t *host, uint32_t level, double scale,
                       vr_plaintext **out);
/* Secret key as int8 coefficients in {-1, 0, 1} (client-side check). */
vr_status vr_sk_export(vr_context *ctx, const vr_secret_key *sk, int8_t *host, size_t n);
/* Switching key in the coefficient domain, uint64 [dnum][2][n_q + n_p][N]
 * (digit j: b_j then a_j; limbs q_0..q_L, p_0..p_{K-1}).  galois = 0 selects
 * the relinearisation key, otherwise the rotation key of that Galois
 * element (VR_ENOKEY if absent).  Synchronises. */
vr_status vr_swk_export(vr_context *ctx, const vr_eval_keys *ek, uint32_t galois, uint64_t *host,
                        size_t cap_words);
/* Ciphertext metadata without a copy. */
vr_status vr_ct_meta(const vr_ciphertext *ct, uint32_t *ncomp, uint32_t *level, double *scale);

/* Negacyclic NTT of raw device limbs in place: data is [n_limbs][N] on the
 * device, limb i reduced modulo moduli[mod_index[i]] (host array).  Forward
 * output is in bit-reversed evaluation order: out[i] = sum_t a_t
 * psi^((2 brev(i) + 1) t).  For kernel tests and benchmarks. */
vr_status vr_ntt(vr_context *ctx, uint64_t *data, uint32_t n_limbs, const uint32_t *mod_index,
                 int inverse, void *stream);

/* Device-side timing of one kernel class: while started, every launch of that
 * class (on whatever stream it runs) is bracketed by HIP events.  Classes:
 * "ntt" (one forward/inverse NTT call; units = limbs), "ks_inner" (key-switch
 * inner product; units = ciphertexts x extended limbs), "base_convert" (units
 * = output limbs), "lincomb" (fused MulConst/AddConst accumulation; units =
 * output limbs), "moddown" (ModDown combine; units = output limbs), "tensor"
 * (units = input limbs).  At most max_launches launches are recorded. */
vr_status vr_profile_start(vr_context *ctx, const char *kernel_class, size_t max_launches);
/* Synchronises the device and returns the summed event time, launch count,
 * unit count and whether launches were dropped; profiling stops. */
vr_status vr_profile_stop(vr_context *ctx, double *total_ms, uint64_t *launches, uint64_t *units,
                          uint32_t *dropped);

/* ------------------------------------------------------- whole networks
 * The encrypted CNN of "Convolutional Neural Networks" with the column-wise
 * layout: conv (as vr_conv2d), then x^2 when square != 0, then the FC layer
 * (as vr_fc) when fc_w != NULL.  fc_w holds fc_out * C_out * w_out weight
 * plaintexts in vr_fc's order; the FC runs at min(its input's level, the
 * plaintexts' level).  x^2 followed by the FC is evaluated with lazy
 * relinearisation when the FC level l >= 2 has room for the unrelinearised
 * products (with e the binary exponent of y_scale^2 * pt_scale and b the
 * total bit length of q_0..q_l: e + l + 12 <= b): each input's tensor,
 * formed on the FC level's limbs, is multiplied by the weights and summed,
 * and each FC output is relinearised once (RelinRescale, then Rescale): two
 * levels from the conv output.  Otherwise x^2 and the FC run as the layer
 * calls do. */
typedef struct {
    uint32_t C_in, h, w, pad, C_out, k, stride;
    const double *K;                  /* [C_out][C_in][k][k] */
    const double *bias;               /* [C_out] */
    uint32_t square;
    const vr_plaintext *const *fc_w;  /* NULL: no FC layer */
    const double *fc_bias;            /* [fc_out] */
    uint32_t fc_out, fc_block;        /* fc_block: slot block H' of the images */
} vr_cnn_desc;
typedef struct vr_graph vr_graph;

/* The network on n_sets image sets (in[s*C_in*w + c*w + j]) in one call:
 * out receives n_sets * (fc_w ? fc_out : C_out*w_out) handles, set after
 * set.  Identical limbs to the per-layer calls, except that with lazy
 * relinearisation (above) x^2 and the FC form one fused stage. */
vr_status vr_cnn_forward(vr_context *ctx, const vr_eval_keys *ek, const vr_cnn_desc *desc,
                         const vr_ciphertext *const *in, uint32_t n_sets, vr_ciphertext **out,
                         void *stream);
/* Captures the same schedule into a HIP graph: copies `in` into the graph's
 * own input slab, runs the network once eagerly (building every cached
 * constant), then records it on a private stream.  The graph owns its
 * intermediate and output memory until vr_graph_destroy.  Needs the built-in
 * allocator and the profiler stopped.  Synchronises. */
vr_status vr_graph_create(vr_context *ctx, const vr_eval_keys *ek, const vr_cnn_desc *desc,
                          const vr_ciphertext *const *in, uint32_t n_sets, vr_graph **out);
/* Copies new inputs (same count, level and scale) into the graph's input
 * slab on `stream`. */
vr_status vr_graph_set_inputs(vr_graph *g, const vr_ciphertext *const *in, size_t n, void *stream);
/* One replay on `stream`: rewrites the output slab from the input slab. */
vr_status vr_graph_launch(vr_graph *g, void *stream);
/* New handles viewing the graph's outputs (valid after a launch completes;
 * the next launch rewrites them). */
vr_status vr_graph_outputs(vr_graph *g, vr_ciphertext **out, size_t cap, size_t *n_out);
/* Synchronises the device and frees the graph (output handles stay valid). */
void vr_graph_destroy(vr_graph *g);

/* An uneven batch in one launch graph: requests of different kinds and sizes
 * (networks as vr_cnn_desc over their own image sets, column-split products
 * as vr_matmul).  Networks with the same description, input level and scale
 * run as one multi-set evaluation; products at one level and scale share one
 * hoisted ModUp and, per rotation step, one shared-key inner product and one
 * ModDown for every request still needing that step.  A request's inputs are
 * referenced in place (the batch shares their allocation) when they are one
 * contiguous run of ciphertexts of one allocation, else gathered into the
 * batch when added.  Every request's output limbs are identical to its own
 * vr_cnn_forward / vr_matmul call. */
typedef struct vr_batch vr_batch;
vr_status vr_batch_create(vr_context *ctx, const vr_eval_keys *ek, vr_batch **out);
/* *req_id indexes the request for vr_batch_outputs. */
vr_status vr_batch_add_cnn(vr_batch *b, const vr_cnn_desc *desc, const vr_ciphertext *const *in,
                           uint32_t n_sets, uint32_t *req_id);
vr_status vr_batch_add_matmul(vr_batch *b, const vr_ciphertext *const *A,
                              const vr_ciphertext *const *Bbar, uint32_t m, uint32_t n, uint32_t p,
                              uint32_t *req_id);
/* An outer-product product (operands as for vr_matmul_outer: T n and n
 * handles).  Outer-product requests at one level and scale share one
 * relinearisation and rescale of all their tiles; limbs identical to each
 * request's own vr_matmul_outer call. */
vr_status vr_batch_add_matmul_outer(vr_batch *b, const vr_ciphertext *const *A,
                                    const vr_ciphertext *const *B, uint32_t m, uint32_t n, uint32_t p,
                                    uint32_t *req_id);
/* Evaluates every request eagerly on `stream` (no graph). */
vr_status vr_batch_run(vr_batch *b, void *stream);
/* Runs the batch once eagerly (building and tuning every cached constant),
 * then captures it into one HIP graph that owns the intermediate and output
 * memory.  No request can be added afterwards.  Synchronises. */
vr_status vr_batch_capture(vr_batch *b);
/* One replay of the captured graph on `stream`. */
vr_status vr_batch_launch(vr_batch *b, void *stream);
/* New handles viewing request req_id's outputs (after a run or a completed
 * launch; the next one rewrites them): a network's n_sets * (fc_out or
 * C_out*w_out) outputs, or a product's P' ciphertexts. */
vr_status vr_batch_outputs(vr_batch *b, uint32_t req_id, vr_ciphertext **out, size_t cap,
                           size_t *n_out);
/* Synchronises the device and frees the batch (output handles stay valid). */
void vr_batch_destroy(vr_batch *b);

/* ---------------------------------------------------------------- serving
 * Continuous batching of encrypted inference requests ("Secure Inference":
 * a model owner evaluates a client's encrypted mini-batches).  A request is
 * one image set (the C_in*w column ciphertexts of up to B' images, from
 * vr_encrypt_columns) for a registered model under a session whose keys stay
 * resident.  A worker thread forms waves: the oldest pending request plus
 * later pending requests of the same session, model, level and scale, up to
 * max_batch, while the estimated device bytes of the in-flight waves stay
 * within the budget.  A wave is one batched multi-set evaluation (as
 * vr_conv2d_sets, then vr_square when the model has the activation); up to
 * two waves are in flight, on two streams of their own.  Every request's
 * output limbs are identical to evaluating it alone.  While a server runs,
 * the context's other calls may be used from the submitting thread; the
 * kernel profiler (vr_profile_*) must not be. */

/* hbm_budget_bytes bounds resident session keys plus in-flight requests.
 * Starts the worker thread.  *out owned by the caller (vr_srv_destroy). */
vr_status vr_srv_create(vr_context *ctx, size_t hbm_budget_bytes, uint32_t max_batch,
                        vr_server **out);
/* Finishes every submitted request, stops the worker, frees the server
 * (handles already returned by vr_srv_poll stay valid). */
void vr_srv_destroy(vr_server *srv);
/* Makes ek's keys resident for later requests (ek must outlive the server).
 * VR_EBUSY if the keys do not fit the budget. */
vr_status vr_srv_register_session(vr_server *srv, const vr_eval_keys *ek, uint64_t *session_id);
/* A conv layer (arguments as vr_conv2d; weights copied) followed by x^2 when
 * square != 0.  *model_id indexes it for vr_srv_submit. */
vr_status vr_srv_register_conv_model(vr_server *srv, uint32_t C_in, uint32_t h, uint32_t w,
                                     uint32_t pad, const double *K, const double *bias,
                                     uint32_t C_out, uint32_t k, uint32_t stride, uint32_t square,
                                     uint32_t *model_id);
/* Any network of vr_cnn_desc (conv, x^2, FC); the weights are copied, the FC
 * weight plaintexts must outlive the server. */
vr_status vr_srv_register_model(vr_server *srv, const vr_cnn_desc *desc, uint32_t *model_id);
/* Queues one request: in[c*w + j] (n_in = C_in*w), n_images images (for the
 * throughput figure).  The inputs are read after the work already queued on
 * the context's stream; the caller may free its handles at once.  VR_EBUSY
 * if the request alone can never fit the budget, VR_ELEVEL if it has too few
 * levels.  *ticket identifies it. */
vr_status vr_srv_submit(vr_server *srv, uint64_t session_id, uint32_t model_id,
                        const vr_ciphertext *const *in, size_t n_in, uint32_t n_images,
                        uint64_t *ticket);
/* Removes a request that has not started; VR_EINVAL if it already has.  Its
 * poll then returns VR_ECANCELED. */
vr_status vr_srv_cancel(vr_server *srv, uint64_t ticket);
/* *ready = 1 and out[0..*n_out) = the model's output handles (C_out*w_out, or fc_out; caller
 * frees) once the request is done (wait != 0 blocks until then); the ticket
 * is then consumed.  A failed or cancelled request returns its error code. */
vr_status vr_srv_poll(vr_server *srv, uint64_t ticket, int wait, vr_ciphertext **out, size_t cap,
                      size_t *n_out, int *ready);
/* Submit-to-completion latency percentiles (nearest rank) over the requests
 * completed since creation or the last reset, images per second between the
 * first submit and the last completion among them, request and wave counts
 * (batched = requests run in waves). */
/* Forgets the completed requests counted so far (e.g. after a warm-up). */
vr_status vr_srv_reset_stats(vr_server *srv);
vr_status vr_srv_stats(vr_server *srv, double *p50_ms, double *p99_ms, double *images_per_s,
                       uint64_t *completed, uint64_t *waves, uint64_t *batched);

void vr_free_ciphertext(vr_ciphertext *ct);
void vr_free_plaintext(vr_plaintext *pt);
void vr_free_keys(vr_secret_key *sk, vr_eval_keys *ek);

#ifdef __cplusplus
}
#endif

#endif /* VR_H */
