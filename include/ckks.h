/*
 * ckks.h -- C-ABI of the MI355X (gfx950) RNS-CKKS inverse-square-root library
 * (libckks_hip.so).
 *
 * What it computes.  The encrypted inverse square root of the paper
 * (Alg. 1 "CryptoInvSqrt": a Chebyshev initial value y0 (§2.3), then Newton
 * steps y <- y (3 - a y^2) / 2 (§2.2), with bootstrapping when levels run
 * out), on the CKKS operations the paper names in §2.1 (Add, Sub, Mul_P,
 * Mul_C, BTS, levels).  The scheme is RNS-CKKS with hybrid key switching; the
 * paper describes none of its internals, so every convention (prime chain,
 * NTT ordering, sampler, scale management, evaluation trees) is fixed by this
 * library, stated at the calls below, and reproduced bit for bit by an
 * independent CPU oracle.
 *
 * Conventions shared by every call:
 *  - A context owns the parameters, the per-prime tables, the keys and the
 *    device memory pool; it is used by one host thread at a time.  All device
 *    work is ordered on the context's HIP stream.
 *  - A ciphertext lives in device memory as uint64 words laid out
 *    [2][level+1][N] (poly-major, then limb-major), each limb a residue
 *    polynomial in the NTT domain (evaluations at the odd powers of the
 *    prime's 2N-th root psi, stored in bit-reversed order), every word fully
 *    reduced in [0, q_i).  Host-side it carries its level and an exact
 *    binary64 scale.
 *  - Every `ckks_ct **out` receives a NEW ciphertext owned by the caller
 *    (free with ckks_ct_free).  Inputs are never modified.  On error *out is
 *    NULL, inputs are untouched, and ckks_last_error() describes the failure;
 *    nothing aborts across the ABI.
 *  - Primitive operations never bootstrap by themselves: a missing level is
 *    CKKS_E_LEVEL.  Only ckks_bootstrap and ckks_invsqrt* bootstrap.
 *  - Host pointers are plain host memory; "device" pointers are HIP device
 *    memory (for example a torch tensor's data_ptr()) on the context's device.
 */
#ifndef CKKS_H
#define CKKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ckks_ctx ckks_ctx;
typedef struct ckks_ct ckks_ct;

typedef enum {
    CKKS_OK = 0,
    CKKS_E_PARAM = -1,   /* bad argument or parameter set */
    CKKS_E_LEVEL = -2,   /* not enough levels / level mismatch */
    CKKS_E_SCALE = -3,   /* scales of an addition do not match */
    CKKS_E_NOKEY = -4,   /* keys not generated / rotation key missing */
    CKKS_E_OOM = -5,     /* device memory exhausted (pool or arena) */
    CKKS_E_DEVICE = -6,  /* a HIP call failed */
    CKKS_E_RANGE = -7    /* a value does not fit the encoding */
} ckks_status;

/*
 * Parameter set.  Primes: q_0 = largest prime < 2^q0_bits with q = 1 mod 2N;
 * q_L..q_1 chosen top-down so that the canonical scale ladder
 * S_L = 2^log_scale, S_{l-1} = S_l^2 / q_l stays near 2^log_scale; special
 * primes p_0..p_{K-1} = the next primes = 1 mod 2N below q_0.  Key switching
 * uses digits of `digit_size` consecutive q-primes (dnum = ceil((L+1)/alpha)).
 * hamming_weight = 0 selects a dense ternary secret, otherwise a secret with
 * exactly that many +-1 coefficients.  sigma is the error standard deviation.
 *
 * Bootstrapping chain (bts_evalmod_levels > 0): max_level is then the top
 * level of computation, l_afterBTS of the paper (§2.1), and the levels that
 * bootstrapping consumes are added above it: bts_stc_levels for SlotToCoeff
 * (primes nearest 2^log_scale), bts_evalmod_levels for EvalMod (chosen top
 * down like the computation levels but around 2^bts_log_scale) and
 * bts_cts_levels for CoeffToSlot (primes nearest 2^bts_log_scale); the
 * ciphertext modulus then has max_level + bts_stc_levels + bts_evalmod_levels
 * + bts_cts_levels + 1 primes and digits are formed over all of them.
 */
typedef struct {
    uint32_t log_n;           /* ring degree N = 2^log_n, 4..16 */
    uint32_t max_level;       /* L (plain chain) or l_afterBTS (bootstrapping chain) */
    uint32_t num_special;     /* K */
    uint32_t digit_size;      /* alpha */
    uint32_t hamming_weight;  /* 0 = dense ternary */
    double sigma;             /* 3.2 */
    uint32_t log_scale;       /* 40 */
    uint32_t q0_bits;         /* 60 */
    uint32_t p_bits;          /* 60 */
    uint32_t bts_stc_levels;      /* 3, or 0 for a plain chain */
    uint32_t bts_evalmod_levels;  /* 10 for (K 25, r 4, degree 31), or 0 */
    uint32_t bts_cts_levels;      /* 3, or 0 */
    uint32_t bts_log_scale;       /* 52 */
} ckks_params;

/*
 * Create a context on the current HIP device.  `arena` (device memory, may be
 * NULL) of `arena_bytes` bytes, if given, is the only memory the context's
 * pool draws from (the caller keeps it alive until ckks_ctx_destroy; a torch
 * tensor works); with NULL the pool uses hipMalloc.  `hip_stream` (a
 * hipStream_t, may be NULL = default stream) orders all work.
 */
ckks_status ckks_ctx_create(const ckks_params *p, void *arena, size_t arena_bytes,
                            void *hip_stream, ckks_ctx **out);
void ckks_ctx_destroy(ckks_ctx *ctx);
/* Last error message of this context (static text valid until the next call). */
const char *ckks_last_error(const ckks_ctx *ctx);
/* Copy the prime chain (L+1+K words: q_0..q_L, p_0..p_{K-1}, L the top
 * level of the whole chain) and the canonical scale ladder S_0..S_L (L+1
 * doubles).  Either pointer may be NULL. */
ckks_status ckks_ctx_primes(const ckks_ctx *ctx, uint64_t *primes, double *ladder);
/* Change the stream all later work is ordered on. */
ckks_status ckks_set_stream(ckks_ctx *ctx, void *hip_stream);
/* Block until all work queued on the context's stream has finished. */
ckks_status ckks_sync(ckks_ctx *ctx);
/* Non-blocking: *done = 1 when every operation queued on the context's stream
 * has completed on the device, 0 while work is pending. */
ckks_status ckks_stream_done(ckks_ctx *ctx, int *done);

/*
 * Device memory as the context sees it, for admission control (a serving
 * loop admits work while its working set fits):
 *   device_free, device_total  the GPU's free and total bytes (hipMemGetInfo);
 *   pool_cached   bytes of free blocks the context's pool holds for reuse
 *                 (available to this context without a new allocation);
 *   pool_in_use   bytes of the pool's blocks held by live buffers (ciphertexts,
 *                 keys, tables, temporaries of operations being issued);
 *   pool_peak     the high-water mark of pool_in_use since the last reset:
 *                 the working set of the operations issued meanwhile;
 *   arena_left    bytes not yet handed out of a caller arena (0 without one).
 * ct_bytes (host, L+1 entries, may be NULL) receives the size of one
 * ciphertext at each level, 16 (l+1) N bytes.  reset_peak != 0 restarts the
 * high-water mark at the current pool_in_use (after the figures are read).
 */
typedef struct {
    size_t device_free, device_total;
    size_t pool_cached, pool_in_use, pool_peak;
    size_t arena_left;
} ckks_mem_stats;
ckks_status ckks_mem_info(ckks_ctx *ctx, ckks_mem_stats *out, uint64_t *ct_bytes, int reset_peak);

/*
 * Keys from the seeded SHAKE-256 sampler: secret, public key, relinearisation
 * key and one switching key per Galois element in `galois` (odd elements of
 * Z_2N^*: 5^k mod 2N rotates left by k slots, 2N-1 conjugates).  All keys
 * live in device memory.  Replaces any previous keys.
 */
ckks_status ckks_keygen(ckks_ctx *ctx, uint64_t seed, const int32_t *galois, uint32_t n_galois);
/* Galois element of a left rotation by `steps` slots (negative = right). */
int32_t ckks_galois_rotation(const ckks_ctx *ctx, int32_t steps);

/*
 * Public-key encryption of n <= N/2 real slot values (the rest are zero) at
 * `level`, encoded at `scale` (quad-precision canonical embedding, rounded to
 * nearest): the Enc(., l) of Alg. 3, which encrypts its input vector at the
 * level under test.  Randomness from SHAKE-256 on `seed`.  Errors:
 * CKKS_E_NOKEY before ckks_keygen, CKKS_E_PARAM for n > N/2, CKKS_E_LEVEL for
 * level > L, CKKS_E_RANGE when a scaled value does not fit the encoding.
 */
ckks_status ckks_encrypt(ckks_ctx *ctx, const double *x, uint32_t n, uint32_t level,
                         double scale, uint64_t seed, ckks_ct **out);
/* Encrypt n_ct vectors (row i = x + i * n, n <= N/2 slots each) at one
 * level and scale; ciphertext i uses seed seed0 + i and is identical to
 * ckks_encrypt(x + i * n, n, level, scale, seed0 + i).  The host encoding
 * and sampling run on up to 16 threads.  outs[i] receive single ciphertexts. */
ckks_status ckks_encrypt_batch(ckks_ctx *ctx, const double *x, uint32_t n_ct, uint32_t n, uint32_t level,
                               double scale, uint64_t seed0, ckks_ct **outs);
/* Decrypt with the context's secret key and decode N/2 slots (real parts to
 * `re`, imaginary parts to `im`; `im` may be NULL): the Dec of Alg. 2, whose
 * output the MRE of §4.2 is measured on.  `re` / `im` are host arrays of N/2
 * doubles.  Errors: CKKS_E_NOKEY before ckks_keygen. */
ckks_status ckks_decrypt(ckks_ctx *ctx, const ckks_ct *ct, double *re, double *im);

/* Ciphertext transfer: host words [B][2][level+1][N] (fully reduced) <->
 * device (import creates single ciphertexts, B = 1; export writes all B). */
ckks_status ckks_ct_import(ckks_ctx *ctx, const uint64_t *host, uint32_t level, double scale,
                           ckks_ct **out);
ckks_status ckks_ct_export(ckks_ctx *ctx, const ckks_ct *ct, uint64_t *host);
/* Device address of the ciphertext words (valid until ckks_ct_free). */
void *ckks_ct_device_ptr(const ckks_ct *ct);
int32_t ckks_ct_level(const ckks_ct *ct);
double ckks_ct_scale(const ckks_ct *ct);
void ckks_ct_free(ckks_ctx *ctx, ckks_ct *ct);
/*
 * Batches.  A ciphertext object may hold B >= 1 ciphertexts at one level and
 * scale, laid out [B][2][level+1][N]; every operation below accepts such an
 * object (all its operands must hold the same B) and runs each step as one
 * launch over all B, reading each switching-key word once per batch.
 * ckks_ct_pack copies n single ciphertexts (same level, same scale) into one
 * batch; ckks_ct_unpack writes its B members to outs[0..B-1] as new single
 * ciphertexts; ckks_ct_count returns B.
 */
ckks_status ckks_ct_pack(ckks_ctx *ctx, const ckks_ct *const *cts, uint32_t n, ckks_ct **out);
ckks_status ckks_ct_unpack(ckks_ctx *ctx, const ckks_ct *batch, ckks_ct **outs);
int32_t ckks_ct_count(const ckks_ct *ct);

/* Add_C / Sub_C: equal levels, |s_a/s_b - 1| <= 2^-30 (else CKKS_E_SCALE);
 * result scale s_a. */
ckks_status ckks_add(ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, ckks_ct **out);
ckks_status ckks_sub(ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, ckks_ct **out);
/* Multiply by a signed integer (no level, scale unchanged). */
ckks_status ckks_mul_int(ckks_ctx *ctx, const ckks_ct *a, int64_t k, ckks_ct **out);
/* Mul_P by a real constant at plaintext scale s_c (paper §2.1, Mul_P):
 * k = rint(value * s_c), ct' = k ct, scale' = scale * s_c; no rescale. */
ckks_status ckks_mul_const(ckks_ctx *ctx, const ckks_ct *a, double value, double s_c,
                           ckks_ct **out);
/* Mul_P landing on the canonical scale one level down:
 * s_c = (S_{l-1} * q_l) / scale, then rescale. */
ckks_status ckks_mul_const_down(ckks_ctx *ctx, const ckks_ct *a, double value, ckks_ct **out);
/* Add_P of a real constant: rint(value * scale) added to every slot. */
ckks_status ckks_add_const(ckks_ctx *ctx, const ckks_ct *a, double value, ckks_ct **out);
/* Keep limbs 0..level (scale unchanged). */
ckks_status ckks_drop_level(ckks_ctx *ctx, const ckks_ct *a, uint32_t level, ckks_ct **out);
/* Bring to a lower level carrying the canonical scale S_level (drop to
 * level+1, Mul_P by 1 at s_c = (S_level q_{level+1}) / scale, rescale). */
ckks_status ckks_level_to(ckks_ctx *ctx, const ckks_ct *a, uint32_t level, ckks_ct **out);
/* Rescale by q_l: c' = round(c / q_l) coefficient-wise, scale' = scale / q_l. */
ckks_status ckks_rescale(ckks_ctx *ctx, const ckks_ct *a, ckks_ct **out);
/* Mul_C with relinearisation (hybrid key switching), no rescale; scale s_a s_b. */
ckks_status ckks_hmult_relin(ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, ckks_ct **out);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * product of ckks_hmult_relin, word for word, written to caller memory and
 * computed with every temporary in a fixed array of the library,
 * CKKS_SCRATCH_BYTES of device memory on each GPU the library runs on (held
 * until the process ends).  Nothing is allocated: no hipMalloc, no pool, no
 * tables (ckks_keygen builds every level's key-switching tables).
 *   out        device memory of the context's GPU receiving [B][2][l+1][N]
 *              words (B = a's ciphertext count, l = a's level), owned by the
 *              caller; out_scale (host) receives scale(a) * scale(b).
 * Errors: CKKS_E_PARAM when the product needs more scratch than
 * CKKS_SCRATCH_BYTES (at N = 2^16 and K = 7 one ciphertext fits at every
 * level up to 23 with digits of 8 primes and up to 26 with digits of 10:
 * 227 and 251 limbs of 512 KiB; level 27 with digits of 10 would need 259)
 * -- nothing is launched
 * then; CKKS_E_NOKEY, CKKS_E_LEVEL as ckks_hmult_relin; CKKS_E_DEVICE when
 * the current device is not the context's.  Every call on one GPU shares that
 * GPU's array (it keeps the last call's contents; each call writes every word
 * it reads, so none needs clearing): calls that can overlap on one GPU --
 * contexts on different streams without synchronisation between them --
 * race, and must be serialised by the caller.
 */
#define CKKS_SCRATCH_BYTES ((size_t)128 << 20)
ckks_status ckks_hmult_relin_noalloc(ckks_ctx *ctx, const ckks_ct *a, const ckks_ct *b, uint64_t *out,
                                     double *out_scale);
/* Left rotation of the slots by `steps` (automorphism X -> X^(5^steps) and
 * key switch; CKKS_E_NOKEY without the Galois key). */
ckks_status ckks_rotate(ckks_ctx *ctx, const ckks_ct *a, int32_t steps, ckks_ct **out);
/* Rotations of one ciphertext by n step counts sharing one ModUp (hoisting):
 * outs[i] holds the slots rotated left by steps[i] (0: a copy).  Same slot
 * values as ckks_rotate, different key-switching noise (the digits are
 * converted before the automorphism).  On error every outs[i] is NULL. */
ckks_status ckks_rotate_hoisted(ckks_ctx *ctx, const ckks_ct *a, const int32_t *steps, uint32_t n,
                                ckks_ct **outs);
/* Complex conjugation of the slots (X -> X^(2N-1)). */
ckks_status ckks_conjugate(ckks_ctx *ctx, const ckks_ct *a, ckks_ct **out);

/*
 * Chebyshev-basis polynomial sum_k coeffs[k] T_k(t), t = (2x - a - b)/(b - a),
 * evaluated by baby-step/giant-step (paper §2.3 uses such a polynomial as
 * the Newton initial value).  [a, b] = [-1, 1] uses x as t directly.
 * Consumes bitlen(degree) + 1 levels (+1 for the affine map).
 */
ckks_status ckks_cheb_eval(ckks_ctx *ctx, const ckks_ct *x, const double *coeffs, uint32_t degree,
                           double a, double b, ckks_ct **out);
/* Chebyshev interpolation coefficients of 1/sqrt(x) on [a, b] at the
 * degree+1 first-kind nodes (quad precision, rounded once). */
ckks_status ckks_cheb_coeffs_invsqrt(uint32_t degree, double a, double b, double *coeffs);
/* One Newton step for 1/sqrt (paper §2.2, Alg. 1 loop body) given
 * ct_half = x/2: y' = 1.5 y - (ct_half y) y^2, at level c = min(l_x, l_y)
 * (needs c >= 2; result at c - 2, on the scale of the product term).  With
 * raw_x = 0 ct_half is brought to level c on the canonical scale; with
 * raw_x = 1 its limbs are only dropped, so it keeps its own scale (used for
 * the last step of ckks_invsqrt, where x comes straight from the input). */
ckks_status ckks_newton_step(ckks_ctx *ctx, const ckks_ct *y, const ckks_ct *ct_half, int raw_x,
                             ckks_ct **out);

/*
 * Bootstrapping (paper §2.1: BTS resets a ciphertext to level l_afterBTS).
 * The slot transform of n = N/2 slots, z = V w with w_k = p_k + i p_{k+n}
 * the coefficients of the plaintext p, factors into log2(n) butterfly stages
 * (stage k: butterflies of length 2^k with twiddles exp(2 pi i (5^j mod
 * 2^(k+2)) / 2^(k+2))) and a bit reversal; CoeffToSlot applies the inverse
 * stages and SlotToCoeff the forward ones, the bit reversal cancelling.  The
 * stages are grouped into three groups (one level each), each group
 * evaluated as a baby-step giant-step sum over its nonzero diagonals.
 *
 * ckks_bts_setup: EvalMod approximates cos(2 pi (K u - 1/4) / 2^r) on
 * u in [-1, 1] (u = t / K, t the ModRaised coefficient over q_0) by a
 * Chebyshev interpolant of `degree`, then r double-angle steps give
 * sin(2 pi t).  Needs a bootstrapping chain with bts_stc_levels = 3,
 * bts_cts_levels = 3 and bts_evalmod_levels = depth(degree) + r, depth(d) =
 * bitlen(d) + 1 for d >= 4 (the Chebyshev evaluation's consumption).
 * Encodes the diagonal plaintexts of the six groups into device memory.
 * The Galois keys listed by ckks_bts_rotations (left rotations) and the
 * conjugation key (2N - 1) must be generated (ckks_keygen) before
 * bootstrapping; ckks_bts_rotations writes at most cap steps and the count.
 */
ckks_status ckks_bts_setup(ckks_ctx *ctx, double K, uint32_t r, uint32_t degree);
ckks_status ckks_bts_rotations(const ckks_ctx *ctx, int32_t *steps, uint32_t cap, uint32_t *count);
/*
 * ckks_bootstrap: a ciphertext at any level whose slot values are real and
 * bounded by the integer `bound` in magnitude (its residues mod q_0 are
 * used).  Steps: multiply by F = rint(s0 / (scale bound)), s0 = q_0 2^-5
 * (exact integer, so the message fills about 2^-5 of q_0 whatever its
 * scale); ModRaise; CoeffToSlot; re = y + conj(y), im = -i (y - conj(y));
 * EvalMod of both (one batched evaluation); SlotToCoeff(re' + i im');
 * multiply by `bound`.  Output at level l_afterBTS, scale
 * S_out (scale F bound) / s0 with S_out ~ S_{l_afterBTS}.
 * The steps are exposed for testing:
 *   ckks_mod_raise: residues mod q_0 lifted to the centred range and
 *     reduced mod q_0..q_L; declared scale 2 q_0 K.
 *   ckks_coeff_to_slot: a ModRaised (level L) ciphertext -> level L - 3.
 *   ckks_eval_mod: level L - 3 -> level l_afterBTS + 3.
 *   ckks_slot_to_coeff: level l_afterBTS + 3 -> l_afterBTS.
 *   ckks_mul_monomial: multiply by X^k (0 <= k < 2N), exact, no level
 *     (X^(N/2) multiplies every slot by i).
 */
ckks_status ckks_bootstrap(ckks_ctx *ctx, const ckks_ct *a, int64_t bound, ckks_ct **out);
ckks_status ckks_mod_raise(ckks_ctx *ctx, const ckks_ct *a, ckks_ct **out);
ckks_status ckks_coeff_to_slot(ckks_ctx *ctx, const ckks_ct *a, ckks_ct **out);
ckks_status ckks_eval_mod(ckks_ctx *ctx, const ckks_ct *a, ckks_ct **out);
ckks_status ckks_slot_to_coeff(ckks_ctx *ctx, const ckks_ct *a, ckks_ct **out);
ckks_status ckks_mul_monomial(ckks_ctx *ctx, const ckks_ct *a, int32_t k, ckks_ct **out);

typedef struct {
    double a, b;        /* input domain of x (default 2^-10, 1) */
    int32_t literal;    /* 1: bootstrap y0 right after the Chebyshev step, as
                           Alg. 1 is written; 0 (default): bootstrap y only
                           when it has fewer than 2 levels before a step */
    int32_t pre_bts;    /* 1: bootstrap x before the Chebyshev step (the
                           paper's Pre-BTS indicator c = 1); 0: only when x
                           lacks the levels for it */
    int64_t bts_bound;  /* message bound for bootstrapping y (0: 16 ceil(sqrt(B/a))) */
    double B;           /* pre-normalisation constant (§2.3, the scaling of
                           PP-STAT): Alg. 1 runs on u = x/B in [a/B, b/B] and
                           its result is scaled back by 1/sqrt(B), so the
                           output approximates 1/sqrt(x); 0 or 1: none */
} ckks_invsqrt_opts;

/*
 * CryptoInvSqrt (paper Alg. 1): y0 = Chebyshev interpolant of degree `degree`
 * of 1/sqrt on [a, b]; ct_x = x/2; `iters` Newton steps; bootstrapping of y
 * per the policy in opts.  With pre-normalisation (opts.B > 1, §2.3):
 * y0 = interpolant of 1/sqrt(u) on [a/B, b/B] at u = x/B (the division by B
 * folded into the affine map's Mul_P, so the scaling takes the one level the
 * paper counts for it), ct_x = Mul_P(x, 1/(2B)), and the scale-back by
 * 1/sqrt(B) folded into the last Newton step (its constant 1.5/sqrt(B) and
 * the exact scale change of its x operand) or, with no Newton step, into the
 * coefficients: no extra level.  Pre-BTS (the paper's c = 1): with opts.pre_bts,
 * or if x has fewer than depth(degree) + 1 levels or fewer than 3, x is
 * bootstrapped first (bound 16 ceil(b)); otherwise x is never bootstrapped.  The last Newton step takes x/2 directly from the
 * input (limbs dropped, halving as an exact scale change, no rescale), so the
 * result keeps the relative precision of the input's scale; its scale is the
 * product of the step's scales (tracked exactly, not the canonical one).
 * ckks_invsqrt uses the defaults above.
 */
ckks_status ckks_invsqrt(ckks_ctx *ctx, const ckks_ct *x, uint32_t degree, uint32_t iters,
                         ckks_ct **out);
ckks_status ckks_invsqrt_ex(ckks_ctx *ctx, const ckks_ct *x, uint32_t degree, uint32_t iters,
                            const ckks_invsqrt_opts *opts, ckks_ct **out);

/*
 * Batched form: n independent ciphertexts at the same level through the same
 * (degree, iters) chain; each primitive step is one launch over all of them.
 * outs[i] receives the result for xs[i].  Results are bit-identical to n
 * calls of ckks_invsqrt_ex.
 */
ckks_status ckks_invsqrt_batch(ckks_ctx *ctx, const ckks_ct *const *xs, uint32_t n,
                               uint32_t degree, uint32_t iters, const ckks_invsqrt_opts *opts,
                               ckks_ct **outs);

/*
 * HIP graph of the CryptoInvSqrt chain for inputs shaped like x (same level,
 * scale and batch size B).  Creation runs the chain once eagerly (so every
 * table and pool block it needs exists), then captures it on the context's
 * stream; the device memory it uses stays reserved for the graph until
 * ckks_graph_destroy.  ckks_invsqrt_graph_run copies x into the graph's
 * input, replays the graph (no per-kernel host launches) and returns a new
 * ciphertext object with a copy of the result, identical to
 * ckks_invsqrt_ex / ckks_invsqrt_batch on the same input.  A graph is bound
 * to its context and stream; runs are stream-ordered.
 */
typedef struct ckks_graph ckks_graph;
ckks_status ckks_invsqrt_graph_create(ckks_ctx *ctx, const ckks_ct *x, uint32_t degree, uint32_t iters,
                                      const ckks_invsqrt_opts *opts, ckks_graph **out);
ckks_status ckks_invsqrt_graph_run(ckks_ctx *ctx, ckks_graph *g, const ckks_ct *x, ckks_ct **out);
void ckks_graph_destroy(ckks_ctx *ctx, ckks_graph *g);

/*
 * Forward (inverse = 0) or inverse (inverse = 1) negacyclic NTT, in place, of
 * `n_limbs` device-resident limbs of N words each at `data` (limb-major).
 * prime_idx[i] (host array) is the index, in the chain q_0..q_L,p_0..p_{K-1},
 * of limb i's prime.  Definition: NTT(a)[j] = sum_i a_i psi^((2 br(j)+1) i).
 */
ckks_status ckks_ntt_device(ckks_ctx *ctx, uint64_t *data, uint32_t n_limbs,
                            const uint32_t *prime_idx, int inverse);

/*
 * Schedule of the N = 2^16 transforms (a tuning knob; results are identical
 * under every schedule).  A forward or inverse NTT call covering at most
 * `r4_max_limbs` limbs in total runs with 4 words per thread, one of at most
 * `r8_max_limbs` limbs with 8, larger calls with 16: fewer words per thread
 * give more, shorter waves (better for small calls), more words fewer LDS
 * exchanges (better for large ones).  A 4-word call of at most `s4_max_limbs`
 * limbs puts 4 sub-transforms of 256 points in each workgroup instead of 16
 * (four times as many workgroups for calls too small to fill the chip).  -1
 * restores the library's default for that bound (128 limbs for each: 4 words
 * and 4 sub-transforms per workgroup up to 128 limbs, 16 words above); values
 * below -1 give CKKS_E_PARAM.  Takes effect for launches issued after the
 * call.
 */
ckks_status ckks_ntt_schedule(ckks_ctx *ctx, int32_t r4_max_limbs, int32_t r8_max_limbs,
                              int32_t s4_max_limbs);

/*
 * Arithmetic of the N = 2^16 transforms (a tuning knob; results are identical
 * either way): in the 4- and 8-words-per-thread forms (see ckks_ntt_schedule),
 * limbs whose prime is below 2^fp64_max_bits run their butterflies in binary64
 * (an error-free product and a rounded quotient by FMA, exact for primes below
 * 2^42), the others on 64-bit integers; the 16-word form keeps every prime on
 * 64-bit integers.
 * fp64_max_bits = 0: integers for every prime; -1: the default (42); values
 * above 42 or below -1 give CKKS_E_PARAM.  Takes effect for launches issued
 * after the call; a transform's two passes must run under one setting.
 */
ckks_status ckks_ntt_arith(ckks_ctx *ctx, int32_t fp64_max_bits);

/*
 * Measurement aid for the choice of word size (not a step of the method): the
 * rate of forward NTT butterflies (U + w V, U - w V with the lazy reductions
 * of the transforms) held in registers, with no memory traffic, in one of
 * three word forms:
 *   form 0: 64-bit words, odd q < 2^61 (the transforms' integer path);
 *   form 1: binary64 residues, odd q < 2^42 (their binary64 path);
 *   form 2: 32-bit words, odd q < 2^30 (a 30-bit-prime design; no
 *           operation of this library uses it).
 * 2048 x 256 threads each apply `rounds` rounds (1..4096: at most about 20 ms
 * per launch) of an 8-point transform held in registers (3 stages of 4
 * butterflies);
 * `launches` launches (1..1000) after one warm-up launch are timed with HIP
 * events on the context's stream.  *butterflies_per_s receives the rate.
 * Uses a 4 MiB buffer from the context's pool; synchronises the stream.
 * Bad arguments (q out of its form's range, even, or counts out of range)
 * give CKKS_E_PARAM.
 */
ckks_status ckks_butterfly_rate(ckks_ctx *ctx, int32_t form, uint64_t q, uint32_t rounds, uint32_t launches,
                                double *butterflies_per_s);

/*
 * Opt-in timing of kernel families on the context's stream (HIP events
 * recorded around each call; enabling clears previous records).  Families:
 *   "ntt"       every forward/inverse NTT call of the hot path; algorithmic
 *               bytes = 16 N per limb (one read and one write of each word);
 *   "keyswitch" every hybrid key switch; algorithmic bytes =
 *               8 N ((l+1) + 2 beta (l+1+K) + 2 (l+1)): the input polynomial,
 *               the switching key and the two output polynomials.
 * ckks_profile_read returns the number of calls, the summed GPU time in ms
 * and the summed algorithmic bytes of a family (zeros if never recorded).
 */
ckks_status ckks_profile_enable(ckks_ctx *ctx, int on);
/*
 * Opt-in operation trace for the cost model (enabling clears it): one text
 * line "op level B" per primitive executed (op in hmult, rescale, rotate,
 * rotate_hoisted, mul_scalar, mul_plain, add, sub, add_const, drop, copy,
 * mod_raise, bootstrap, lincomb, lincomb_term), in execution order; a
 * bootstrap is one line (its internal operations are not listed).  A fused
 * linear combination (the Chebyshev baby-step sums) is one "lincomb" line for
 * the launch and one "lincomb_term" line for each further term or sum.
 * ckks_trace_read copies at most cap-1 bytes plus a terminating zero and
 * returns the size needed (including the zero).
 */
ckks_status ckks_trace_enable(ckks_ctx *ctx, int on);
size_t ckks_trace_read(const ckks_ctx *ctx, char *buf, size_t cap);
ckks_status ckks_profile_read(ckks_ctx *ctx, const char *family, uint64_t *calls, double *gpu_ms,
                              double *alg_bytes);

#ifdef __cplusplus
}
#endif
#endif /* CKKS_H */
