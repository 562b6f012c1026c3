/*
 * he_mi355x.h - C ABI of the MI355X (gfx950) RNS-CKKS homomorphic matrix
 * product library.
 *
 * The operations follow "Improved Privacy-Preserving PCA Using Optimized
 * Homomorphic Matrix Multiplication" (arXiv 2305.17341):
 *   - full-RNS CKKS (Appendix A: Setparams, Encode/Decode, SecKeyGen,
 *     PubKeyGen, SwitchKeyGen, Enc, Dec, Add, PMult, Mult, Rescale,
 *     KeySwitch, Rot),
 *   - hoisted and double-hoisted BSGS linear transforms (section 3.3.1,
 *     Eq. 2 and Eq. 3'),
 *   - Jiang's matrix product sum_k C^k Z a (.) R^k T b (Eq. 4) with the
 *     hoisting of section 4.1 and the diagonal convergence decomposition of
 *     section 4.2 (Algorithms DCDforZ, DCDforT, DMatrixMult),
 *   - the covariance circuit of section 5 (Algorithm HCovMtrx),
 *   - the PowerMethod round, eigenvalue and eigen-shift of section 6.1
 *     (Algorithms HPowerMethod, HEigenShift) with the interactive refresh.
 *
 * Conventions
 *   - Every call returns he_status (HE_OK = 0); on failure the message of the
 *     last error of the calling thread is available from he_last_error().
 *     Calls never abort the process and no C++ exception crosses the ABI.
 *   - Host pointers are plain CPU memory owned by the caller; the library
 *     copies what it needs before returning.  Ciphertexts (he_ct) and all
 *     keys live in device memory owned by the library.
 *   - Work is issued on the context's HIP stream and is asynchronous; calls
 *     that hand data to the host (he_decrypt, he_ct_export) synchronise.
 *   - Calls that touch one context (or its ciphertexts) are serialised by a
 *     lock held inside the library; different contexts may be driven from
 *     different threads at once, and their work overlaps on the device.
 *     he_ctx_destroy must not race with any other call on that context.
 *   - A ciphertext at level l is u64[2][l+1][N] (limb-major, evaluation
 *     domain, residues in [0, q_i)); its scale is a double tracked exactly.
 *   - Slot vectors hold N/2 reals; a shorter message is replicated with its
 *     own period (a d x d matrix, row-major, uses period d*d).
 *   - Limits: 10 <= log N <= 16, at most 48 Q primes, 1..4 special primes,
 *     at most 16 decomposition digits, prime sizes 30..61 bits.
 */
#ifndef HE_MI355X_H
#define HE_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HE_OK = 0,
  HE_EINVAL = -1,   /* bad argument or shape */
  HE_ELEVEL = -2,   /* not enough levels left / level mismatch */
  HE_ESCALE = -3,   /* scale mismatch for an addition */
  HE_EKEY = -4,     /* a needed switching key was not generated */
  HE_ENOMEM = -5,   /* device allocation failed */
  HE_EDEVICE = -6,  /* HIP runtime error */
  HE_EBUSY = -7,
  HE_ENEEDREFRESH = -8
} he_status;

typedef struct he_ctx he_ctx; /* parameters, tables, keys, plaintext caches */
typedef struct he_ct he_ct;   /* one device-resident ciphertext */

/* Setparams (Appendix A): N = 2^log_n, q_bits[n_q] sizes of q_0..q_L,
 * p_bits[n_p] sizes of the special primes p_0..p_{alpha-1}; every prime is
 * 1 mod 2N (the largest such primes below 2^bits, Q first, then P).
 * Default scale Delta = 2^log2_scale; sigma = error width (support |e| <= 19). */
typedef struct {
  uint32_t log_n;
  const uint32_t* q_bits;
  uint32_t n_q;
  const uint32_t* p_bits;
  uint32_t n_p;
  double log2_scale;
  double sigma;
} he_params;

/* Optional device-memory hooks (e.g. a framework's caching allocator) and the
 * HIP stream to run on.  Any field may be NULL: hipMalloc / a stream owned by
 * the context are used instead. */
typedef struct {
  void* (*alloc)(size_t bytes, void* user);
  void (*release)(void* p, void* user);
  void* user;
  void* hip_stream;
} he_device;

/* Options of the matrix product.  Zero fields take the defaults:
 * n1_z = n1_t = 2^ceil(log2(d)/2) (baby steps of the sigma/tau BSGS),
 * nprime_z = nprime_t = d - 1 (no diagonal convergence decomposition). */
typedef struct {
  uint32_t n1_z, n1_t;
  uint32_t nprime_z, nprime_t;
  uint32_t flags; /* HE_MM_* below */
} he_matmul_opts;
/* he_matmul_batch only: consecutive products of equal d (and equal operand
 * level and scales) run as one stacked batch of up to 8 members, so every
 * kernel launch of the plan serves all of them and each switching-key word is
 * read once per batch.  Results are residue-for-residue identical to the
 * unbatched path.  Costs 8x the temporaries of one product in HBM. */
#define HE_MM_BATCHED 1u
/* he_matmul, he_matmul_batch, he_covariance: lazy relinearisation, a variant
 * of the paper's order (which relinearises every product of Algorithm
 * DMatrixMult): the n tensors (A_k, B_k) are summed in three components and
 * relinearised once, saving n - 1 key switches per product.  Different
 * residues from the default (no more noise); same level and scale. */
#define HE_MM_LAZY_RELIN 2u
/* he_matmul, he_matmul_batch, he_covariance: the A side's ModDown and the
 * Rescale after it (A_k = Rescale(ModDown(...)), section 4.1.1) as one
 * rounding, round(x / (P q_l)), a variant of the paper's two roundings.
 * Rounding twice differs from it only where round(x / P) / q_l lies within
 * about 2^-41 of a half-integer, so the residues almost always agree; the
 * level and scale are the same.  Needs at most 3 special primes (HE_EINVAL
 * otherwise). */
#define HE_MM_FUSED_RESCALE 4u
/* he_matmul_batch only, with HE_MM_BATCHED: 1 to 8 products of one d (one
 * operand level and scale) recorded once as a HIP graph and replayed by later
 * calls with the same operand ciphertexts and options (the last 4 recordings
 * are kept per context).  A replay reads the operands' buffers as they are at
 * that time; results are copied out of the graph's own buffers into new
 * ciphertexts, residue for residue those of the unrecorded call.  The first call runs the product three
 * times (warm-up, arena sizing, recording).  Not while the kernel profile is
 * enabled (HE_EINVAL).  he_trim and he_keygen drop the recordings. */
#define HE_MM_GRAPH 8u
/* he_covariance only: the dataset is not centred (see he_covariance) */
#define HE_COV_UNCENTRED 16u
/* he_matmul, he_matmul_batch, he_matmul_rot_steps: the masks of C^k
 * (section 4.1.1) folded into Z.  phi^k(sigma(A)) is one permutation of A's
 * entries whose diagonals are C^k's masks times Z's diagonals, with Z's
 * diagonal indices, so A_k is a single double-hoisted BSGS transform of a
 * (Z's geometry and keys, no column-shift keys) and the product takes two
 * levels instead of three: for chains with only two rescales, such as q0 +
 * two 40-bit primes.  Costs n transforms in place of Z and the shifts.  Not
 * with HE_MM_FUSED_RESCALE or a decomposition of Z (HE_EINVAL); not for
 * he_covariance. */
#define HE_MM_FOLDED 32u
/* he_matmul_batch only: products of any sizes and levels run together.
 * Products of equal d, level and scales are stacked (up to 8, wherever they
 * stand in the list); the stacks run concurrently on the context's stream,
 * taking turns, and their key inner products (the hoisted rotations of every
 * transform and shift, the relinearisations) are merged: each merged launch
 * (one per member count) serves one key-switch step of every product at
 * once, items of different levels and rotation sets side by side.  Results
 * are residue-for-residue those of each product computed alone.  Not with
 * HE_MM_GRAPH. */
#define HE_MM_MERGED 64u

/* Host only (no device needed): the moduli a context with these parameters
 * uses, q_0..q_L then p_0..p_{alpha-1} (Setparams of Appendix A: the largest
 * primes 1 mod 2N below 2^bits, Q first in chain order, then P), and each
 * modulus's NTT root psi = x^((q-1)/2N) for the smallest x >= 2 whose power
 * has order 2N (the smallest quadratic non-residue).  Both arrays hold at
 * least n_q + n_p words (`cap`). */
he_status he_params_moduli(const he_params* p, uint64_t* moduli, uint64_t* psi, size_t cap);

/* Create a context on the current HIP device.  `dev` may be NULL.  `seed`
 * keys every random draw of the context (Philox4x64-10 streams).
 * Returns HE_EINVAL for unsupported parameters, HE_EDEVICE without a device. */
he_status he_ctx_create(const he_params* params, const he_device* dev, uint64_t seed, he_ctx** out);
he_status he_ctx_destroy(he_ctx* ctx);
/* number of primes (Q then P) and their values */
he_status he_ctx_moduli(const he_ctx* ctx, uint64_t* out, size_t cap, size_t* n);

/* SecKeyGen + PubKeyGen + relinearisation key + rotation keys for each left
 * rotation step in rot_steps (Appendix A).  Calling it again only adds keys
 * that are missing. */
he_status he_keygen(he_ctx* ctx, const int32_t* rot_steps, size_t n_steps);
/* rotation steps the d x d product needs with these options (for keygen);
 * writes at most cap entries and the total count to *n */
he_status he_matmul_rot_steps(const he_ctx* ctx, uint32_t d, const he_matmul_opts* opts, int32_t* steps,
                              size_t cap, size_t* n);
/* Planner, no context or device needed: rotation steps of one transform of a
 * d x d product (kind 0 = Z, 1 = T, 2 = transposition G) by double-hoisted
 * BSGS with n1 baby steps, decomposed (section 4.2) when 0 < nprime < d - 1
 * (MinRotKeys of Tables 1 and 2). */
he_status he_lintrans_rot_steps(uint32_t kind, uint32_t d, uint32_t n1, uint32_t nprime, int32_t* steps, size_t cap,
                                size_t* n);
/* Planner, no context or device needed: rotation steps of Z (kind 0) or T
 * (kind 1) by double-hoisted BSGS with the simple key substitution of section
 * 4.2.1 (see he_lintrans_smpkeysub): of the inner loop only the prefix a j',
 * 0 < j' < n1p (a = 1 for Z, d for T); n1p = 0 or >= n1 gives the plain
 * dh-BSGS steps; n1p = 1 is rejected (HE_EINVAL). */
he_status he_smpkeysub_rot_steps(uint32_t kind, uint32_t d, uint32_t n1, uint32_t n1p, int32_t* steps, size_t cap,
                                 size_t* n);
/* rotation steps of the transposition (G) with baby-step count n1 (0 = default) */
he_status he_transpose_rot_steps(const he_ctx* ctx, uint32_t d, uint32_t n1, int32_t* steps, size_t cap, size_t* n);

/* Encode (Appendix A): m_i = floor(v_i + 1/2 + 2^-30) with
 * v_i = (2 Delta/N) sum_j z_j cos(pi 5^j i / N); z replicated to N/2 slots.
 * `n` must divide N/2.  Output: N signed coefficients (host). */
he_status he_encode(he_ctx* ctx, const double* z, size_t n, double delta, int64_t* out);

/* Enc at `level` with the public key; randomness is a pure function of
 * (context seed, nonce).  he_encrypt_matrix packs a d x d row-major matrix. */
he_status he_encrypt_slots(he_ctx* ctx, const double* z, size_t n, uint32_t level, uint64_t nonce, he_ct** out);
he_status he_encrypt_matrix(he_ctx* ctx, const double* a_rowmajor, uint32_t d, uint32_t level, uint64_t nonce,
                            he_ct** out);
/* Dec + Decode of the first n slots (client side, holds the secret key).
 * Uses the residue mod q_0, exact while |message * scale| < q_0 / 2. */
he_status he_decrypt(he_ctx* ctx, const he_ct* ct, double* out, size_t n);

/* ciphertext metadata, transfer and lifetime */
he_status he_ct_info(const he_ct* ct, uint32_t* level, double* scale);
he_status he_ct_export(const he_ct* ct, uint64_t* host, size_t words, uint32_t* level, double* scale);
he_status he_ct_import(he_ctx* ctx, const uint64_t* host, size_t words, uint32_t level, double scale, he_ct** out);
he_status he_ct_free(he_ct* ct);

/* Add / Sub (equal level and scale), Mult = tensor + relinearisation (no
 * rescale), Rescale, Rot (left rotation by `step` slots), level drop. */
he_status he_add(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct** out);
he_status he_sub(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct** out);
he_status he_mult(he_ctx* ctx, const he_ct* a, const he_ct* b, he_ct** out);
he_status he_rescale(he_ctx* ctx, const he_ct* a, he_ct** out);
he_status he_rotate(he_ctx* ctx, const he_ct* a, int32_t step, he_ct** out);
he_status he_drop_level(he_ctx* ctx, const he_ct* a, uint32_t level, he_ct** out);
/* Hoisted rotations (section 3.3.1) of `count` ciphertexts (1..64, one level
 * and scale) by `nsteps` steps each: one Decompose of the whole batch, the key
 * inner products of all steps in one multi-rotation launch (per 64 steps),
 * one ModDown per step for the whole batch.  out[i * nsteps + r] (caller's
 * array of count * nsteps handles) = Rot(a[i], steps[r]), residue for residue
 * what he_rotate gives.  HE_EKEY before any launch if a step's key is
 * missing; on any error no handle is returned. */
he_status he_rotate_many(he_ctx* ctx, const he_ct* const* a, size_t count, const int32_t* steps, size_t nsteps,
                         he_ct** out);

/* Rotation that allocates no device memory, for callers that cannot call
 * hipMalloc: code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation.  Same residues as he_rotate(ctx, a, step).
 *   out  an existing ciphertext (from any call of this library) at a's level
 *        and batch size; its residues are overwritten and its scale set to
 *        a's.  out == a is allowed.
 *   Workspace: a file-scope device array of HE_NOALLOC_WS_BYTES per GPU,
 *        allocated when the library's code is loaded and held until the
 *        process ends.  Every temporary of the rotation (Decompose digits,
 *        the R_{Q_l P} hoisted rotation, ModDown's lift) lives there; no
 *        kernel reads a workspace word before writing it, so nothing needs
 *        clearing.  All contexts on one GPU share that GPU's array, which
 *        keeps the last call's contents: calls that overlap on one GPU
 *        (different contexts on different host threads, or streams running
 *        concurrently) race and must be serialised by the caller.
 *   Errors: HE_EINVAL if the rotation at a's level needs more workspace than
 *        HE_NOALLOC_WS_BYTES (he_rotate_workspace_bytes gives the need; about
 *        48 MiB at N = 2^15 with 15 Q and 3 P primes, 288 MiB at N = 2^16
 *        with 31 and 3, which is rejected), or if out does not match a;
 *        HE_EKEY if the step's key is missing (nothing is launched then). */
#define HE_NOALLOC_WS_BYTES (64ull << 20)
he_status he_rotate_noalloc(he_ctx* ctx, const he_ct* a, int32_t step, he_ct* out);
/* Measured VALU ceiling of the modular products the kernels use, on the
 * current device: blocks x 256 threads each run `iters` steps of eight
 * independent product chains in registers (no memory traffic), timed with HIP
 * events.  kind 0 = lazy signed FP64 product a w - k q (the arithmetic of
 * moduli below 2^46), 1 = Shoup product by a constant (60-bit moduli), 2 =
 * Barrett product of two residues (60-bit moduli), 3 = lazy FP64 butterfly
 * (one product, one add, one subtract, the re-centring of both outputs).
 * *products_per_s = blocks * 256 * iters * 8 / elapsed; *ms (may be NULL) the
 * elapsed time.  Allocates and frees its own small output buffer. */
he_status he_modmul_peak(uint32_t kind, uint64_t iters, uint32_t blocks, double* products_per_s, double* ms);

/* Workspace bytes he_rotate_noalloc needs for a single ciphertext at `level`
 * (host-side arithmetic only). */
he_status he_rotate_workspace_bytes(const he_ctx* ctx, uint32_t level, size_t* bytes);
/* PMult by the encoding of z (n slots, replicated) at scale pt_scale */
he_status he_pmult_slots(he_ctx* ctx, const he_ct* a, const double* z, size_t n, double pt_scale, he_ct** out);

/* Linear transforms of section 4 on a d x d matrix ciphertext by
 * double-hoisted BSGS, one level consumed: kind 0 = sigma (Z), 1 = tau (T),
 * 2 = transposition (G); `weight` multiplies every diagonal (1.0 = plain). */
he_status he_lintrans(he_ctx* ctx, const he_ct* a, uint32_t kind, uint32_t d, uint32_t n1, double weight,
                      he_ct** out);
/* Z (kind 0) or T (kind 1) decomposed by diagonal convergence (section 4.2,
 * Algorithms DCDforZ / DCDforT) when 0 < nprime < d - 1, as the product's
 * sides apply them: ceil((d - 1) / nprime) levels consumed (1 without
 * decomposition).  Keys: he_lintrans_rot_steps(kind, d, n1, nprime). */
he_status he_lintrans_dcd(he_ctx* ctx, const he_ct* a, uint32_t kind, uint32_t d, uint32_t n1, uint32_t nprime,
                          he_ct** out);
/* Z (kind 0) or T (kind 1) by double-hoisted BSGS with the simple key
 * substitution of section 4.2.1, one level consumed: the baby steps
 * a (b n1p + j'), j' < n1p, are hoisted in blocks from bases
 * x_b = Rot(x_{b-1}, a n1p), each formed with the prefix keys alone (ModDown
 * of HR(x_{b-1}, a (n1p - 1)), then a rotation by a), so only the keys of
 * he_smpkeysub_rot_steps are needed.  2 <= n1p < n1 (n1 = 0: default);
 * n1p = 0 or >= n1 is plain dh-BSGS; n1p = 1 gives HE_EINVAL; a missing key
 * gives HE_EKEY.  `out` receives a new ciphertext owned by the caller. */
he_status he_lintrans_smpkeysub(he_ctx* ctx, const he_ct* a, uint32_t kind, uint32_t d, uint32_t n1, uint32_t n1p,
                                he_ct** out);

/* The homomorphic d x d product (Eq. 4, Algorithm DMatrixMult): a and b at
 * the same level l >= 3 (more with decomposition); result at level l - 3. */
he_status he_matmul(he_ctx* ctx, const he_ct* a, const he_ct* b, uint32_t d, const he_matmul_opts* opts,
                    he_ct** out);
/* `count` independent products; out[count] receives new ciphertexts */
he_status he_matmul_batch(he_ctx* ctx, const he_ct* const* a, const he_ct* const* b, const uint32_t* d,
                          size_t count, const he_matmul_opts* opts, he_ct** out);

/* Block covariance of a centred dataset (Algorithm HCovMtrx): x holds
 * row_blocks * k ciphertexts, x[r*k + j] = block (row block r, feature block
 * j) of size d x d.  cov[a*k + b] receives block (a, b) of X^T X / n_samples.
 * With HE_COV_UNCENTRED in opts->flags the dataset need not be centred
 * (section 5.2): the means mu[j] = Aggregate(sum_r x[r*k + j]; 0) / n_samples
 * (every row of the block holds its features' means) are computed
 * homomorphically, and block (a, b) of mu^T mu (transposition of mu[a] times
 * mu[b]) is subtracted after being brought to the level and scale of the
 * X^T X blocks (drop, constant 1 at the scale ratio, rescale).  Needs the
 * rotation keys d, 2d, .. < d^2 besides those of the covariance. */
he_status he_covariance(he_ctx* ctx, const he_ct* const* x, uint32_t row_blocks, uint32_t k, uint32_t d,
                        uint64_t n_samples, const he_matmul_opts* opts, he_ct** cov);

/* The block covariance of he_covariance in parts (Algorithm HCovMtrx), for
 * a dataset that arrives, or is to be scheduled, a few row blocks at a time.
 * he_covariance_begin fixes k, d, n_samples and the product options (a
 * centred dataset: HE_COV_UNCENTRED is refused) and returns a state in *st;
 * each he_covariance_add takes row_blocks * k more blocks in he_covariance's
 * layout (x[r*k + j] = row block r, feature block j), every block of every
 * call at one level; he_covariance_end writes the k*k blocks of
 * X^T X / n_samples to cov[k*k] as new ciphertexts and empties the state (it
 * may then take another dataset).  Any split of the row blocks over calls
 * gives exactly he_covariance's residues: the products of the row blocks
 * are summed exactly, mod q, before the one relinearisation and rescale.
 * The state holds device memory of its context: free it with
 * he_covariance_free before he_ctx_destroy.  Calls on one state, and on its
 * context, are serialised by the context's lock. */
typedef struct he_cov he_cov;
he_status he_covariance_begin(he_ctx* ctx, uint32_t k, uint32_t d, uint64_t n_samples, const he_matmul_opts* opts,
                              he_cov** st);
he_status he_covariance_add(he_cov* st, const he_ct* const* x, uint32_t row_blocks);
he_status he_covariance_end(he_cov* st, he_ct** cov);
he_status he_covariance_free(he_cov* st);

/* ------------------------------------------------------------------------
 * PowerMethod (section 6.1; Algorithms Aggregate, TaylorInit,
 * IterativeInvSRTbyNewton, AxisFlipping, HPowerMethod, HEigenShift).
 *
 * A replicated vector of t = k d components is k ciphertexts of d x d
 * blocks: axis 0 = every row of block i holds segment i (a row vector),
 * axis 1 = every column does (a column vector).  cov[r*k + c] is block
 * (row block r, column block c) of the symmetric t x t covariance (the
 * layout he_covariance returns).  d is a power of two; the rotation keys of
 * he_power_rot_steps(d) must exist.
 * ------------------------------------------------------------------------ */

/* Interactive refresh (client side, needs the secret key): ct is replaced in
 * place by a fresh encryption at the top level, with the nominal scale Delta,
 * of its message: the centred residue m mod q_0 of the decryption (exact
 * while |m| < q_0/2), re-scaled exactly to m' = round(m Delta / scale)
 * (halves away from zero).  Randomness from (context seed, nonce). */
he_status he_refresh(he_ctx* ctx, he_ct* ct, uint64_t nonce);

/* Called by the library when an operand sits at level 0; must replace *ct in
 * place by a ciphertext with levels left (he_refresh does) and return HE_OK. */
typedef he_status (*he_refresh_fn)(he_ct* ct, void* user);

/* Rotation steps of Aggregate for d x d blocks: +-2^j and d 2^j, 2^j < d. */
he_status he_power_rot_steps(uint32_t d, int32_t* steps, size_t cap, size_t* n);

/* he_power_step flags: the inverse square root by Goldschmidt's iteration
 * (section 3.5: h = y / 2, g = x y; the same iterates as Newton's, two levels
 * per step instead of three; v_out = 2 (y h) by an addition) */
#define HE_PM_GOLDSCHMIDT 1u
/* he_power_step flags: when a block of v enters the round with fewer than 3
 * levels left (but at least 1) and all k > 1 blocks share level and scale,
 * v is refreshed through one ciphertext (Appendix C): block i's segment kept
 * in column i (axis 1) or row i (axis 0) by a mask, the blocks summed, one
 * call of `refresh`, then each block recovered by rotation, mask and
 * spreading rotations (keys of he_power_rot_steps); the blocks of v are
 * replaced in place.  Otherwise operands are refreshed one by one at level 0. */
#define HE_PM_PACK_REFRESH 2u

/* One round of HPowerMethod on the replicated vector v[k] in `axis` form:
 *   y = Cov v (block products, Aggregate along the other axis), x = <y, y>;
 *   last == 0: v_out = y * Newton_{newton_iters}(T(x), x) in the flipped
 *              form, with T the order-1 Taylor expansion of x^-1/2 at
 *              taylor_x0 (taylor_order must be 1) and the Newton step
 *              y <- y (3 - x y^2) / 2 (Lazy Normalization: the caller picks
 *              newton_iters per round); with HE_PM_GOLDSCHMIDT in flags the
 *              same iterates by Goldschmidt's form (other bits: HE_EINVAL);
 *   last != 0: lambda_out = <y, v> (eigenvalue, every slot) and vt_out[k] =
 *              v flipped to the other axis (AxisFlipping); v stays the result.
 * *axis_out receives the form of v_out (last: of v).  Operands at level 0
 * are handed to `refresh` (NULL: HE_ENEEDREFRESH), which may thus replace
 * entries of cov and v in place.  Outputs are new ciphertexts owned by the
 * caller. */
he_status he_power_step(he_ctx* ctx, he_ct* const* cov, uint32_t k, uint32_t d, he_ct* const* v, uint32_t axis,
                        uint32_t newton_iters, double taylor_x0, uint32_t taylor_order, int last, uint32_t flags,
                        he_refresh_fn refresh, void* user, he_ct** v_out, uint32_t* axis_out, he_ct** lambda_out,
                        he_ct** vt_out);

/* HEigenShift: cov_out[r*k + c] = cov[r*k + c] - lambda (v v^T)_(r,c), with v
 * in `axis` form and vt its flip (as the last power step returns them).
 * Each covariance block is first taken to the level and scale of the
 * subtracted term (drop, multiplication by the constant 1 encoded at the
 * scale ratio, rescale).  Same refresh rule as he_power_step. */
he_status he_eigen_shift(he_ctx* ctx, he_ct* const* cov, uint32_t k, uint32_t d, he_ct* lambda, he_ct* const* v,
                         he_ct* const* vt, uint32_t axis, he_refresh_fn refresh, void* user, he_ct** cov_out);

/* Launch-shape knobs (process-wide; they regroup work into launches and never
 * change a residue): "ms_members" (1..8, batch members per key inner product
 * launch), "mr_members" (1..8) and "mr_rotations" (1..64) (members and
 * rotations per multi-rotation launch), "ntt_interleave" (0/1: the NTT's
 * block pass visits the limbs of one modulus back to back, so their twiddles
 * come from L2) and "ew_interleave" (0/1: the same for the limbs that share a
 * broadcast plaintext in the multiply-sums), "mr_group" (1/2/4, default 4:
 * rotations per work-group of a multi-rotation launch, which then read the
 * digits once for all of them), "cov_row_blocks" (1..8, default
 * 4: row blocks of he_covariance stacked into one batch through the
 * transposition and both sides; device memory for the sides grows with it),
 * "ntt_split_13/14/15" (0/1: the NTT's alternative stage split for that ring
 * size), and for the 60-bit limbs (q0, the special primes) of a
 * multi-rotation launch: "mr_int_split" (0/1, default 1: in a kernel of their
 * own), "mr_int_pass" (4/8: members per pass of that kernel), "mr_int_chunk"
 * (1..64: rotations per dispatch chunk) and "mr_int_concurrent" (0/1, default
 * 0: that kernel on a second stream of the context, beside the FP64 one);
 * "fbc_mfma" (0/1, default 1: ModDown's basis conversion into targets of 33
 * to 46 bits as an int8 matrix product of 7-bit digits, else six exact FP64
 * products per value) and "xcd_map" (0/1, default 1: that lift's work-groups
 * renumbered so that those of one polynomial run on one XCD and share its L2);
 * "sum_streams" (1/2/4, default 4: term streams that share their plaintexts
 * per thread of the multi-output multiply-sums, each plaintext word loaded
 * once for all of them) and "mr_pair" (0/1, default 1: the two masked
 * multi-rotation launches of a shift block of the product's A side as one
 * launch over both decompositions, each key word loaded once).
 * Set them between calls, not while
 * another thread drives the library.  The autotuner in the Python package
 * picks them by timing. */
he_status he_knob_set(const char* name, int32_t value);
he_status he_knob_get(const char* name, int32_t* value);

/* wait for all work of the context */
he_status he_sync(he_ctx* ctx);
/* device bytes held by the context (live, cached, peak) */
he_status he_mem_info(const he_ctx* ctx, size_t* live, size_t* cached, size_t* peak);
/* free and total bytes of the current HIP device */
he_status he_device_memory(size_t* free_bytes, size_t* total_bytes);
/* wait for the context's work, return its cached (free) device blocks to the
 * allocator and restart the peak mark at the live bytes */
he_status he_trim(he_ctx* ctx);

/* Raw limb transforms for parity checks: host in/out u64[nlimbs][N]; limb k
 * uses modulus mod_idx[k] (index into he_ctx_moduli order). */
he_status he_ntt_limbs(he_ctx* ctx, const uint64_t* in, uint64_t* out, size_t nlimbs, const int32_t* mod_idx,
                       int inverse);
/* Raw automorphism X -> X^g on evaluation-domain limbs (host in/out). */
he_status he_automorph_limbs(he_ctx* ctx, const uint64_t* in, uint64_t* out, size_t nlimbs, uint64_t galois);
/* Hoisted rotation left in R_{Q_l P} (section 3.3.1), exported to host as
 * u64[2][l+1+alpha][N]: the double-hoisting building block. */
he_status he_hoisted_rotate_export(he_ctx* ctx, const he_ct* a, int32_t step, uint64_t* host, size_t words);

/* time spent in the last he_matmul / he_matmul_batch call, milliseconds
 * (HIP events around the call's stream work) */
he_status he_last_op_ms(const he_ctx* ctx, double* ms);

/* Device-time profile by kernel: "ntt_fwd_cols", "ntt_fwd_rows",
 * "ntt_inv_rows", "ntt_inv_cols" (the two passes of each transform),
 * "ntt_fwd_rows_sub" (the forward block pass that ends ModDown and Rescale:
 * (x - y) c), "ntt_fwd_cols_modup" (the forward column pass of Decompose's
 * digits, basis conversion included), "ntt_fwd_cols_fbc" (the forward
 * column pass of ModDown, P-to-Q conversion included), "fbc_prep" (its
 * per-coefficient quotient), "ntt_fwd_cols_lift" (the forward column pass of
 * Rescale, lift of the top limb included), "multsum", "multsum_rot"
 * (several rotations of one decomposition), "modup", "fbc_to_q",
 * "moddown_final", "rescale_lift", "rescale_final", "elementwise", "tensor",
 * "plift".  While enabled, HIP
 * events are recorded on the launching stream around every launch of the
 * kernel.  Enabling clears the totals.  `bytes` (may be NULL) receives the
 * kernel's algorithmic HBM bytes: every input read once, every output written
 * once (for an NTT pass: every active limb read and written once).  The
 * profile is process-wide: enable it only while a single thread drives the
 * library. */
he_status he_profile_enable(he_ctx* ctx, int on);
he_status he_profile_read(he_ctx* ctx, const char* family, double* total_ms, uint64_t* launches, double* bytes);
/* Algorithmic modular products of a kernel family since enabling, by the
 * arithmetic of their moduli: lazy FP64 (moduli below 2^46) and 64-bit
 * integer (the others).  Counted per launch from its shape: (N/2) x stages
 * butterflies per limb of an NTT pass, the basis conversions' terms (one
 * product per source and target value, plus the quotient's), 2 beta key
 * products per output value of a key inner product (plus P c_0 and masks),
 * four per tensor value, one per elementwise or multiply-sum product.  With
 * he_modmul_peak's measured rates this gives the VALU side of a roofline.
 * `unit_bytes` (may be NULL): the family's bytes in the key switch's unit
 * of work, each switching key read once per launch (2 beta_l (l+1+alpha)
 * limbs) and each member's ciphertext read and written once per rotation
 * (4 (l+1) limbs); for other families the algorithmic bytes of
 * he_profile_read. */
he_status he_profile_read_ops(he_ctx* ctx, const char* family, double* modmuls_f64, double* modmuls_int,
                              double* unit_bytes);
/* counts of Decompose / MultSum / ModDown operations issued by the context */
he_status he_op_counts(const he_ctx* ctx, uint64_t* decompose, uint64_t* multsum, uint64_t* moddown);

const char* he_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HE_MI355X_H */
