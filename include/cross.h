/*
 * cross.h -- C ABI of libcross: the CROSS hot path (arXiv 2501.07047) on AMD
 * MI355X (gfx950): RNS negacyclic NTT/INTT and the CKKS modular matrix
 * products rewritten as exact int8 MFMA matrix multiplies (BAT + MAT).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Residues are uint32 values in [0, q).  Inputs outside that range give
 *    unspecified (but memory-safe) results, unless the debug mode
 *    (cross_set_debug_check, or CROSS_DEBUG_CHECK=1 in the environment when the
 *    context is created) is on: then every entry point checks its residue
 *    inputs on the device first and fails with CROSS_EDOMAIN, naming the first
 *    offending polynomial, limb and coefficient, before enqueueing any work.
 *  - Polynomial data is device memory laid out [batch][L][N] (limb-major per
 *    polynomial, N contiguous coefficients per limb).  Pointers must be
 *    16-byte aligned.  The caller owns every data buffer.
 *  - NTT form ("evaluation form") stores slot p = a(psi^(2*brv_N(p)+1)) in
 *    position p (bit-reversed order; Sec. MAT: the layout-invariant 3-step
 *    NTT delivers its output directly in bit-reversed order).  psi is the
 *    canonical primitive 2N-th root g^((q-1)/2N), g the smallest generator of
 *    Z_q^* (see cross_root).
 *  - Primes: 2 < q < 2^28, prime, q = 1 (mod 2N).  The NTT entry points
 *    (cross_ntt_forward/inverse and their butterfly forms), cross_bconv and the
 *    CKKS operators (cross_keyswitch_modup/moddown, cross_he_mult, cross_rotate,
 *    cross_rescale) also take wide primes 2^28 <= q < 2^31 (see
 *    cross_ntt_forward and cross_bconv; with a wide prime the CKKS operators run
 *    their separate, unfused kernels); the batch runtime does not.  Arrays of
 *    primes are host memory.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls return
 *    after enqueueing; argument errors are reported synchronously and nothing
 *    is enqueued; device faults surface at the caller's next synchronisation.
 *  - A context is bound to one HIP device and is not thread-safe: use one per
 *    host thread.  It owns the precomputed tables and an internal workspace
 *    (device memory, grown on demand and freed by cross_ctx_destroy).
 *  - Every function returns a cross_status; cross_last_error() describes the
 *    most recent failure on that context.
 */
#ifndef CROSS_H
#define CROSS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum cross_status {
  CROSS_OK = 0,
  CROSS_EINVAL = -1,       /* bad argument (null pointer, size, alignment, layout) */
  CROSS_ENOTPRIME = -2,    /* a modulus is not prime */
  CROSS_ENOROOT = -3,      /* q != 1 (mod 2N): no primitive 2N-th root of unity */
  CROSS_ERANGE = -4,       /* q >= 2^28 (residues must split into four 7-bit chunks); for
                              the entry points that take wide primes q >= 2^31 */
  CROSS_ENOMEM = -5,       /* device allocation failed */
  CROSS_EDEVICE = -6,      /* HIP runtime error while enqueueing */
  CROSS_EUNSUPPORTED = -7, /* valid but unsupported shape */
  CROSS_EDOMAIN = -8       /* debug mode (cross_set_debug_check): an input residue is not below
                              its limb's prime */
} cross_status;

#define CROSS_MAX_LIMBS 64   /* L + K limit per call */
#define CROSS_MIN_LOG_N 4
#define CROSS_MAX_LOG_N 16

typedef struct cross_ctx_s* cross_ctx;

/* Create a context on HIP device `hip_device`.  *out receives the handle. */
cross_status cross_ctx_create(int hip_device, cross_ctx* out);
/* Free tables, workspace and the context.  Waits for the device to go idle. */
void cross_ctx_destroy(cross_ctx ctx);
/* Text of the last error on ctx (valid until the next call on ctx). */
const char* cross_last_error(cross_ctx ctx);

/* Canonical psi for (q, N = 2^log_n): *psi_out = g^((q-1)/2N).  Validates q
 * (any prime the NTT takes, q < 2^31). */
cross_status cross_root(uint32_t q, uint32_t log_n, uint32_t* psi_out);

/* Force the 3-step split N = R x C with R = 2^log_r for transforms of size
 * 2^log_n on this context (the autotuner's choice otherwise; default
 * R = 2^floor(log_n/2)).  4 <= log_r and 4 <= log_n - log_r. */
cross_status cross_set_ntt_split(cross_ctx ctx, uint32_t log_n, uint32_t log_r);

/*
 * Three-factor NTT for size 2^log_n (MAT applied to a third dimension, Sec.
 * MAT): the R x C split with R = 2^log_r, and the C-point row transform of
 * step 3 split once more as C1 x C2 (C1 = 2^log_c1) -- same input/output layout
 * and bit-reversed order as the two-factor form, about (R + C1 + C2) / (R + C)
 * of its int8 MAC work.  Needs 16 <= C1, C2 <= 64, R >= 16 and R * C1 * C2 >=
 * 8192 (the row kernel takes 8192 / C rows per workgroup).  log_c1 = 0 with
 * log_r > 0 selects the two-factor form with R = 2^log_r; log_r = log_c1 = 0
 * restores the size's default (three factors R x C1 x C2 = 2^5 x 2^4 x 2^4,
 * 2^5 x 2^5 x 2^4, 2^6 x 2^5 x 2^4, 2^6 x 2^5 x 2^5 for log_n = 13, 14, 15, 16;
 * two factors below).  cross_set_ntt_split also selects two factors.  Applies
 * to cross_ntt_forward/inverse, the CKKS entry points and cross_poly_mul; the
 * batch runtime keeps two factors.
 * Errors: CROSS_EINVAL for an unsupported split.
 */
cross_status cross_set_ntt_split3(cross_ctx ctx, uint32_t log_n, uint32_t log_r, uint32_t log_c1);
/* The split cross_ntt_forward uses for size 2^log_n on ctx: *log_c1 = 0 for two
 * factors (8 <= log_n <= 16; sizes below 2^8 run on the butterfly kernels). */
cross_status cross_get_ntt_split(cross_ctx ctx, uint32_t log_n, uint32_t* log_r, uint32_t* log_c1);

/* Autotuner: time forward + inverse NTTs of `batch` x L limbs of size 2^log_n
 * (8 <= log_n <= 16) for every two-factor split R = 2^log_r within a factor of
 * four of square (R, C >= 64 from log_n = 12 up, so the batch runtime can use
 * it) with every GEMM tile, and every three-factor split R x C1 x C2 with
 * 16 <= C1, C2 <= 32 (the paper sweeps (R, C) and keeps the best); keep the
 * fastest on this context for that size (as cross_set_ntt_split3 plus a
 * per-size tile; the best two-factor split also becomes the batch runtime's).
 * *log_c1_out = 0 reports a two-factor choice.  For 12 <= log_n it also times
 * the batch runtime's NTT of the same shape with every work-list tile that fits
 * and keeps the fastest per direction (cross_batch_create uses it for that size;
 * see cross_get_batch_tile; a cached line restores only the per-call choice).
 * If cache_path is non-NULL a
 * matching line "<device> <log_n> <L> <batch> <log_r> <log_c1> <tile> <us>
 * <two-factor log_r>" is reused without timing, else the new choice is
 * appended.  Any out pointer may be NULL.  Allocates batch*L*N*4 bytes of
 * scratch while timing; synchronises the device. */
cross_status cross_autotune(cross_ctx ctx, uint32_t log_n, uint32_t L, uint32_t batch, const char* cache_path,
                            uint32_t* log_r_out, uint32_t* log_c1_out, int* tile_out, double* us_out);

/* Workgroup tile of the BAT int8 GEMM steps on this context (autotuner knob):
 * 0 = automatic (by shape and grid size), 1 = 256x256 (8 waves of 128x64),
 * 2 = 256x128 (4 waves of 128x64), 3 = 128x64, 4 = 64x64, 5 = 256x128 (8 waves
 * of 64x64), 6 = 256x256 (16 waves of 64x64), 7 = as 6 with 128-deep K
 * stages; 8 = 256x128 (8 waves of 64x64) and 9 = 256x128 (4 waves of 64x128),
 * where each wave reads its rows of the pre-known table straight from global
 * memory instead of through LDS (steps contracting at most 512 inputs).  A
 * tile that does not fit a step falls back to auto.
 * Results are identical for every tile; only speed changes. */
cross_status cross_set_gemm_tile(cross_ctx ctx, int tile);

/*
 * Forward negacyclic NTT, in place, of `batch` polynomials of L limbs each
 * (Sec. MAT, layout-invariant 3-step NTT; Sec. BAT for the int8 products):
 * for every b < batch and limb i < L, data[b][i][:] (coefficients, natural
 * order) is replaced by its NTT form modulo primes[i] (bit-reversed order).
 * Steps 1 and 3 run as BAT-expanded int8 MFMA GEMMs; step 2 is fused into the
 * epilogue of step 1.  Uses batch*L*N*4 bytes of context workspace.
 *   log_n  : 4..16 (log_n >= 8 runs on MFMA; smaller sizes use the butterfly kernels)
 *   primes : host array of L primes (see conventions); q < 2^31
 *   L      : 1..CROSS_MAX_LIMBS;  batch >= 1
 *   data   : device, uint32 [batch][L][2^log_n]
 * Wide primes (2^28 <= q < 2^31; Sec. BAT with bp = 8 as the paper uses it):
 * the runtime side is cut into its four bytes, fed to the signed int8 MFMA as
 * b - 128, the pre-known side into balanced signed 8-bit digits, and each
 * accumulator starts at a per-row correction 128 * (row sum); the partial sums
 * are merged (in 32 bits where a contraction is at most 64 inputs deep, else
 * in 64) and reduced with a signed Montgomery step.  Limbs of
 * both kinds may be mixed in one call (they run as two groups).  With
 * CROSS_NTT_RED_BARRETT, wide primes fail with CROSS_EUNSUPPORTED.
 */
cross_status cross_ntt_forward(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L,
                               uint32_t batch, uint32_t* data, void* stream);
/* Inverse of cross_ntt_forward (NTT form in bit-reversed order -> coefficients),
 * N^-1 included.  Same arguments. */
cross_status cross_ntt_inverse(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L,
                               uint32_t batch, uint32_t* data, void* stream);

/* Baseline: the same transforms as plain radix-2 butterflies on the vector
 * ALUs, one launch per stage (App. "Radix-2 Cooley-Tukey NTT").  Bit-identical
 * results to cross_ntt_forward / cross_ntt_inverse.  Same arguments. */
cross_status cross_ntt_forward_butterfly(cross_ctx ctx, uint32_t log_n, const uint32_t* primes,
                                         uint32_t L, uint32_t batch, uint32_t* data, void* stream);
cross_status cross_ntt_inverse_butterfly(cross_ctx ctx, uint32_t log_n, const uint32_t* primes,
                                         uint32_t L, uint32_t batch, uint32_t* data, void* stream);

/*
 * Negacyclic polynomial product (config-1 check of the convolution theorem):
 * out = INTT(NTT(a) * NTT(b)) limb-wise, i.e. a*b in Z_q[x]/(x^N + 1).
 * a, b, out: device [batch][L][N] coefficient form (a and b are read before out is
 * written, so out may alias either).  Uses 2*batch*L*N*4 bytes of workspace.
 */
cross_status cross_poly_mul(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L,
                            uint32_t batch, const uint32_t* a, const uint32_t* b, uint32_t* out,
                            void* stream);

/*
 * Fast basis conversion (App. "Basis Conversion (BConv)"): for every
 * coefficient n, out_j = sum_i [in_i * qhat_i^-1]_{q_i} * [qhat_i]_{p_j} mod p_j with
 * qhat_i = prod_{i' != i} q_{i'} over src_primes.  Step 1 is fused into the
 * prologue of step 2, which runs as a BAT-expanded int8 MFMA GEMM.  This is
 * the approximate ("fast") conversion: the result may differ from the exact
 * CRT value by a multiple u*Q, 0 <= u < l.
 *   in : device [batch][l][N] coefficient form mod src_primes (1 <= l <= 32, distinct)
 *   out: device [batch][lp][N] mod dst_primes (1 <= lp <= 64); must not overlap in
 *        (CROSS_EINVAL otherwise)
 *   log_n: 5..16
 * Primes are odd primes below 2^31 (CROSS_ERANGE at or above): with any of them at
 * or above 2^28 the whole conversion takes the byte form (residue bytes as
 * b - 128 against balanced signed 8-bit digits with per-row corrections, the
 * paper's full-byte BAT), otherwise 7-bit chunks.
 */
cross_status cross_bconv(cross_ctx ctx, uint32_t log_n, const uint32_t* src_primes, uint32_t l,
                         const uint32_t* dst_primes, uint32_t lp, const uint32_t* in, uint32_t* out,
                         uint32_t batch, void* stream);

/*
 * CKKS parameters for hybrid key switching (Tab. perf_cmp "L, log2 q, Dnum").
 * Digit j holds limbs [j*alpha, min((j+1)*alpha, L)), alpha = ceil(L/dnum);
 * a digit with no limb is inactive (its ModUp output is zero).  Limits:
 * 5 <= log_n <= 16, L + K <= 64, alpha <= 32, K <= 32; primes pairwise distinct.
 */
typedef struct cross_ckks_params {
  uint32_t log_n;           /* N = 2^log_n */
  uint32_t L;               /* ciphertext limbs (the Q primes) */
  uint32_t K;               /* special primes (P = product of the last K primes) */
  uint32_t dnum;            /* key-switch digits */
  const uint32_t* primes;   /* host array of L + K primes: Q first, then P */
} cross_ckks_params;

/*
 * ModUp (hybrid key switching): in = d, NTT form [batch][L][N] (not modified);
 * out = [batch][dnum][L+K][N] NTT form with, for digit j, out[j][t] = d[t] for
 * limbs t of the digit and out[j][t] = NTT_t(BConv_{digit j -> t}(INTT(d))) for
 * every other limb t < L+K.  out must not alias in.
 */
cross_status cross_keyswitch_modup(cross_ctx ctx, const cross_ckks_params* params, const uint32_t* in,
                                   uint32_t* out, uint32_t batch, void* stream);
/*
 * ModDown: in = x, NTT form [batch][L+K][N] (not modified); out = [batch][L][N]
 * with out_i = (x_i - NTT_{q_i}(BConv_{P -> q_i}(INTT_P(x_P)))) * P^-1 mod q_i.
 */
cross_status cross_keyswitch_moddown(cross_ctx ctx, const cross_ckks_params* params,
                                     const uint32_t* in, uint32_t* out, uint32_t batch, void* stream);

/*
 * HE-Mult with relinearisation, no rescale (Tab. perf_cmp "HE-Mult"):
 * d0 = a0 b0, d1 = a0 b1 + a1 b0, d2 = a1 b1 (NTT form, limb-wise), then
 * out = (d0 + ModDown(sum_j ModUp(d2)_j * key_j.b), d1 + ModDown(sum_j ModUp(d2)_j * key_j.a)).
 *   ct_a, ct_b, out: device [batch][2][L][N] NTT form; out must not overlap ct_a,
 *                    ct_b or relin_key (ct_a and ct_b may be the same buffer)
 *   relin_key      : device [dnum][2][L+K][N] NTT form, index 0 = b, 1 = a
 * Errors: CROSS_EINVAL for null / misaligned / overlapping buffers or bad
 * parameters, prime checks as cross_ntt_forward (q < 2^31).
 */
cross_status cross_he_mult(cross_ctx ctx, const cross_ckks_params* params, const uint32_t* ct_a,
                           const uint32_t* ct_b, const uint32_t* relin_key, uint32_t* out,
                           uint32_t batch, void* stream);

/*
 * Rotate by `steps` slots (Tab. perf_cmp "Rotate"): Galois element
 * g = 5^steps mod 2N (steps taken mod N/2); automorphism first, in NTT form
 * (slot p <- slot brv(((2 brv(p)+1) g mod 2N - 1)/2)), then the key switch of
 * the second component with rot_key (the key for g, layout as relin_key):
 * out = (sigma(c0) + ModDown(acc_b), ModDown(acc_a)).  ct, out: [batch][2][L][N];
 * out must not overlap ct or rot_key (CROSS_EINVAL otherwise).
 */
cross_status cross_rotate(cross_ctx ctx, const cross_ckks_params* params, int32_t steps,
                          const uint32_t* ct, const uint32_t* rot_key, uint32_t* out, uint32_t batch,
                          void* stream);

/*
 * HE-Add (Tab. perf_cmp "HE-Add"; limb-wise by the RNS isomorphism, Sec.
 * Background): out = a + b mod q_i limb by limb.
 *   a, b, out: device [npoly][L][N], 16-byte aligned; any of them may alias
 *              (a ciphertext is two consecutive polynomials; NTT or coefficient
 *              form alike)
 *   primes   : host array of L primes (as cross_ntt_forward); 4 <= log_n <= 16
 * Errors: CROSS_EINVAL for null / misaligned pointers or bad shape, prime
 * checks as cross_ntt_forward.  Asynchronous on `stream`.
 */
cross_status cross_he_add(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L,
                          uint32_t npoly, const uint32_t* a, const uint32_t* b, uint32_t* out,
                          void* stream);

/*
 * Rescale (Tab. perf_cmp "Rescale"; dropping two primes per level is the
 * paper's double rescaling, Sec. Evaluation "Security Parameter Selection"):
 * division by P = product of the last `drop` primes, read as ModDown with
 * those primes in the role of the special primes:
 *   out_i = (in_i - NTT_{q_i}(BConv_{P -> q_i}(INTT_P(in_P)))) * P^-1 mod q_i,  i < L - drop.
 * For drop = 1 each coefficient becomes exactly floor(C / q_{L-1}) of its CRT
 * value C; for more primes the fast conversion may leave it one lower.
 *   in     : device [npoly][L][N] NTT form over primes[0..L-1], not modified
 *   out    : device [npoly][L-drop][N] NTT form over primes[0..L-drop-1];
 *            must not overlap in (a ciphertext is two consecutive polynomials)
 *   primes : host array of L distinct primes; 5 <= log_n <= 16; 1 <= drop < L <= 64,
 *            drop <= 32
 * Uses context workspace of npoly * N * (L + max(drop, L - drop)) words.
 * Errors: CROSS_EINVAL (null / misaligned / overlapping buffers, bad shape),
 * prime checks as cross_he_mult.  Asynchronous on `stream`.
 */
cross_status cross_rescale(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L,
                           uint32_t drop, uint32_t npoly, const uint32_t* in, uint32_t* out,
                           void* stream);

/*
 * VecModMul with a pre-known operand under a chosen modular reduction (Sec.
 * Evaluation "Impact of Modular Reduction Algorithm", Fig. diff_modred:
 * Barrett, Montgomery, Shoup; App. "BAT for Modular Reduction": the lazy
 * partial reduction as an int8 matrix product on the MFMA units):
 *   out[p][l][n] = a[p][l][n] * w[l][n] mod q_l   for p < npoly, l < L, n < N.
 * Every method returns the canonical residue, so results are identical.
 *   CROSS_MODRED_BARRETT    Alg. barrett on the 56-bit product
 *   CROSS_MODRED_MONTGOMERY REDC (Alg. montgomery_reduction) with w in Montgomery form
 *   CROSS_MODRED_SHOUP      Shoup multiplication with precomputed quotients
 *   CROSS_MODRED_BAT_LAZY   the product's four 7-bit chunks above bit 28 times the
 *                           chunk matrix of 2^(7(4+j)) mod q on one int8 MFMA per 256
 *                           elements, then Barrett on the lazy sum (< 2^38); N >= 256
 */
typedef enum {
  CROSS_MODRED_BARRETT = 0,
  CROSS_MODRED_MONTGOMERY = 1,
  CROSS_MODRED_SHOUP = 2,
  CROSS_MODRED_BAT_LAZY = 3
} cross_modred;

/*
 * Prepare the pre-known operand once for `method`.
 *   w      : device [L][N] residues (not modified)
 *   w_prep : device 2*L*N words, must not overlap w: [L][N] prepared values
 *            (w * 2^32 mod q for Montgomery, w otherwise), then [L][N] Shoup
 *            quotients floor(w * 2^32 / q) (written for Shoup only)
 * Errors: CROSS_EINVAL (null / overlapping buffers, bad shape or method),
 * CROSS_EUNSUPPORTED (BAT-lazy with N < 256), prime checks as cross_ntt_forward.
 */
cross_status cross_vec_modmul_prepare(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L,
                                      int method, const uint32_t* w, uint32_t* w_prep, void* stream);
/*
 * out = a * w mod q limb-wise with w_prep from cross_vec_modmul_prepare (same
 * method, primes and N).  a, out: device [npoly][L][N] residues, 16-byte
 * aligned; out may alias a.  Asynchronous on `stream`.
 */
cross_status cross_vec_modmul(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L,
                              uint32_t npoly, int method, const uint32_t* a, const uint32_t* w_prep,
                              uint32_t* out, void* stream);

/*
 * Chunked forms of the two key-switching vector streams, beside their plain VALU
 * forms (App. "Applying BAT to Preknown Parameters", closing remark: evaluation
 * keys through BAT on a fine-grained matrix engine; App. "Fall-back Algorithm for
 * unknown parameters": runtime x runtime products as a chunk-wise 1D convolution).
 * Both chunked forms use 8-bit chunks on the VALU byte dot product; every form
 * returns the canonical residues, so the results are identical.
 *   CROSS_STREAM_VALU    : 32-bit products with Barrett reduction (Alg. barrett)
 *   CROSS_STREAM_CHUNKED : inner product from the BAT-expanded key (E[l][i] = byte l
 *                          of k 2^(32+8i) mod p, dot products over dnum x 4 bytes,
 *                          ChunkMerge, Montgomery reduction); tensor product from
 *                          the seven partial sums of the byte convolution, then Barrett
 */
typedef enum { CROSS_STREAM_VALU = 0, CROSS_STREAM_CHUNKED = 1 } cross_stream_form;

/*
 * Expand an evaluation key for CROSS_STREAM_CHUNKED (once per key).
 *   primes  : host, LK limb primes (Q then P), as cross_ntt_forward
 *   key     : device [dnum][2][LK][N] residues
 *   key_bat : device [dnum][2][LK][N][4] words (16 bytes per residue), must not
 *             overlap key; word l packs bytes E[l][0..3]
 * Errors: CROSS_EINVAL (null, misaligned or overlapping buffers, bad shape:
 * 1 <= LK <= CROSS_MAX_LIMBS, 1 <= dnum <= 64), prime checks as cross_ntt_forward.
 */
cross_status cross_evk_bat_prepare(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t LK,
                                   uint32_t dnum, const uint32_t* key, uint32_t* key_bat, void* stream);
/*
 * Key-switch inner product: out[b][s][t] = sum_j ext[b][j][t] * key_j.s[t] mod p_t
 * (s = 0 for b, 1 for a; the step between ModUp and ModDown of the hybrid key switch).
 *   ext : device [batch][dnum][LK][N];  out : device [batch][2][LK][N], must not
 *         overlap ext or key
 *   key : device [dnum][2][LK][N] (CROSS_STREAM_VALU) or the cross_evk_bat_prepare
 *         output (CROSS_STREAM_CHUNKED)
 * All buffers 16-byte aligned.  Asynchronous on `stream`.
 */
cross_status cross_keyswitch_inner_product(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t LK,
                                           uint32_t dnum, uint32_t batch, int form, const uint32_t* ext,
                                           const uint32_t* key, uint32_t* out, void* stream);
/*
 * HE-Mult tensor product limb-wise mod q_l: out[b][0] = a0 b0, out[b][1] = a0 b1 +
 * a1 b0, d2[b] = a1 b1.  a, b, out: device [batch][2][L][N]; d2: device
 * [batch][L][N]; out and d2 must not overlap each other or the inputs; 16-byte
 * aligned.  Asynchronous on `stream`.
 */
cross_status cross_tensor(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L, uint32_t batch,
                          int form, const uint32_t* a, const uint32_t* b, uint32_t* out, uint32_t* d2,
                          void* stream);

/*
 * Batch runtime (many jobs of uneven N and limb count in one pass).
 * Jobs are lowered onto a fixed sequence of phases (one per step of the hot
 * path, each covering that step for every job), each a few work-list launches:
 * the BAT GEMM steps run as persistent grids over (task, tile) lists, one
 * launch per list tile shape, and the three-factor row transform (R x 32 x 32,
 * used from N = 2^14 up; 2^12 and 2^13 run in two factors) as one persistent
 * launch over a task list -- at most 7 + 4 x 14 launches whatever the number of
 * jobs -- optionally captured once into a hipGraph so that a run is a single
 * graph launch.  The list tile per (N, direction) is the autotuner's choice
 * where it has made one.  Results are bit-identical to the per-call entry points.
 *   op CROSS_OP_NTT_FORWARD / _INVERSE: params.log_n, params.L, params.primes (L
 *        primes); data = device [batch][L][N], transformed in place.
 *   op CROSS_OP_HE_MULT: params as cross_he_mult; ct_a, ct_b, key, out as there.
 *   op CROSS_OP_ROTATE : params, steps, ct_a (the ciphertext), key (rotation key), out.
 * Limits: 12 <= log_n <= 16 and both R, C >= 64 for every job.  All buffers
 * must stay allocated while the batch exists; their contents may change
 * between runs.  A batch owns its workspace; concurrent runs of one batch race.
 */
enum { CROSS_OP_NTT_FORWARD = 1, CROSS_OP_NTT_INVERSE = 2, CROSS_OP_HE_MULT = 3, CROSS_OP_ROTATE = 4 };
typedef struct cross_job {
  uint32_t op;
  cross_ckks_params params;
  uint32_t batch;           /* polynomials (NTT) or ciphertexts */
  int32_t steps;            /* rotation steps (CROSS_OP_ROTATE) */
  uint32_t* data;           /* NTT jobs */
  const uint32_t* ct_a;
  const uint32_t* ct_b;
  const uint32_t* key;
  uint32_t* out;
} cross_job;
typedef struct cross_batch_s* cross_batch;
/* Plan the jobs (tables, task lists, workspace) and, if use_graph, capture the
 * launch sequence into a hipGraph.  No device work runs until cross_batch_run.
 * Primes below 2^28 only (CROSS_ERANGE for a wide prime in any job). */
cross_status cross_batch_create(cross_ctx ctx, const cross_job* jobs, uint32_t njobs, int use_graph,
                                cross_batch* out);
/* Bytes of device workspace a batch of these jobs needs when the caller provides it.
 * Never more than the sum of the bytes of each job alone (a batch's scratch is the
 * sum of its jobs', its merged task lists no larger than theirs apart), so a caller
 * may size a group of jobs from sizes it keeps per job shape. */
cross_status cross_batch_workspace_bytes(cross_ctx ctx, const cross_job* jobs, uint32_t njobs,
                                         uint64_t* bytes);
/* As cross_batch_create, but all of the batch's device memory (scratch and task
 * lists) is carved from the caller's `workspace` (256-byte aligned, at least
 * cross_batch_workspace_bytes): the batch allocates and frees no device memory
 * and destroying it does not synchronise the device, so the caller must know
 * that its last run has finished.  Task lists are copied on `stream`, in one copy
 * from a pinned host buffer of the context (held by the batch until it is
 * destroyed, then reused by later batches once that copy has finished); run the
 * batch on the same stream (or order it after that copy).  CROSS_ENOMEM if no
 * pinned buffer can be allocated. */
cross_status cross_batch_create_in(cross_ctx ctx, const cross_job* jobs, uint32_t njobs, int use_graph,
                                   void* workspace, uint64_t workspace_bytes, void* stream,
                                   cross_batch* out);
/* Work-list tile the batch runtime uses on ctx for the GEMM steps of a transform of
 * size 2^log_n in one direction (inverse != 0): 0 = 256 x 128, 1 = 128 x 64,
 * 2 = 64 x 64 (rows x columns of the int8 product per workgroup); *tuned = 1 if
 * cross_autotune chose it, 0 for the default (the largest tile whose rows divide
 * the step's 4U rows; here reported for the first step's U).
 * Errors: CROSS_EINVAL for a null pointer or log_n outside 12..16. */
cross_status cross_get_batch_tile(cross_ctx ctx, uint32_t log_n, int inverse, int* tile, int* tuned);
/* Enqueue one pass over every job on `stream` (graph launch or eager launches). */
cross_status cross_batch_run(cross_batch batch, void* stream);
/* Launch count per run (eager), workspace bytes and total GEMM tiles per run. */
cross_status cross_batch_info(cross_batch batch, uint32_t* launches, uint64_t* workspace_bytes,
                              uint64_t* gemm_tiles);
void cross_batch_destroy(cross_batch batch);

/*
 * Kernel timing with HIP events (tracing aid).  While enabled, every kernel
 * launch the library makes (or, after cross_profile_only, every launch of one
 * kernel family) carries a pair of events that the dispatch itself stamps at
 * kernel start and end on the launch stream (hipExtLaunchKernel; graph launches
 * of the batch runtime are bracketed by recorded events instead).
 * cross_profile_report synchronises on the events and writes one line per
 * kernel family, "name launches total_ms\n", into `buf` (NUL-terminated,
 * truncated to `len`), then clears the record.  cross_profile_only(ctx, name)
 * limits timing to the family `name` (NULL or "": all families).
 */
cross_status cross_profile_enable(cross_ctx ctx, int enable);
cross_status cross_profile_only(cross_ctx ctx, const char* family);
cross_status cross_profile_report(cross_ctx ctx, char* buf, uint64_t len);

/*
 * Measured machine peaks (roofline reference, synchronous): which = 0 -> int8
 * MFMA TOP/s from registers (v_mfma_i32_16x16x64_i8, 8 independent chains per
 * wave, 8 waves per SIMD); which = 1 -> streaming copy GB/s (bytes read +
 * written, 1 GiB buffers, allocated and freed by the call); which = 2 -> int8
 * MFMA TOP/s with v_mfma_i32_32x32x32_i8.
 */
cross_status cross_measure_peak(cross_ctx ctx, int which, double* out);

/*
 * Host-only introspection of the offline-compiled tables (no device work):
 * copies one table of the (q, N = 2^log_n, R = 2^log_r) plan into host memory
 * `out` of `*bytes` bytes.  If out is NULL, *bytes receives the size needed.
 *   which 0/1/2/3: BAT-expanded int8 matrices, forward step 1 / forward step 3 /
 *                  inverse step 3 (applied last) / inverse step 1 (applied first),
 *                  entry chunk_i((T[x][u] * 2^32 * 2^(7j)) mod q), m = 4u+i, k = 4x+j,
 *                  stored in MFMA fragment order: byte (m, k) at
 *                  ((k/64)*(M/32) + m/32)*2048 + ((k%64)/32)*1024
 *                  + 16*(m%32 + 32*((k%32)/16)) + k%16
 *                  (Alg. bat_deployment, DirectScalarBAT with the Montgomery factor folded in)
 *                  For a wide prime (2^28 <= q < 2^31): entry = balanced digit i (in
 *                  [-128, 127]) of the representative of (T[x][u] * 2^32 * 2^(8j)) mod q
 *                  in [-128*0x1010101, 127*0x1010101] (the residue itself unless above
 *                  that range), same order, followed by M int32 row corrections
 *                  128 * sum_k (m, k) at byte M*K + 4m
 *   which 4/5    : uint32 step-2 twiddles as (w, floor(w*2^32/q)) pairs (Shoup
 *                  multiplication), forward [R][C][2] and inverse transposed [C][R][2]
 *                  (Sec. MAT, layout-invariant 3-step NTT)
 *   which 7/8/9/10: the tables of which 0/1/2/3 without the Montgomery factor 2^32
 *                  (CROSS_NTT_RED_BARRETT; CROSS_EINVAL for wide primes)
 *   which 6      : the 1 KB int8 A operand of the BAT lazy reduction for q
 *                  (cross_vec_modmul, CROSS_MODRED_BAT_LAZY): lane l (0..63), byte e
 *                  at 16*l + e holds, for row = l%32, K byte kb = 16*(l/32) + e,
 *                  s = kb/4, j = kb%4, chunk row%4 of 2^(7(4+j)) mod q if
 *                  row/4 == 2*(s%4) + s/4, else 0 (App. "BAT for Modular Reduction")
 * Returns CROSS_EINVAL for a bad `which`, split or buffer size, CROSS_ERANGE for
 * q >= 2^31 (which 6: q >= 2^28).
 */
cross_status cross_host_tables(uint32_t q, uint32_t log_n, uint32_t log_r, uint32_t which,
                               void* out, uint64_t* bytes);

/*
 * Epilogue reduction of every MFMA NTT step on ctx (the row-side step and both
 * row-kernel sub-steps of the three-factor form, both steps of the two-factor
 * form), for the NTT side of the modular-reduction comparison (Sec. Evaluation,
 * Fig. diff_modred).  The butterfly kernels (N < 2^8 and the butterfly entry
 * points) and the batch runtime always use Montgomery reduction.  Results are
 * identical either way.
 *   CROSS_NTT_RED_MONTGOMERY (default): tables carry the factor 2^32, REDC of the
 *                            merged chunk sums (Alg. montgomery_reduction)
 *   CROSS_NTT_RED_BARRETT    : tables without the factor, Barrett reduction of the
 *                            merged sums (Alg. barrett); NTT calls whose primes lie
 *                            below 2^21 or at or above 2^28 then fail with
 *                            CROSS_EUNSUPPORTED
 * Returns CROSS_EINVAL for another method.
 */
typedef enum { CROSS_NTT_RED_MONTGOMERY = 0, CROSS_NTT_RED_BARRETT = 1 } cross_ntt_reduction;
cross_status cross_set_ntt_reduction(cross_ctx ctx, int method);

/*
 * Allocation-free NTT, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the transform of cross_ntt_forward (inverse = 0) or
 * cross_ntt_inverse (inverse != 0) with the same arguments, results and
 * kernels, but no device allocation and no free.  Its scratch (the NTT
 * intermediate and the call's job lists) is a file-scope device array of the
 * library, CROSS_NOALLOC_MAX_BYTES plus 64 KiB, of which each device the library
 * runs on holds one copy until the process ends; every call on a device shares
 * it, so calls that overlap on one device (on different streams, or from
 * different host threads) race.  Calls in one stream are ordered and safe.
 * The tables for the primes must already exist on ctx (built, and allocated, by
 * an earlier cross_ntt_forward or cross_ntt_inverse call with the same primes and
 * N on the same context and split).  Job lists are copied to the device with
 * stream-ordered host-to-device copies.
 * Errors: as cross_ntt_forward, plus CROSS_EINVAL when batch * L * N * 4 exceeds
 * CROSS_NOALLOC_MAX_BYTES and CROSS_EUNSUPPORTED when a prime's tables are not
 * on ctx yet; nothing is enqueued then.
 */
#define CROSS_NOALLOC_MAX_BYTES (128ull << 20)
cross_status cross_ntt_noalloc(cross_ctx ctx, uint32_t log_n, const uint32_t* primes, uint32_t L, uint32_t batch,
                               uint32_t* data, int inverse, void* stream);

/*
 * Debug mode (the preconditions check): while enabled, each entry point that
 * takes residues checks every input residue against its limb's prime with a
 * device kernel before its own work and returns CROSS_EDOMAIN (cross_last_error
 * names the input, polynomial, limb and coefficient) if one is not below it.
 * The check synchronises the stream (not for use under graph capture); the
 * chunked evaluation key, the prepared VecModMul operand, the batch runtime and
 * cross_ntt_noalloc are not checked.  Off by default; CROSS_DEBUG_CHECK=1 in the
 * environment turns it on for contexts created afterwards.
 */
cross_status cross_set_debug_check(cross_ctx ctx, int enable);

/*
 * Engine of every NTT the context runs (cross_ntt_forward/inverse and those
 * inside HE-Mult, Rotate, ModUp, ModDown, Rescale and cross_poly_mul): the BAT
 * int8-MFMA form (default) or the plain radix-2 butterfly kernels of
 * cross_ntt_forward_butterfly (App. "Radix-2 Cooley-Tukey NTT"), for the
 * comparison of whole HE operations on the two NTT paths.  Results are
 * identical either way.  The batch runtime always uses the MFMA form.
 * Returns CROSS_EINVAL for another value.
 */
typedef enum { CROSS_NTT_ENGINE_MFMA = 0, CROSS_NTT_ENGINE_BUTTERFLY = 1 } cross_ntt_engine;
cross_status cross_set_ntt_engine(cross_ctx ctx, int engine);

/*
 * Host-only introspection of the three-factor row tables (split as in
 * cross_set_ntt_split3), same calling convention as cross_host_tables:
 *   which 0/1 : int8 BAT tables of the forward row sub-steps, TB (over c1, 4C1 x 4C1)
 *               and TC (over c2, 4C2 x 4C2), in the fragment order of cross_host_tables
 *   which 2/3 : the inverse ones, ITC (over c2', first) and ITB (over m, second)
 *   which 4/5 : uint32 (w, floor(w*2^32/q)) pairs of T3, [C1][C2][2] (m, c2), and of
 *               IT3, [C2][C1][2] (c2, m)
 *   which 6/7 : uint32 pairs of the inverse / forward step-2 twiddles, row-major [R][C][2]
 *   which 8-11: the tables of which 0-3 without the Montgomery factor 2^32
 *               (CROSS_NTT_RED_BARRETT; CROSS_EINVAL for wide primes, which have none)
 *   which 12  : uint32 pairs of T3 * 2^32 mod q, [C1][C2][2]: with them the forward
 *               row transform yields its outputs times 2^32 (Montgomery form), as the
 *               fused ModUp NTT + key-switch inner product uses them
 */
cross_status cross_host_row_tables(uint32_t q, uint32_t log_n, uint32_t log_r, uint32_t log_c1, uint32_t which,
                                   void* out, uint64_t* bytes);

#ifdef __cplusplus
}
#endif
#endif /* CROSS_H */
