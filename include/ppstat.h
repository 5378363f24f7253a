/*
 * ppstat.h -- C ABI of an MI355X (gfx950) implementation of the RNS-CKKS
 * ciphertext arithmetic behind PP-STAT's encrypted statistics
 * (H. Choi, "PP-STAT: An Efficient Privacy-Preserving Statistical Analysis
 * Framework using Homomorphic Encryption", CIKM 2025).
 *
 * The paper's roles (Sec. 4): the client generates keys, encrypts its data
 * with the public key and sends ciphertexts plus evaluation keys; the server
 * evaluates statistics with pre-normalisation bounds B (Sec. 5.1); the client
 * decrypts.  All three roles are available here.
 *
 * Conventions
 *   - Every function returns PPST_OK (0) or a negative status; the message of
 *     the last failure on the calling thread is ppst_last_error().
 *   - Objects returned through `T** out` belong to the caller and are released
 *     with the matching *_destroy function.  Inputs are borrowed for the call.
 *   - Device work is enqueued on the context's HIP stream and is asynchronous;
 *     functions that return host data (decode, export, *_sync) synchronise.
 *     A context is used by one thread at a time.
 *   - Polynomials are limb-major: limb i of a ciphertext polynomial at level l
 *     holds N residues modulo q_i, i = 0..l, in the canonical NTT order in
 *     which slot j holds a(psi_i^(2 brv(j) + 1)).  A ciphertext is
 *     [2][l+1][N] uint64 words; every ciphertext at level l has the canonical
 *     scale Delta_l (Delta_L = Delta, Delta_{l-1} = Delta_l^2 / q_l).
 *   - Binary operations require equal levels (and hence scales); there is no
 *     silent alignment: use ppst_level_align.
 */
#ifndef PPSTAT_H
#define PPSTAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
enum {
  PPST_OK = 0,
  PPST_EINVAL = -1,   /* malformed argument (null pointer, size mismatch) */
  PPST_ELEVEL = -2,   /* an operation would go below level 0 (Sec. 3.1: beyond the
                         depth, decryption is not guaranteed) */
  PPST_ESCALE = -3,   /* operands at different levels or scales */
  PPST_ENOKEY = -4,   /* missing relinearisation or Galois key */
  PPST_ENOMEM = -5,   /* device memory or serving budget exhausted */
  PPST_EDEVICE = -6,  /* HIP runtime error */
  PPST_EDOMAIN = -7   /* parameter outside the documented domain */
};

/* message of the last failure on this thread (valid until the next call) */
const char* ppst_last_error(void);

/* ------------------------------------------------------------- parameters */
/* Ring degree N = 2^logN, L+1 ciphertext primes (q_0 of q0_bits bits, q_1..q_L
 * chosen so that the scale stays at Delta), K special primes of p_bits bits
 * for hybrid key switching with dnum digits, and the scale Delta.
 * Presets: "c1" (N=2^12, 40/30/30-bit chain, Delta=2^30, one 60-bit special
 * prime); "c2" (N=2^16, Delta=2^40, 24 scale primes + 60-bit q_0, 7 special
 * primes, dnum=3: the paper's N, Delta and log2 PQ <= 1443 budget, Sec. 6.1);
 * "t1", "t2" (N=2^12 test sets with the c2 prime shapes, L=6 and L=24);
 * "b2" (N=2^16) and "b1" (N=2^12), bootstrappable: L = 27 levels of which
 * the top 16 serve bootstrapping (3 CoeffToSlot, 10 EvalMod at scale 2^58,
 * 3 SlotToCoeff) and 11 computation (Delta = 2^40; the paper's depth 27
 * with 11 levels between bootstraps, Sec. 6.1), a sparse secret of weight
 * 64, a 55-bit q_0, 8 special primes, dnum = 4.
 * Every prime must stay below 2^60 (q0_bits, p_bits <= 60 and Delta well
 * below 2^60), K <= 8, dnum <= 8 and ceil((L+1)/dnum) <= 16; other sets are
 * rejected with PPST_EINVAL.
 * h: secret weight (0: uniform ternary).  boot_cts, boot_evalmod, boot_stc:
 * levels of the bootstrapping stages at the top of the chain (all 0 for a
 * chain without bootstrapping), boot_scale: EvalMod's scale.  Their primes:
 * the largest unused primes below 2^p_bits for the two transforms (labels
 * boot_scale on top, Delta 2^(i e / stc) between, e the difference of the
 * binary exponents), an EvalMod chain near boot_scale. */
typedef struct {
  int32_t logN, L, K, dnum, q0_bits, p_bits;
  double scale;
  int32_t h, boot_cts, boot_evalmod, boot_stc;
  double boot_scale;
} ppst_params;

int ppst_params_preset(const char* name, ppst_params* out);

/* Optional device-memory hooks.  alloc/free receive the context's stream and
 * `user`; when absent the library allocates with hipMalloc and caches blocks
 * per stream. */
typedef struct {
  void* (*alloc)(size_t bytes, void* stream, void* user);
  void (*free)(void* ptr, size_t bytes, void* stream, void* user);
  void* user;
} ppst_device_hooks;

/* Host-only derivations (no device needed): the combined prime list, the
 * canonical scales and the 2N-th roots of a parameter set, following the
 * prime rule of the presets (q_0 the largest prime < 2^q0_bits that is
 * 1 mod 2N; q_L..q_1 the unused such prime nearest Delta_l^2 / Delta with
 * Delta_{l-1} = Delta_l^2 / q_l; the K largest unused primes < 2^p_bits). */
int ppst_params_derive(const ppst_params* params, uint64_t* primes, uint64_t* roots,
                       double* scales, size_t cap);
/* discrete-Gaussian sampler thresholds (19 entries), host only */
int ppst_dg_thresholds(uint64_t* out, size_t cap);
/* integer coefficients of the canonical-embedding encoding of n values at
 * (level, Delta_level), host only (N outputs) */
int ppst_encode_coeffs(const ppst_params* params, const double* values, size_t n, int32_t level,
                       int64_t* out, size_t cap);
/* the rotation steps whose Galois keys ppst_rotsum needs (the keys
 * ppst_evk_add_rotsum makes), host only: *n receives their number; with
 * out == NULL and cap == 0 only the count is returned, otherwise cap must be
 * at least that count (EINVAL) */
int ppst_rotsum_steps(const ppst_params* params, int32_t* out, size_t cap, size_t* n);
/* Host only: the Chebyshev coefficients c_0..c_degree (first kind, in
 * t = (2v - a - b) / (b - a)) of 1/sqrt(B' v) on [a, b], interpolated at the
 * first-kind nodes cos(pi (j + 1/2) / (degree + 1)): the initial value of
 * CryptoInvSqrt (Sec. 4.1 Alg. 3, Sec. 4.2 Eq. 1 and Eq. 3 with a = 0, b = 2)
 * that the statistics use when their configuration brings no coefficients.
 * EDOMAIN unless 0 <= a < b, B' > 0 and 1 <= degree <= 511; EINVAL when cap <
 * degree + 1. */
int ppst_chebyshev_invsqrt(double a, double b, int32_t degree, double Bp, double* out, size_t cap);
/* SplitMix64 stream state for (seed, purpose, limb), host only */
uint64_t ppst_stream_key(uint64_t seed, uint64_t purpose, uint64_t limb);

typedef struct ppst_context ppst_context;
typedef struct ppst_secret_key ppst_secret_key;
typedef struct ppst_public_key ppst_public_key;
typedef struct ppst_eval_keys ppst_eval_keys;
typedef struct ppst_plaintext ppst_plaintext;
typedef struct ppst_ciphertext ppst_ciphertext;

/* Creates the primes, roots, twiddle and CRT tables on the current HIP device.
 * stream: a hipStream_t to run on, or NULL for a private stream.
 * hooks: may be NULL. */
int ppst_context_create(const ppst_params* params, const ppst_device_hooks* hooks, void* stream,
                        ppst_context** out);
/* A second context sharing tables with `base`, running on its own stream.
 * Work on different contexts is not ordered: an object made on one context
 * may be used on another after ppst_sync of the first, and must not be
 * destroyed while another context's queued work still reads it. */
int ppst_context_fork(const ppst_context* base, void* stream, ppst_context** out);
/* waits for the context's stream; ciphertexts and plaintexts it produced stay
 * valid (their memory is released when the last of them is destroyed) */
int ppst_context_destroy(ppst_context* ctx);
/* waits for all work enqueued on the context's stream */
int ppst_sync(ppst_context* ctx);

typedef struct {
  int32_t logN, N, L, K, dnum, alpha, nprimes, slots;
} ppst_info;
int ppst_context_info(const ppst_context* ctx, ppst_info* out);
/* combined prime list q_0..q_L, p_0..p_{K-1} (cap >= nprimes) */
int ppst_context_primes(const ppst_context* ctx, uint64_t* out, size_t cap);
/* canonical scales Delta_0..Delta_L (cap >= L+1) */
int ppst_context_scales(const ppst_context* ctx, double* out, size_t cap);
/* discrete-Gaussian thresholds of the sampler (19 entries), for auditing */
int ppst_context_dg_table(const ppst_context* ctx, uint64_t* out, size_t cap);

/* --------------------------------------------------------------- keys */
/* Seeded key generation (client side, Sec. 4).  Randomness is a counter-based
 * SplitMix64 stream keyed by (seed, purpose, limb): ternary s, uniform a
 * drawn in NTT form, discrete Gaussian errors (sigma 3.2, |e| <= 19). */
int ppst_keygen(ppst_context* ctx, uint64_t seed, ppst_secret_key** sk, ppst_public_key** pk);
int ppst_secret_key_destroy(ppst_secret_key* sk);
int ppst_public_key_destroy(ppst_public_key* pk);
int ppst_evk_create(ppst_context* ctx, ppst_eval_keys** out);
int ppst_evk_destroy(ppst_eval_keys* evk);
/* relinearisation key (s^2 -> s) */
int ppst_evk_add_relin(ppst_context* ctx, const ppst_secret_key* sk, uint64_t seed,
                       ppst_eval_keys* evk);
/* Galois keys for rotations by steps[i] slots (s(X^g) -> s, g = 5^r mod 2N) */
int ppst_evk_add_galois(ppst_context* ctx, const ppst_secret_key* sk, const int32_t* steps,
                        size_t n, uint64_t seed, ppst_eval_keys* evk);
/* Galois keys that rotate-and-sum needs: steps k 8^i (k = 1..7) while
 * 8^(i+1) <= N/2, then k 8^i for k below the remaining 4 or 2 (35 keys at
 * N = 2^16, 24 at N = 2^12) */
int ppst_evk_add_rotsum(ppst_context* ctx, const ppst_secret_key* sk, uint64_t seed,
                        ppst_eval_keys* evk);
/* copy a key to the host: galois = 0 selects the relinearisation key.
 * Layout [dnum][2][nprimes][N] (b, a per digit, NTT form). */
int ppst_evk_export(ppst_context* ctx, const ppst_eval_keys* evk, uint64_t galois, uint64_t* host,
                    size_t cap_words);
/* The server side of the paper's roles (Sec. 4: the client sends the
 * evaluation keys with its ciphertexts): a key in ppst_evk_export's layout,
 * `words` = dnum * 2 * nprimes * N, added to `evk` as the relinearisation key
 * (galois = 0) or the Galois key of element `galois` (odd, 1 < g < 2N),
 * replacing one already there.  The words are copied (the host buffer is not
 * kept); every residue must be below its prime (EINVAL otherwise, nothing
 * changed).  Synchronises. */
int ppst_evk_import(ppst_context* ctx, ppst_eval_keys* evk, uint64_t galois, const uint64_t* host,
                    size_t words);
/* [2][L+1][N] (b, a over q_0..q_L, NTT form) */
int ppst_pk_export(ppst_context* ctx, const ppst_public_key* pk, uint64_t* host, size_t cap_words);
/* a public key from ppst_pk_export's words (`words` = 2 (L+1) N, each below
 * its prime, else EINVAL); the caller owns *out.  Synchronises. */
int ppst_pk_import(ppst_context* ctx, const uint64_t* host, size_t words, ppst_public_key** out);
/* s in NTT form over every prime, [nprimes][N] */
int ppst_sk_export(ppst_context* ctx, const ppst_secret_key* sk, uint64_t* host, size_t cap_words);

/* ------------------------------------------------------------ plaintexts */
/* Canonical-embedding encoding of n <= N/2 real values (the rest zero) at
 * (level, Delta_level): coefficient k = round_half_away(Delta_level * p_k). */
int ppst_encode(ppst_context* ctx, const double* values, size_t n, int32_t level,
                ppst_plaintext** out);
/* plaintext from signed integer coefficients (N of them), at a given scale */
int ppst_plaintext_from_coeffs(ppst_context* ctx, const int64_t* coeffs, int32_t level,
                               double scale, ppst_plaintext** out);
/* integer coefficients of an encoded plaintext (N values) */
int ppst_plaintext_coeffs(const ppst_plaintext* pt, int64_t* out, size_t cap);
/* [level+1][N] residues, NTT form */
int ppst_plaintext_export(ppst_context* ctx, const ppst_plaintext* pt, uint64_t* host,
                          size_t cap_words);
/* a plaintext from ppst_plaintext_export's words at (level, scale): usable
 * wherever an encoded one is (ppst_mul_plain, ppst_decode); it carries no
 * integer coefficients (ppst_plaintext_coeffs gives EINVAL).  Residues must be
 * below their primes and scale positive (EINVAL), level in 0..L (ELEVEL).
 * Synchronises; the caller owns *out. */
int ppst_plaintext_import(ppst_context* ctx, const uint64_t* host, int32_t level, double scale,
                          ppst_plaintext** out);
/* decode slots (the centred lift uses q_0, or q_0 q_1 above level 0) */
int ppst_decode(ppst_context* ctx, const ppst_plaintext* pt, double* out, size_t n);
int ppst_plaintext_destroy(ppst_plaintext* pt);

/* ----------------------------------------------------------- ciphertexts */
/* public-key encryption (Sec. 4): (v b + e0 + m, v a + e1), v ternary */
int ppst_encrypt(ppst_context* ctx, const ppst_public_key* pk, const ppst_plaintext* pt,
                 uint64_t seed, ppst_ciphertext** out);
/* secret-key encryption: (-a s + e + m, a) */
int ppst_encrypt_sk(ppst_context* ctx, const ppst_secret_key* sk, const ppst_plaintext* pt,
                    uint64_t seed, ppst_ciphertext** out);
/* c0 + c1 s */
int ppst_decrypt(ppst_context* ctx, const ppst_secret_key* sk, const ppst_ciphertext* ct,
                 ppst_plaintext** out);
int ppst_ciphertext_destroy(ppst_ciphertext* ct);
int ppst_ct_info(const ppst_ciphertext* ct, int32_t* level, double* scale, int32_t* npoly);
/* copy [npoly][level+1][N] words to / from the host */
int ppst_ct_export(ppst_context* ctx, const ppst_ciphertext* ct, uint64_t* host, size_t cap_words);
int ppst_ct_import(ppst_context* ctx, const uint64_t* host, int32_t level, double scale,
                   int32_t npoly, ppst_ciphertext** out);
/* device address of the residues (valid while the ciphertext lives) */
int ppst_ct_device_ptr(const ppst_ciphertext* ct, uint64_t** out);

/* ------------------------------------------------------------- evaluator */
/* Add(C), Sub(C) (Sec. 3.1) */
int ppst_add(ppst_context* ctx, const ppst_ciphertext* a, const ppst_ciphertext* b,
             ppst_ciphertext** out);
int ppst_sub(ppst_context* ctx, const ppst_ciphertext* a, const ppst_ciphertext* b,
             ppst_ciphertext** out);
/* Add(P) with a constant: adds round_half_away(c Delta_level) */
int ppst_add_const(ppst_context* ctx, const ppst_ciphertext* a, double c, ppst_ciphertext** out);
/* Mul(P) with a constant: multiply by round_half_away(c Delta_l), then rescale */
int ppst_mul_const(ppst_context* ctx, const ppst_ciphertext* a, double c, ppst_ciphertext** out);
/* multiply by a signed integer; no rescale, scale unchanged */
int ppst_mul_int(ppst_context* ctx, const ppst_ciphertext* a, int64_t k, ppst_ciphertext** out);
/* Mul(P) with a plaintext encoded at the ciphertext's level, then rescale */
int ppst_mul_plain(ppst_context* ctx, const ppst_ciphertext* a, const ppst_plaintext* pt,
                   ppst_ciphertext** out);
/* Mul(C): tensor, relinearise (hybrid key switching), rescale: level l -> l-1 */
int ppst_mul(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* a,
             const ppst_ciphertext* b, ppst_ciphertext** out);
/* ppst_mul into caller memory, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): no hipMalloc, hipFree or pool allocation happens in it.
 *   a, b   device addresses of two ciphertexts at `level` (1..L), each
 *          [2][level+1][N] words in the layout above, scale Delta_level (the
 *          layout ppst_ct_device_ptr exposes); borrowed, read on the stream.
 *   out    device address of [2][level][N] words receiving the product at
 *          scale Delta_{level-1}, bit for bit ppst_mul's; must not overlap
 *          a or b (EINVAL).
 * The key-switching intermediates live in one library-wide device array of
 * 144 MiB per GPU, held from the first context on that GPU until the process
 * ends; a product whose intermediates exceed it is refused with EINVAL (at
 * N = 2^16, K = 7, dnum = 3 every level up to 24 fits).  All calls on one GPU
 * share that array: calls that overlap in time (other contexts' streams,
 * other threads) race, and the caller must order them.  Nothing in the array
 * needs clearing between calls.  Asynchronous on the context's stream;
 * ELEVEL outside 1..L, ENOKEY without a relinearisation key, EDEVICE when
 * the runtime could not resolve the array. */
int ppst_mul_noalloc(ppst_context* ctx, const ppst_eval_keys* evk, const uint64_t* a,
                     const uint64_t* b, int32_t level, uint64_t* out);
/* the three steps of ppst_mul separately (tensor output has npoly = 3) */
int ppst_tensor(ppst_context* ctx, const ppst_ciphertext* a, const ppst_ciphertext* b,
                ppst_ciphertext** out);
int ppst_relin(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* d,
               ppst_ciphertext** out);
int ppst_rescale(ppst_context* ctx, const ppst_ciphertext* a, ppst_ciphertext** out);
/* Rot (Sec. 3.1): slot j of the result holds slot (j + r) mod N/2 */
int ppst_rotate(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* a, int32_t r,
                ppst_ciphertext** out);
/* n rotations sharing one ModUp of c1 (the automorphism acts on the extended
 * digits); a different but equally valid key switch than ppst_rotate */
int ppst_rotate_hoisted(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* a,
                        const int32_t* rs, size_t n, ppst_ciphertext** outs);
/* ppst_rotate of n ciphertexts of one level by the same step r as one key
 * switch over the batch (the Galois key read once per group of items);
 * outs[i] is bit-identical to ppst_rotate(cts[i], r). */
int ppst_rotate_batch(ppst_context* ctx, const ppst_eval_keys* evk,
                      const ppst_ciphertext* const* cts, size_t n, int32_t r,
                      ppst_ciphertext** outs);
/* ppst_rotate_hoisted over n ciphertexts of one level: all ModUps first, then
 * each rotation over the whole batch, so a Galois key is read once per group
 * of ciphertexts.  outs[i * m + k] = rotation of cts[i] by rs[k], bit-identical
 * to ppst_rotate_hoisted(cts[i], rs).  Device memory: about
 * n (beta (l+1+K) + 2 (l+1+K) + 2 (l+1)) limbs of scratch besides the n m
 * outputs (beta = ceil((l+1)/alpha) digits). */
int ppst_rotate_hoisted_batch(ppst_context* ctx, const ppst_eval_keys* evk,
                              const ppst_ciphertext* const* cts, size_t n, const int32_t* rs,
                              size_t m, ppst_ciphertext** outs);
/* rotate-and-sum: every slot ends up holding the sum of all N/2 slots (the
 * sums of Eq. 2, Sec. 5.1).  Steps of three bits, ct += rot(ct, s) + ... +
 * rot(ct, 7s) for s = 1, 8, 64, ..., then one step of two bits or one bit
 * for what remains; each step's key switches share one ModUp of c1 and one
 * rounding ModDown of the summed inner products (keys: ppst_evk_add_rotsum). */
int ppst_rotsum(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* a,
                ppst_ciphertext** out);
/* rotate-and-sum by its plain definition (the slot sums of Eq. 2, with
 * Sec. 3.1's Rot): for k = 0 .. log2(N/2) - 1, ct <- ct + Rot(ct, 2^k), each
 * Rot an ordinary (unhoisted) rotation.  Fifteen key switches at N = 2^16
 * instead of ppst_rotsum's five hoisted steps; the same sum up to the
 * key-switching rounding.  Galois keys for the steps 2^k (ppst_evk_add_rotsum
 * makes them, or ppst_evk_add_galois); ENOKEY when one is missing. */
int ppst_rotsum_serial(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* a,
                       ppst_ciphertext** out);
/* ppst_rotsum of n ciphertexts of one level: each step's ModUp, inner
 * product (a thread serves up to 5 ciphertexts per key read) and ModDown
 * run once for the whole group.  Bit for bit the same as n calls of
 * ppst_rotsum.  outs: n handles written on success; PPST_ESCALE for mixed
 * levels. */
int ppst_rotsum_batch(ppst_context* ctx, const ppst_eval_keys* evk,
                      const ppst_ciphertext* const* cts, size_t n, ppst_ciphertext** outs);
/* bring a ciphertext down to `level`: keep q_0..q_{level+1}, multiply by
 * round(Delta_level q_{level+1} / Delta_l), rescale by q_{level+1} */
int ppst_level_align(ppst_context* ctx, const ppst_ciphertext* a, int32_t level,
                     ppst_ciphertext** out);
/* sum_i cs[i] cts[i] at `level` with a single rescale (the Chebyshev sum of
 * Alg. 3 uses it): every cts[i] (level > `level`, any mix of levels) is cut
 * to q_0..q_{level+1} and multiplied by round(cs[i] Delta_{level+1}
 * (Delta_{level+1} / Delta_{l_i})); the products are added and the sum is
 * rescaled by q_{level+1}.  One term one level up gives exactly
 * ppst_mul_const.  ELEVEL when a term is not above `level`. */
int ppst_lincomb(ppst_context* ctx, const ppst_ciphertext* const* cts, const double* cs, size_t n,
                 int32_t level, ppst_ciphertext** out);
/* ppst_mul_const(cts[i], c) for i < n, all ciphertexts at one level and of
 * one degree: the rescales of up to 16 ciphertexts run as one launch
 * sequence (the dropped limbs gathered, one inverse NTT, one conversion, one
 * forward NTT whose last pass multiplies by c and divides by q_l).  Bit for
 * bit the same as n calls of ppst_mul_const.  outs: n handles written on
 * success.  PPST_ESCALE when levels or degrees differ, PPST_ELEVEL at level
 * 0, PPST_EDOMAIN when c does not fit the scale. */
int ppst_mul_const_batch(ppst_context* ctx, const ppst_ciphertext* const* cts, size_t n, double c,
                         ppst_ciphertext** outs);
/* n independent products a[i] * b[i] (same level): each stage of tensor,
 * relinearisation and rescale runs once per group of 16 products (the key
 * is read once per 8 products inside the inner product) */
int ppst_mul_batch(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* const* a,
                   const ppst_ciphertext* const* b, size_t n, ppst_ciphertext** outs);

/* ----------------------------------------------------------------- graphs */
/* Recording of evaluation work into a HIP graph (stream capture on the
 * context's stream), for callers that replay a fixed sequence many times.
 * Between ppst_graph_begin and ppst_graph_end the evaluation calls (add, sub,
 * add_const, mul_const, mul_const_batch, mul_int, mul_plain, mul, tensor,
 * relin, rescale, rotate, rotate_batch, rotate_hoisted(_batch), rotsum, rotsum_serial,
 * rotsum_batch, level_align, mul_batch) are recorded, not run: their output handles are valid at once, and each
 * ppst_graph_launch writes them again.  Calls that wait for the device or
 * move data to or from the host (keygen, encode, encrypt, decrypt, exports,
 * imports, statistics, ppst_sync, context create/fork/destroy) fail with
 * PPST_EINVAL while a recording is open.  Device memory handed out while
 * recording is owned by the graph until ppst_graph_destroy, so releasing a
 * recorded output early is safe; the recorded inputs must stay alive for as
 * long as the graph is launched.  Launches are asynchronous on the
 * context's stream; ppst_graph_destroy waits for them and must come before
 * the context's destruction.  While a recording is open no other context
 * may be created or destroyed in the process: that synchronises or frees
 * device memory, which invalidates the capture (the calls of the
 * recording then fail with PPST_EDEVICE). */
typedef struct ppst_graph ppst_graph;
int ppst_graph_begin(ppst_context* ctx);
int ppst_graph_end(ppst_context* ctx, ppst_graph** out);
int ppst_graph_launch(ppst_graph* g);
int ppst_graph_destroy(ppst_graph* g);

/* ------------------------------------------------------------- statistics */
typedef struct ppst_boot ppst_boot;   /* bootstrapping material, see below */
/* CryptoInvSqrt configuration (Sec. 4, Alg. 2-3; Sec. 5.1, Eq. 3): Chebyshev
 * initial value of degree `degree` for 1/sqrt(B' v) on [a, b] (first-kind
 * interpolation; degree 0..511), then `iters` Newton steps (0..32; EDOMAIN
 * outside these ranges).  coeffs, when non-NULL, gives
 * c_0..c_degree of 1/sqrt(v) on [a, b] (B' = 1), divided by sqrt(B') per call.
 * sign_k: number of g_3 compositions of the sign in CV (Sec. 6.2).
 * boot, when non-NULL (a bootstrappable context's ppst_boot, its keys in the
 * call's evk), lets InvSqrt refresh levels by bootstrapping (Alg. 3 bootstraps
 * the initial value; each refresh brings a ciphertext to level 0 and
 * bootstraps it): the argument when it lacks the levels of the initial
 * value's polynomial, the initial value itself, w = (B'/2) v or y before a
 * Newton step that lacks its two levels, and the result when the statistic
 * needs more levels after it than remain; CV also refreshes its sign
 * before a g_3 step it lacks the levels for.  The statistics then need only
 * their own levels around InvSqrt.
 * degree 0: the initial value is the constant c_0 (with coeffs = {1}, the
 * y_0 = 1 of HEaaN-STAT's Newton iteration, the paper's Tab. 2 baseline). */
typedef struct {
  double a, b;
  int32_t degree, iters, sign_k;
  const double* coeffs;
  const ppst_boot* boot;
} ppst_invsqrt_cfg;
/* a, b = 1e-3, 1; degree 7; 3 iterations; sign_k 2; coeffs NULL; boot NULL */
int ppst_invsqrt_cfg_default(ppst_invsqrt_cfg* out);

/* CryptoInvSqrt slot by slot (Sec. 4, Alg. 2-3; Sec. 6.2, Exp. 1): each of
 * the nct ciphertexts x (one level) is scaled to v = x/B and its inverse
 * square root InvSqrt(v; B) ~ 1/sqrt(x) written to outs[i] (caller frees).
 * Consumes 1 + (m + ceil(log2(degree + 1)) + 1 + 2 iters) levels, m = 0 when
 * b - a = 2 (the map onto [-1, 1] is then a shift, as Eq. 1's x - 1 on
 * [0, 2]) and 1 otherwise; a Chebyshev degree of up to 511 holds degree + 1
 * ciphertexts per input while it runs.  B > 0; the interval needs
 * 0 <= a < b. */
int ppst_stat_invsqrt(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* const* x,
                      size_t nct, double B, const ppst_invsqrt_cfg* cfg,
                      ppst_ciphertext** outs /* nct */);

/* A column is `nct` ciphertexts at one level holding `nrows` values (slots
 * past nrows are zero).  Each statistic writes ciphertexts whose every slot
 * holds the result (ZNorm: one output per input ciphertext).
 * Preconditions that cannot be checked on encrypted data (Var/B^2 and
 * |mean|/B inside [a, b]) are the caller's (Sec. 5.1).  ZNorm, kurtosis,
 * skewness and CV form the mean and the variance's slot sum with one
 * two-lane rotate-and-sum; PCC forms all five of its slot sums (both means,
 * both second moments, the cross moment) with one five-lane rotate-and-sum,
 * so its two columns must have the same length and level (EINVAL). */
int ppst_stat_mean(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* const* col,
                   size_t nct, size_t nrows, double B, ppst_ciphertext** out);          /* Mean/B */
int ppst_stat_variance(ppst_context* ctx, const ppst_eval_keys* evk,
                       const ppst_ciphertext* const* col, size_t nct, size_t nrows, double B,
                       ppst_ciphertext** out);                                         /* Var/B^2 */
int ppst_stat_zscore(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* const* col,
                     size_t nct, size_t nrows, double B, const ppst_invsqrt_cfg* cfg,
                     ppst_ciphertext** outs /* nct */);                                /* Alg. 4 */
int ppst_stat_kurtosis(ppst_context* ctx, const ppst_eval_keys* evk,
                       const ppst_ciphertext* const* col, size_t nct, size_t nrows, double B,
                       const ppst_invsqrt_cfg* cfg, int32_t excess, ppst_ciphertext** out); /* Alg. 5 */
int ppst_stat_skewness(ppst_context* ctx, const ppst_eval_keys* evk,
                       const ppst_ciphertext* const* col, size_t nct, size_t nrows, double B,
                       const ppst_invsqrt_cfg* cfg, ppst_ciphertext** out);
int ppst_stat_cv(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* const* col,
                 size_t nct, size_t nrows, double B_mean, double B_var, const ppst_invsqrt_cfg* cfg,
                 ppst_ciphertext** out);                                               /* Alg. 6 */
int ppst_stat_pearson(ppst_context* ctx, const ppst_eval_keys* evk,
                      const ppst_ciphertext* const* colx, const ppst_ciphertext* const* coly,
                      size_t nct, size_t nrows, double Bx, double By, const ppst_invsqrt_cfg* cfg,
                      ppst_ciphertext** out);                                          /* Sec. 5.5 */

/* ---------------------------------------------------------- bootstrapping */
/* CKKS bootstrapping (Sec. 3.2: it refreshes a ciphertext whose levels are
 * spent; Alg. 3 refreshes the InvSqrt initial value with it; Tab. 1 gives its
 * cost), built as in the work the paper cites, for the bootstrappable
 * presets "b1"/"b2" (EINVAL on other parameter sets):
 *   ModRaise     a level-0 ciphertext read over q_0..q_L (centred lift):
 *                it decrypts to t = c + q_0 I, I small;
 *   CoeffToSlot  the inverse decoding map in three levels, each a
 *                baby-step giant-step sum of rotated diagonals (baby
 *                rotations hoisted) and one rescale: slots
 *                (t_k + i t_{k+N/2}) / (2 K q_0), K = 16, in bit-reversed order;
 *   split        re = w + conj(w), im = -X^{N/2} (w - conj(w));
 *   EvalMod      per lane, the degree-27 Chebyshev series of
 *                cos(2 pi (K u - 1/4) / 16) and four double angles:
 *                sin(2 pi K u), i.e. 2 pi c_k / q_0 near the integers;
 *   SlotToCoeff  re + X^{N/2} im through the decoding map in three levels,
 *                times q_0 / (2 pi Delta_0): the message at level Lc = L - 16.
 * A refreshed [-1, 1] message carries a max error of about 2^-21 at
 * N = 2^12 and 2^-17 at N = 2^16 (q_0 of 55 bits: q_0 / Delta_0 = 2^15).
 * The diagonals' plaintexts are encoded on the host in binary128 (each
 * integer the correctly rounded one), then transformed on the device;
 * ppst_boot_create takes seconds at N = 2^16 and holds about 3.3 GiB there.
 * Every call is enqueued on the context's stream; outputs are new handles. */
/* coeffs: EvalMod's c_0..c_27 (NULL: the library's interpolation, see
 * ppst_evalmod_coeffs); ncoeffs must be 28 when coeffs is given */
int ppst_boot_create(ppst_context* ctx, const double* coeffs, size_t ncoeffs, ppst_boot** out);
int ppst_boot_destroy(ppst_boot* bt);
/* the number of bootstraps enqueued with bt so far (ppst_bootstrap and the
 * refreshes of statistics whose cfg carries bt) */
int ppst_boot_count(const ppst_boot* bt, uint64_t* n);
/* the Galois keys bootstrapping needs: every rotation step of
 * ppst_boot_rotations and conjugation (Galois element 2N - 1) */
int ppst_evk_add_boot(ppst_context* ctx, const ppst_secret_key* sk, uint64_t seed,
                      ppst_eval_keys* evk);
/* host only: the nonzero rotation steps (mod N/2, ascending) of the
 * transforms; *n receives their count (out == NULL with cap == 0: count only) */
int ppst_boot_rotations(const ppst_params* params, int32_t* out, size_t cap, size_t* n);
/* host only: group `group` (0..2, in the order applied) of CoeffToSlot
 * (transform 0) or SlotToCoeff (1) as 9 integers: inverse, lo, hi (layers
 * len = 2^lo..2^hi), level, constant kind, offset unit u, first offset m0,
 * baby steps b, giant steps G */
int ppst_boot_group_info(const ppst_params* params, int32_t transform, int32_t group, int32_t* desc);
/* host only: the integer coefficients of that group's b G plaintexts, out
 * [b G][N] (row j b + i: the diagonal of offset u (m0 + b j + i) rotated by
 * -u (m0 + b j), encoded at Delta_{l-1} q_l / Delta_l times the group's
 * constant), used[b G] (0: no such diagonal, row left zero); cap_cells >= b G */
int ppst_boot_group_coeffs(const ppst_params* params, int32_t transform, int32_t group,
                           int64_t* out, uint8_t* used, size_t cap_cells);
/* host only: first-kind Chebyshev interpolation of cos(2 pi (K u - 1/4) / 2^r)
 * on [-1, 1], c_0..c_degree (EDOMAIN for degree < 1, K < 1 or r < 0) */
int ppst_evalmod_coeffs(int32_t K, int32_t r, int32_t degree, double* out, size_t cap);
/* the refresh: level 0 in, level L - 16 out (ELEVEL otherwise) */
int ppst_bootstrap(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_boot* bt,
                   const ppst_ciphertext* a, ppst_ciphertext** out);
/* its stages, for inspection: ModRaise (level 0 -> L); X -> X^g with the key
 * switch back (g odd, < 2N; g = 2N - 1 conjugates every slot); a * (sign
 * X^k), exact; CoeffToSlot (level L -> L - 3); the split into re and im;
 * EvalMod of n lanes of one level; SlotToCoeff of (re, im) */
int ppst_mod_raise(ppst_context* ctx, const ppst_ciphertext* a, ppst_ciphertext** out);
int ppst_apply_galois(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* a,
                      uint64_t g, ppst_ciphertext** out);
int ppst_mul_monomial(ppst_context* ctx, const ppst_ciphertext* a, int32_t k, int32_t sign,
                      ppst_ciphertext** out);
int ppst_boot_coeff_to_slot(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_boot* bt,
                            const ppst_ciphertext* a, ppst_ciphertext** out);
int ppst_boot_split(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_boot* bt,
                    const ppst_ciphertext* w, ppst_ciphertext** re, ppst_ciphertext** im);
int ppst_boot_eval_mod(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_boot* bt,
                       const ppst_ciphertext* const* lanes, size_t n, ppst_ciphertext** outs);
int ppst_boot_slot_to_coeff(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_boot* bt,
                            const ppst_ciphertext* re, const ppst_ciphertext* im,
                            ppst_ciphertext** out);

/* ------------------------------------------------------------ raw kernels */
/* In-place forward / inverse negacyclic NTT of `nlimbs` limbs of N words at
 * device address `dev`; limb i uses combined prime first_prime + i (0..L are
 * q_i, L+1.. the special primes).  Enqueued on the context stream. */
int ppst_ntt_forward(ppst_context* ctx, uint64_t* dev, int32_t nlimbs, int32_t first_prime);
int ppst_ntt_inverse(ppst_context* ctx, uint64_t* dev, int32_t nlimbs, int32_t first_prime);
/* Re-run the NTT autotuner (it also runs at context creation unless the
 * environment sets PPST_NTT_AUTOTUNE=0 or forces PPST_NTT_PLAN="col,row" or a
 * whole plan):
 * every register-radix / workgroup-shape variant of the column and row passes
 * is timed per limb-count bucket and the fastest is kept for this parameter
 * set.  ppst_ntt_plan writes the choice as text. */
int ppst_ntt_autotune(ppst_context* ctx);
int ppst_ntt_plan(const ppst_context* ctx, char* buf, size_t cap);
/* force one variant for every bucket and direction (col ignored at N = 2^12);
 * returns PPST_EINVAL for an index outside the variant tables */
int ppst_ntt_set_plan(ppst_context* ctx, int32_t col, int32_t row);
/* install a plan in the text form ppst_ntt_plan writes (e.g. one saved from
 * an earlier autotuning); the environment variable PPST_NTT_PLAN may hold the
 * same text.  PPST_EINVAL for an unknown variant name or a missing bucket
 * (the plan is then unchanged). */
int ppst_ntt_load_plan(ppst_context* ctx, const char* plan);
/* hipStream_t of the context */
int ppst_context_stream(const ppst_context* ctx, void** stream);

/* ---------------------------------------------------------------- serving */
/* A server owns worker contexts (one HIP stream each) over resident columns
 * and evaluation keys.  Queries are admitted while the number of in-flight
 * queries is below `slots` and their estimated device memory fits within
 * `hbm_budget` bytes; later queries wait in arrival order and are admitted as
 * earlier ones finish, so their work overlaps on the device. */
typedef struct ppst_server ppst_server;
enum { PPST_Q_MEAN = 0, PPST_Q_VARIANCE = 1, PPST_Q_ZSCORE = 2, PPST_Q_CV = 3, PPST_Q_PEARSON = 4,
       PPST_Q_SKEWNESS = 5, PPST_Q_KURTOSIS = 6 };
typedef struct {
  int32_t kind;
  uint64_t col_x, col_y;     /* column handles; col_y only for Pearson */
  double B, B2;              /* bounds: B (and By for Pearson, B_var for CV) */
  ppst_invsqrt_cfg cfg;
} ppst_query;
typedef struct {
  double t_submit, t_admit, t_done;   /* seconds, monotonic clock */
  uint64_t bytes_reserved;            /* the admission estimate */
  uint64_t bytes_peak;                /* device bytes its worker's pool held at most */
} ppst_query_stats;
enum { PPST_SERVER_NO_MERGE = 1 };
/* Waits until the device is idle (the keys may still be in generation on the
 * caller's stream), then starts `slots` workers (1..16) with streams of their
 * own.  Queries are admitted while the sum of their estimated peak device
 * memory stays within hbm_budget; hbm_budget = 0 takes the device's free
 * memory at creation less 2 GiB.  Unless flags has PPST_SERVER_NO_MERGE, the
 * rotate-and-sums of queries running at once are merged into shared launches
 * (the lanes of every worker that reaches one at the same level within
 * 0.5 ms, up to 10 lanes, one key read per step for up to five of them);
 * each result is bit for bit the one the query gets alone. */
int ppst_server_create(ppst_context* ctx, const ppst_eval_keys* evk, size_t hbm_budget,
                       int32_t slots, uint32_t flags, ppst_server** out);
/* the admission budget in force, and the merged rotate-and-sum launches run,
 * the lanes they served and how many carried more than one query's lanes
 * (any pointer may be NULL) */
int ppst_server_info(ppst_server* srv, uint64_t* budget, uint64_t* merged_launches,
                     uint64_t* merged_lanes, uint64_t* multi_query_launches);
/* the server keeps its own copy of the ciphertexts; the call waits until the
 * device is idle first, so ciphertexts still being produced on any stream
 * (e.g. an asynchronous encryption) are complete when they are copied */
int ppst_server_register_column(ppst_server* srv, const ppst_ciphertext* const* cts, size_t nct,
                                size_t nrows, uint64_t* col_id);
/* EINVAL for a query whose cfg carries a bootstrapper (the admission
 * estimates do not cover bootstrapping) */
int ppst_server_submit(ppst_server* srv, const ppst_query* q, uint64_t* ticket);
/* *done = 1 once the query has finished, 0 while it is pending or running;
 * never blocks.  The result stays with the server until ppst_server_wait
 * collects it.  EINVAL for an unknown (or already collected) ticket. */
int ppst_server_poll(ppst_server* srv, uint64_t ticket, int32_t* done);
/* blocks until the query has finished; out receives the result ciphertext
 * (ZNorm: the first output ciphertext).  Returns the query's own status. */
int ppst_server_wait(ppst_server* srv, uint64_t ticket, ppst_ciphertext** out,
                     ppst_query_stats* stats);
/* number of result ciphertexts of a submitted query: for ZNorm the column's
 * ciphertext count (one z-score ciphertext per input ciphertext), else 1.
 * EINVAL for an unknown or collected ticket. */
int ppst_server_output_count(ppst_server* srv, uint64_t ticket, size_t* n);
/* like ppst_server_wait, but every result ciphertext: outs (cap entries)
 * receives *n_out handles on success.  EINVAL, without collecting the query,
 * when cap is below ppst_server_output_count. */
int ppst_server_wait_all(ppst_server* srv, uint64_t ticket, ppst_ciphertext** outs, size_t cap,
                         size_t* n_out, ppst_query_stats* stats);
/* lets the queries being run finish, drops those still waiting for
 * admission, and releases the server's streams; result ciphertexts already
 * collected stay valid */
int ppst_server_destroy(ppst_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* PPSTAT_H */
