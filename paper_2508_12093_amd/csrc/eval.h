// eval.h -- the RNS-CKKS evaluator of the ppstat library (host orchestration
// of the device kernels).  Every operation is enqueued on the context's
// stream; nothing synchronises except the functions that return host data.
#pragma once

#include "core.h"

namespace ppst {

typedef std::shared_ptr<Ciphertext> CtPtr;
typedef std::shared_ptr<Plaintext> PtPtr;

std::shared_ptr<Shared> make_shared_state(const ParamSpec& spec, const Hooks* hooks);
std::unique_ptr<Context> make_context(std::shared_ptr<Shared> sh, hipStream_t stream);
void destroy_context(Context* cx);
// time the NTT kernel variants and keep the fastest per limb-count bucket
void autotune_ntt(Shared& sh);

// galois element of a rotation by r slots: 5^(r mod N/2) mod 2N
u64 galois_elt(const Params& P, long r);

// ------------------------------------------------------------------ keys
std::unique_ptr<SecretKey> keygen_secret(Context& cx, u64 seed);
std::unique_ptr<PublicKey> keygen_public(Context& cx, const SecretKey& sk, u64 seed);
std::shared_ptr<KsKey> keygen_relin(Context& cx, const SecretKey& sk, u64 seed);
std::shared_ptr<KsKey> keygen_galois(Context& cx, const SecretKey& sk, u64 seed, u64 g);

// ----------------------------------------------------------- plaintexts
PtPtr encode(Context& cx, const double* v, size_t n, int level);
// encode at `level` from encode_embed's values: the same plaintext as encode
PtPtr encode_embedded(Context& cx, const std::vector<long double>& p, int level);
PtPtr plaintext_from_coeffs(Context& cx, const int64_t* coeffs, int level, double scale);
void decode(Context& cx, const Plaintext& pt, double* out, size_t n);

// --------------------------------------------------------- ciphertexts
CtPtr new_ct(Context& cx, int level, double scale, int npoly = 2);
CtPtr encrypt_pk(Context& cx, const PublicKey& pk, const Plaintext& pt, u64 seed);
CtPtr encrypt_sk(Context& cx, const SecretKey& sk, const Plaintext& pt, u64 seed);
PtPtr decrypt(Context& cx, const SecretKey& sk, const Ciphertext& ct);

// ------------------------------------------------------------ operations
CtPtr add(Context& cx, const Ciphertext& a, const Ciphertext& b);
// the sum of ciphertexts of one level and scale in one launch per 64 terms
CtPtr add_n(Context& cx, const std::vector<const Ciphertext*>& a);
CtPtr sub(Context& cx, const Ciphertext& a, const Ciphertext& b);
int64_t const_int(const Params& P, double c, int level);
CtPtr add_const(Context& cx, const Ciphertext& a, double c);
CtPtr mul_int(Context& cx, const Ciphertext& a, int64_t k);
CtPtr mul_const(Context& cx, const Ciphertext& a, double c);
// mul_const of each ciphertext, all at one level and of one degree; the
// rescales of up to 16 ciphertexts share each launch.  Bit for bit the same
// as mul_const of each.
std::vector<CtPtr> mul_const_n(Context& cx, const std::vector<const Ciphertext*>& a, double c);
CtPtr mul_plain(Context& cx, const Ciphertext& a, const Plaintext& pt);
CtPtr tensor(Context& cx, const Ciphertext& a, const Ciphertext& b);
CtPtr relin(Context& cx, const EvalKeys& evk, const Ciphertext& d);
CtPtr rescale(Context& cx, const Ciphertext& a);
CtPtr mul(Context& cx, const EvalKeys& evk, const Ciphertext& a, const Ciphertext& b);
// mul() of raw device ciphertexts a, b ([2][l+1][N] at scale Delta_l) into
// out ([2][l][N]) with no allocation: every intermediate lives in `scratch`
// (mul_scratch_words(P, l) words: the tensor, the extended digits, the
// accumulators, and d2's coefficient copy whose space the ModDown
// correction takes over).  Bit for bit mul()'s result.
size_t mul_scratch_words(const Params& P, int level);
void mul_into(Context& cx, const EvalKeys& evk, const u64* a, const u64* b, int level, u64* out,
              u64* scratch);
CtPtr rotate(Context& cx, const EvalKeys& evk, const Ciphertext& a, long r);
// X -> X^g (g odd, below 2N) and the key switch back to s: rotate() for
// g = 5^r; conjugation of every slot for g = 2N - 1
CtPtr apply_galois(Context& cx, const EvalKeys& evk, const Ciphertext& a, u64 g);
// rescale by q_l whose result carries `scale` (for products whose plaintext
// factor was chosen to land on that scale)
CtPtr rescale_as(Context& cx, const Ciphertext& a, double scale);
// the product with a plaintext (limbs 0..a.level of it), no rescale
CtPtr mul_plain_raw(Context& cx, const Ciphertext& a, const Plaintext& pt);
// a * (sign X^k), exact (no level)
CtPtr mul_monomial(Context& cx, const Ciphertext& a, int k, int sign);
// ModRaise: a level-0 ciphertext read over q_0..q_L, each residue mod q_0
// lifted to (-q_0/2, q_0/2]; it decrypts to the old plaintext plus q_0 I for
// a small integer polynomial I
CtPtr mod_raise(Context& cx, const Ciphertext& a);
std::vector<CtPtr> rotate_hoisted(Context& cx, const EvalKeys& evk, const Ciphertext& a,
                                  const std::vector<long>& rs);
// rotate_hoisted for many ciphertexts of one level: every ModUp first, then
// each rotation over the whole batch (outputs ordered [ciphertext][rotation])
std::vector<CtPtr> rotate_hoisted_batch(Context& cx, const EvalKeys& evk,
                                        const std::vector<const Ciphertext*>& cts,
                                        const std::vector<long>& rs);
// rotate() of several ciphertexts of one level by the same step: one key
// switch over the batch (the key read once per group of items)
std::vector<CtPtr> rotate_batch(Context& cx, const EvalKeys& evk,
                                const std::vector<const Ciphertext*>& cts, long r);
// Rotate-and-sum (every slot ends up holding the sum of all N/2 slots) in
// the steps of rotsum_plan: ct <- ct + sum_{0<k<radix} rot(ct, k s), each
// step's key switches hoisted (one ModUp of c1, the permuted inner products
// added in the extended basis, one ModDown).
CtPtr rotsum(Context& cx, const EvalKeys& evk, const Ciphertext& a);
// Rotate-and-sum by its definition: log2(N/2) steps ct <- ct + Rot(ct, 2^k),
// each a plain rotation (key switch of c1(X^g), ModDown adding c0(X^g))
// whose last pass also adds the step's input
CtPtr rotsum_serial(Context& cx, const EvalKeys& evk, const Ciphertext& a);
// rotsum() of several ciphertexts of one level, each step batched
std::vector<CtPtr> rotsum_batch(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& cts);
// rotsum_batch whose results are written into `outs` (caller-allocated, one
// per input, of its level and scale; empty: new ones), for a caller whose
// lanes come from other streams and must land in memory they own
std::vector<CtPtr> rotsum_batch_into(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& cts,
                                     const std::vector<CtPtr>& outs);
// (s, radix) per step: radix 8 while three or more bits of the slot index
// remain, then radix 4 or 2 for the rest; the Galois keys needed are those of
// k s, 0 < k < radix
std::vector<std::pair<long, int>> rotsum_plan(const Params& P);
CtPtr level_align(Context& cx, const Ciphertext& a, int level);
// level_align of each ciphertext, all at one level and of one degree; the
// rescales of up to 16 ciphertexts share each launch.  Bit for bit the same
// as level_align of each.
std::vector<CtPtr> level_align_n(Context& cx, const std::vector<const Ciphertext*>& a, int level);
// sum_k cs[k] cts[k] at `level` with one rescale: each term (level > level)
// cut to q_0..q_{level+1}, multiplied by round(c Delta_{level+1}
// (Delta_{level+1} / Delta_term)), the products added, then rescaled by
// q_{level+1}
CtPtr lincomb(Context& cx, const std::vector<const Ciphertext*>& cts,
              const std::vector<double>& cs, int level);
CtPtr copy_ct(Context& cx, const Ciphertext& a);

// many independent products a[i] * b[i], one launch per stage for each group
// of 16 products (the inner product reads the key once per 8 of them)
std::vector<CtPtr> mul_batch(Context& cx, const EvalKeys& evk, const std::vector<const Ciphertext*>& a,
                             const std::vector<const Ciphertext*>& b);

// Recording of evaluation calls into a HIP graph (stream capture on the
// context's stream).  The graph owns every block handed out while recording
// until it is destroyed; destruction waits for its launches.
struct Graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t stream = nullptr;
  std::shared_ptr<Pool> pool;
  std::vector<void*> blocks;
  Graph() = default;
  Graph(const Graph&) = delete;
  Graph& operator=(const Graph&) = delete;
  ~Graph();
};
void graph_begin(Context& cx);
std::unique_ptr<Graph> graph_end(Context& cx);
void graph_launch(Graph& g);

// raw NTT on device memory (canonical order), limb i on prime first_prime + i
void ntt_raw(Context& cx, u64* data, int nlimbs, int first_prime, bool inverse);

}  // namespace ppst
