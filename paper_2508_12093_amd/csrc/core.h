// core.h -- internal types of the ppstat library (RNS-CKKS on gfx950).
//
// Layout conventions used everywhere:
//   * a polynomial over a list of primes is limb-major: limb t occupies
//     N consecutive uint64 residues in [0, q_t);
//   * a ciphertext at level l is [npoly][l+1][N] (npoly = 2, or 3 after a
//     tensor product), every polynomial in NTT form;
//   * prime indices are "combined": 0..L are the ciphertext primes q_0..q_L,
//     L+1..L+K the special primes p_0..p_{K-1} of hybrid key switching.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

namespace ppst {

typedef uint64_t u64;
typedef unsigned __int128 u128;

constexpr int kMaxPrimes = 64;

// -------------------------------------------------------------------------
// errors: every entry point converts these into a status code + message
// -------------------------------------------------------------------------
enum Status {
  ST_OK = 0, ST_EINVAL = -1, ST_ELEVEL = -2, ST_ESCALE = -3, ST_ENOKEY = -4, ST_ENOMEM = -5,
  ST_EDEVICE = -6, ST_EDOMAIN = -7
};

struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define PPST_THROW(code, msg) throw ::ppst::Error((code), (msg))
#define HIP_CHECK(expr)                                                          \
  do {                                                                           \
    hipError_t _e = (expr);                                                      \
    if (_e != hipSuccess)                                                        \
      PPST_THROW(::ppst::ST_EDEVICE, std::string(#expr " failed: ") + hipGetErrorString(_e)); \
  } while (0)

// -------------------------------------------------------------------------
// host modular arithmetic (64-bit residues, 128-bit products)
// -------------------------------------------------------------------------
inline u64 h_mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
inline u64 h_addmod(u64 a, u64 b, u64 q) { u64 s = a + b; return s >= q ? s - q : s; }
inline u64 h_submod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + (q - b); }
u64 h_powmod(u64 b, u64 e, u64 q);
inline u64 h_invmod(u64 a, u64 q) { return h_powmod(a % q, q - 2, q); }
inline u64 h_signed_mod(int64_t x, u64 q) {
  if (x >= 0) return (u64)x % q;
  u64 m = (u64)(-(x + 1)) % q;
  return q - 1 - m;
}
// floor(w * 2^64 / q): the Shoup companion of a constant w < q
inline u64 shoup(u64 w, u64 q) { return (u64)(((u128)w << 64) / q); }

// -------------------------------------------------------------------------
// parameters
// -------------------------------------------------------------------------
struct ParamSpec {
  int logN = 0, L = 0, K = 0, dnum = 0, q0_bits = 0, p_bits = 0;
  double scale = 0.0;
  // bootstrappable chains: secret weight (0: uniform ternary), the levels of
  // CoeffToSlot, EvalMod and SlotToCoeff at the top of the chain (counted in
  // L; all zero for a chain without bootstrapping) and EvalMod's scale
  int h = 0, boot_cts = 0, boot_evalmod = 0, boot_stc = 0;
  double boot_scale = 0.0;
};

struct Params {
  ParamSpec spec;
  int logN = 0, N = 0, L = 0, K = 0, dnum = 0, alpha = 0, nprimes = 0;
  int Lc = 0;                 // top level of computation (L without bootstrapping levels)
  std::vector<u64> q;         // combined: q_0..q_L, p_0..p_{K-1}
  std::vector<u64> psi;       // primitive 2N-th roots
  std::vector<double> scale;  // Delta_l, l = 0..L
  // canon[l]: Delta_{l-1} = Delta_l^2 / q_l, so a product at level l rescales
  // onto level l-1's scale; false only on the levels of the bootstrapping
  // linear transforms, whose scales are set by their plaintexts
  std::vector<uint8_t> canon;
  int slots() const { return N / 2; }
  bool bootstrappable() const { return spec.boot_cts > 0; }
  int digit_lo(int j) const { return j * alpha; }
  int digit_hi(int j, int level) const {  // one past the last limb of digit j at level
    int h = (j + 1) * alpha;
    return h < level + 1 ? h : level + 1;
  }
  int beta(int level) const { return (level + 1 + alpha - 1) / alpha; }
};

Params make_params(const ParamSpec& s);
bool preset_spec(const std::string& name, ParamSpec* out);
bool is_prime_u64(u64 n);

// -------------------------------------------------------------------------
// seeded sampling specification (counter-based SplitMix64)
// -------------------------------------------------------------------------
enum Purpose : u64 {
  P_SK = 1, P_PK_A = 2, P_PK_E = 3, P_KSK_A = 4, P_KSK_E = 5,
  P_ENC_V = 6, P_ENC_E0 = 7, P_ENC_E1 = 8, P_SKE_A = 9, P_SKE_E = 10
};
inline u64 purpose_code(u64 tag, u64 keyid, u64 digit) { return (tag << 40) | (keyid << 8) | digit; }
u64 stream_key(u64 seed, u64 purpose, u64 limb);
constexpr int kDgMax = 19;                  // |e| <= 19 (about 6 sigma)
void dg_thresholds(u64 thr[kDgMax]);        // cumulative thresholds, x = 0..18
// sparse ternary secret with exactly h nonzero coefficients, from the
// secret-key stream (seed, P_SK, 0): positions by a partial Fisher-Yates
// shuffle driven by its first h words, signs by the top bits of the next h
void sparse_ternary(u64 seed, int N, int h, int32_t* out);

// -------------------------------------------------------------------------
// encoding (host, extended precision)
// -------------------------------------------------------------------------
// encode_coeffs = encode_embed (the scale-free values p_k, N of them) then
// encode_round (coefficient k = round_half_away(scale p_k))
void encode_embed(const Params& P, const double* m, int n_used, std::vector<long double>& p);
void encode_round(const std::vector<long double>& p, double scale, int64_t* out);
void encode_coeffs(const Params& P, const double* m, int n_used, double scale, int64_t* out);
void decode_coeffs(const Params& P, const long double* coeffs, double scale, double* out, int n);

// -------------------------------------------------------------------------
// device prime descriptor: q and R = floor(2^128 / q) for 128-bit Barrett
// -------------------------------------------------------------------------
struct Mod {
  u64 q;
  u64 r_hi, r_lo;   // floor(2^128 / q)
  u64 mneg;         // -q^-1 mod 2^64 (Montgomery reduction)
};

// -------------------------------------------------------------------------
// device memory: a caching pool on one stream, optionally backed by caller
// hooks (e.g. a framework's caching allocator)
// -------------------------------------------------------------------------
struct Hooks {
  void* (*alloc)(size_t bytes, void* stream, void* user) = nullptr;
  void (*free)(void* ptr, size_t bytes, void* stream, void* user) = nullptr;
  void* user = nullptr;
};

class Pool;
// Every pool of one set of device tables (all contexts forked from one
// another, the key pool): when an allocation fails after a pool has freed its
// own cache, the others free theirs too.
class PoolRegistry {
 public:
  void add(const std::shared_ptr<Pool>& p);
  void trim_others(const Pool* except);
 private:
  std::mutex mu_;
  std::vector<std::weak_ptr<Pool>> pools_;
};

class Pool {
 public:
  Pool(hipStream_t s, const Hooks& h, std::shared_ptr<PoolRegistry> reg = nullptr)
      : stream_(s), hooks_(h), registry_(std::move(reg)) {}
  ~Pool();
  void* get(size_t bytes);
  void put(void* p, size_t bytes);
  size_t in_use() const { return in_use_; }
  size_t cached() const { return cached_; }
  // the largest in_use() since the last reset_peak() (the serving loop checks
  // its per-query estimates against it)
  size_t peak() const { return peak_; }
  void reset_peak();
  void trim();
  // The owning context is going away (its stream drained, about to be
  // destroyed): blocks still held by callers may outlive it, so from now on
  // the pool never touches that stream again.
  void detach();
  // Graph recording: every block handed out between begin_capture and
  // end_capture is pinned for the graph (end_capture returns them); a pinned
  // block released by its owner is not reused until unpin(), so the memory a
  // graph writes on each launch stays out of other hands.
  void begin_capture();
  std::vector<void*> end_capture();
  void unpin(const std::vector<void*>& blocks);
 private:
  // Blocks up to kSlabBlockMax bytes are carved from slabs of kSlabBytes (one
  // device allocation serves many ciphertexts); larger ones are allocations
  // of their own.  A slab is returned to the device by trim() once none of
  // its blocks is in use.
  static constexpr size_t kSlabBytes = (size_t)256 << 20;
  static constexpr size_t kSlabBlockMax = (size_t)32 << 20;
  struct Slab {
    char* base;
    size_t offset;
    int inuse;      // carved blocks currently handed out (or pinned)
    bool dead;
  };
  void* raw_alloc(size_t bytes);
  void raw_free(void* p, size_t bytes);
  void* alloc_retry(size_t bytes);
  void* hand_out(void* p, size_t bytes);   // bookkeeping of a block leaving the pool (mu_ held)

  hipStream_t stream_;
  bool detached_ = false;
  Hooks hooks_;
  std::shared_ptr<PoolRegistry> registry_;
  std::mutex mu_;
  std::multimap<size_t, void*> free_;
  std::map<void*, size_t> sizes_;
  std::map<void*, int> slab_of_;   // carved block -> slab index
  std::vector<Slab> slabs_;
  int cur_ = -1;                   // slab being carved
  size_t in_use_ = 0, cached_ = 0, nalloc_ = 0, peak_ = 0;
  bool capturing_ = false;
  std::vector<void*> captured_;
  std::map<void*, bool> pinned_;   // block -> released by its owner
};

struct Buf {
  u64* p = nullptr;
  size_t bytes = 0;
  std::shared_ptr<Pool> pool;
  Buf() = default;
  Buf(std::shared_ptr<Pool> pl, size_t nbytes) : bytes(nbytes), pool(std::move(pl)) {
    p = (u64*)pool->get(nbytes);
  }
  Buf(const Buf&) = delete;
  Buf& operator=(const Buf&) = delete;
  Buf(Buf&& o) noexcept : p(o.p), bytes(o.bytes), pool(std::move(o.pool)) { o.p = nullptr; o.bytes = 0; }
  Buf& operator=(Buf&& o) noexcept {
    release();
    p = o.p; bytes = o.bytes; pool = std::move(o.pool);
    o.p = nullptr; o.bytes = 0;
    return *this;
  }
  ~Buf() { release(); }
  void release() {
    if (p && pool) pool->put(p, bytes);
    p = nullptr;
    bytes = 0;
  }
};

// -------------------------------------------------------------------------
// per-device constant tables shared by every context of one parameter set
// -------------------------------------------------------------------------
struct Tables {
  Buf mods;        // Mod[nprimes]
  Buf fwd;         // [nprimes][N][2] (w, w') with w = psi^brv(k)
  Buf inv;         // [nprimes][N][2] (w, w') with w = psi^-brv(k)
  // row passes of the two-pass transform (N = 2^16, rows of 2^8 points) form
  // the entries they need from two small tables (ntt.hip, row_twiddles):
  // rowf [nprimes][2^8][8] = entry (2^8 + r) 2^s as a double (FP64 primes),
  // comm [nprimes][2^8][2] = (psi^(brv_s(j) N / 2^s), its quotient by q) at
  // index 2^s + j; the _inv tables the same for psi^-1
  Buf rowf_fwd, rowf_inv, comm_fwd, comm_inv;
  Buf ninv;        // [nprimes][2] (N^-1, Shoup)
  // ModUp constants per level: see modup_table()
  std::map<int, std::shared_ptr<Buf>> modup;
  // per level: [l+1][2] final factors N^-1 Qhat_i^-1 mod q_i (digit of limb i)
  // of the inverse transforms that feed ModUp, in the twiddle table format
  std::map<int, std::shared_ptr<Buf>> modup_ninv;
  // ModDown constants (one table for all levels)
  Buf moddown;
  // [nprimes][2] final factors of the inverse NTT before a ModDown's
  // conversion: N^-1 Phat_k^-1 on special prime p_k, N^-1 elsewhere
  Buf md_ninv;
  // host copy of (P mod q_i, Shoup companion), i = 0..L, for kernel arguments
  std::vector<u64> pmod_host;
  // rescale constants per level
  std::map<int, std::shared_ptr<Buf>> rescale;
  std::mutex mu;
};

// NTT variant choice per [inverse][pass: 0 column, 1 row][limb-count bucket]
struct NttPlan {
  int v[2][2][5] = {};
  bool tuned = false;
};

struct Shared {
  Params P;
  NttPlan ntt_plan;
  int device = 0;
  Hooks hooks;
  std::shared_ptr<PoolRegistry> pools = std::make_shared<PoolRegistry>();
  std::shared_ptr<Pool> const_pool;  // long-lived tables and keys
  Tables tab;
  u64 dg_thr[kDgMax];
};

struct Context;
struct Ciphertext {
  Buf buf;          // [npoly][level+1][N]
  int level = 0;
  double scale = 0;
  int npoly = 2;
  int N = 0;
  u64* poly(int c) const { return buf.p + (size_t)c * (level + 1) * N; }
};
struct Plaintext {
  Buf buf;          // [level+1][N], NTT form
  int level = 0;
  double scale = 0;
  std::vector<int64_t> coeffs;   // integer coefficients when produced by encode
};
struct SecretKey {
  std::vector<int8_t> s;   // ternary coefficients (host)
  Buf s_ntt;               // [nprimes][N]
};
struct PublicKey {
  Buf pk;                  // [2][L+1][N]
};
struct KsKey {
  Buf k;                   // [dnum][2][nprimes][N]
};
struct EvalKeys {
  std::shared_ptr<KsKey> relin;
  std::map<u64, std::shared_ptr<KsKey>> galois;   // keyed by Galois element
};

struct Context;
// Where a statistics circuit's rotate-and-sums go: with none set, straight to
// rotsum_batch on the context's stream; a server installs one that merges the
// lanes of concurrent queries into shared launches (results bit for bit the
// same: the batched form equals the one-lane form).
struct RotSumRouter {
  virtual ~RotSumRouter() = default;
  virtual std::vector<std::shared_ptr<Ciphertext>> rotsum(
      Context& cx, const EvalKeys& evk, const std::vector<std::shared_ptr<Ciphertext>>& lanes) = 0;
};

struct Context {
  std::shared_ptr<Shared> sh;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::shared_ptr<Pool> pool;    // temporaries and results on this stream
  bool recording = false;        // a graph recording is open on the stream
  RotSumRouter* router = nullptr;
  const Params& P() const { return sh->P; }
};

// -------------------------------------------------------------------------
// kernel launchers (kernels.hip)
// -------------------------------------------------------------------------
// NTT autotuner (ntt.hip): times the kernel variants on `scratch` (at least
// max_limbs * N words) and records the fastest per limb-count bucket
void ntt_autotune(Shared& sh, hipStream_t st, u64* scratch, int max_limbs);
std::string ntt_plan_string(const Shared& sh);
void ntt_set_plan(Shared& sh, int col, int row);
// the plan ntt_plan_string wrote (EINVAL for unknown names or a missing bucket)
void ntt_load_plan(Shared& sh, const std::string& text);

}  // namespace ppst
