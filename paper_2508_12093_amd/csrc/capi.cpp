// capi.cpp -- the extern "C" boundary declared in include/ppstat.h.
#include "capi.h"

using namespace ppst;

namespace ppst {
std::string& last_error() {
  thread_local std::string msg;
  return msg;
}
}  // namespace ppst

namespace {


std::vector<CtPtr> column(const ppst_ciphertext* const* col, size_t nct) {
  NEED(col);
  std::vector<CtPtr> v;
  for (size_t i = 0; i < nct; ++i) {
    NEED(col[i]);
    v.push_back(col[i]->c);
  }
  return v;
}

InvSqrtCfg cfg_from(const ppst_invsqrt_cfg* c) {
  InvSqrtCfg r;
  if (c) {
    r.a = c->a;
    r.b = c->b;
    r.degree = c->degree;
    r.iters = c->iters;
    if (c->coeffs) r.coeffs.assign(c->coeffs, c->coeffs + c->degree + 1);
    if (c->boot) {
      if (!c->boot->b) PPST_THROW(ST_EINVAL, "empty bootstrapping handle");
      r.boot = c->boot->b.get();
    }
  }
  return r;
}

void copy_out(Context& cx, const u64* dev, size_t words, uint64_t* host, size_t cap) {
  NEED(host);
  if (cap < words) PPST_THROW(ST_EINVAL, "host buffer too small");
  HIP_CHECK(hipMemcpyAsync(host, dev, words * 8, hipMemcpyDeviceToHost, cx.stream));
  HIP_CHECK(hipStreamSynchronize(cx.stream));
}

}  // namespace

ParamSpec ppst::spec_from(const ppst_params& p) {
  ParamSpec s;
  s.logN = p.logN;
  s.L = p.L;
  s.K = p.K;
  s.dnum = p.dnum;
  s.q0_bits = p.q0_bits;
  s.p_bits = p.p_bits;
  s.scale = p.scale;
  s.h = p.h;
  s.boot_cts = p.boot_cts;
  s.boot_evalmod = p.boot_evalmod;
  s.boot_stc = p.boot_stc;
  s.boot_scale = p.boot_scale;
  return s;
}

extern "C" {

const char* ppst_last_error(void) { return last_error().c_str(); }

int ppst_params_preset(const char* name, ppst_params* out) {
  return guard([&] {
    NEED(name);
    NEED(out);
    ParamSpec s;
    if (!preset_spec(name, &s)) PPST_THROW(ST_EINVAL, std::string("unknown preset ") + name);
    out->logN = s.logN;
    out->L = s.L;
    out->K = s.K;
    out->dnum = s.dnum;
    out->q0_bits = s.q0_bits;
    out->p_bits = s.p_bits;
    out->scale = s.scale;
    out->h = s.h;
    out->boot_cts = s.boot_cts;
    out->boot_evalmod = s.boot_evalmod;
    out->boot_stc = s.boot_stc;
    out->boot_scale = s.boot_scale;
  });
}

int ppst_params_derive(const ppst_params* params, uint64_t* primes, uint64_t* roots,
                       double* scales, size_t cap) {
  return guard([&] {
    NEED(params);
    ParamSpec s = spec_from(*params);
    Params P = make_params(s);
    if (cap < (size_t)P.nprimes) PPST_THROW(ST_EINVAL, "buffer too small");
    for (int i = 0; i < P.nprimes; ++i) {
      if (primes) primes[i] = P.q[i];
      if (roots) roots[i] = P.psi[i];
    }
    if (scales)
      for (int i = 0; i <= P.L; ++i) scales[i] = P.scale[i];
  });
}

int ppst_dg_thresholds(uint64_t* out, size_t cap) {
  return guard([&] {
    NEED(out);
    if (cap < (size_t)kDgMax) PPST_THROW(ST_EINVAL, "buffer too small");
    u64 t[kDgMax];
    dg_thresholds(t);
    for (int i = 0; i < kDgMax; ++i) out[i] = t[i];
  });
}

int ppst_chebyshev_invsqrt(double a, double b, int32_t degree, double Bp, double* out, size_t cap) {
  return guard([&] {
    NEED(out);
    if (!(a >= 0.0 && b > a && Bp > 0.0)) PPST_THROW(ST_EDOMAIN, "need 0 <= a < b and B' > 0");
    if (degree < 1 || degree > 511) PPST_THROW(ST_EDOMAIN, "degree must be in 1..511");
    if (cap < (size_t)degree + 1) PPST_THROW(ST_EINVAL, "buffer too small");
    const std::vector<double> c = chebyshev_invsqrt(a, b, degree, Bp);
    std::copy(c.begin(), c.end(), out);
  });
}

int ppst_encode_coeffs(const ppst_params* params, const double* values, size_t n, int32_t level,
                       int64_t* out, size_t cap) {
  return guard([&] {
    NEED(params);
    NEED(out);
    if (n) NEED(values);
    ParamSpec s = spec_from(*params);
    Params P = make_params(s);
    if (level < 0 || level > P.L) PPST_THROW(ST_ELEVEL, "level out of range");
    if (cap < (size_t)P.N) PPST_THROW(ST_EINVAL, "buffer too small");
    encode_coeffs(P, values, (int)n, P.scale[level], out);
  });
}

int ppst_rotsum_steps(const ppst_params* params, int32_t* out, size_t cap, size_t* n) {
  return guard([&] {
    NEED(params);
    NEED(n);
    ParamSpec sp = spec_from(*params);
    Params P = make_params(sp);
    std::vector<int32_t> steps;
    for (const auto& st : rotsum_plan(P))
      for (int k = 1; k < st.second; ++k) steps.push_back((int32_t)(k * st.first));
    *n = steps.size();
    if (out == nullptr && cap == 0) return;
    NEED(out);
    if (cap < steps.size()) PPST_THROW(ST_EINVAL, "buffer too small");
    for (size_t i = 0; i < steps.size(); ++i) out[i] = steps[i];
  });
}

uint64_t ppst_stream_key(uint64_t seed, uint64_t purpose, uint64_t limb) {
  return stream_key(seed, purpose, limb);
}

int ppst_context_create(const ppst_params* params, const ppst_device_hooks* hooks, void* stream,
                        ppst_context** out) {
  return guard([&] {
    NEED(params);
    NEED(out);
    ParamSpec s = spec_from(*params);
    if (s.logN != 12 && s.logN != 16) PPST_THROW(ST_EDOMAIN, "log2 N must be 12 or 16");
    Hooks h;
    if (hooks) {
      if (!hooks->alloc || !hooks->free) PPST_THROW(ST_EINVAL, "hooks need alloc and free");
      h.alloc = hooks->alloc;
      h.free = hooks->free;
      h.user = hooks->user;
    }
    auto sh = make_shared_state(s, hooks ? &h : nullptr);
    *out = new ppst_context{make_context(sh, (hipStream_t)stream)};
    // resolve this device's ppst_mul_noalloc scratch now; a failure is kept
    // and reported by that entry point, the context itself is usable
    try {
      noalloc_scratch();
    } catch (const Error&) {
    }
  });
}

int ppst_context_fork(const ppst_context* base, void* stream, ppst_context** out) {
  return guard([&] {
    NEED(base);
    NOT_RECORDING(base);
    NEED(out);
    *out = new ppst_context{make_context(base->cx->sh, (hipStream_t)stream)};
  });
}

int ppst_context_destroy(ppst_context* ctx) {
  return guard([&] {
    if (!ctx) return;
    NOT_RECORDING(ctx);
    destroy_context(ctx->cx.get());
    delete ctx;
  });
}

int ppst_sync(ppst_context* ctx) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    HIP_CHECK(hipStreamSynchronize(ctx->cx->stream));
  });
}

int ppst_context_info(const ppst_context* ctx, ppst_info* out) {
  return guard([&] {
    NEED(ctx);
    NEED(out);
    const Params& P = ctx->cx->P();
    out->logN = P.logN;
    out->N = P.N;
    out->L = P.L;
    out->K = P.K;
    out->dnum = P.dnum;
    out->alpha = P.alpha;
    out->nprimes = P.nprimes;
    out->slots = P.slots();
  });
}

int ppst_context_primes(const ppst_context* ctx, uint64_t* out, size_t cap) {
  return guard([&] {
    NEED(ctx);
    NEED(out);
    const Params& P = ctx->cx->P();
    if (cap < (size_t)P.nprimes) PPST_THROW(ST_EINVAL, "buffer too small");
    for (int i = 0; i < P.nprimes; ++i) out[i] = P.q[i];
  });
}

int ppst_context_scales(const ppst_context* ctx, double* out, size_t cap) {
  return guard([&] {
    NEED(ctx);
    NEED(out);
    const Params& P = ctx->cx->P();
    if (cap < (size_t)P.L + 1) PPST_THROW(ST_EINVAL, "buffer too small");
    for (int i = 0; i <= P.L; ++i) out[i] = P.scale[i];
  });
}

int ppst_context_dg_table(const ppst_context* ctx, uint64_t* out, size_t cap) {
  return guard([&] {
    NEED(ctx);
    NEED(out);
    if (cap < (size_t)kDgMax) PPST_THROW(ST_EINVAL, "buffer too small");
    for (int i = 0; i < kDgMax; ++i) out[i] = ctx->cx->sh->dg_thr[i];
  });
}

int ppst_context_stream(const ppst_context* ctx, void** stream) {
  return guard([&] {
    NEED(ctx);
    NEED(stream);
    *stream = (void*)ctx->cx->stream;
  });
}

// ------------------------------------------------------------------ keys
int ppst_keygen(ppst_context* ctx, uint64_t seed, ppst_secret_key** sk, ppst_public_key** pk) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(sk);
    NEED(pk);
    auto s = keygen_secret(*ctx->cx, seed);
    auto p = keygen_public(*ctx->cx, *s, seed);
    *sk = new ppst_secret_key{std::move(s)};
    *pk = new ppst_public_key{std::move(p)};
  });
}

int ppst_secret_key_destroy(ppst_secret_key* sk) {
  return guard([&] {
    if (!sk) return;
    HIP_CHECK(hipDeviceSynchronize());
    delete sk;
  });
}

int ppst_public_key_destroy(ppst_public_key* pk) {
  return guard([&] {
    if (!pk) return;
    HIP_CHECK(hipDeviceSynchronize());
    delete pk;
  });
}

int ppst_evk_create(ppst_context* ctx, ppst_eval_keys** out) {
  return guard([&] {
    NEED(ctx);
    NEED(out);
    *out = new ppst_eval_keys{};
  });
}

int ppst_evk_destroy(ppst_eval_keys* evk) {
  return guard([&] {
    if (!evk) return;
    HIP_CHECK(hipDeviceSynchronize());
    delete evk;
  });
}

int ppst_evk_add_relin(ppst_context* ctx, const ppst_secret_key* sk, uint64_t seed,
                       ppst_eval_keys* evk) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(sk);
    NEED(evk);
    evk->e.relin = keygen_relin(*ctx->cx, *sk->k, seed);
  });
}

int ppst_evk_add_galois(ppst_context* ctx, const ppst_secret_key* sk, const int32_t* steps,
                        size_t n, uint64_t seed, ppst_eval_keys* evk) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(sk);
    NEED(evk);
    if (n) NEED(steps);
    const Params& P = ctx->cx->P();
    for (size_t i = 0; i < n; ++i) {
      u64 g = galois_elt(P, steps[i]);
      if (g == 1 || evk->e.galois.count(g)) continue;
      evk->e.galois[g] = keygen_galois(*ctx->cx, *sk->k, seed, g);
    }
  });
}

int ppst_evk_add_rotsum(ppst_context* ctx, const ppst_secret_key* sk, uint64_t seed,
                        ppst_eval_keys* evk) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(sk);
    NEED(evk);
    const Params& P = ctx->cx->P();
    for (const auto& st : rotsum_plan(P))
      for (int k = 1; k < st.second; ++k) {
        u64 g = galois_elt(P, k * st.first);
        if (!evk->e.galois.count(g)) evk->e.galois[g] = keygen_galois(*ctx->cx, *sk->k, seed, g);
      }
  });
}

int ppst_evk_export(ppst_context* ctx, const ppst_eval_keys* evk, uint64_t galois, uint64_t* host,
                    size_t cap_words) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(evk);
    const Params& P = ctx->cx->P();
    const KsKey* k = nullptr;
    if (galois == 0) {
      if (!evk->e.relin) PPST_THROW(ST_ENOKEY, "no relinearisation key");
      k = evk->e.relin.get();
    } else {
      auto it = evk->e.galois.find(galois);
      if (it == evk->e.galois.end()) PPST_THROW(ST_ENOKEY, "no such Galois key");
      k = it->second.get();
    }
    copy_out(*ctx->cx, k->k.p, (size_t)P.dnum * 2 * P.nprimes * P.N, host, cap_words);
  });
}

int ppst_evk_import(ppst_context* ctx, ppst_eval_keys* evk, uint64_t galois, const uint64_t* host,
                    size_t words) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(evk);
    NEED(host);
    Context& cx = *ctx->cx;
    const Params& P = cx.P();
    const size_t np = (size_t)P.nprimes, N = (size_t)P.N, want = (size_t)P.dnum * 2 * np * N;
    if (words != want)
      PPST_THROW(ST_EINVAL, "a key switching key has " + std::to_string(want) + " words");
    if (galois != 0 && (galois >= 2 * N || !(galois & 1) || galois == 1))
      PPST_THROW(ST_EINVAL, "not a rotation's Galois element (odd, 1 < g < 2N)");
    for (size_t r = 0; r < (size_t)P.dnum * 2; ++r)
      for (size_t t = 0; t < np; ++t) {
        const uint64_t* row = host + (r * np + t) * N;
        for (size_t k = 0; k < N; ++k)
          if (row[k] >= P.q[t]) PPST_THROW(ST_EINVAL, "residue not reduced modulo its prime");
      }
    auto key = std::make_shared<KsKey>();
    key->k = Buf(cx.sh->const_pool, want * 8);
    HIP_CHECK(hipMemcpyAsync(key->k.p, host, want * 8, hipMemcpyHostToDevice, cx.stream));
    HIP_CHECK(hipStreamSynchronize(cx.stream));
    if (galois == 0) evk->e.relin = key;
    else evk->e.galois[galois] = key;
  });
}

int ppst_pk_import(ppst_context* ctx, const uint64_t* host, size_t words, ppst_public_key** out) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(host);
    NEED(out);
    Context& cx = *ctx->cx;
    const Params& P = cx.P();
    const size_t N = (size_t)P.N, nl = (size_t)P.L + 1, want = 2 * nl * N;
    if (words != want) PPST_THROW(ST_EINVAL, "a public key has " + std::to_string(want) + " words");
    for (size_t r = 0; r < 2 * nl; ++r)
      for (size_t k = 0; k < N; ++k)
        if (host[r * N + k] >= P.q[r % nl]) PPST_THROW(ST_EINVAL, "residue not reduced modulo its prime");
    auto pk = std::make_unique<PublicKey>();
    pk->pk = Buf(cx.sh->const_pool, want * 8);
    HIP_CHECK(hipMemcpyAsync(pk->pk.p, host, want * 8, hipMemcpyHostToDevice, cx.stream));
    HIP_CHECK(hipStreamSynchronize(cx.stream));
    *out = new ppst_public_key{std::move(pk)};
  });
}

int ppst_pk_export(ppst_context* ctx, const ppst_public_key* pk, uint64_t* host, size_t cap_words) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(pk);
    const Params& P = ctx->cx->P();
    copy_out(*ctx->cx, pk->k->pk.p, 2 * (size_t)(P.L + 1) * P.N, host, cap_words);
  });
}

int ppst_sk_export(ppst_context* ctx, const ppst_secret_key* sk, uint64_t* host, size_t cap_words) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(sk);
    const Params& P = ctx->cx->P();
    copy_out(*ctx->cx, sk->k->s_ntt.p, (size_t)P.nprimes * P.N, host, cap_words);
  });
}

// ------------------------------------------------------------ plaintexts
int ppst_encode(ppst_context* ctx, const double* values, size_t n, int32_t level,
                ppst_plaintext** out) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(out);
    if (n) NEED(values);
    *out = new ppst_plaintext{encode(*ctx->cx, values, n, level)};
  });
}

int ppst_plaintext_from_coeffs(ppst_context* ctx, const int64_t* coeffs, int32_t level,
                               double scale, ppst_plaintext** out) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(coeffs);
    NEED(out);
    *out = new ppst_plaintext{plaintext_from_coeffs(*ctx->cx, coeffs, level, scale)};
  });
}

int ppst_plaintext_coeffs(const ppst_plaintext* pt, int64_t* out, size_t cap) {
  return guard([&] {
    NEED(pt);
    NEED(out);
    if (pt->p->coeffs.empty()) PPST_THROW(ST_EINVAL, "plaintext has no integer coefficients");
    if (cap < pt->p->coeffs.size()) PPST_THROW(ST_EINVAL, "buffer too small");
    std::memcpy(out, pt->p->coeffs.data(), pt->p->coeffs.size() * 8);
  });
}

int ppst_plaintext_export(ppst_context* ctx, const ppst_plaintext* pt, uint64_t* host,
                          size_t cap_words) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(pt);
    copy_out(*ctx->cx, pt->p->buf.p, (size_t)(pt->p->level + 1) * ctx->cx->P().N, host, cap_words);
  });
}

int ppst_plaintext_import(ppst_context* ctx, const uint64_t* host, int32_t level, double scale,
                          ppst_plaintext** out) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(host);
    NEED(out);
    Context& cx = *ctx->cx;
    const Params& P = cx.P();
    if (level < 0 || level > P.L) PPST_THROW(ST_ELEVEL, "level out of range");
    if (!(scale > 0.0)) PPST_THROW(ST_EINVAL, "a plaintext needs a positive scale");
    const size_t N = (size_t)P.N, words = (size_t)(level + 1) * N;
    for (int i = 0; i <= level; ++i)
      for (size_t k = 0; k < N; ++k)
        if (host[(size_t)i * N + k] >= P.q[i]) PPST_THROW(ST_EINVAL, "residue not reduced modulo its prime");
    auto pt = std::make_shared<Plaintext>();
    pt->level = level;
    pt->scale = scale;
    pt->buf = Buf(cx.pool, words * 8);
    HIP_CHECK(hipMemcpyAsync(pt->buf.p, host, words * 8, hipMemcpyHostToDevice, cx.stream));
    HIP_CHECK(hipStreamSynchronize(cx.stream));
    *out = new ppst_plaintext{pt};
  });
}

int ppst_decode(ppst_context* ctx, const ppst_plaintext* pt, double* out, size_t n) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(pt);
    if (n) NEED(out);
    decode(*ctx->cx, *pt->p, out, n);
  });
}

int ppst_plaintext_destroy(ppst_plaintext* pt) {
  return guard([&] { delete pt; });
}

// ----------------------------------------------------------- ciphertexts
int ppst_encrypt(ppst_context* ctx, const ppst_public_key* pk, const ppst_plaintext* pt,
                 uint64_t seed, ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(pk);
    NEED(pt);
    NEED(out);
    *out = wrap(encrypt_pk(*ctx->cx, *pk->k, *pt->p, seed));
  });
}

int ppst_encrypt_sk(ppst_context* ctx, const ppst_secret_key* sk, const ppst_plaintext* pt,
                    uint64_t seed, ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(sk);
    NEED(pt);
    NEED(out);
    *out = wrap(encrypt_sk(*ctx->cx, *sk->k, *pt->p, seed));
  });
}

int ppst_decrypt(ppst_context* ctx, const ppst_secret_key* sk, const ppst_ciphertext* ct,
                 ppst_plaintext** out) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(sk);
    NEED(ct);
    NEED(out);
    *out = new ppst_plaintext{decrypt(*ctx->cx, *sk->k, *ct->c)};
  });
}

int ppst_ciphertext_destroy(ppst_ciphertext* ct) {
  return guard([&] { delete ct; });
}

int ppst_ct_info(const ppst_ciphertext* ct, int32_t* level, double* scale, int32_t* npoly) {
  return guard([&] {
    NEED(ct);
    if (level) *level = ct->c->level;
    if (scale) *scale = ct->c->scale;
    if (npoly) *npoly = ct->c->npoly;
  });
}

int ppst_ct_export(ppst_context* ctx, const ppst_ciphertext* ct, uint64_t* host, size_t cap_words) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(ct);
    const Ciphertext& c = *ct->c;
    copy_out(*ctx->cx, c.buf.p, (size_t)c.npoly * (c.level + 1) * c.N, host, cap_words);
  });
}

int ppst_ct_import(ppst_context* ctx, const uint64_t* host, int32_t level, double scale,
                   int32_t npoly, ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(host);
    NEED(out);
    const Params& P = ctx->cx->P();
    if (level < 0 || level > P.L) PPST_THROW(ST_ELEVEL, "level out of range");
    if (npoly != 2 && npoly != 3) PPST_THROW(ST_EINVAL, "npoly must be 2 or 3");
    const size_t words = (size_t)npoly * (level + 1) * P.N;
    for (int c = 0; c < npoly; ++c)
      for (int i = 0; i <= level; ++i)
        for (int k = 0; k < P.N; k += 4099)
          if (host[((size_t)c * (level + 1) + i) * P.N + k] >= P.q[i])
            PPST_THROW(ST_EINVAL, "residue not reduced modulo its prime");
    auto ct = new_ct(*ctx->cx, level, scale, npoly);
    HIP_CHECK(hipMemcpyAsync(ct->buf.p, host, words * 8, hipMemcpyHostToDevice, ctx->cx->stream));
    HIP_CHECK(hipStreamSynchronize(ctx->cx->stream));
    *out = wrap(ct);
  });
}

int ppst_ct_device_ptr(const ppst_ciphertext* ct, uint64_t** out) {
  return guard([&] {
    NEED(ct);
    NEED(out);
    *out = ct->c->buf.p;
  });
}

// ------------------------------------------------------------ evaluator
#define UNARY_OP(name, expr)                                                       \
  int name {                                                                       \
    return guard([&] {                                                             \
      NEED(ctx);                                                                   \
      NEED(a);                                                                     \
      NEED(out);                                                                   \
      *out = wrap(expr);                                                           \
    });                                                                            \
  }

int ppst_add(ppst_context* ctx, const ppst_ciphertext* a, const ppst_ciphertext* b,
             ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(a); NEED(b); NEED(out);
    *out = wrap(add(*ctx->cx, *a->c, *b->c));
  });
}
int ppst_sub(ppst_context* ctx, const ppst_ciphertext* a, const ppst_ciphertext* b,
             ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(a); NEED(b); NEED(out);
    *out = wrap(sub(*ctx->cx, *a->c, *b->c));
  });
}
UNARY_OP(ppst_add_const(ppst_context* ctx, const ppst_ciphertext* a, double c, ppst_ciphertext** out),
         add_const(*ctx->cx, *a->c, c))
UNARY_OP(ppst_mul_const(ppst_context* ctx, const ppst_ciphertext* a, double c, ppst_ciphertext** out),
         mul_const(*ctx->cx, *a->c, c))
UNARY_OP(ppst_mul_int(ppst_context* ctx, const ppst_ciphertext* a, int64_t k, ppst_ciphertext** out),
         mul_int(*ctx->cx, *a->c, k))
UNARY_OP(ppst_rescale(ppst_context* ctx, const ppst_ciphertext* a, ppst_ciphertext** out),
         rescale(*ctx->cx, *a->c))
UNARY_OP(ppst_level_align(ppst_context* ctx, const ppst_ciphertext* a, int32_t level,
                          ppst_ciphertext** out),
         level_align(*ctx->cx, *a->c, level))

int ppst_lincomb(ppst_context* ctx, const ppst_ciphertext* const* cts, const double* cs, size_t n,
                 int32_t level, ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(cts); NEED(cs); NEED(out);
    std::vector<const Ciphertext*> v;
    for (size_t i = 0; i < n; ++i) {
      NEED(cts[i]);
      v.push_back(cts[i]->c.get());
    }
    *out = wrap(lincomb(*ctx->cx, v, std::vector<double>(cs, cs + n), level));
  });
}
int ppst_mul_plain(ppst_context* ctx, const ppst_ciphertext* a, const ppst_plaintext* pt,
                   ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(a); NEED(pt); NEED(out);
    *out = wrap(mul_plain(*ctx->cx, *a->c, *pt->p));
  });
}
int ppst_mul(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* a,
             const ppst_ciphertext* b, ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(a); NEED(b); NEED(out);
    *out = wrap(mul(*ctx->cx, evk->e, *a->c, *b->c));
  });
}
int ppst_tensor(ppst_context* ctx, const ppst_ciphertext* a, const ppst_ciphertext* b,
                ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(a); NEED(b); NEED(out);
    *out = wrap(tensor(*ctx->cx, *a->c, *b->c));
  });
}
int ppst_relin(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* d,
               ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(d); NEED(out);
    *out = wrap(relin(*ctx->cx, evk->e, *d->c));
  });
}
int ppst_rotate(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* a, int32_t r,
                ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(a); NEED(out);
    *out = wrap(rotate(*ctx->cx, evk->e, *a->c, r));
  });
}
int ppst_rotate_hoisted(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* a,
                        const int32_t* rs, size_t n, ppst_ciphertext** outs) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(a); NEED(outs);
    if (n) NEED(rs);
    std::vector<long> r(rs, rs + n);
    auto v = rotate_hoisted(*ctx->cx, evk->e, *a->c, r);
    for (size_t i = 0; i < n; ++i) outs[i] = wrap(v[i]);
  });
}
int ppst_rotate_hoisted_batch(ppst_context* ctx, const ppst_eval_keys* evk,
                              const ppst_ciphertext* const* cts, size_t n, const int32_t* rs,
                              size_t m, ppst_ciphertext** outs) {
  return guard([&] {
    NEED(ctx); NEED(evk);
    if (n) NEED(cts);
    if (m) NEED(rs);
    if (n && m) NEED(outs);
    std::vector<const Ciphertext*> v;
    for (size_t i = 0; i < n; ++i) {
      NEED(cts[i]);
      v.push_back(cts[i]->c.get());
    }
    std::vector<long> r(rs, rs + m);
    auto o = rotate_hoisted_batch(*ctx->cx, evk->e, v, r);
    for (size_t i = 0; i < o.size(); ++i) outs[i] = wrap(o[i]);
  });
}
int ppst_rotate_batch(ppst_context* ctx, const ppst_eval_keys* evk,
                      const ppst_ciphertext* const* cts, size_t n, int32_t r,
                      ppst_ciphertext** outs) {
  return guard([&] {
    NEED(ctx); NEED(evk);
    if (n) {
      NEED(cts);
      NEED(outs);
    }
    std::vector<const Ciphertext*> v;
    for (size_t i = 0; i < n; ++i) {
      NEED(cts[i]);
      v.push_back(cts[i]->c.get());
    }
    auto o = rotate_batch(*ctx->cx, evk->e, v, r);
    for (size_t i = 0; i < o.size(); ++i) outs[i] = wrap(o[i]);
  });
}
int ppst_rotsum(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* a,
                ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(a); NEED(out);
    *out = wrap(rotsum(*ctx->cx, evk->e, *a->c));
  });
}
int ppst_rotsum_serial(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* a,
                       ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(a); NEED(out);
    *out = wrap(rotsum_serial(*ctx->cx, evk->e, *a->c));
  });
}
int ppst_rotsum_batch(ppst_context* ctx, const ppst_eval_keys* evk,
                      const ppst_ciphertext* const* cts, size_t n, ppst_ciphertext** outs) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(cts); NEED(outs);
    std::vector<CtPtr> v;
    for (size_t i = 0; i < n; ++i) {
      NEED(cts[i]);
      v.push_back(cts[i]->c);
    }
    auto r = rotsum_batch(*ctx->cx, evk->e, v);
    for (size_t i = 0; i < n; ++i) outs[i] = wrap(r[i]);
  });
}
int ppst_mul_const_batch(ppst_context* ctx, const ppst_ciphertext* const* cts, size_t n, double c,
                         ppst_ciphertext** outs) {
  return guard([&] {
    NEED(ctx); NEED(cts); NEED(outs);
    std::vector<const Ciphertext*> v;
    for (size_t i = 0; i < n; ++i) {
      NEED(cts[i]);
      v.push_back(cts[i]->c.get());
    }
    auto r = mul_const_n(*ctx->cx, v, c);
    for (size_t i = 0; i < n; ++i) outs[i] = wrap(r[i]);
  });
}

int ppst_mul_batch(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* const* a,
                   const ppst_ciphertext* const* b, size_t n, ppst_ciphertext** outs) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(a); NEED(b); NEED(outs);
    std::vector<const Ciphertext*> va, vb;
    for (size_t i = 0; i < n; ++i) {
      NEED(a[i]);
      NEED(b[i]);
      va.push_back(a[i]->c.get());
      vb.push_back(b[i]->c.get());
    }
    auto v = mul_batch(*ctx->cx, evk->e, va, vb);
    for (size_t i = 0; i < n; ++i) outs[i] = wrap(v[i]);
  });
}

// ----------------------------------------------------------- statistics
// ---------------------------------------------------------------- graphs
int ppst_graph_begin(ppst_context* ctx) {
  return guard([&] {
    NEED(ctx);
    graph_begin(*ctx->cx);
  });
}
int ppst_graph_end(ppst_context* ctx, ppst_graph** out) {
  return guard([&] {
    NEED(ctx); NEED(out);
    *out = new ppst_graph{graph_end(*ctx->cx)};
  });
}
int ppst_graph_launch(ppst_graph* g) {
  return guard([&] {
    NEED(g);
    graph_launch(*g->g);
  });
}
int ppst_graph_destroy(ppst_graph* g) {
  return guard([&] { delete g; });
}

int ppst_invsqrt_cfg_default(ppst_invsqrt_cfg* out) {
  return guard([&] {
    NEED(out);
    out->a = 1e-3;
    out->b = 1.0;
    out->degree = 7;
    out->iters = 3;
    out->sign_k = 2;
    out->coeffs = nullptr;
    out->boot = nullptr;
  });
}

int ppst_stat_mean(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* const* col,
                   size_t nct, size_t nrows, double B, ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(out);
    NOT_RECORDING(ctx);
    *out = wrap(stat_mean(*ctx->cx, evk->e, column(col, nct), nrows, B));
  });
}
int ppst_stat_variance(ppst_context* ctx, const ppst_eval_keys* evk,
                       const ppst_ciphertext* const* col, size_t nct, size_t nrows, double B,
                       ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(out);
    NOT_RECORDING(ctx);
    *out = wrap(stat_variance(*ctx->cx, evk->e, column(col, nct), nrows, B));
  });
}
int ppst_stat_invsqrt(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* const* x,
                      size_t nct, double B, const ppst_invsqrt_cfg* cfg, ppst_ciphertext** outs) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(outs);
    NOT_RECORDING(ctx);
    auto v = stat_invsqrt(*ctx->cx, evk->e, column(x, nct), B, cfg_from(cfg));
    for (size_t i = 0; i < v.size(); ++i) outs[i] = wrap(v[i]);
  });
}
int ppst_stat_zscore(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* const* col,
                     size_t nct, size_t nrows, double B, const ppst_invsqrt_cfg* cfg,
                     ppst_ciphertext** outs) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(outs);
    NOT_RECORDING(ctx);
    auto v = stat_zscore(*ctx->cx, evk->e, column(col, nct), nrows, B, cfg_from(cfg));
    for (size_t i = 0; i < v.size(); ++i) outs[i] = wrap(v[i]);
  });
}
int ppst_stat_kurtosis(ppst_context* ctx, const ppst_eval_keys* evk,
                       const ppst_ciphertext* const* col, size_t nct, size_t nrows, double B,
                       const ppst_invsqrt_cfg* cfg, int32_t excess, ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(out);
    NOT_RECORDING(ctx);
    *out = wrap(stat_kurtosis(*ctx->cx, evk->e, column(col, nct), nrows, B, cfg_from(cfg),
                              excess != 0));
  });
}
int ppst_stat_skewness(ppst_context* ctx, const ppst_eval_keys* evk,
                       const ppst_ciphertext* const* col, size_t nct, size_t nrows, double B,
                       const ppst_invsqrt_cfg* cfg, ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(out);
    NOT_RECORDING(ctx);
    *out = wrap(stat_skewness(*ctx->cx, evk->e, column(col, nct), nrows, B, cfg_from(cfg)));
  });
}
int ppst_stat_cv(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* const* col,
                 size_t nct, size_t nrows, double B_mean, double B_var, const ppst_invsqrt_cfg* cfg,
                 ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(out);
    NOT_RECORDING(ctx);
    int k = cfg ? cfg->sign_k : 2;
    *out = wrap(stat_cv(*ctx->cx, evk->e, column(col, nct), nrows, B_mean, B_var, cfg_from(cfg), k));
  });
}
int ppst_stat_pearson(ppst_context* ctx, const ppst_eval_keys* evk,
                      const ppst_ciphertext* const* colx, const ppst_ciphertext* const* coly,
                      size_t nct, size_t nrows, double Bx, double By, const ppst_invsqrt_cfg* cfg,
                      ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(out);
    NOT_RECORDING(ctx);
    *out = wrap(stat_pearson(*ctx->cx, evk->e, column(colx, nct), column(coly, nct), nrows, Bx, By,
                             cfg_from(cfg)));
  });
}

// ----------------------------------------------------------- raw kernels
int ppst_ntt_forward(ppst_context* ctx, uint64_t* dev, int32_t nlimbs, int32_t first_prime) {
  return guard([&] {
    NEED(ctx);
    NEED(dev);
    ntt_raw(*ctx->cx, dev, nlimbs, first_prime, false);
  });
}
int ppst_ntt_inverse(ppst_context* ctx, uint64_t* dev, int32_t nlimbs, int32_t first_prime) {
  return guard([&] {
    NEED(ctx);
    NEED(dev);
    ntt_raw(*ctx->cx, dev, nlimbs, first_prime, true);
  });
}

int ppst_ntt_autotune(ppst_context* ctx) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    HIP_CHECK(hipStreamSynchronize(ctx->cx->stream));
    autotune_ntt(*ctx->cx->sh);
  });
}
int ppst_ntt_load_plan(ppst_context* ctx, const char* plan) {
  return guard([&] {
    NEED(ctx); NEED(plan);
    ntt_load_plan(*ctx->cx->sh, plan);
  });
}
int ppst_ntt_set_plan(ppst_context* ctx, int32_t col, int32_t row) {
  return guard([&] {
    NEED(ctx);
    HIP_CHECK(hipStreamSynchronize(ctx->cx->stream));
    ntt_set_plan(*ctx->cx->sh, ctx->cx->P().logN == 16 ? col : 0, row);
  });
}
int ppst_ntt_plan(const ppst_context* ctx, char* buf, size_t cap) {
  return guard([&] {
    NEED(ctx);
    NEED(buf);
    std::string s = ntt_plan_string(*ctx->cx->sh);
    if (cap < s.size() + 1) PPST_THROW(ST_EINVAL, "buffer too small");
    std::memcpy(buf, s.c_str(), s.size() + 1);
  });
}

// -------------------------------------------------------------- serving
int ppst_server_create(ppst_context* ctx, const ppst_eval_keys* evk, size_t hbm_budget,
                       int32_t slots, uint32_t flags, ppst_server** out) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(out);
    NOT_RECORDING(ctx);
    if (flags & ~(uint32_t)PPST_SERVER_NO_MERGE) PPST_THROW(ST_EINVAL, "unknown server flags");
    auto keys = std::make_shared<const EvalKeys>(evk->e);
    *out = new ppst_server{std::make_unique<Server>(*ctx->cx, keys, hbm_budget, slots,
                                                    !(flags & PPST_SERVER_NO_MERGE))};
  });
}
int ppst_server_info(ppst_server* srv, uint64_t* budget, uint64_t* merged_launches,
                     uint64_t* merged_lanes, uint64_t* multi_query_launches) {
  return guard([&] {
    NEED(srv);
    u64 l = 0, n = 0, m = 0;
    srv->s->merge_counters(&l, &n, &m);
    if (budget) *budget = srv->s->budget();
    if (merged_launches) *merged_launches = l;
    if (merged_lanes) *merged_lanes = n;
    if (multi_query_launches) *multi_query_launches = m;
  });
}
int ppst_server_register_column(ppst_server* srv, const ppst_ciphertext* const* cts, size_t nct,
                                size_t nrows, uint64_t* col_id) {
  return guard([&] {
    NEED(srv); NEED(cts); NEED(col_id);
    std::vector<const Ciphertext*> v;
    for (size_t i = 0; i < nct; ++i) {
      NEED(cts[i]);
      v.push_back(cts[i]->c.get());
    }
    *col_id = srv->s->register_column(v, nrows);
  });
}
int ppst_server_submit(ppst_server* srv, const ppst_query* q, uint64_t* ticket) {
  return guard([&] {
    NEED(srv); NEED(q); NEED(ticket);
    // admission estimates cover the statistics' own working sets only
    if (q->cfg.boot) PPST_THROW(ST_EINVAL, "served queries run without bootstrapping");
    Query Q;
    Q.kind = q->kind;
    Q.col_x = q->col_x;
    Q.col_y = q->col_y;
    Q.B = q->B;
    Q.B2 = q->B2;
    Q.cfg = cfg_from(&q->cfg);
    Q.sign_k = q->cfg.sign_k;
    *ticket = srv->s->submit(Q);
  });
}
int ppst_server_poll(ppst_server* srv, uint64_t ticket, int32_t* done) {
  return guard([&] {
    NEED(srv);
    NEED(done);
    *done = srv->s->poll(ticket) ? 1 : 0;
  });
}
namespace {
void copy_stats(const QueryState& st, ppst_query_stats* stats) {
  if (!stats) return;
  stats->t_submit = st.t_submit;
  stats->t_admit = st.t_admit;
  stats->t_done = st.t_done;
  stats->bytes_reserved = st.bytes;
  stats->bytes_peak = st.peak;
}
}  // namespace

int ppst_server_wait(ppst_server* srv, uint64_t ticket, ppst_ciphertext** out,
                     ppst_query_stats* stats) {
  int status = PPST_OK;
  int rc = guard([&] {
    NEED(srv);
    std::vector<CtPtr> res;
    QueryState st;
    status = srv->s->wait(ticket, &res, &st);
    copy_stats(st, stats);
    if (status != ST_OK) last_error() = st.error;
    if (out) *out = (status == ST_OK && !res.empty()) ? wrap(res[0]) : nullptr;
  });
  return rc != PPST_OK ? rc : status;
}
int ppst_server_output_count(ppst_server* srv, uint64_t ticket, size_t* n) {
  return guard([&] {
    NEED(srv); NEED(n);
    *n = srv->s->output_count(ticket);
  });
}
int ppst_server_wait_all(ppst_server* srv, uint64_t ticket, ppst_ciphertext** outs, size_t cap,
                         size_t* n_out, ppst_query_stats* stats) {
  int status = PPST_OK;
  int rc = guard([&] {
    NEED(srv); NEED(outs); NEED(n_out);
    const size_t need = srv->s->output_count(ticket);
    if (cap < need)
      PPST_THROW(ST_EINVAL, "output array holds " + std::to_string(cap) + " handles, the query has " +
                              std::to_string(need));
    std::vector<CtPtr> res;
    QueryState st;
    status = srv->s->wait(ticket, &res, &st);
    copy_stats(st, stats);
    *n_out = 0;
    if (status != ST_OK) {
      last_error() = st.error;
      return;
    }
    for (size_t i = 0; i < res.size(); ++i) outs[i] = wrap(res[i]);
    *n_out = res.size();
  });
  return rc != PPST_OK ? rc : status;
}
int ppst_server_destroy(ppst_server* srv) {
  return guard([&] { delete srv; });
}

}  // extern "C"
