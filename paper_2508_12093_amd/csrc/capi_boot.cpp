// capi_boot.cpp -- the extern "C" bootstrapping calls of include/ppstat.h.
#include "boot.h"
#include "capi.h"

using namespace ppst;

ppst_boot::~ppst_boot() = default;

namespace {

const BootGroup& pick_group(const BootPlan& plan, int32_t transform, int32_t group) {
  if (transform != 0 && transform != 1) PPST_THROW(ST_EINVAL, "transform must be 0 or 1");
  const auto& v = transform == 0 ? plan.cts : plan.stc;
  if (group < 0 || group >= (int32_t)v.size()) PPST_THROW(ST_EINVAL, "no such group");
  return v[group];
}

const Bootstrapper& boot_of(const ppst_boot* bt) {
  NEED(bt);
  NEED(bt->b);
  return *bt->b;
}

}  // namespace

int ppst_boot_create(ppst_context* ctx, const double* coeffs, size_t ncoeffs, ppst_boot** out) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(out);
    std::vector<double> c;
    if (coeffs) c.assign(coeffs, coeffs + ncoeffs);
    else if (ncoeffs) PPST_THROW(ST_EINVAL, "coefficient count without coefficients");
    auto b = boot_create(*ctx->cx, c);
    HIP_CHECK(hipStreamSynchronize(ctx->cx->stream));
    *out = new ppst_boot{std::move(b)};
  });
}

int ppst_boot_destroy(ppst_boot* bt) {
  return guard([&] { delete bt; });
}

int ppst_boot_count(const ppst_boot* bt, uint64_t* n) {
  return guard([&] {
    NEED(n);
    *n = boot_of(bt).runs.load(std::memory_order_relaxed);
  });
}

int ppst_evk_add_boot(ppst_context* ctx, const ppst_secret_key* sk, uint64_t seed,
                      ppst_eval_keys* evk) {
  return guard([&] {
    NEED(ctx);
    NOT_RECORDING(ctx);
    NEED(sk);
    NEED(evk);
    const Params& P = ctx->cx->P();
    std::vector<u64> gs;
    for (long r : boot_rotations(P)) gs.push_back(galois_elt(P, r));
    gs.push_back(2 * (u64)P.N - 1);
    for (u64 g : gs)
      if (!evk->e.galois.count(g)) evk->e.galois[g] = keygen_galois(*ctx->cx, *sk->k, seed, g);
  });
}

int ppst_boot_rotations(const ppst_params* params, int32_t* out, size_t cap, size_t* n) {
  return guard([&] {
    NEED(params);
    NEED(n);
    const Params P = make_params(spec_from(*params));
    const std::vector<long> r = boot_rotations(P);
    *n = r.size();
    if (out == nullptr && cap == 0) return;
    NEED(out);
    if (cap < r.size()) PPST_THROW(ST_EINVAL, "buffer too small");
    for (size_t i = 0; i < r.size(); ++i) out[i] = (int32_t)r[i];
  });
}

int ppst_boot_group_info(const ppst_params* params, int32_t transform, int32_t group, int32_t* desc) {
  return guard([&] {
    NEED(params);
    NEED(desc);
    const Params P = make_params(spec_from(*params));
    const BootPlan plan = boot_plan(P);
    const BootGroup& g = pick_group(plan, transform, group);
    const int32_t v[9] = {g.inverse, g.lo, g.hi, g.level, g.ckind, g.u, g.m0, g.b, g.G};
    std::copy(v, v + 9, desc);
  });
}

int ppst_boot_group_coeffs(const ppst_params* params, int32_t transform, int32_t group,
                           int64_t* out, uint8_t* used, size_t cap_cells) {
  return guard([&] {
    NEED(params);
    NEED(out);
    NEED(used);
    const Params P = make_params(spec_from(*params));
    const BootPlan plan = boot_plan(P);
    const BootGroup& g = pick_group(plan, transform, group);
    if (cap_cells < (size_t)g.G * g.b) PPST_THROW(ST_EINVAL, "buffer too small");
    std::fill(out, out + (size_t)g.G * g.b * P.N, 0);
    const int threads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    try {
      boot_group_coeffs(P.logN, g, boot_factor(P, plan, g), out, used, threads);
    } catch (const std::runtime_error& e) {
      PPST_THROW(ST_EINVAL, e.what());
    }
  });
}

int ppst_evalmod_coeffs(int32_t K, int32_t r, int32_t degree, double* out, size_t cap) {
  return guard([&] {
    NEED(out);
    const std::vector<double> c = evalmod_coeffs(K, r, degree);
    if (cap < c.size()) PPST_THROW(ST_EINVAL, "buffer too small");
    std::copy(c.begin(), c.end(), out);
  });
}

int ppst_bootstrap(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_boot* bt,
                   const ppst_ciphertext* a, ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(a); NEED(out);
    *out = wrap(bootstrap(*ctx->cx, evk->e, boot_of(bt), *a->c));
  });
}

int ppst_mod_raise(ppst_context* ctx, const ppst_ciphertext* a, ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(a); NEED(out);
    *out = wrap(mod_raise(*ctx->cx, *a->c));
  });
}

int ppst_apply_galois(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_ciphertext* a,
                      uint64_t g, ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(a); NEED(out);
    *out = wrap(apply_galois(*ctx->cx, evk->e, *a->c, g));
  });
}

int ppst_mul_monomial(ppst_context* ctx, const ppst_ciphertext* a, int32_t k, int32_t sign,
                      ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(a); NEED(out);
    *out = wrap(mul_monomial(*ctx->cx, *a->c, k, sign));
  });
}

int ppst_boot_coeff_to_slot(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_boot* bt,
                            const ppst_ciphertext* a, ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(a); NEED(out);
    *out = wrap(coeff_to_slot(*ctx->cx, evk->e, boot_of(bt), *a->c));
  });
}

int ppst_boot_split(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_boot* bt,
                    const ppst_ciphertext* w, ppst_ciphertext** re, ppst_ciphertext** im) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(w); NEED(re); NEED(im);
    auto r = boot_split(*ctx->cx, evk->e, boot_of(bt), *w->c);
    *re = wrap(r.first);
    *im = wrap(r.second);
  });
}

int ppst_boot_eval_mod(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_boot* bt,
                       const ppst_ciphertext* const* lanes, size_t n, ppst_ciphertext** outs) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(lanes); NEED(outs);
    if (n == 0) PPST_THROW(ST_EINVAL, "no lanes");
    std::vector<CtPtr> v;
    for (size_t i = 0; i < n; ++i) {
      NEED(lanes[i]);
      if (lanes[i]->c->level != lanes[0]->c->level) PPST_THROW(ST_ESCALE, "lanes at different levels");
      v.push_back(lanes[i]->c);
    }
    auto y = eval_mod(*ctx->cx, evk->e, boot_of(bt), v);
    for (size_t i = 0; i < n; ++i) outs[i] = wrap(y[i]);
  });
}

int ppst_boot_slot_to_coeff(ppst_context* ctx, const ppst_eval_keys* evk, const ppst_boot* bt,
                            const ppst_ciphertext* re, const ppst_ciphertext* im,
                            ppst_ciphertext** out) {
  return guard([&] {
    NEED(ctx); NEED(evk); NEED(re); NEED(im); NEED(out);
    *out = wrap(slot_to_coeff(*ctx->cx, evk->e, boot_of(bt), *re->c, *im->c));
  });
}
