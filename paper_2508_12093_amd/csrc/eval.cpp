// eval.cpp -- context, tables, keys, encryption and the RNS-CKKS operations.
#include "eval.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "kern.h"
#include "tables.h"

namespace ppst {

// =========================================================== memory pool
Pool::~Pool() {
  if (std::getenv("PPST_POOL_LOG"))
    std::fprintf(stderr, "[ppstat] pool: %zu device allocations (%zu slabs), %zu blocks (%zu bytes) cached at exit\n",
                 nalloc_, slabs_.size(), free_.size(), cached_);
  trim();
}

namespace {
// Block sizes come in classes so that cached blocks are reused across
// requests of similar size (ciphertexts of neighbouring levels, batches of
// different lengths) instead of piling up one block per distinct size:
// 4 KiB granules up to 64 KiB, then four classes per power of two
// (2^k, 1.25, 1.5, 1.75 x 2^k), at most 25 % above the request.
size_t size_class(size_t bytes) {
  if (bytes <= ((size_t)1 << 16)) return (bytes + 4095) & ~(size_t)4095;
  const int k = 63 - __builtin_clzll((unsigned long long)bytes);
  const size_t step = ((size_t)1 << k) / 4;
  return (bytes + step - 1) / step * step;
}
}  // namespace

void* Pool::raw_alloc(size_t bytes) {
  void* p = nullptr;
  if (hooks_.alloc) return hooks_.alloc(bytes, (void*)stream_, hooks_.user);
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void Pool::raw_free(void* p, size_t bytes) {
  if (hooks_.free) hooks_.free(p, bytes, (void*)stream_, hooks_.user);
  else (void)hipFree(p);
}

// a device allocation; on failure this pool's cache is released, then the
// other pools' of the same tables, before giving up
void* Pool::alloc_retry(size_t bytes) {
  void* p = raw_alloc(bytes);
  if (p) return p;
  if (capturing_)   // no synchronisation is possible while a recording is open
    PPST_THROW(ST_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  if (std::getenv("PPST_POOL_LOG")) {
    std::lock_guard<std::mutex> g(mu_);
    std::fprintf(stderr, "[ppstat] allocation of %zu bytes failed; freeing %zu cached bytes\n",
                 bytes, cached_);
  }
  trim();
  p = raw_alloc(bytes);
  if (!p && registry_) {
    registry_->trim_others(this);
    p = raw_alloc(bytes);
  }
  if (!p) PPST_THROW(ST_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  return p;
}

void Pool::reset_peak() {
  std::lock_guard<std::mutex> g(mu_);
  peak_ = in_use_;
}

void* Pool::hand_out(void* p, size_t bytes) {
  in_use_ += bytes;
  if (in_use_ > peak_) peak_ = in_use_;
  sizes_[p] = bytes;
  auto s = slab_of_.find(p);
  if (s != slab_of_.end()) ++slabs_[s->second].inuse;
  if (capturing_) {
    captured_.push_back(p);
    pinned_[p] = false;
  }
  return p;
}

void* Pool::get(size_t bytes) {
  if (bytes == 0) bytes = 256;
  bytes = size_class(bytes);
  std::unique_lock<std::mutex> g(mu_);
  auto it = free_.find(bytes);
  if (it != free_.end()) {
    void* p = it->second;
    free_.erase(it);
    cached_ -= bytes;
    return hand_out(p, bytes);
  }
  if (bytes <= kSlabBlockMax) {
    if (cur_ < 0 || slabs_[cur_].offset + bytes > kSlabBytes) {
      g.unlock();
      char* base = (char*)alloc_retry(kSlabBytes);
      g.lock();
      ++nalloc_;
      slabs_.push_back(Slab{base, 0, 0, false});
      cur_ = (int)slabs_.size() - 1;
    }
    Slab& sl = slabs_[cur_];
    void* p = sl.base + sl.offset;
    sl.offset += bytes;
    slab_of_[p] = cur_;
    return hand_out(p, bytes);
  }
  g.unlock();
  void* p = alloc_retry(bytes);
  g.lock();
  ++nalloc_;
  return hand_out(p, bytes);
}

void Pool::put(void* p, size_t) {
  std::lock_guard<std::mutex> g(mu_);
  auto pin = pinned_.find(p);
  if (pin != pinned_.end()) {   // the graph still writes this block
    pin->second = true;
    return;
  }
  auto it = sizes_.find(p);
  size_t sz = it->second;
  sizes_.erase(it);
  in_use_ -= sz;
  cached_ += sz;
  free_.emplace(sz, p);
  auto s = slab_of_.find(p);
  if (s != slab_of_.end()) --slabs_[s->second].inuse;
}

void Pool::begin_capture() {
  std::lock_guard<std::mutex> g(mu_);
  capturing_ = true;
  captured_.clear();
}

std::vector<void*> Pool::end_capture() {
  std::lock_guard<std::mutex> g(mu_);
  capturing_ = false;
  std::vector<void*> v;
  v.swap(captured_);
  return v;
}

void Pool::unpin(const std::vector<void*>& blocks) {
  std::lock_guard<std::mutex> g(mu_);
  for (void* p : blocks) {
    auto pin = pinned_.find(p);
    if (pin == pinned_.end()) continue;
    const bool released = pin->second;
    pinned_.erase(pin);
    if (released) {
      auto it = sizes_.find(p);
      size_t sz = it->second;
      sizes_.erase(it);
      in_use_ -= sz;
      cached_ += sz;
      free_.emplace(sz, p);
      auto s = slab_of_.find(p);
      if (s != slab_of_.end()) --slabs_[s->second].inuse;
    }
  }
}

void PoolRegistry::add(const std::shared_ptr<Pool>& p) {
  std::lock_guard<std::mutex> g(mu_);
  pools_.erase(std::remove_if(pools_.begin(), pools_.end(),
                              [](const std::weak_ptr<Pool>& w) { return w.expired(); }),
               pools_.end());
  pools_.push_back(p);
}

void PoolRegistry::trim_others(const Pool* except) {
  std::lock_guard<std::mutex> g(mu_);
  for (auto& w : pools_)
    if (auto p = w.lock())
      if (p.get() != except) p->trim();
}

// Returns every cached block of its own and every slab none of whose blocks
// is in use; blocks of slabs still in use stay cached.
void Pool::detach() {
  std::lock_guard<std::mutex> g(mu_);
  detached_ = true;
  stream_ = nullptr;
}

void Pool::trim() {
  std::lock_guard<std::mutex> g(mu_);
  if (capturing_) return;   // a recording stream cannot be synchronised
  // cached blocks may still be read by work in flight: on the pool's stream,
  // or, once detached, on whichever stream last used a caller's block
  if (!free_.empty()) {
    if (detached_) (void)hipDeviceSynchronize();
    else (void)hipStreamSynchronize(stream_);
  }
  for (auto it = free_.begin(); it != free_.end();) {
    auto s = slab_of_.find(it->second);
    if (s == slab_of_.end()) {
      raw_free(it->second, it->first);
    } else if (slabs_[s->second].inuse == 0) {
      slab_of_.erase(s);
    } else {
      ++it;
      continue;
    }
    cached_ -= it->first;
    it = free_.erase(it);
  }
  for (size_t i = 0; i < slabs_.size(); ++i) {
    Slab& sl = slabs_[i];
    if (sl.dead || sl.inuse != 0) continue;
    raw_free(sl.base, kSlabBytes);
    sl.dead = true;
    if (cur_ == (int)i) cur_ = -1;
  }
}

namespace {

Buf dev_buf(const std::shared_ptr<Pool>& pool, size_t words) { return Buf(pool, words * 8); }

Buf upload(const std::shared_ptr<Pool>& pool, const std::vector<u64>& v) {
  Buf b = dev_buf(pool, v.size());
  HIP_CHECK(hipMemcpy(b.p, v.data(), v.size() * 8, hipMemcpyHostToDevice));
  return b;
}

// 2^64 mod q: a constant c stored as c 2^64 mod q comes out of Acc30::redc
// as c itself
u64 mont_r(u64 q) { return (u64)(((u128)1 << 64) % q); }

unsigned brv(unsigned x, int bits) {
  unsigned r = 0;
  for (int i = 0; i < bits; ++i) r |= ((x >> i) & 1u) << (bits - 1 - i);
  return r;
}

}  // namespace

// ============================================================== tables
void build_tables(Shared& sh) {
  const Params& P = sh.P;
  const int N = P.N, np = P.nprimes;
  auto& pool = sh.const_pool;
  static_assert(sizeof(Mod) == 4 * sizeof(u64), "Mod layout");
  std::vector<u64> mods(4 * np);
  for (int i = 0; i < np; ++i) {
    const u64 q = P.q[i];
    u128 R = (~(u128)0) / q;
    u64 inv = q;                            // q^-1 mod 2^64 by Newton (q odd)
    for (int k = 0; k < 6; ++k) inv *= 2 - q * inv;
    if (q * inv != 1) PPST_THROW(ST_EINVAL, "Montgomery inverse");
    mods[4 * i] = q;
    mods[4 * i + 1] = (u64)(R >> 64);
    mods[4 * i + 2] = (u64)R;
    mods[4 * i + 3] = 0 - inv;
  }
  sh.tab.mods = upload(pool, mods);

  // Twiddle pairs: (w, floor(w 2^64 / q)) for the 64-bit integer path;
  // (double w, double w/q) bit patterns for primes below kFpPrimeBound, which
  // the NTT runs in FP64 (ntt.hip).
  std::vector<u64> fwd((size_t)np * N * 2), inv((size_t)np * N * 2), ninv(2 * np);
  auto pair = [](u64 w, u64 q, u64* out) {
    if (q < kFpPrimeBound) {
      double d = (double)w, s = (double)w / (double)q;
      std::memcpy(out, &d, 8);
      std::memcpy(out + 1, &s, 8);
    } else {
      out[0] = w;
      out[1] = shoup(w, q);
    }
  };
  for (int i = 0; i < np; ++i) {
    u64 q = P.q[i], psi = P.psi[i], ipsi = h_invmod(psi, q);
    u64 a = 1, b = 1;
    for (int k = 0; k < N; ++k) {
      size_t pos = ((size_t)i * N + brv((unsigned)k, P.logN)) * 2;
      pair(a, q, &fwd[pos]);
      pair(b, q, &inv[pos]);
      a = h_mulmod(a, psi, q);
      b = h_mulmod(b, ipsi, q);
    }
    pair(h_invmod((u64)N % q, q), q, &ninv[2 * i]);
  }
  sh.tab.fwd = upload(pool, fwd);
  sh.tab.inv = upload(pool, inv);
  sh.tab.ninv = upload(pool, ninv);

  // Row-pass factor tables of N = 2^16 (rows of M = 2^8 points, R = 2^8
  // rows).  Entry (R + r) 2^s + j (j < 2^s) of the table is psi^e with
  // e = brv((R + r) 2^s) + brv_s(j) N / 2^s (the two bit fields reverse
  // separately), i.e. rowf[r][s] times comm[2^s + j]; every product is
  // checked against the full table here.
  if (P.logN == 16) {
    constexpr int LM = 8, M = 1 << LM, R = 1 << LM;
    std::vector<double> rf((size_t)np * R * LM, 0.0), ri((size_t)np * R * LM, 0.0);
    std::vector<u64> cf((size_t)np * M * 2, 0), ci((size_t)np * M * 2, 0);
    for (int p = 0; p < np; ++p) {
      const u64 q = P.q[p];
      if (q >= kFpPrimeBound) continue;       // only the FP64 path forms its entries
      const u64 psi = P.psi[p], ipsi = h_invmod(psi, q);
      auto tab_w = [&](const std::vector<u64>& t, size_t m) {
        double d;
        std::memcpy(&d, &t[((size_t)p * N + m) * 2], 8);
        return (u64)d;
      };
      for (int dir = 0; dir < 2; ++dir) {
        const std::vector<u64>& full = dir ? inv : fwd;
        std::vector<double>& rowf = dir ? ri : rf;
        std::vector<u64>& comm = dir ? ci : cf;
        const u64 root = dir ? ipsi : psi;
        std::vector<u64> cw(M, 1);
        for (int s = 0; s < LM; ++s) {
          const u64 b = h_powmod(root, (u64)N >> s, q);   // a primitive 2^(s+1)-th root
          for (int j = 0; j < (1 << s); ++j) {
            cw[(1 << s) + j] = h_powmod(b, brv((unsigned)j, s), q);
            pair(cw[(1 << s) + j], q, &comm[((size_t)p * M + (1 << s) + j) * 2]);
          }
        }
        for (int r = 0; r < R; ++r)
          for (int s = 0; s < LM; ++s) {
            const u64 f = tab_w(full, (size_t)(R + r) << s);
            rowf[((size_t)p * R + r) * LM + s] = (double)f;
            for (int j = 0; j < (1 << s); ++j)
              if (h_mulmod(f, cw[(1 << s) + j], q) != tab_w(full, ((size_t)(R + r) << s) + j))
                PPST_THROW(ST_EINVAL, "row twiddle factorisation does not reproduce the table");
          }
      }
    }
    sh.tab.rowf_fwd = upload(pool, std::vector<u64>((const u64*)rf.data(), (const u64*)rf.data() + rf.size()));
    sh.tab.rowf_inv = upload(pool, std::vector<u64>((const u64*)ri.data(), (const u64*)ri.data() + ri.size()));
    sh.tab.comm_fwd = upload(pool, cf);
    sh.tab.comm_inv = upload(pool, ci);
  }

  // ModDown
  const int L = P.L, K = P.K;
  MdLayout lay(K, L);
  std::vector<u64> md(lay.size());
  for (int k = 0; k < K; ++k) {
    u64 pk = P.q[L + 1 + k];
    u64 ph = 1;
    for (int k2 = 0; k2 < K; ++k2)
      if (k2 != k) ph = h_mulmod(ph, P.q[L + 1 + k2] % pk, pk);
    u64 phi = h_invmod(ph, pk);
    md[lay.phinv(k)] = phi;
    md[lay.phinv(k) + 1] = shoup(phi, pk);
    for (int i = 0; i <= L; ++i) {
      u64 qi = P.q[i], v = 1;
      for (int k2 = 0; k2 < K; ++k2)
        if (k2 != k) v = h_mulmod(v, P.q[L + 1 + k2] % qi, qi);
      md[lay.phat(k, i)] = h_mulmod(v, mont_r(qi), qi);   // Montgomery form
    }
  }
  for (int i = 0; i <= L; ++i) {
    u64 qi = P.q[i], pm = 1;
    for (int k = 0; k < K; ++k) pm = h_mulmod(pm, P.q[L + 1 + k] % qi, qi);
    u64 pinv = h_invmod(pm, qi);
    md[lay.pinv(i)] = pinv;
    md[lay.pinv(i) + 1] = shoup(pinv, qi);
  }
  for (int i = 0; i <= L; ++i) {   // P mod q_i
    u64 qi = P.q[i], pm = 1;
    for (int k = 0; k < K; ++k) pm = h_mulmod(pm, P.q[L + 1 + k] % qi, qi);
    md[lay.pmod(i)] = pm;
    md[lay.pmod(i) + 1] = shoup(pm, qi);
    sh.tab.pmod_host.push_back(pm);
    sh.tab.pmod_host.push_back(shoup(pm, qi));
  }
  for (int p = 0; p < np; ++p) {   // h = (P - 1) / 2 reduced mod every prime
    u64 q = P.q[p], pm = 1;
    for (int k = 0; k < K; ++k) pm = h_mulmod(pm, P.q[L + 1 + k] % q, q);
    md[lay.hmod(p)] = h_mulmod(h_submod(pm, 1, q), h_invmod(2, q), q);
  }
  for (int i = 0; i <= L; ++i) {   // the same constants times P^-1 mod q_i
    const u64 qi = P.q[i], pinv = md[lay.pinv(i)];
    for (int k = 0; k < K; ++k) md[lay.phatp(k, i)] = h_mulmod(md[lay.phat(k, i)], pinv, qi);
    md[lay.hpinv(i)] = h_mulmod(md[lay.hmod(i)], pinv, qi);
  }
  std::vector<u64> mdn(ninv);   // N^-1 in the table format, special primes scaled
  for (int k = 0; k < K; ++k) {
    const int p = L + 1 + k;
    const u64 pk = P.q[p], phi = md[lay.phinv(k)];
    md[lay.hphinv(k)] = h_mulmod(md[lay.hmod(p)], phi, pk);
    pair(h_mulmod(h_invmod((u64)N % pk, pk), phi, pk), pk, &mdn[2 * (size_t)p]);
  }
  sh.tab.moddown = upload(pool, md);
  sh.tab.md_ninv = upload(pool, mdn);

  // ModUp per (level, digit)
  for (int l = 0; l <= L; ++l) {
    const int nl = l + 1, ne = nl + K;
    const size_t dw = modup_digit_words(ne);
    std::vector<u64> all(dw * P.beta(l), 0), nv(2 * (size_t)nl, 0);
    for (int j = 0; j < P.beta(l); ++j) {
      const int lo = P.digit_lo(j), hi = P.digit_hi(j, l);
      u64* t = all.data() + dw * j;
      for (int i = lo; i < hi; ++i) {
        u64 qi = P.q[i], qh = 1;
        for (int i2 = lo; i2 < hi; ++i2)
          if (i2 != i) qh = h_mulmod(qh, P.q[i2] % qi, qi);
        u64 inv_ = h_invmod(qh, qi);
        t[2 * (i - lo)] = inv_;
        t[2 * (i - lo) + 1] = shoup(inv_, qi);
        pair(h_mulmod(h_invmod((u64)N % qi, qi), inv_, qi), qi, &nv[2 * (size_t)i]);
        for (int tt = 0; tt < ne; ++tt) {
          int p = tt < nl ? tt : L + 1 + (tt - nl);
          u64 qt = P.q[p], v = 1;
          for (int i2 = lo; i2 < hi; ++i2)
            if (i2 != i) v = h_mulmod(v, P.q[i2] % qt, qt);
          // Montgomery form: the kernel's sum comes out times 2^-64
          t[2 * kMaxAlpha + (size_t)tt * kMaxAlpha + (i - lo)] = h_mulmod(v, mont_r(qt), qt);
        }
      }
    }
    sh.tab.modup[l] = std::make_shared<Buf>(upload(pool, all));
    sh.tab.modup_ninv[l] = std::make_shared<Buf>(upload(pool, nv));
  }
  // rescale per level
  for (int l = 1; l <= L; ++l) {
    std::vector<u64> t(3 * (size_t)l);
    u64 ql = P.q[l];
    for (int i = 0; i < l; ++i) {
      u64 qi = P.q[i];
      u64 inv_ = h_invmod(ql % qi, qi);
      t[3 * i] = inv_;
      t[3 * i + 1] = shoup(inv_, qi);
      t[3 * i + 2] = ql % qi;
    }
    sh.tab.rescale[l] = std::make_shared<Buf>(upload(pool, t));
  }
}

const u64* modup_table(const Shared& sh, int level) {
  auto it = sh.tab.modup.find(level);
  if (it == sh.tab.modup.end()) PPST_THROW(ST_EINVAL, "no ModUp table");
  return it->second->p;
}
const u64* modup_ninv(const Shared& sh, int level) {
  auto it = sh.tab.modup_ninv.find(level);
  if (it == sh.tab.modup_ninv.end()) PPST_THROW(ST_EINVAL, "no ModUp factor table");
  return it->second->p;
}
const u64* rescale_table(const Shared& sh, int level) {
  auto it = sh.tab.rescale.find(level);
  if (it == sh.tab.rescale.end()) PPST_THROW(ST_EINVAL, "no rescale table");
  return it->second->p;
}

// ============================================================ contexts
void autotune_ntt(Shared& sh) {
  const int max_limbs = 200;
  hipStream_t st;
  HIP_CHECK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  {
    Buf scratch = dev_buf(sh.const_pool, (size_t)max_limbs * sh.P.N);
    HIP_CHECK(hipMemsetAsync(scratch.p, 0, (size_t)max_limbs * sh.P.N * 8, st));
    ntt_autotune(sh, st, scratch.p, max_limbs);
    HIP_CHECK(hipStreamSynchronize(st));
  }
  HIP_CHECK(hipStreamDestroy(st));
}

std::shared_ptr<Shared> make_shared_state(const ParamSpec& spec, const Hooks* hooks) {
  auto sh = std::make_shared<Shared>();
  sh->P = make_params(spec);
  HIP_CHECK(hipGetDevice(&sh->device));
  if (hooks) sh->hooks = *hooks;
  sh->const_pool = std::make_shared<Pool>((hipStream_t)0, sh->hooks, sh->pools);
  sh->pools->add(sh->const_pool);
  dg_thresholds(sh->dg_thr);
  build_tables(*sh);
  HIP_CHECK(hipDeviceSynchronize());
  // "col,row" variant indices, or a whole plan as ntt_plan_string writes it
  const char* force = std::getenv("PPST_NTT_PLAN");
  const char* tune = std::getenv("PPST_NTT_AUTOTUNE");
  if (force && std::strchr(force, '[')) {
    ntt_load_plan(*sh, force);
  } else if (force) {
    int c = 0, r = 0;
    if (std::sscanf(force, "%d,%d", &c, &r) != 2)
      PPST_THROW(ST_EINVAL, "PPST_NTT_PLAN is col,row or a plan as ppst_ntt_plan writes it");
    ntt_set_plan(*sh, c, r);
  } else if (!(tune && tune[0] == '0')) {
    autotune_ntt(*sh);
  }
  return sh;
}

std::unique_ptr<Context> make_context(std::shared_ptr<Shared> sh, hipStream_t stream) {
  auto cx = std::make_unique<Context>();
  cx->sh = std::move(sh);
  if (stream) {
    cx->stream = stream;
  } else {
    HIP_CHECK(hipStreamCreateWithFlags(&cx->stream, hipStreamNonBlocking));
    cx->own_stream = true;
  }
  cx->pool = std::make_shared<Pool>(cx->stream, cx->sh->hooks, cx->sh->pools);
  cx->sh->pools->add(cx->pool);
  return cx;
}

void destroy_context(Context* cx) {
  if (!cx) return;
  (void)hipStreamSynchronize(cx->stream);
  // ciphertexts the caller still holds keep the pool alive past the stream;
  // its cache of free blocks goes back to the device now
  if (cx->pool) {
    cx->pool->trim();
    cx->pool->detach();
  }
  cx->pool.reset();
  if (cx->own_stream) (void)hipStreamDestroy(cx->stream);
}

u64 galois_elt(const Params& P, long r) {
  const long n = P.N / 2;
  long rr = ((r % n) + n) % n;
  return h_powmod(5, (u64)rr, 2 * (u64)P.N);
}

// =============================================================== helpers
namespace {

inline size_t limb_words(const Params& P) { return (size_t)P.N; }

void ntt_ct_limbs(Context& cx, u64* data, int nl, int npoly, size_t stride, bool inverse) {
  NttLaunch L{};
  L.src = data;
  L.dst = data;
  L.nlimbs = nl;
  L.nbatch = npoly;
  L.batch_stride = stride;
  L.nq = nl;
  L.pofs = cx.P().L + 1;
  ntt(*cx.sh, L, inverse, cx.stream);
}

void require_same(const Ciphertext& a, const Ciphertext& b) {
  if (a.level != b.level)
    PPST_THROW(ST_ESCALE, "operands at different levels (" + std::to_string(a.level) + " vs " +
                           std::to_string(b.level) + ")");
  if (a.scale != b.scale) PPST_THROW(ST_ESCALE, "operands at different scales");
  if (a.npoly != 2 || b.npoly != 2) PPST_THROW(ST_EINVAL, "expected degree-1 ciphertexts");
}

// products rescaled at `level` land on Delta_{level-1} only where the scale
// rule holds; the levels of the bootstrapping transforms are excluded
void require_canon(const Params& P, int level) {
  if (level >= 1 && level <= P.L && !P.canon[level])
    PPST_THROW(ST_ESCALE, "level " + std::to_string(level) +
                              " is reserved for the bootstrapping linear transforms");
}

const KsKey& relin_key(const EvalKeys& evk) {
  if (!evk.relin) PPST_THROW(ST_ENOKEY, "no relinearisation key");
  return *evk.relin;
}
const KsKey& galois_key(const EvalKeys& evk, u64 g) {
  auto it = evk.galois.find(g);
  if (it == evk.galois.end()) PPST_THROW(ST_ENOKEY, "no Galois key for element " + std::to_string(g));
  return *it->second;
}

// Forward NTT of the ModUp output [nbatch][beta][ne][N] in one launch: it is
// [nbatch * beta][ne][N] with each digit's own limbs skipped.
void ntt_ext_digits(Context& cx, u64* ext, int level, int nbatch) {
  const Params& P = cx.P();
  const int nl = level + 1, ne = nl + P.K, beta = P.beta(level);
  NttLaunch L{};
  L.src = ext;
  L.dst = ext;
  int most = 0;
  for (int j = 0; j < beta; ++j) most = std::max(most, ne - (P.digit_hi(j, level) - P.digit_lo(j)));
  L.nlimbs = most;
  L.nbatch = nbatch * beta;
  L.batch_stride = (size_t)ne * P.N;
  L.nq = nl;
  L.pofs = P.L + 1;
  L.digit_alpha = P.alpha;
  L.digit_count = beta;
  L.digit_total = ne;
  ntt(*cx.sh, L, false, cx.stream);
}

// Hybrid key switching, first half: coefficient form of the input d (NTT
// form, level l, nbatch items at stride sd), ModUp of every digit back to NTT
// form, inner product with the key.  Returns the accumulators u,
// [nbatch][2][ne][N] over q_0..q_l, p_0..p_{K-1}.
// With prep_d (products), limb q_l of u also receives (P mod q_l) times the
// tensor's d0, d1 (prep_d: [nbatch][3][nl][N] at stride sd), the first step
// of the fused ModDown + rescale.
// The scratch is caller memory: x ([nbatch][l+1][N], free again once this
// returns), ext ([nbatch][beta][ne][N]) and the result u.
// With pa, pb (a product on the fused path; d, sd, prep_d unused) the input
// is the operands' d2 = a1 b1, formed in the inverse transform's first pass
// and, for the digits' own limbs and P d0, P d1, in the fused kernel: the
// tensor is never written.
void ks_accumulate_into(Context& cx, const KsKey& key, const u64* d, size_t sd, int level,
                        int nbatch, uint32_t g, const u64* prep_d, u64* x, u64* ext, u64* u,
                        const u64* const* pa = nullptr, const u64* const* pb = nullptr) {
  const Params& P = cx.P();
  const Shared& sh = *cx.sh;
  const int N = P.N, nl = level + 1, K = P.K, ne = nl + K, beta = P.beta(level);
  const size_t sx = (size_t)nl * N, sext = (size_t)beta * ne * N, su = 2 * (size_t)ne * N;
  if (pa) {
    if (!ks_fused_ok(P, level) || g != 0) PPST_THROW(ST_EINVAL, "operand form needs the fused key switch");
    ntt_inv_prod(sh, pa, pb, x, level, nbatch, modup_ninv(sh, level), cx.stream);
  } else {
    NttLaunch L{};
    L.src = d;
    L.dst = x;
    L.nlimbs = nl;
    L.nbatch = nbatch;
    L.batch_stride = sd;
    L.dst_stride = sx;
    L.nq = nl;
    L.pofs = P.L + 1;
    L.galois = g;
    L.ninv = modup_ninv(sh, level);
    ntt(sh, L, true, cx.stream);
  }
  // ModUp inside the column pass saves the extended digits' round trip
  // through memory but re-reads each digit limb once per target (from L2):
  // a gain for a few items, a loss for large batches
  const bool fused = ks_fused_ok(P, level), modup_in_col = fused && nbatch <= 4 && modup_col_ok();
  if (!modup_in_col) k_modup(sh, x, ext, level, nbatch, sx, sext, cx.stream);
  if (fused) {
    // the digits' row pass and the inner product in one kernel (and ModUp
    // in their column pass)
    KsTail kt{};
    kt.x = modup_in_col ? x : nullptr;
    kt.sx = sx;
    kt.ext = ext;
    kt.d = pa ? nullptr : d;
    kt.sd = sd;
    kt.pa = pa;
    kt.pb = pb;
    kt.key = key.k.p;
    kt.u = u;
    kt.pd = prep_d;
    kt.spd = sd;
    if (prep_d || pa) {
      kt.pmod = sh.tab.pmod_host[2 * level];
      kt.pmods = sh.tab.pmod_host[2 * level + 1];
    }
    kt.gd = g;
    ntt_fwd_ks_fused(sh, kt, level, nbatch, cx.stream);
    return;
  }
  ntt_ext_digits(cx, ext, level, nbatch);
  k_ks_inner(sh, d, ext, key.k.p, u, level, nbatch, sd, sext, su, g, 0, cx.stream, prep_d, sd);
}

Buf ks_accumulate(Context& cx, const KsKey& key, const u64* d, size_t sd, int level, int nbatch,
                  uint32_t g = 0, const u64* prep_d = nullptr) {
  const Params& P = cx.P();
  const int N = P.N, nl = level + 1, ne = nl + P.K, beta = P.beta(level);
  const size_t sx = (size_t)nl * N, sext = (size_t)beta * ne * N, su = 2 * (size_t)ne * N;
  Buf x = dev_buf(cx.pool, sx * nbatch);
  Buf ext = dev_buf(cx.pool, sext * nbatch);
  Buf u = dev_buf(cx.pool, su * nbatch);
  ks_accumulate_into(cx, key, d, sd, level, nbatch, g, prep_d, x.p, ext.p, u.p);
  return u;
}

// Second half, plain: for each item b, out[b] = (u/P rounded) + (add0[b],
// add1[b]) [+ acc[b]] with the rounding ModDown; the final step runs in the
// last pass of the conversion's NTT.  add0 is read through X -> X^gadd.
void ks_moddown_ptr(Context& cx, Buf& u, int level, int nbatch, const u64* const* add0,
                    const u64* const* add1, const u64* const* acc, u64* const* out,
                    uint32_t gadd) {
  const Params& P = cx.P();
  const Shared& sh = *cx.sh;
  const int N = P.N, nl = level + 1, K = P.K, ne = nl + K;
  const size_t su = 2 * (size_t)ne * N, sc = 2 * (size_t)nl * N;
  {
    NttLaunch L{};
    L.dst = u.p + (size_t)nl * N;
    L.src = L.dst;
    L.nlimbs = K;
    L.nbatch = 2 * nbatch;
    L.batch_stride = (size_t)ne * N;   // [batch][2][ne][N] is [2 nbatch][ne][N]
    L.nq = 0;
    L.pofs = P.L + 1;
    L.ninv = sh.tab.md_ninv.p;         // the conversion's weights need z_k Phat_k^-1
    ntt(sh, L, true, cx.stream);
  }
  Buf conv = dev_buf(cx.pool, sc * nbatch);
  k_moddown_conv(sh, u.p, conv.p, level, nbatch, su, sc, cx.stream);
  MdTail t{u.p, su, add0, add1, acc, out, gadd};
  ntt_fwd_md_final(sh, conv.p, level, nbatch, t, cx.stream);
}

// the same with addends and outputs at fixed strides (sa, so) from one base
void ks_moddown(Context& cx, Buf& u, int level, const u64* add0, const u64* add1, size_t sa,
                u64* out, size_t so, int nbatch, uint32_t gadd = 0) {
  std::vector<const u64*> a0(nbatch), a1(nbatch);
  std::vector<u64*> o(nbatch);
  for (int b = 0; b < nbatch; ++b) {
    a0[b] = add0 ? add0 + (size_t)b * sa : nullptr;
    a1[b] = add1 ? add1 + (size_t)b * sa : nullptr;
    o[b] = out + (size_t)b * so;
  }
  ks_moddown_ptr(cx, u, level, nbatch, a0.data(), a1.data(), nullptr, o.data(), gadd);
}

// g != 0: switch the key of the automorphism X -> X^g applied to d and add0
// (the permutation is folded into their reads)
void keyswitch(Context& cx, const KsKey& key, const u64* d, size_t sd, int level,
               const u64* add0, const u64* add1, size_t sa, u64* out, size_t so, int nbatch,
               uint32_t g = 0) {
  Buf u = ks_accumulate(cx, key, d, sd, level, nbatch, g);
  ks_moddown(cx, u, level, add0, add1, sa, out, so, nbatch, g);
}

// Second half for a product: rescale(d + ModDown(u)) in one pass, bit-exact
// with relinearisation followed by rescale (kern.h, k_mdr_*).  D is the
// tensor [3][nl][N] per item (stride sd); out: one device pointer per item,
// each [2][l][N].
// corr: caller scratch of [nbatch][2][l][N] words
// pa, pb: a product's operands in place of the tensor D (d0, d1 formed in
// the last pass)
void ks_moddown_rescale_into(Context& cx, u64* u, const u64* D, size_t sd, int level,
                             u64* const* out, int nbatch, u64* corr,
                             const u64* const* pa = nullptr, const u64* const* pb = nullptr) {
  const Params& P = cx.P();
  const Shared& sh = *cx.sh;
  const int N = P.N, nl = level + 1, K = P.K, ne = nl + K;
  const size_t su = 2 * (size_t)ne * N, sc = 2 * (size_t)level * N;
  {
    NttLaunch L{};                    // limbs q_l, p_0..p_{K-1} of both polynomials
    L.src = u;
    L.dst = u;
    L.nlimbs = K + 1;
    L.nbatch = 2 * nbatch;
    L.batch_stride = (size_t)ne * N;
    L.nq = nl;
    L.pofs = P.L + 1;
    L.skip_lo = 0;
    L.skip_hi = level;
    L.ninv = sh.tab.md_ninv.p;         // N^-1 on q_l, N^-1 Phat_k^-1 on the special limbs
    ntt(sh, L, true, cx.stream);
  }
  k_mdr_corr(sh, u, corr, level, nbatch, su, sc, cx.stream);
  MdrTail tail{u, pa ? nullptr : D, su, sd, rescale_table(sh, level), out, pa, pb};
  ntt_fwd_mdr_final(sh, corr, level, nbatch, tail, cx.stream);
}

void ks_moddown_rescale(Context& cx, Buf& u, const u64* D, size_t sd, int level,
                        u64* const* out, int nbatch, const u64* const* pa = nullptr,
                        const u64* const* pb = nullptr) {
  Buf corr = dev_buf(cx.pool, 2 * (size_t)level * cx.P().N * nbatch);
  ks_moddown_rescale_into(cx, u.p, D, sd, level, out, nbatch, corr.p, pa, pb);
}

// A product on the fused path straight from its operands (pa[b], pb[b]):
// out[b] = rescale(relin(tensor)) with the tensor never written
void mul_from_operands(Context& cx, const KsKey& key, const u64* const* pa, const u64* const* pb,
                       int level, u64* const* out, int nbatch) {
  const Params& P = cx.P();
  const int N = P.N, nl = level + 1, ne = nl + P.K, beta = P.beta(level);
  const size_t sx = (size_t)nl * N, sext = (size_t)beta * ne * N, su = 2 * (size_t)ne * N;
  Buf u = dev_buf(cx.pool, su * nbatch);
  {
    Buf x = dev_buf(cx.pool, sx * nbatch);
    Buf ext = dev_buf(cx.pool, sext * nbatch);
    ks_accumulate_into(cx, key, nullptr, 0, level, nbatch, 0, nullptr, x.p, ext.p, u.p, pa, pb);
  }
  ks_moddown_rescale(cx, u, nullptr, 0, level, out, nbatch, pa, pb);
}

// ciphertexts per batched launch group
constexpr size_t kMulChunk = 16;
// products per group of ppst_mul_batch: as many as one launch's pointer
// arrays take, so that a batch of up to 64 reads the relinearisation key once
// (key-switching scratch: about 154 MiB per product at level 24, under 10 GiB
// for a full group)
constexpr size_t kMulBatchGroup = kPtrBatch;

// Rescale npoly polynomials at `level`: polynomial c at a[c] (limbs 0..level)
// into out[c] (limbs 0..level-1).  With k (host arrays of level+1 constant
// residues and Shoup companions) the input is first multiplied by that
// constant; the result is bit for bit rescale(k a).  The dropped limbs are
// read strided from a[0] when pstride is nonzero (a[c] = a[0] + c pstride),
// else gathered; they are transformed out of place, so the input is never
// modified.
void rescale_ptrs(Context& cx, const u64* const* a, u64* const* out, int level, int npoly,
                  size_t pstride, const u64* k, const u64* kp) {
  const Params& P = cx.P();
  const Shared& sh = *cx.sh;
  const int N = P.N;
  Buf top = dev_buf(cx.pool, (size_t)npoly * N);
  Buf tmp = dev_buf(cx.pool, (size_t)npoly * level * N);
  {
    NttLaunch L{};
    if (pstride) {
      L.src = a[0] + (size_t)level * N;
      L.batch_stride = pstride;
    } else {
      std::vector<const u64*> rows(npoly);
      for (int c = 0; c < npoly; ++c) rows[c] = a[c] + (size_t)level * N;
      k_gather_rows(sh, rows.data(), top.p, npoly, cx.stream);
      L.src = top.p;
      L.batch_stride = N;
    }
    L.dst = top.p;
    L.nlimbs = 1;
    L.nbatch = npoly;
    L.dst_stride = N;
    L.nq = 0;
    L.pofs = level;     // every row is on q_level
    ntt(sh, L, true, cx.stream);
  }
  const u64 kl[2] = {k ? k[level] : 0, k ? kp[level] : 0};
  k_rescale_conv(sh, top.p, tmp.p, level, npoly, N, cx.stream, k ? kl : nullptr);
  RsTail tail{a, out, rescale_table(sh, level), k, kp};
  ntt_fwd_rescale_final(sh, tmp.p, level, npoly, tail, cx.stream);
}

// Rescale npoly polynomials at `level` (polynomial c at a + c pstride) into
// out ([npoly][level][N]); k, kp as for rescale_ptrs.
void rescale_raw(Context& cx, const u64* a, size_t pstride, int level, int npoly, u64* out,
                 const u64* k = nullptr, const u64* kp = nullptr) {
  const size_t N = (size_t)cx.P().N;
  std::vector<const u64*> ap(npoly);
  std::vector<u64*> op(npoly);
  for (int c = 0; c < npoly; ++c) {
    ap[c] = a + (size_t)c * pstride;
    op[c] = out + (size_t)c * level * N;
  }
  rescale_ptrs(cx, ap.data(), op.data(), level, npoly, pstride, k, kp);
}

void scalar_residues(const Params& P, int64_t k, int nl, std::vector<u64>& v, std::vector<u64>& vp) {
  v.resize(nl);
  vp.resize(nl);
  for (int t = 0; t < nl; ++t) {
    v[t] = h_signed_mod(k, P.q[t]);
    vp[t] = shoup(v[t], P.q[t]);
  }
}

}  // namespace

// ================================================================= keys
std::unique_ptr<SecretKey> keygen_secret(Context& cx, u64 seed) {
  const Params& P = cx.P();
  const Shared& sh = *cx.sh;
  auto sk = std::make_unique<SecretKey>();
  Buf s32(cx.pool, (size_t)P.N * 4);
  std::vector<int32_t> sparse;
  if (P.spec.h > 0) {
    sparse.resize(P.N);
    sparse_ternary(seed, P.N, P.spec.h, sparse.data());
    HIP_CHECK(hipMemcpyAsync(s32.p, sparse.data(), (size_t)P.N * 4, hipMemcpyHostToDevice,
                             cx.stream));
  } else {
    k_sample_ternary(sh, (int32_t*)s32.p, seed, purpose_code(P_SK, 0, 0), cx.stream);
  }
  sk->s_ntt = dev_buf(sh.const_pool, (size_t)P.nprimes * P.N);
  k_small_to_rns(sh, (int32_t*)s32.p, sk->s_ntt.p, P.nprimes, P.nprimes, 0, cx.stream);
  NttLaunch L{};
  L.src = L.dst = sk->s_ntt.p;
  L.nlimbs = P.nprimes;
  L.nq = P.nprimes;
  L.pofs = 0;
  ntt(sh, L, false, cx.stream);
  std::vector<int32_t> h(P.N);
  HIP_CHECK(hipMemcpyAsync(h.data(), s32.p, (size_t)P.N * 4, hipMemcpyDeviceToHost, cx.stream));
  HIP_CHECK(hipStreamSynchronize(cx.stream));
  sk->s.assign(h.begin(), h.end());
  return sk;
}

std::unique_ptr<PublicKey> keygen_public(Context& cx, const SecretKey& sk, u64 seed) {
  const Params& P = cx.P();
  const Shared& sh = *cx.sh;
  const int nq = P.L + 1, N = P.N;
  auto pk = std::make_unique<PublicKey>();
  pk->pk = dev_buf(sh.const_pool, 2 * (size_t)nq * N);
  u64* b = pk->pk.p;
  u64* a = b + (size_t)nq * N;
  k_sample_uniform(sh, a, nq, nq, 0, seed, purpose_code(P_PK_A, 0, 0), cx.stream);
  Buf e32(cx.pool, (size_t)N * 4);
  Buf e = dev_buf(cx.pool, (size_t)nq * N);
  k_sample_dg(sh, (int32_t*)e32.p, seed, purpose_code(P_PK_E, 0, 0), cx.stream);
  k_small_to_rns(sh, (int32_t*)e32.p, e.p, nq, nq, 0, cx.stream);
  ntt_ct_limbs(cx, e.p, nq, 1, 0, false);
  k_keyform(sh, a, sk.s_ntt.p, e.p, nullptr, nullptr, b, nq, nq, 0, cx.stream);
  HIP_CHECK(hipStreamSynchronize(cx.stream));
  return pk;
}

namespace {

std::shared_ptr<KsKey> keygen_ks(Context& cx, const SecretKey& sk, u64 seed, u64 keyid,
                                 const u64* sp) {
  const Params& P = cx.P();
  const Shared& sh = *cx.sh;
  const int np = P.nprimes, N = P.N;
  auto key = std::make_shared<KsKey>();
  key->k = dev_buf(sh.const_pool, (size_t)P.dnum * 2 * np * N);
  Buf e32(cx.pool, (size_t)N * 4);
  Buf e = dev_buf(cx.pool, (size_t)np * N);
  std::vector<u64> pmod(np);
  for (int t = 0; t < np; ++t) {
    u64 q = P.q[t], v = 1;
    for (int k = 0; k < P.K; ++k) v = h_mulmod(v, P.q[P.L + 1 + k] % q, q);
    pmod[t] = v;
  }
  for (int j = 0; j < P.dnum; ++j) {
    u64* b = key->k.p + (size_t)(2 * j) * np * N;
    u64* a = key->k.p + (size_t)(2 * j + 1) * np * N;
    k_sample_uniform(sh, a, np, np, 0, seed, purpose_code(P_KSK_A, keyid, j), cx.stream);
    k_sample_dg(sh, (int32_t*)e32.p, seed, purpose_code(P_KSK_E, keyid, j), cx.stream);
    k_small_to_rns(sh, (int32_t*)e32.p, e.p, np, np, 0, cx.stream);
    NttLaunch L{};
    L.src = L.dst = e.p;
    L.nlimbs = np;
    L.nq = np;
    L.pofs = 0;
    ntt(sh, L, false, cx.stream);
    std::vector<u64> f(np, 0);
    for (int t = 0; t <= P.L; ++t)
      if (t / P.alpha == j) f[t] = pmod[t];
    k_keyform(sh, a, sk.s_ntt.p, e.p, sp, f.data(), b, np, np, 0, cx.stream);
  }
  HIP_CHECK(hipStreamSynchronize(cx.stream));
  return key;
}

}  // namespace

std::shared_ptr<KsKey> keygen_relin(Context& cx, const SecretKey& sk, u64 seed) {
  const Params& P = cx.P();
  Buf s2 = dev_buf(cx.pool, (size_t)P.nprimes * P.N);
  k_mul_poly(*cx.sh, sk.s_ntt.p, sk.s_ntt.p, s2.p, 1, P.nprimes, 0, 0, cx.stream);
  return keygen_ks(cx, sk, seed, 0, s2.p);
}

std::shared_ptr<KsKey> keygen_galois(Context& cx, const SecretKey& sk, u64 seed, u64 g) {
  const Params& P = cx.P();
  Buf sp = dev_buf(cx.pool, (size_t)P.nprimes * P.N);
  k_automorph(*cx.sh, sk.s_ntt.p, sp.p, P.nprimes, P.N, P.N, g, cx.stream);
  return keygen_ks(cx, sk, seed, g, sp.p);
}

// ========================================================== plaintexts
PtPtr plaintext_from_coeffs(Context& cx, const int64_t* coeffs, int level, double scale) {
  const Params& P = cx.P();
  if (level < 0 || level > P.L) PPST_THROW(ST_ELEVEL, "level out of range");
  auto pt = std::make_shared<Plaintext>();
  pt->level = level;
  pt->scale = scale;
  pt->coeffs.assign(coeffs, coeffs + P.N);
  Buf c64(cx.pool, (size_t)P.N * 8);
  HIP_CHECK(hipMemcpyAsync(c64.p, pt->coeffs.data(), (size_t)P.N * 8, hipMemcpyHostToDevice,
                           cx.stream));
  pt->buf = dev_buf(cx.pool, (size_t)(level + 1) * P.N);
  k_int64_to_rns(*cx.sh, (const int64_t*)c64.p, pt->buf.p, level + 1, level + 1, 0, cx.stream);
  ntt_ct_limbs(cx, pt->buf.p, level + 1, 1, 0, false);
  // the host vector must stay alive until the copy has run
  HIP_CHECK(hipStreamSynchronize(cx.stream));
  return pt;
}

PtPtr encode(Context& cx, const double* v, size_t n, int level) {
  const Params& P = cx.P();
  if (level < 0 || level > P.L) PPST_THROW(ST_ELEVEL, "level out of range");
  if (n > (size_t)P.slots()) PPST_THROW(ST_EINVAL, "more values than slots");
  std::vector<int64_t> c(P.N);
  encode_coeffs(P, v, (int)n, P.scale[level], c.data());
  return plaintext_from_coeffs(cx, c.data(), level, P.scale[level]);
}

PtPtr encode_embedded(Context& cx, const std::vector<long double>& p, int level) {
  const Params& P = cx.P();
  if (level < 0 || level > P.L) PPST_THROW(ST_ELEVEL, "level out of range");
  if (p.size() != (size_t)P.N) PPST_THROW(ST_EINVAL, "embedding of the wrong length");
  std::vector<int64_t> c(P.N);
  encode_round(p, P.scale[level], c.data());
  return plaintext_from_coeffs(cx, c.data(), level, P.scale[level]);
}

void decode(Context& cx, const Plaintext& pt, double* out, size_t n) {
  const Params& P = cx.P();
  const int N = P.N;
  const int nl = pt.level >= 1 ? 2 : 1;
  Buf tmp = dev_buf(cx.pool, (size_t)nl * N);
  NttLaunch L{};
  L.src = pt.buf.p;
  L.dst = tmp.p;
  L.nlimbs = nl;
  L.nq = nl;
  L.pofs = 0;
  ntt(*cx.sh, L, true, cx.stream);
  std::vector<u64> h((size_t)nl * N);
  HIP_CHECK(hipMemcpyAsync(h.data(), tmp.p, h.size() * 8, hipMemcpyDeviceToHost, cx.stream));
  HIP_CHECK(hipStreamSynchronize(cx.stream));
  std::vector<long double> c(N);
  const u64 q0 = P.q[0];
  if (nl == 1) {
    for (int k = 0; k < N; ++k)
      c[k] = h[k] > q0 / 2 ? -(long double)(q0 - h[k]) : (long double)h[k];
  } else {
    // two-limb CRT, exact while |coefficient| < q_0 q_1 / 2
    const u64 q1 = P.q[1];
    const u64 q0inv = h_invmod(q0 % q1, q1);
    const u128 Q = (u128)q0 * q1;
    for (int k = 0; k < N; ++k) {
      u64 x0 = h[k], x1 = h[(size_t)N + k];
      u64 t = h_mulmod(h_submod(x1, x0 % q1, q1), q0inv, q1);
      u128 X = (u128)x0 + (u128)q0 * t;
      c[k] = X > Q / 2 ? -(long double)(Q - X) : (long double)X;
    }
  }
  std::vector<double> all(P.slots());
  decode_coeffs(P, c.data(), pt.scale, all.data(), P.slots());
  for (size_t j = 0; j < n && j < all.size(); ++j) out[j] = all[j];
}

// ========================================================= ciphertexts
CtPtr new_ct(Context& cx, int level, double scale, int npoly) {
  const Params& P = cx.P();
  auto ct = std::make_shared<Ciphertext>();
  ct->level = level;
  ct->scale = scale;
  ct->npoly = npoly;
  ct->N = P.N;
  ct->buf = dev_buf(cx.pool, (size_t)npoly * (level + 1) * P.N);
  return ct;
}

CtPtr encrypt_pk(Context& cx, const PublicKey& pk, const Plaintext& pt, u64 seed) {
  const Params& P = cx.P();
  const Shared& sh = *cx.sh;
  const int nl = pt.level + 1, N = P.N;
  Buf s32(cx.pool, (size_t)N * 4);
  Buf v = dev_buf(cx.pool, (size_t)nl * N);
  Buf e0 = dev_buf(cx.pool, (size_t)nl * N);
  Buf e1 = dev_buf(cx.pool, (size_t)nl * N);
  k_sample_ternary(sh, (int32_t*)s32.p, seed, purpose_code(P_ENC_V, 0, 0), cx.stream);
  k_small_to_rns(sh, (int32_t*)s32.p, v.p, nl, nl, 0, cx.stream);
  k_sample_dg(sh, (int32_t*)s32.p, seed, purpose_code(P_ENC_E0, 0, 0), cx.stream);
  k_small_to_rns(sh, (int32_t*)s32.p, e0.p, nl, nl, 0, cx.stream);
  k_sample_dg(sh, (int32_t*)s32.p, seed, purpose_code(P_ENC_E1, 0, 0), cx.stream);
  k_small_to_rns(sh, (int32_t*)s32.p, e1.p, nl, nl, 0, cx.stream);
  ntt_ct_limbs(cx, v.p, nl, 1, 0, false);
  ntt_ct_limbs(cx, e0.p, nl, 1, 0, false);
  ntt_ct_limbs(cx, e1.p, nl, 1, 0, false);
  auto ct = new_ct(cx, pt.level, pt.scale);
  const u64* b = pk.pk.p;
  const u64* a = pk.pk.p + (size_t)(P.L + 1) * N;
  k_fma3(sh, e0.p, v.p, b, pt.buf.p, ct->poly(0), nl, cx.stream);
  k_fma3(sh, e1.p, v.p, a, nullptr, ct->poly(1), nl, cx.stream);
  return ct;
}

CtPtr encrypt_sk(Context& cx, const SecretKey& sk, const Plaintext& pt, u64 seed) {
  const Params& P = cx.P();
  const Shared& sh = *cx.sh;
  const int nl = pt.level + 1, N = P.N;
  auto ct = new_ct(cx, pt.level, pt.scale);
  k_sample_uniform(sh, ct->poly(1), nl, nl, 0, seed, purpose_code(P_SKE_A, 0, 0), cx.stream);
  Buf e32(cx.pool, (size_t)N * 4);
  Buf e = dev_buf(cx.pool, (size_t)nl * N);
  k_sample_dg(sh, (int32_t*)e32.p, seed, purpose_code(P_SKE_E, 0, 0), cx.stream);
  k_small_to_rns(sh, (int32_t*)e32.p, e.p, nl, nl, 0, cx.stream);
  ntt_ct_limbs(cx, e.p, nl, 1, 0, false);
  k_keyform(sh, ct->poly(1), sk.s_ntt.p, e.p, nullptr, nullptr, ct->poly(0), nl, nl, 0, cx.stream);
  k_add(sh, ct->poly(0), pt.buf.p, ct->poly(0), 1, nl, 0, 0, 0, false, cx.stream);
  return ct;
}

PtPtr decrypt(Context& cx, const SecretKey& sk, const Ciphertext& ct) {
  if (ct.npoly != 2) PPST_THROW(ST_EINVAL, "decrypt expects a degree-1 ciphertext");
  const Params& P = cx.P();
  auto pt = std::make_shared<Plaintext>();
  pt->level = ct.level;
  pt->scale = ct.scale;
  pt->buf = dev_buf(cx.pool, (size_t)(ct.level + 1) * P.N);
  k_fma3(*cx.sh, ct.poly(0), ct.poly(1), sk.s_ntt.p, nullptr, pt->buf.p, ct.level + 1, cx.stream);
  return pt;
}

// =========================================================== operations
CtPtr copy_ct(Context& cx, const Ciphertext& a) {
  auto out = new_ct(cx, a.level, a.scale, a.npoly);
  HIP_CHECK(hipMemcpyAsync(out->buf.p, a.buf.p, (size_t)a.npoly * (a.level + 1) * a.N * 8,
                           hipMemcpyDeviceToDevice, cx.stream));
  return out;
}

CtPtr add(Context& cx, const Ciphertext& a, const Ciphertext& b) {
  require_same(a, b);
  auto out = new_ct(cx, a.level, a.scale);
  size_t st = (size_t)(a.level + 1) * a.N;
  k_add(*cx.sh, a.buf.p, b.buf.p, out->buf.p, 2, a.level + 1, st, st, st, false, cx.stream);
  return out;
}

CtPtr add_n(Context& cx, const std::vector<const Ciphertext*>& a) {
  if (a.empty()) PPST_THROW(ST_EINVAL, "empty sum");
  std::vector<const u64*> src;
  for (const Ciphertext* x : a) {
    require_same(*a[0], *x);
    src.push_back(x->buf.p);
  }
  auto out = new_ct(cx, a[0]->level, a[0]->scale);
  k_sum(*cx.sh, src.data(), (int)src.size(), out->buf.p, 2, a[0]->level + 1, cx.stream);
  return out;
}

CtPtr sub(Context& cx, const Ciphertext& a, const Ciphertext& b) {
  require_same(a, b);
  auto out = new_ct(cx, a.level, a.scale);
  size_t st = (size_t)(a.level + 1) * a.N;
  k_add(*cx.sh, a.buf.p, b.buf.p, out->buf.p, 2, a.level + 1, st, st, st, true, cx.stream);
  return out;
}

int64_t const_int(const Params& P, double c, int level) {
  double v = c * P.scale[level];
  if (!(std::fabs(v) < 9.0e18)) PPST_THROW(ST_EDOMAIN, "constant too large for the scale");
  return llround(v);
}

CtPtr add_const(Context& cx, const Ciphertext& a, double c) {
  const Params& P = cx.P();
  int64_t k = const_int(P, c, a.level);
  std::vector<u64> v, vp;
  scalar_residues(P, k, a.level + 1, v, vp);
  auto out = new_ct(cx, a.level, a.scale, a.npoly);
  size_t per = (size_t)(a.level + 1) * a.N;
  k_add_scalar(*cx.sh, a.poly(0), out->poly(0), a.level + 1, v.data(), cx.stream);
  HIP_CHECK(hipMemcpyAsync(out->buf.p + per, a.buf.p + per, (a.npoly - 1) * per * 8,
                           hipMemcpyDeviceToDevice, cx.stream));
  return out;
}

CtPtr mul_int(Context& cx, const Ciphertext& a, int64_t k) {
  const Params& P = cx.P();
  std::vector<u64> v, vp;
  scalar_residues(P, k, a.level + 1, v, vp);
  auto out = new_ct(cx, a.level, a.scale, a.npoly);
  size_t per = (size_t)(a.level + 1) * a.N;
  k_mul_scalar(*cx.sh, a.buf.p, out->buf.p, a.npoly, a.level + 1, per, per, v.data(), vp.data(),
               cx.stream);
  return out;
}

CtPtr rescale(Context& cx, const Ciphertext& a) {
  if (a.level < 1) PPST_THROW(ST_ELEVEL, "no level left to rescale");
  const Params& P = cx.P();
  require_canon(P, a.level);
  auto out = new_ct(cx, a.level - 1, P.scale[a.level - 1], a.npoly);
  rescale_raw(cx, a.buf.p, (size_t)(a.level + 1) * a.N, a.level, a.npoly, out->buf.p);
  return out;
}

CtPtr mul_const(Context& cx, const Ciphertext& a, double c) {
  if (a.level < 1) PPST_THROW(ST_ELEVEL, "no level left for a constant product");
  const Params& P = cx.P();
  require_canon(P, a.level);
  std::vector<u64> v, vp;
  scalar_residues(P, const_int(P, c, a.level), a.level + 1, v, vp);
  auto out = new_ct(cx, a.level - 1, P.scale[a.level - 1], a.npoly);
  rescale_raw(cx, a.buf.p, (size_t)(a.level + 1) * a.N, a.level, a.npoly, out->buf.p, v.data(),
              vp.data());
  return out;
}

namespace {
// Ciphertexts of one level and degree, each multiplied by the constant with
// residues v, vp and rescaled from rlevel (limbs above rlevel are not read):
// the group-wise form of rescale_raw
std::vector<CtPtr> rescale_group(Context& cx, const std::vector<const Ciphertext*>& a, int rlevel,
                                 const std::vector<u64>& v, const std::vector<u64>& vp) {
  const Params& P = cx.P();
  std::vector<CtPtr> outs;
  const size_t per = (size_t)(a[0]->level + 1) * P.N, per_out = (size_t)rlevel * P.N;
  for (size_t i0 = 0; i0 < a.size(); i0 += kMulChunk) {
    const size_t n = std::min(kMulChunk, a.size() - i0);
    std::vector<const u64*> ap;
    std::vector<u64*> op;
    for (size_t i = 0; i < n; ++i) {
      const Ciphertext& x = *a[i0 + i];
      auto o = new_ct(cx, rlevel - 1, P.scale[rlevel - 1], x.npoly);
      for (int p = 0; p < x.npoly; ++p) {
        ap.push_back(x.buf.p + p * per);
        op.push_back(o->buf.p + p * per_out);
      }
      outs.push_back(o);
    }
    rescale_ptrs(cx, ap.data(), op.data(), rlevel, (int)ap.size(), 0, v.data(), vp.data());
  }
  return outs;
}

// Level alignment from `from` to `level` multiplies by
// K = round(Delta_level q_{level+1} / Delta_from) and rescales by q_{level+1}:
// K's residues on q_0..q_{level+1}
void align_residues(const Params& P, int from, int level, std::vector<u64>& v,
                    std::vector<u64>& vp) {
  const int64_t K = llround((P.scale[level] * (double)P.q[level + 1]) / P.scale[from]);
  scalar_residues(P, K, level + 2, v, vp);
}

void check_group(const std::vector<const Ciphertext*>& a) {
  for (const Ciphertext* x : a)
    if (x->level != a[0]->level || x->npoly != a[0]->npoly)
      PPST_THROW(ST_ESCALE, "ciphertexts of different levels or degrees");
}
}  // namespace

std::vector<CtPtr> mul_const_n(Context& cx, const std::vector<const Ciphertext*>& a, double c) {
  if (a.empty()) return {};
  check_group(a);
  const int level = a[0]->level;
  if (level < 1) PPST_THROW(ST_ELEVEL, "no level left for a constant product");
  require_canon(cx.P(), level);
  std::vector<u64> v, vp;
  scalar_residues(cx.P(), const_int(cx.P(), c, level), level + 1, v, vp);
  return rescale_group(cx, a, level, v, vp);
}

std::vector<CtPtr> level_align_n(Context& cx, const std::vector<const Ciphertext*>& a, int level) {
  if (a.empty()) return {};
  check_group(a);
  const int from = a[0]->level;
  std::vector<CtPtr> outs;
  if (level == from) {
    for (const Ciphertext* x : a) outs.push_back(copy_ct(cx, *x));
    return outs;
  }
  if (level > from || level < 0) PPST_THROW(ST_ELEVEL, "cannot raise a ciphertext's level");
  std::vector<u64> v, vp;
  align_residues(cx.P(), from, level, v, vp);
  return rescale_group(cx, a, level + 1, v, vp);
}

CtPtr lincomb(Context& cx, const std::vector<const Ciphertext*>& cts,
              const std::vector<double>& cs, int level) {
  const Params& P = cx.P();
  if (cts.empty() || cts.size() != cs.size())
    PPST_THROW(ST_EINVAL, "need matching ciphertexts and constants");
  if (level < 0) PPST_THROW(ST_ELEVEL, "combination level below 0");
  if (level + 1 <= P.L) require_canon(P, level + 1);
  const int lv1 = level + 1, nl = lv1 + 1, N = P.N;
  const size_t nt = cts.size();
  std::vector<const u64*> src(nt);
  std::vector<size_t> ps(nt);
  std::vector<u64> k(nt * nl), kp(nt * nl);
  for (size_t j = 0; j < nt; ++j) {
    const Ciphertext& a = *cts[j];
    if (a.npoly != 2) PPST_THROW(ST_EINVAL, "linear combination of degree-1 ciphertexts only");
    if (a.level < lv1) PPST_THROW(ST_ELEVEL, "a term is below the combination's level + 1");
    const double v = cs[j] * P.scale[lv1] * (P.scale[lv1] / P.scale[a.level]);
    if (!(std::fabs(v) < 9.0e18)) PPST_THROW(ST_EDOMAIN, "constant too large for the scale");
    std::vector<u64> r, rp;
    scalar_residues(P, llround(v), nl, r, rp);
    for (int t = 0; t < nl; ++t) {
      k[j * nl + t] = r[t];
      kp[j * nl + t] = rp[t];
    }
    src[j] = a.buf.p;
    ps[j] = (size_t)(a.level + 1) * N;
  }
  Buf sum = dev_buf(cx.pool, 2 * (size_t)nl * N);
  k_lincomb(*cx.sh, src.data(), ps.data(), k.data(), kp.data(), (int)nt, nl, sum.p, (size_t)nl * N,
            cx.stream);
  auto out = new_ct(cx, level, P.scale[level], 2);
  rescale_raw(cx, sum.p, (size_t)nl * N, lv1, 2, out->buf.p);
  return out;
}

CtPtr mul_plain(Context& cx, const Ciphertext& a, const Plaintext& pt) {
  if (a.level < 1) PPST_THROW(ST_ELEVEL, "no level left for a plaintext product");
  if (pt.level != a.level) PPST_THROW(ST_ESCALE, "plaintext level differs from the ciphertext's");
  auto t = new_ct(cx, a.level, a.scale, a.npoly);
  size_t per = (size_t)(a.level + 1) * a.N;
  k_mul_poly(*cx.sh, a.buf.p, pt.buf.p, t->buf.p, a.npoly, a.level + 1, per, per, cx.stream);
  return rescale(cx, *t);
}

CtPtr tensor(Context& cx, const Ciphertext& a, const Ciphertext& b) {
  require_same(a, b);
  auto d = new_ct(cx, a.level, a.scale * b.scale, 3);
  const u64* pa = a.buf.p;
  const u64* pb = b.buf.p;
  k_tensor(*cx.sh, &pa, &pb, d->buf.p, a.level + 1, 1, 0, cx.stream);
  return d;
}

CtPtr relin(Context& cx, const EvalKeys& evk, const Ciphertext& d) {
  if (d.npoly != 3) PPST_THROW(ST_EINVAL, "relinearisation expects a degree-2 ciphertext");
  const KsKey& key = relin_key(evk);
  auto out = new_ct(cx, d.level, d.scale);
  keyswitch(cx, key, d.poly(2), 0, d.level, d.poly(0), d.poly(1), 0, out->buf.p, 0, 1);
  return out;
}

CtPtr mul(Context& cx, const EvalKeys& evk, const Ciphertext& a, const Ciphertext& b) {
  require_same(a, b);
  if (a.level < 1) PPST_THROW(ST_ELEVEL, "no level left for a product");
  require_canon(cx.P(), a.level);
  const KsKey& key = relin_key(evk);
  const Params& P = cx.P();
  auto out = new_ct(cx, a.level - 1, P.scale[a.level - 1]);
  u64* op = out->buf.p;
  if (ks_fused_ok(P, a.level)) {
    const u64* pa = a.buf.p;
    const u64* pb = b.buf.p;
    mul_from_operands(cx, key, &pa, &pb, a.level, &op, 1);
    return out;
  }
  auto d = tensor(cx, a, b);
  Buf u = ks_accumulate(cx, key, d->poly(2), 0, a.level, 1, 0, d->buf.p);
  ks_moddown_rescale(cx, u, d->buf.p, 0, a.level, &op, 1);
  return out;
}

size_t mul_scratch_words(const Params& P, int level) {
  const size_t nl = (size_t)level + 1, ne = nl + P.K, beta = (size_t)P.beta(level);
  return (3 * nl + beta * ne + 2 * ne + std::max(nl, 2 * (size_t)level)) * (size_t)P.N;
}

void mul_into(Context& cx, const EvalKeys& evk, const u64* a, const u64* b, int level, u64* out,
              u64* scratch) {
  const Params& P = cx.P();
  if (level < 1 || level > P.L) PPST_THROW(ST_ELEVEL, "no level left for a product");
  require_canon(P, level);
  const KsKey& key = relin_key(evk);
  const size_t N = (size_t)P.N, nl = (size_t)level + 1, ne = nl + P.K;
  u64* D = scratch;                                   // tensor [3][l+1][N]
  u64* ext = D + 3 * nl * N;                          // extended digits [beta][ne][N]
  u64* u = ext + (size_t)P.beta(level) * ne * N;      // accumulators [2][ne][N]
  u64* xc = u + 2 * ne * N;                           // d2's coefficients, later the correction
  if (ks_fused_ok(P, level)) {                        // the tensor region stays unused
    ks_accumulate_into(cx, key, nullptr, 0, level, 1, 0, nullptr, xc, ext, u, &a, &b);
    ks_moddown_rescale_into(cx, u, nullptr, 0, level, &out, 1, xc, &a, &b);
    return;
  }
  k_tensor(*cx.sh, &a, &b, D, (int)nl, 1, 0, cx.stream);
  ks_accumulate_into(cx, key, D + 2 * nl * N, 0, level, 1, 0, D, xc, ext, u);
  ks_moddown_rescale_into(cx, u, D, 0, level, &out, 1, xc);
}

CtPtr apply_galois(Context& cx, const EvalKeys& evk, const Ciphertext& a, u64 g) {
  if (a.npoly != 2) PPST_THROW(ST_EINVAL, "an automorphism expects a degree-1 ciphertext");
  const Params& P = cx.P();
  if (g % 2 == 0 || g >= 2 * (u64)P.N) PPST_THROW(ST_EINVAL, "Galois element must be odd and below 2N");
  if (g == 1) return copy_ct(cx, a);
  const KsKey& key = galois_key(evk, g);
  auto out = new_ct(cx, a.level, a.scale);
  keyswitch(cx, key, a.poly(1), 0, a.level, a.poly(0), nullptr, 0, out->buf.p, 0, 1,
            (uint32_t)g);
  return out;
}

CtPtr rotate(Context& cx, const EvalKeys& evk, const Ciphertext& a, long r) {
  if (a.npoly != 2) PPST_THROW(ST_EINVAL, "rotation expects a degree-1 ciphertext");
  return apply_galois(cx, evk, a, galois_elt(cx.P(), r));
}

CtPtr rescale_as(Context& cx, const Ciphertext& a, double scale) {
  if (a.level < 1) PPST_THROW(ST_ELEVEL, "no level left to rescale");
  auto out = new_ct(cx, a.level - 1, scale, a.npoly);
  rescale_raw(cx, a.buf.p, (size_t)(a.level + 1) * a.N, a.level, a.npoly, out->buf.p);
  return out;
}

CtPtr mod_raise(Context& cx, const Ciphertext& a) {
  if (a.npoly != 2) PPST_THROW(ST_EINVAL, "ModRaise expects a degree-1 ciphertext");
  if (a.level != 0) PPST_THROW(ST_ELEVEL, "ModRaise takes a level-0 ciphertext");
  const Params& P = cx.P();
  const Shared& sh = *cx.sh;
  const size_t N = (size_t)P.N;
  Buf x = dev_buf(cx.pool, 2 * N);
  {
    NttLaunch L{};                      // limb q_0 of both polynomials to coefficients
    L.src = a.buf.p;
    L.dst = x.p;
    L.nlimbs = 1;
    L.nbatch = 2;
    L.batch_stride = N;
    L.dst_stride = N;
    L.nq = 1;
    L.pofs = P.L + 1;
    ntt(sh, L, true, cx.stream);
  }
  auto out = new_ct(cx, P.L, P.scale[P.L]);
  k_mod_raise(sh, x.p, out->buf.p, P.L + 1, 2, cx.stream);
  ntt_ct_limbs(cx, out->buf.p, P.L + 1, 2, (size_t)(P.L + 1) * N, false);
  return out;
}

CtPtr mul_monomial(Context& cx, const Ciphertext& a, int k, int sign) {
  const Params& P = cx.P();
  if (k < 0 || k >= P.N || (sign != 1 && sign != -1)) PPST_THROW(ST_EINVAL, "monomial out of range");
  std::vector<int64_t> e(P.N, 0);
  e[k] = sign;
  auto pt = plaintext_from_coeffs(cx, e.data(), a.level, 1.0);
  return mul_plain_raw(cx, a, *pt);
}

CtPtr mul_plain_raw(Context& cx, const Ciphertext& a, const Plaintext& pt) {
  if (pt.level < a.level) PPST_THROW(ST_ESCALE, "plaintext has fewer limbs than the ciphertext");
  auto t = new_ct(cx, a.level, a.scale, a.npoly);
  const size_t per = (size_t)(a.level + 1) * a.N;
  k_mul_poly(*cx.sh, a.buf.p, pt.buf.p, t->buf.p, a.npoly, a.level + 1, per, per, cx.stream);
  return t;
}

std::vector<CtPtr> rotate_hoisted(Context& cx, const EvalKeys& evk, const Ciphertext& a,
                                  const std::vector<long>& rs) {
  if (a.npoly != 2) PPST_THROW(ST_EINVAL, "rotation expects a degree-1 ciphertext");
  const Params& P = cx.P();
  const Shared& sh = *cx.sh;
  const int level = a.level, N = P.N, nl = level + 1, K = P.K, ne = nl + K, beta = P.beta(level);
  const size_t per = (size_t)nl * N, sext = (size_t)beta * ne * N;
  std::vector<CtPtr> outs;
  // shared ModUp of c1
  Buf x = dev_buf(cx.pool, per);
  Buf ext = dev_buf(cx.pool, sext);
  {
    NttLaunch L{};
    L.src = a.poly(1);
    L.dst = x.p;
    L.nlimbs = nl;
    L.nq = nl;
    L.pofs = P.L + 1;
    L.ninv = modup_ninv(sh, level);
    ntt(sh, L, true, cx.stream);
  }
  k_modup(sh, x.p, ext.p, level, 1, per, sext, cx.stream);
  x.release();
  ntt_ext_digits(cx, ext.p, level, 1);
  Buf u = dev_buf(cx.pool, 2 * (size_t)ne * N);
  for (long r : rs) {
    u64 g = galois_elt(P, r);
    if (g == 1) {
      outs.push_back(copy_ct(cx, a));
      continue;
    }
    const KsKey& key = galois_key(evk, g);
    k_ks_inner(sh, a.poly(1), ext.p, key.k.p, u.p, level, 1, 0, 0, 0, (uint32_t)g, (uint32_t)g,
               cx.stream);
    auto out = new_ct(cx, level, a.scale);
    const u64* add0 = a.poly(0);
    u64* op = out->buf.p;
    ks_moddown_ptr(cx, u, level, 1, &add0, nullptr, nullptr, &op, (uint32_t)g);
    outs.push_back(out);
  }
  return outs;
}

std::vector<CtPtr> rotate_hoisted_batch(Context& cx, const EvalKeys& evk,
                                        const std::vector<const Ciphertext*>& cts,
                                        const std::vector<long>& rs) {
  const size_t n = cts.size(), m = rs.size();
  if (n == 0 || m == 0) return {};
  const Params& P = cx.P();
  const Shared& sh = *cx.sh;
  const int level = cts[0]->level;
  for (const Ciphertext* c : cts) {
    if (c->npoly != 2) PPST_THROW(ST_EINVAL, "rotation expects a degree-1 ciphertext");
    if (c->level != level) PPST_THROW(ST_ESCALE, "batch members at different levels");
  }
  const int N = P.N, nl = level + 1, K = P.K, ne = nl + K, beta = P.beta(level);
  const size_t per = (size_t)nl * N, sext = (size_t)beta * ne * N;
  std::vector<const KsKey*> keys(m, nullptr);
  std::vector<u64> gs(m);
  for (size_t r = 0; r < m; ++r) {
    gs[r] = galois_elt(P, rs[r]);
    if (gs[r] != 1) keys[r] = &galois_key(evk, gs[r]);
  }
  std::vector<CtPtr> outs(n * m);
  // ModUp of every c1, with each digit's own limbs copied in beside the
  // extension so that the inner product reads one buffer; groups of
  // kMulChunk ciphertexts share each launch
  Buf ext = dev_buf(cx.pool, sext * n);
  {
    const size_t grp = std::min(n, kMulChunk);
    Buf x = dev_buf(cx.pool, per * grp);
    for (size_t i0 = 0; i0 < n; i0 += grp) {
      const int nb = (int)std::min(grp, n - i0);
      u64* e0 = ext.p + sext * i0;
      std::vector<const u64*> c1(nb);
      for (int i = 0; i < nb; ++i) c1[i] = cts[i0 + i]->poly(1);
      for (int j = 0; j < beta; ++j) {
        const int lo = P.digit_lo(j), hi = P.digit_hi(j, level);
        std::vector<const u64*> own(nb);
        for (int i = 0; i < nb; ++i) own[i] = c1[i] + (size_t)lo * N;
        k_gather_rows(sh, own.data(), e0 + ((size_t)j * ne + lo) * N, nb, cx.stream,
                      (size_t)(hi - lo) * N, sext);
      }
      NttLaunch L{};
      if (nb == 1) {
        L.src = c1[0];
      } else {
        k_gather_rows(sh, c1.data(), x.p, nb, cx.stream, per);
        L.src = x.p;
      }
      L.dst = x.p;
      L.nlimbs = nl;
      L.nbatch = nb;
      L.batch_stride = per;
      L.nq = nl;
      L.pofs = P.L + 1;
      L.ninv = modup_ninv(sh, level);
      ntt(sh, L, true, cx.stream);
      k_modup(sh, x.p, e0, level, nb, per, sext, cx.stream);
    }
    ntt_ext_digits(cx, ext.p, level, (int)n);   // the copied own limbs are skipped
  }
  // one rotation at a time over chunks of the batch: the key is read once
  // per group of items of the inner product
  const int chunk = (int)std::min<size_t>(n, kPtrBatch);
  const size_t su = 2 * (size_t)ne * N;
  Buf u = dev_buf(cx.pool, su * chunk);
  for (size_t r = 0; r < m; ++r) {
    if (gs[r] == 1) {
      for (size_t i = 0; i < n; ++i) outs[i * m + r] = copy_ct(cx, *cts[i]);
      continue;
    }
    const uint32_t g = (uint32_t)gs[r];
    for (size_t b0 = 0; b0 < n; b0 += chunk) {
      const int nb = (int)std::min<size_t>(chunk, n - b0);
      k_ks_inner(sh, nullptr, ext.p + sext * b0, keys[r]->k.p, u.p, level, nb, 0, sext, su, g, g,
                 cx.stream);
      std::vector<const u64*> add(nb);
      std::vector<u64*> po(nb);
      for (int i = 0; i < nb; ++i) {
        auto o = new_ct(cx, level, cts[b0 + i]->scale);
        add[i] = cts[b0 + i]->poly(0);
        po[i] = o->buf.p;
        outs[(b0 + i) * m + r] = o;
      }
      ks_moddown_ptr(cx, u, level, nb, add.data(), nullptr, nullptr, po.data(), g);
    }
  }
  return outs;
}

// one key switch over the batch: the c1 polynomials side by side, the
// automorphism folded into the reads
std::vector<CtPtr> rotate_batch(Context& cx, const EvalKeys& evk,
                                const std::vector<const Ciphertext*>& cts, long r) {
  const size_t n = cts.size();
  if (n == 0) return {};
  const Params& P = cx.P();
  const Shared& sh = *cx.sh;
  const int level = cts[0]->level;
  for (const Ciphertext* c : cts) {
    if (c->npoly != 2) PPST_THROW(ST_EINVAL, "rotation expects a degree-1 ciphertext");
    if (c->level != level) PPST_THROW(ST_ESCALE, "batch members at different levels");
  }
  const u64 g = galois_elt(P, r);
  std::vector<CtPtr> outs;
  if (g == 1) {
    for (const Ciphertext* c : cts) outs.push_back(copy_ct(cx, *c));
    return outs;
  }
  const KsKey& key = galois_key(evk, g);
  const int N = P.N, nl = level + 1;
  const size_t per = (size_t)nl * N;
  // the c1 polynomials side by side (one gather launch unless there is
  // one), then one key switch
  Buf d;
  const u64* dp = cts[0]->poly(1);
  if (n > 1) {
    d = dev_buf(cx.pool, per * n);
    std::vector<const u64*> c1(n);
    for (size_t i = 0; i < n; ++i) c1[i] = cts[i]->poly(1);
    k_gather_rows(*cx.sh, c1.data(), d.p, (int)n, cx.stream, per);
    dp = d.p;
  }
  Buf u = ks_accumulate(cx, key, dp, per, level, (int)n, (uint32_t)g);
  d.release();
  std::vector<const u64*> add0(n);
  std::vector<u64*> po(n);
  for (size_t i = 0; i < n; ++i) {
    outs.push_back(new_ct(cx, level, cts[i]->scale));
    add0[i] = cts[i]->poly(0);
    po[i] = outs.back()->buf.p;
  }
  ks_moddown_ptr(cx, u, level, (int)n, add0.data(), nullptr, nullptr, po.data(), (uint32_t)g);
  return outs;
}

std::vector<std::pair<long, int>> rotsum_plan(const Params& P) {
  std::vector<std::pair<long, int>> plan;
  int bits = 0;
  while ((1L << bits) < P.slots()) ++bits;
  for (int b = 0; b < bits;) {
    const int take = std::min(3, bits - b);
    plan.emplace_back(1L << b, 1 << take);
    b += take;
  }
  return plan;
}

namespace {

// One hoisted rotate-and-sum step for every item: out_i = ct_i +
// sum_{0<k<radix} rot(ct_i, k s), with one ModUp of each c1, the radix - 1
// permuted inner products (and P times c0's permutations) added in the
// extended basis, and one ModDown whose last pass adds the item itself.
// into: when given, the outputs are these ciphertexts (allocated by the
// caller, same level and scale as the inputs) instead of new ones
std::vector<CtPtr> rotsum_step(Context& cx, const EvalKeys& evk,
                               const std::vector<const Ciphertext*>& cts, long s, int radix,
                               const std::vector<CtPtr>* into = nullptr) {
  const Params& P = cx.P();
  const Shared& sh = *cx.sh;
  const size_t n = cts.size();
  const int level = cts[0]->level;
  const int N = P.N, nl = level + 1, ne = nl + P.K, beta = P.beta(level);
  const size_t per = (size_t)nl * N, sext = (size_t)beta * ne * N, su = 2 * (size_t)ne * N;
  const int nk = radix - 1;
  if (nk < 1 || nk > kMaxHoistKeys) PPST_THROW(ST_EINVAL, "radix out of range");
  const u64* keys[kMaxHoistKeys];
  uint32_t gs[kMaxHoistKeys];
  for (int k = 0; k < nk; ++k) {
    const u64 g = galois_elt(P, (k + 1) * s);
    if (g == 1) PPST_THROW(ST_EINVAL, "rotate-and-sum step wraps around");
    gs[k] = (uint32_t)g;
    keys[k] = galois_key(evk, g).k.p;
  }
  std::vector<CtPtr> outs(n);
  const int chunk = (int)std::min<size_t>(n, kPtrBatch);
  Buf ext = dev_buf(cx.pool, sext * chunk);
  Buf x = dev_buf(cx.pool, per * chunk);
  Buf u = dev_buf(cx.pool, su * chunk);
  for (size_t b0 = 0; b0 < n; b0 += chunk) {
    const int nb = (int)std::min<size_t>(chunk, n - b0);
    std::vector<const u64*> d(nb), add(nb), acc(nb);
    std::vector<u64*> po(nb);
    for (int i = 0; i < nb; ++i) {
      const Ciphertext& c = *cts[b0 + i];
      d[i] = c.poly(1);
      add[i] = c.poly(0);
      acc[i] = c.buf.p;
      outs[b0 + i] = into ? (*into)[b0 + i] : new_ct(cx, level, c.scale);
      po[i] = outs[b0 + i]->buf.p;
    }
    // the c1 polynomials side by side (one gather launch unless there is
    // one), then one inverse NTT and one ModUp launch over the group
    if (nb == 1) {
      NttLaunch L{};
      L.src = d[0];
      L.dst = x.p;
      L.nlimbs = nl;
      L.nq = nl;
      L.pofs = P.L + 1;
      L.ninv = modup_ninv(sh, level);
      ntt(sh, L, true, cx.stream);
    } else {
      k_gather_rows(sh, d.data(), x.p, nb, cx.stream, per);
      NttLaunch L{};
      L.src = x.p;
      L.dst = x.p;
      L.nlimbs = nl;
      L.nbatch = nb;
      L.batch_stride = per;
      L.nq = nl;
      L.pofs = P.L + 1;
      L.ninv = modup_ninv(sh, level);
      ntt(sh, L, true, cx.stream);
    }
    k_modup(sh, x.p, ext.p, level, nb, per, sext, cx.stream);
    ntt_ext_digits(cx, ext.p, level, nb);   // the digits' own limbs are skipped
    // c0's permutations enter u0 as P sum_r c0(X^g_r) (exact through ModDown);
    // the ModDown's last pass adds the input itself
    k_ks_inner_multi(sh, d.data(), ext.p, keys, gs, nk, u.p, level, nb, sext, su, cx.stream,
                     add.data());
    ks_moddown_ptr(cx, u, level, nb, nullptr, nullptr, acc.data(), po.data(), 0);
  }
  return outs;
}

}  // namespace

std::vector<CtPtr> rotsum_batch(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& cts) {
  return rotsum_batch_into(cx, evk, cts, {});
}

std::vector<CtPtr> rotsum_batch_into(Context& cx, const EvalKeys& evk, const std::vector<CtPtr>& cts,
                                     const std::vector<CtPtr>& outs) {
  std::vector<CtPtr> cur = cts;
  if (cur.empty()) return cur;
  for (const CtPtr& c : cur) {
    if (c->npoly != 2) PPST_THROW(ST_EINVAL, "rotate-and-sum expects degree-1 ciphertexts");
    if (c->level != cur[0]->level) PPST_THROW(ST_ESCALE, "batch members at different levels");
  }
  if (!outs.empty()) {
    if (outs.size() != cts.size()) PPST_THROW(ST_EINVAL, "rotate-and-sum outputs differ in number");
    for (size_t i = 0; i < outs.size(); ++i)
      if (outs[i]->level != cts[i]->level || outs[i]->npoly != 2 || outs[i]->N != cts[i]->N)
        PPST_THROW(ST_EINVAL, "rotate-and-sum output of the wrong shape");
  }
  const auto plan = rotsum_plan(cx.P());
  if (plan.empty()) {                      // one slot: the sum is the input
    if (outs.empty()) {
      std::vector<CtPtr> r;
      for (const CtPtr& c : cts) r.push_back(copy_ct(cx, *c));
      return r;
    }
    for (size_t i = 0; i < outs.size(); ++i)
      HIP_CHECK(hipMemcpyAsync(outs[i]->buf.p, cts[i]->buf.p, cts[i]->buf.bytes,
                               hipMemcpyDeviceToDevice, cx.stream));
    return outs;
  }
  for (size_t k = 0; k < plan.size(); ++k) {
    std::vector<const Ciphertext*> v;
    for (const CtPtr& c : cur) v.push_back(c.get());
    const bool last = k + 1 == plan.size();
    cur = rotsum_step(cx, evk, v, plan[k].first, plan[k].second,
                      last && !outs.empty() ? &outs : nullptr);
  }
  return cur;
}

CtPtr rotsum(Context& cx, const EvalKeys& evk, const Ciphertext& a) {
  if (a.npoly != 2) PPST_THROW(ST_EINVAL, "rotate-and-sum expects a degree-1 ciphertext");
  std::vector<const Ciphertext*> v{&a};
  CtPtr cur;
  for (const auto& st : rotsum_plan(cx.P())) {
    cur = rotsum_step(cx, evk, v, st.first, st.second)[0];
    v = {cur.get()};
  }
  return cur ? cur : copy_ct(cx, a);
}

CtPtr rotsum_serial(Context& cx, const EvalKeys& evk, const Ciphertext& a) {
  if (a.npoly != 2) PPST_THROW(ST_EINVAL, "rotate-and-sum expects a degree-1 ciphertext");
  const Params& P = cx.P();
  CtPtr cur;
  const Ciphertext* in = &a;
  for (long s = 1; s < (long)P.slots(); s <<= 1) {
    const u64 g = galois_elt(P, s);
    const KsKey& key = galois_key(evk, g);
    // in + Rot(in, s): the key switch of c1(X^g), whose ModDown's last pass
    // adds c0(X^g) and the step's input
    auto out = new_ct(cx, in->level, in->scale);
    Buf u = ks_accumulate(cx, key, in->poly(1), 0, in->level, 1, (uint32_t)g);
    const u64* add0 = in->poly(0);
    const u64* acc = in->buf.p;
    u64* op = out->buf.p;
    ks_moddown_ptr(cx, u, in->level, 1, &add0, nullptr, &acc, &op, (uint32_t)g);
    cur = out;
    in = cur.get();
  }
  return cur ? cur : copy_ct(cx, a);
}

CtPtr level_align(Context& cx, const Ciphertext& a, int level) {
  if (level == a.level) return copy_ct(cx, a);
  if (level > a.level || level < 0) PPST_THROW(ST_ELEVEL, "cannot raise a ciphertext's level");
  const Params& P = cx.P();
  std::vector<u64> v, vp;
  align_residues(P, a.level, level, v, vp);
  // limbs q_0..q_{level+1} of a, multiplied by K and rescaled by q_{level+1}
  auto out = new_ct(cx, level, P.scale[level], a.npoly);
  rescale_raw(cx, a.buf.p, (size_t)(a.level + 1) * P.N, level + 1, a.npoly, out->buf.p, v.data(),
              vp.data());
  return out;
}


std::vector<CtPtr> mul_batch(Context& cx, const EvalKeys& evk,
                             const std::vector<const Ciphertext*>& a,
                             const std::vector<const Ciphertext*>& b) {
  const size_t n = a.size();
  if (n == 0) return {};
  if (b.size() != n) PPST_THROW(ST_EINVAL, "batch operands differ in length");
  const Params& P = cx.P();
  const int level = a[0]->level;
  for (size_t i = 0; i < n; ++i) {
    require_same(*a[i], *b[i]);
    if (a[i]->level != level) PPST_THROW(ST_ESCALE, "batch members at different levels");
  }
  if (level < 1) PPST_THROW(ST_ELEVEL, "no level left for a product");
  require_canon(P, level);
  const KsKey& key = relin_key(evk);
  const int nl = level + 1, N = P.N;
  const size_t per = (size_t)nl * N;
  std::vector<const u64*> pa(n), pb(n);
  for (size_t i = 0; i < n; ++i) {
    pa[i] = a[i]->buf.p;
    pb[i] = b[i]->buf.p;
  }
  std::vector<CtPtr> outs;
  for (size_t i = 0; i < n; ++i) outs.push_back(new_ct(cx, level - 1, P.scale[level - 1]));
  // groups of kMulBatchGroup products: one launch per stage and one read of
  // the key per group
  const bool operands = ks_fused_ok(P, level);
  for (size_t b0 = 0; b0 < n; b0 += kMulBatchGroup) {
    const int nb = (int)std::min<size_t>(kMulBatchGroup, n - b0);
    if (operands) {
      std::vector<u64*> po(nb);
      for (int i = 0; i < nb; ++i) po[i] = outs[b0 + i]->buf.p;
      mul_from_operands(cx, key, pa.data() + b0, pb.data() + b0, level, po.data(), nb);
      continue;
    }
    Buf D = dev_buf(cx.pool, 3 * per * nb);
    k_tensor(*cx.sh, pa.data() + b0, pb.data() + b0, D.p, nl, nb, 3 * per, cx.stream);
    Buf u = ks_accumulate(cx, key, D.p + 2 * per, 3 * per, level, nb, 0, D.p);
    std::vector<u64*> po(nb);
    for (int i = 0; i < nb; ++i) po[i] = outs[b0 + i]->buf.p;
    ks_moddown_rescale(cx, u, D.p, 3 * per, level, po.data(), nb);
  }
  return outs;
}

// ============================================================ graphs
void graph_begin(Context& cx) {
  if (cx.recording) PPST_THROW(ST_EINVAL, "a graph recording is already open");
  cx.pool->begin_capture();
  hipError_t e = hipStreamBeginCapture(cx.stream, hipStreamCaptureModeRelaxed);
  if (e != hipSuccess) {
    cx.pool->unpin(cx.pool->end_capture());
    PPST_THROW(ST_EDEVICE, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
  }
  cx.recording = true;
}

std::unique_ptr<Graph> graph_end(Context& cx) {
  if (!cx.recording) PPST_THROW(ST_EINVAL, "no graph recording is open");
  cx.recording = false;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(cx.stream, &g);
  std::vector<void*> blocks = cx.pool->end_capture();
  if (e != hipSuccess || g == nullptr) {
    if (g) (void)hipGraphDestroy(g);
    // nothing of the recording ever ran: wait for earlier work, then release
    (void)hipStreamSynchronize(cx.stream);
    cx.pool->unpin(blocks);
    PPST_THROW(ST_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  }
  auto out = std::make_unique<Graph>();
  out->graph = g;
  out->stream = cx.stream;
  out->pool = cx.pool;
  out->blocks = std::move(blocks);
  e = hipGraphInstantiate(&out->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    out->exec = nullptr;
    PPST_THROW(ST_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  return out;
}

void graph_launch(Graph& g) { HIP_CHECK(hipGraphLaunch(g.exec, g.stream)); }

Graph::~Graph() {
  (void)hipStreamSynchronize(stream);
  if (exec) (void)hipGraphExecDestroy(exec);
  if (graph) (void)hipGraphDestroy(graph);
  if (pool) pool->unpin(blocks);
}

void ntt_raw(Context& cx, u64* data, int nlimbs, int first_prime, bool inverse) {
  const Params& P = cx.P();
  if (first_prime < 0 || first_prime + nlimbs > P.nprimes)
    PPST_THROW(ST_EINVAL, "prime range out of bounds");
  NttLaunch L{};
  L.src = data;
  L.dst = data;
  L.nlimbs = nlimbs;
  L.nq = 0;
  L.pofs = first_prime;
  ntt(*cx.sh, L, inverse, cx.stream);
}

}  // namespace ppst
