// host_math.cpp -- parameter generation, sampling specification and the
// canonical-embedding encoder of the ppstat library (host side).
#include <algorithm>
#include <cmath>
#include <functional>
#include <thread>

#include "core.h"
#include "tables.h"

namespace ppst {

u64 h_powmod(u64 b, u64 e, u64 q) {
  u64 r = 1 % q;
  b %= q;
  for (; e; e >>= 1) {
    if (e & 1) r = h_mulmod(r, b, q);
    b = h_mulmod(b, b, q);
  }
  return r;
}

// Miller-Rabin with the seven bases of Jaeschke / Sinclair, exact for all
// 64-bit integers.
bool is_prime_u64(u64 n) {
  if (n < 4) return n == 2 || n == 3;
  if (!(n & 1)) return false;
  for (u64 p : {3ULL, 5ULL, 7ULL, 11ULL, 13ULL, 17ULL, 19ULL, 23ULL, 29ULL, 31ULL, 37ULL})
    if (n % p == 0) return n == p;
  u64 d = n - 1;
  int r = 0;
  while (!(d & 1)) { d >>= 1; ++r; }
  static const u64 bases[7] = {2ULL, 325ULL, 9375ULL, 28178ULL, 450775ULL, 9780504ULL,
                               1795265022ULL};
  for (u64 a0 : bases) {
    u64 a = a0 % n;
    if (a == 0) continue;
    u64 x = h_powmod(a, d, n);
    if (x == 1 || x == n - 1) continue;
    bool comp = true;
    for (int i = 1; i < r && comp; ++i) {
      x = h_mulmod(x, x, n);
      if (x == n - 1) comp = false;
    }
    if (comp) return false;
  }
  return true;
}

namespace {

bool used_in(const std::vector<u64>& v, u64 x) {
  for (u64 y : v) if (y == x) return true;
  return false;
}

// the largest unused prime p < 2^bits with p = 1 (mod 2N)
u64 top_prime(int bits, u64 m, const std::vector<u64>& used) {
  u64 lim = bits >= 64 ? ~0ULL : ((1ULL << bits) - 1);
  u64 x = lim - ((lim - 1) % m);              // largest x <= lim with x = 1 mod m
  for (; x > m; x -= m)
    if (!used_in(used, x) && is_prime_u64(x)) return x;
  PPST_THROW(ST_EINVAL, "no prime found");
}

// the unused prime p = 1 (mod 2N) closest to target; on a tie the smaller
u64 closest_prime(double target, u64 m, const std::vector<u64>& used) {
  u64 below = (u64)std::floor((target - 1.0) / (double)m) * m + 1;
  u64 above = below + m;
  while (below > m && (used_in(used, below) || !is_prime_u64(below))) below -= m;
  while (used_in(used, above) || !is_prime_u64(above)) above += m;
  double db = target - (double)below, da = (double)above - target;
  return da < db ? above : below;
}

// smallest x >= 2 whose power x^((q-1)/2N) has order exactly 2N
u64 root_2n(u64 q, u64 n) {
  for (u64 x = 2;; ++x) {
    u64 r = h_powmod(x, (q - 1) / (2 * n), q);
    if (h_powmod(r, n, q) == q - 1) return r;
  }
}

}  // namespace

Params make_params(const ParamSpec& s) {
  if (s.logN < 2 || s.logN > 17 || s.L < 0 || s.K < 1 || s.dnum < 1 ||
      s.L + 1 + s.K > kMaxPrimes || s.scale <= 1.0)
    PPST_THROW(ST_EINVAL, "invalid parameter specification");
  Params P;
  P.spec = s;
  P.logN = s.logN;
  P.N = 1 << s.logN;
  P.L = s.L;
  P.K = s.K;
  P.dnum = s.dnum;
  P.alpha = (s.L + 1 + s.dnum - 1) / s.dnum;
  // key-switching kernels keep a digit's limbs and the special primes in registers
  if (s.K > kMaxSpecial || P.alpha > kMaxAlpha || s.dnum > 8)
    PPST_THROW(ST_EINVAL, "at most 8 special primes, 8 digits and 16 limbs per digit");
  P.nprimes = s.L + 1 + s.K;
  const u64 m = 2 * (u64)P.N;
  std::vector<u64> used;
  P.q.assign(P.nprimes, 0);
  P.scale.assign(P.L + 1, 0.0);
  P.canon.assign(P.L + 1, 1);
  P.q[0] = top_prime(s.q0_bits, m, used);
  used.push_back(P.q[0]);
  // a segment of levels hi..lo+1 whose scale stays near `target`:
  // Delta_{l-1} = (Delta_l * Delta_l) / q_l with q_l the unused prime
  // nearest Delta_l^2 / target
  auto chain = [&](int hi, int lo, double target) {
    for (int l = hi; l > lo; --l) {
      double sq = P.scale[l] * P.scale[l];
      u64 p = closest_prime(sq / target, m, used);
      P.q[l] = p;
      used.push_back(p);
      P.scale[l - 1] = sq / (double)p;
    }
  };
  if (s.boot_cts <= 0) {
    P.Lc = P.L;
    P.scale[P.L] = s.scale;
    chain(P.L, 0, s.scale);
  } else {
    // Bootstrappable chain, top down: CoeffToSlot levels (the largest unused
    // primes below 2^p_bits, scale boot_scale), EvalMod levels (a chain at
    // boot_scale), SlotToCoeff levels (the largest unused primes, scales
    // stepping from boot_scale down to Delta by powers of two), then the
    // computation levels (a chain at Delta).
    const int C = s.boot_cts, E = s.boot_evalmod, S = s.boot_stc;
    if (E < 1 || S < 1 || !(s.boot_scale > 1.0)) PPST_THROW(ST_EINVAL, "invalid bootstrapping levels");
    P.Lc = P.L - C - E - S;
    if (P.Lc < 1) PPST_THROW(ST_EINVAL, "no computation level under the bootstrapping levels");
    for (int l = P.L; l > P.L - C; --l) {
      P.q[l] = top_prime(s.p_bits, m, used);
      used.push_back(P.q[l]);
      P.scale[l] = s.boot_scale;
      P.canon[l] = 0;
    }
    P.scale[P.L - C] = s.boot_scale;
    chain(P.L - C, P.Lc + S, s.boot_scale);
    for (int l = P.Lc + S; l > P.Lc; --l) {
      P.q[l] = top_prime(s.p_bits, m, used);
      used.push_back(P.q[l]);
      P.canon[l] = 0;
    }
    const int e = std::ilogb(s.boot_scale) - std::ilogb(s.scale);
    for (int i = 1; i < S; ++i) P.scale[P.Lc + i] = std::ldexp(s.scale, (i * e) / S);
    P.scale[P.Lc] = s.scale;
    chain(P.Lc, 0, s.scale);
  }
  for (int k = 0; k < P.K; ++k) {
    u64 p = top_prime(s.p_bits, m, used);
    P.q[P.L + 1 + k] = p;
    used.push_back(p);
  }
  P.psi.resize(P.nprimes);
  for (int i = 0; i < P.nprimes; ++i) {
    if (P.q[i] >= (1ULL << 60)) PPST_THROW(ST_EINVAL, "primes must stay below 2^60");
    P.psi[i] = root_2n(P.q[i], P.N);
  }
  return P;
}

bool preset_spec(const std::string& name, ParamSpec* out) {
  ParamSpec s;
  if (name == "c1") {          // N=2^12, 40-bit q0, two 30-bit primes, one 60-bit special prime
    s = {12, 2, 1, 3, 40, 60, 1073741824.0};
  } else if (name == "c2") {   // N=2^16, 60-bit q0, 24 primes near 2^40, 7 special primes
    s = {16, 24, 7, 3, 60, 60, 1099511627776.0};
  } else if (name == "t1") {   // N=2^12 with the c2 prime shapes, L=6
    s = {12, 6, 3, 3, 60, 60, 1099511627776.0};
  } else if (name == "t2") {   // N=2^12 with the full c2 chain, L=24
    s = {12, 24, 7, 3, 60, 60, 1099511627776.0};
  } else if (name == "b2" || name == "b1") {
    // bootstrappable: 11 computation levels at 2^40 under 3 SlotToCoeff,
    // 10 EvalMod (2^58) and 3 CoeffToSlot levels; sparse secret of weight 64;
    // q_0 of 55 bits (q_0 / Delta_0 = 2^15: a refresh multiplies EvalMod's
    // error by that ratio); b1 is the same chain at N=2^12
    s = {name == "b2" ? 16 : 12, 27, 8, 4, 55, 60, 1099511627776.0, 64, 3, 10, 3,
         288230376151711744.0};
  } else {
    return false;
  }
  *out = s;
  return true;
}

// ---------------------------------------------------------------- sampling
// SplitMix64 step: advance the state by the golden-ratio increment, mix.
static inline u64 splitmix(u64& state) {
  state += 0x9E3779B97F4A7C15ULL;
  u64 z = state;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline u64 mix_once(u64 x) { return splitmix(x); }

u64 stream_key(u64 seed, u64 purpose, u64 limb) {
  return mix_once(mix_once(mix_once(seed) ^ purpose) ^ limb);
}

void sparse_ternary(u64 seed, int N, int h, int32_t* out) {
  if (h < 1 || h > N) PPST_THROW(ST_EINVAL, "secret weight out of range");
  u64 state = stream_key(seed, purpose_code(P_SK, 0, 0), 0);
  std::vector<int32_t> idx(N);
  for (int k = 0; k < N; ++k) idx[k] = k;
  for (int i = 0; i < h; ++i) {
    const u64 w = splitmix(state);
    std::swap(idx[i], idx[i + (int)(w % (u64)(N - i))]);
  }
  std::fill(out, out + N, 0);
  for (int i = 0; i < h; ++i) out[idx[i]] = (splitmix(state) >> 63) ? -1 : 1;
}

void dg_thresholds(u64 thr[kDgMax]) {
  const double sigma = 3.2;
  const double two_s2 = 2.0 * sigma * sigma;
  double w[kDgMax + 1];
  w[0] = 1.0;
  for (int x = 1; x <= kDgMax; ++x) w[x] = 2.0 * std::exp(-((double)(x * x)) / two_s2);
  double tot = 0.0;
  for (int x = 0; x <= kDgMax; ++x) tot += w[x];
  double c = 0.0;
  for (int x = 0; x < kDgMax; ++x) {
    c += w[x];
    thr[x] = (u64)((c / tot) * 18446744073709551616.0);
  }
}

// ---------------------------------------------------------------- encoding
namespace {

typedef long double ld;
const ld kPi = 3.141592653589793238462643383279502884L;

// cos and sin of sign 2 pi J / n for J < n/2, computed once per (n, sign)
// and shared by every later call (threads included).  Stage len of the FFT
// uses the angle sign 2 pi j / len = sign 2 pi (j n/len) / n: the two
// expressions scale the same rounded factors by a power of two, so the
// table entry is bit for bit the value the stage would compute itself.
struct Twiddles {
  std::vector<ld> c, s;
};

const Twiddles& twiddles(size_t n, int sign) {
  static std::mutex mu;
  static std::map<std::pair<size_t, int>, std::unique_ptr<Twiddles>> cache;
  std::lock_guard<std::mutex> g(mu);
  auto& t = cache[{n, sign}];
  if (!t) {
    t.reset(new Twiddles);
    t->c.resize(n / 2);
    t->s.resize(n / 2);
    for (size_t j = 0; j < n / 2; ++j) {
      ld ang = (ld)sign * 2.0L * kPi * (ld)j / (ld)n;
      t->c[j] = cosl(ang);
      t->s[j] = sinl(ang);
    }
  }
  return *t;
}

// Butterflies of the stage of block length len over j in [j0, j1) and the
// blocks starting at i in [i0, i1)
void dif_stage(ld* re, ld* im, size_t len, size_t step, const Twiddles& tw, size_t j0, size_t j1,
               size_t i0, size_t i1) {
  const size_t h = len / 2;
  for (size_t j = j0; j < j1; ++j) {
    const ld c = tw.c[j * step], s = tw.s[j * step];
    for (size_t i = i0; i < i1; i += len) {
      ld ur = re[i + j], ui = im[i + j];
      ld vr = re[i + j + h], vi = im[i + j + h];
      re[i + j] = ur + vr;
      im[i + j] = ui + vi;
      ld dr = ur - vr, di = ui - vi;
      re[i + j + h] = dr * c - di * s;
      im[i + j + h] = dr * s + di * c;
    }
  }
}

// in-place decimation-in-frequency FFT of length n (power of two);
// output X_k = sum_j x_j exp(sign 2 pi i j k / n) lands at position brv(k).
// Long transforms run on T threads: the first log2 T stages split each
// block's butterflies by j, after which the n/T-point blocks are independent
// transforms, one per thread.  Every butterfly is computed as in the serial
// loop, so the result does not depend on T.
void dif_fft(std::vector<ld>& re, std::vector<ld>& im, int sign) {
  const size_t n = re.size();
  const Twiddles& tw = twiddles(n, sign);
  size_t T = 1;
  if (n >= ((size_t)1 << 14)) {
    const size_t hw = std::max<unsigned>(1u, std::thread::hardware_concurrency());
    while (T * 2 <= std::min<size_t>(hw, 8)) T *= 2;
  }
  size_t len = n, step = 1;
  auto run = [&](const std::function<void(size_t)>& f) {
    std::vector<std::thread> th;
    for (size_t t = 1; t < T; ++t) th.emplace_back(f, t);
    f(0);
    for (auto& x : th) x.join();
  };
  for (; T > 1 && len > n / T; len >>= 1, step <<= 1) {
    const size_t h = len / 2, l = len, st = step;
    run([&, h, l, st](size_t t) {
      dif_stage(re.data(), im.data(), l, st, tw, t * h / T, (t + 1) * h / T, 0, n);
    });
  }
  if (T > 1) {
    const size_t len0 = len, step0 = step, blk = n / T;
    run([&, len0, step0, blk](size_t t) {
      for (size_t l = len0, st = step0; l >= 2; l >>= 1, st <<= 1)
        dif_stage(re.data(), im.data(), l, st, tw, 0, l / 2, t * blk, (t + 1) * blk);
    });
    return;
  }
  for (; len >= 2; len >>= 1, step <<= 1)
    dif_stage(re.data(), im.data(), len, step, tw, 0, len / 2, 0, n);
}

size_t bitrev(size_t x, int bits) {
  size_t r = 0;
  for (int b = 0; b < bits; ++b) r |= ((x >> b) & 1) << (bits - 1 - b);
  return r;
}

}  // namespace

// Canonical embedding inverse: slot j is the evaluation at zeta^(5^j),
// zeta = exp(i pi / N); p_k = (2/N) Re sum_j m_j zeta^(-5^j k);
// coefficient k = round_half_away(scale * p_k).
void encode_embed(const Params& P, const double* m, int n_used, std::vector<long double>& p) {
  const int N = P.N, n = N / 2;
  if (n_used < 0 || n_used > n) PPST_THROW(ST_EINVAL, "more values than slots");
  const size_t M2 = 2 * (size_t)N;
  std::vector<ld> re(M2, 0.0L), im(M2, 0.0L);
  u64 e = 1;
  for (int j = 0; j < n_used; ++j) {
    re[e] = (ld)m[j];
    e = (e * 5) % M2;
  }
  dif_fft(re, im, -1);
  const int bits = P.logN + 1;
  p.resize(N);
  for (int k = 0; k < N; ++k) p[k] = (2.0L / (ld)N) * re[bitrev((size_t)k, bits)];
}

void encode_round(const std::vector<long double>& p, double scale, int64_t* out) {
  for (size_t k = 0; k < p.size(); ++k) out[k] = llroundl((ld)scale * p[k]);
}

void encode_coeffs(const Params& P, const double* m, int n_used, double scale, int64_t* out) {
  std::vector<ld> p;
  encode_embed(P, m, n_used, p);
  encode_round(p, scale, out);
}

// m_j = Re sum_k c_k zeta^(5^j k) / scale
void decode_coeffs(const Params& P, const long double* c, double scale, double* out, int n) {
  const int N = P.N;
  const size_t M2 = 2 * (size_t)N;
  std::vector<ld> re(M2, 0.0L), im(M2, 0.0L);
  for (int k = 0; k < N; ++k) re[k] = c[k];
  dif_fft(re, im, +1);
  const int bits = P.logN + 1;
  u64 e = 1;
  for (int j = 0; j < n; ++j) {
    out[j] = (double)(re[bitrev((size_t)e, bits)] / (ld)scale);
    e = (e * 5) % M2;
  }
}

}  // namespace ppst
