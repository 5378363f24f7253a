// boot_host.cpp -- the plaintexts of CKKS bootstrapping's linear transforms.
//
// Slot s of a CKKS plaintext holds m(xi_s), xi_s = zeta^(5^s mod 2N),
// zeta = exp(i pi / N).  As the n = N/2 values c_k + i c_{k+n} this is the
// n x n map U0[s, k] = xi_s^k (xi_s^n = i for every slot).  With the input in
// bit-reversed order U0 is a product of log2(n) butterfly layers ("special
// FFT", Cheon et al., cited for bootstrapping in Sec. 3.2): layer len pairs
// (x_j, x_{j+len/2}) of every block of len entries into
//   (x_j + w x_{j+len/2}, x_j - w x_{j+len/2}),  w = zeta^((n/len) (5^j mod 4 len)),
// so that SlotToCoeff is the layers len = 2 .. n in that order, and
// CoeffToSlot (U0^-1 = U0^H / n) is the conjugate-transposed layers, each
// halved, len = n .. 2.  A layer is a sum of diagonal matrices times slot
// rotations (offsets 0, +-len/2); a merged group of layers is again one,
// since diag(a) R^x diag(b) R^y = diag(a . R^x b) R^(x+y), (R^x v)_s = v_{s+x}.
//
// Everything here is binary128 (__float128 with libquadmath) so that every
// integer coefficient is the correctly rounded value of the exact real one
// (the rounding is off only for a value within about 2^-40 of a
// half-integer).
#include "boot_host.h"

#include <quadmath.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <stdexcept>
#include <thread>

namespace ppst {
namespace {

typedef __float128 R;

struct Cx {
  R re, im;
};
inline Cx operator+(Cx a, Cx b) { return {a.re + b.re, a.im + b.im}; }
inline Cx operator-(Cx a, Cx b) { return {a.re - b.re, a.im - b.im}; }
inline Cx operator*(Cx a, Cx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
inline Cx conj(Cx a) { return {a.re, -a.im}; }
inline Cx half(Cx a) { return {a.re / 2, a.im / 2}; }
inline bool is_zero(Cx a) { return a.re == 0 && a.im == 0; }

// zeta^t = exp(i pi t / N), t in [0, 2N)
struct Roots {
  int N;
  std::vector<Cx> z;
  explicit Roots(int n2) : N(n2), z(2 * (size_t)n2) {
    for (int t = 0; t < 2 * N; ++t) {
      const R a = M_PIq * (R)t / (R)N;
      z[t] = {cosq(a), sinq(a)};
    }
  }
  Cx pow(long e) const {
    const long m = 2L * N;
    e %= m;
    return z[e < 0 ? e + m : e];
  }
};

template <class F>
void parallel_for(size_t n, int threads, F&& f) {
  threads = std::max(1, std::min<int>(threads, (int)std::min<size_t>(n, 64)));
  if (threads == 1) {
    for (size_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<size_t> next(0);
  std::vector<std::thread> pool;
  for (int t = 0; t < threads; ++t)
    pool.emplace_back([&] {
      for (size_t i; (i = next.fetch_add(1)) < n;) f(i);
    });
  for (auto& th : pool) th.join();
}

// sum_k diag(D[k]) R^k over n slots (k reduced mod n)
typedef std::map<int, std::vector<Cx>> Diags;

std::vector<Cx>& diag(Diags& D, int off, int n) {
  off %= n;
  if (off < 0) off += n;
  auto it = D.find(off);
  if (it == D.end()) it = D.emplace(off, std::vector<Cx>((size_t)n, Cx{0, 0})).first;
  return it->second;
}

Diags layer(const Roots& Z, int len, bool inverse) {
  const int n = Z.N / 2, h = len / 2;
  std::vector<Cx> w(h);
  long e = 1;
  for (int j = 0; j < h; ++j) {
    w[j] = Z.pow((long)(n / len) * e);
    e = e * 5 % (4L * len);
  }
  Diags D;
  auto& d0 = diag(D, 0, n);
  auto& dp = diag(D, h, n);
  auto& dm = diag(D, -h, n);     // the same diagonal as dp when len = n
  const Cx one{1, 0};
  for (int s = 0; s < n; ++s) {
    const int p = s % len;
    if (!inverse) {
      if (p < h) {
        d0[s] = one;
        dp[s] = w[p];
      } else {
        dm[s] = one;
        d0[s] = Cx{0, 0} - w[p - h];
      }
    } else {
      // (L^H)[j][j] = 1, [j][j+h] = 1, [j+h][j] = conj w, [j+h][j+h] = -conj w; halved
      if (p < h) {
        d0[s] = half(one);
        dp[s] = half(one);
      } else {
        dm[s] = half(conj(w[p - h]));
        d0[s] = Cx{0, 0} - half(conj(w[p - h]));
      }
    }
  }
  return D;
}

// A B, the rows split over threads
Diags compose(const Diags& A, const Diags& B, int n, int threads) {
  Diags C;
  for (const auto& a : A)
    for (const auto& b : B) diag(C, a.first + b.first, n);
  const int chunk = 1024;
  const size_t nchunks = ((size_t)n + chunk - 1) / chunk;
  parallel_for(nchunks, threads, [&](size_t c) {
    const int s0 = (int)c * chunk, s1 = std::min(n, s0 + chunk);
    for (const auto& a : A)
      for (const auto& b : B) {
        std::vector<Cx>& out = C.find((a.first + b.first) % n)->second;
        for (int s = s0; s < s1; ++s) out[s] = out[s] + a.second[s] * b.second[(s + a.first) % n];
      }
  });
  return C;
}

Diags group_matrix(const Roots& Z, const BootGroup& g, int threads) {
  // the layers in the order they act: SlotToCoeff from len = 2^lo up,
  // CoeffToSlot from len = 2^hi down
  std::vector<int> order;
  for (int e = g.lo; e <= g.hi; ++e) order.push_back(e);
  if (g.inverse) std::reverse(order.begin(), order.end());
  Diags M = layer(Z, 1 << order[0], g.inverse != 0);
  for (size_t t = 1; t < order.size(); ++t)
    M = compose(layer(Z, 1 << order[t], g.inverse != 0), M, Z.N / 2, threads);
  return M;
}

R factor_q(const BootGroup& g, const BootFactor& f) {
  R c = 1;
  if (g.ckind == 1) c = (R)f.scale_top / ((R)2 * (R)f.K * (R)f.q0);
  if (g.ckind == 2) c = expq(logq((R)f.q0 / ((R)2 * M_PIq * (R)f.scale0)) / (R)f.nsplit);
  return (R)f.scale_out * (R)f.q_l / (R)f.scale_in * c;
}

// coefficient k = round_half_away(S (2/N) Re X_k), X_k = sum_s v_s xi_s^(-k):
// the slot exponents are odd, so X_k = zeta^(-k) Y_k with Y the N-point DFT
// (sign -1) of a_((e-1)/2) = v_s for e = 5^s mod 2N
void encode(const Roots& Z, const std::vector<Cx>& v, R S, int64_t* out) {
  const int N = Z.N, n = N / 2;
  int logN = 0;
  while ((1 << logN) < N) ++logN;
  std::vector<Cx> a((size_t)N, Cx{0, 0});
  long e = 1;
  for (int s = 0; s < n; ++s) {
    a[(e - 1) / 2] = v[s];
    e = e * 5 % (2L * N);
  }
  for (int i = 0; i < N; ++i) {
    int r = 0;
    for (int bit = 0; bit < logN; ++bit) r |= ((i >> bit) & 1) << (logN - 1 - bit);
    if (r > i) std::swap(a[i], a[r]);
  }
  for (int len = 2; len <= N; len <<= 1) {
    const int h = len / 2, step = N / len;
    for (int i = 0; i < N; i += len)
      for (int j = 0; j < h; ++j) {
        const Cx t = conj(Z.z[2 * (size_t)j * step]);     // exp(-2 pi i j step / N)
        const Cx x = a[i + j], y = a[i + j + h] * t;
        a[i + j] = x + y;
        a[i + j + h] = x - y;
      }
  }
  const R f = S * (R)2 / (R)N;
  const R lim = (R)9.2e18;
  for (int k = 0; k < N; ++k) {
    const Cx X = conj(Z.z[k]) * a[k];
    const R x = f * X.re;
    const R r = x >= 0 ? floorq(x + (R)0.5) : -floorq(-x + (R)0.5);
    if (!(r < lim && r > -lim)) throw std::runtime_error("bootstrapping plaintext coefficient leaves int64");
    out[k] = (int64_t)r;
  }
}

}  // namespace

double boot_group_factor(const BootGroup& g, const BootFactor& f) { return (double)factor_q(g, f); }

void boot_group_coeffs(int logN, const BootGroup& g, const BootFactor& f, int64_t* out,
                       uint8_t* used, int threads) {
  const int N = 1 << logN, n = N / 2;
  if (g.lo < 1 || g.hi < g.lo || (1 << g.hi) > n || g.u < 1 || g.b < 1 || g.G < 1)
    throw std::runtime_error("invalid bootstrapping group");
  const Roots Z(N);
  const Diags M = group_matrix(Z, g, threads);
  const R S = factor_q(g, f);
  const size_t cells = (size_t)g.G * g.b;
  std::vector<const std::vector<Cx>*> src(cells, nullptr);
  std::map<long, int> hits;
  size_t covered = 0;
  for (size_t c = 0; c < cells; ++c) {
    const long m = g.m0 + (long)c;                  // m0 + b j + i with c = j b + i
    long k = ((long)g.u * m) % n;
    if (k < 0) k += n;
    auto it = M.find((int)k);
    used[c] = 0;
    if (it == M.end()) continue;
    bool nz = false;
    for (const Cx& x : it->second) nz = nz || !is_zero(x);
    if (!nz) continue;
    src[c] = &it->second;
    used[c] = 1;
    ++covered;
    ++hits[k];
  }
  size_t nonzero = 0;
  for (const auto& d : M) {
    bool nz = false;
    for (const Cx& x : d.second) nz = nz || !is_zero(x);
    nonzero += nz;
  }
  if (covered != nonzero || hits.size() != covered)
    throw std::runtime_error("the baby-step grid does not cover each diagonal once");
  parallel_for(cells, threads, [&](size_t c) {
    if (!src[c]) return;
    const long j = (long)c / g.b;
    long rot = ((long)g.u * (g.m0 + (long)g.b * j)) % n;
    if (rot < 0) rot += n;
    std::vector<Cx> v((size_t)n);
    const std::vector<Cx>& d = *src[c];
    for (int s = 0; s < n; ++s) v[s] = d[(size_t)((s - rot + n) % n)];
    encode(Z, v, S, out + c * (size_t)N);
  });
}

}  // namespace ppst
