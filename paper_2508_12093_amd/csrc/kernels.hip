// kernels.hip -- element-wise, base-conversion, key-switching, rescale and
// sampling kernels.  All of them are HBM-streaming: one thread per residue
// (or per coefficient, looping over the limbs it produces), consecutive
// threads on consecutive words of a limb.
#include "dev.h"
#include "kern.h"
#include "tables.h"

namespace ppst {

namespace {

constexpr int kBlock = 256;

inline dim3 grid_for(size_t n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

struct ScalarArr {
  u64 v[kMaxLimbArgs];
  u64 vp[kMaxLimbArgs];
};

// ------------------------------------------------------------------ basic
__global__ void k_add_kernel(const u64* __restrict__ a, const u64* __restrict__ b, u64* out,
                             const Mod* mods, int logN, int nl, int npoly, size_t sa, size_t sb,
                             size_t so, int sub) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t per = (size_t)nl << logN;
  if (i >= per * npoly) return;
  int c = (int)(i / per);
  size_t r = i - (size_t)c * per;
  int t = (int)(r >> logN);
  u64 q = mods[t].q;
  u64 x = a[c * sa + r], y = b[c * sb + r];
  out[c * so + r] = sub ? subm(x, y, q) : addm(x, y, q);
}

__global__ void k_mul_scalar_kernel(const u64* __restrict__ a, u64* out, const Mod* mods, int logN,
                                    int nl, int npoly, size_t sa, size_t so, ScalarArr k) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t per = (size_t)nl << logN;
  if (i >= per * npoly) return;
  int c = (int)(i / per);
  size_t r = i - (size_t)c * per;
  int t = (int)(r >> logN);
  out[c * so + r] = mul_shoup(a[c * sa + r], k.v[t], k.vp[t], mods[t].q);
}

__global__ void k_add_scalar_kernel(const u64* __restrict__ a, u64* out, const Mod* mods, int logN,
                                    int nl, ScalarArr k) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ((size_t)nl << logN)) return;
  int t = (int)(i >> logN);
  out[i] = addm(a[i], k.v[t], mods[t].q);
}

__global__ void k_mul_poly_kernel(const u64* __restrict__ a, const u64* __restrict__ pt, u64* out,
                                  const Mod* mods, int logN, int nl, int npoly, size_t sa,
                                  size_t so) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t per = (size_t)nl << logN;
  if (i >= per * npoly) return;
  int c = (int)(i / per);
  size_t r = i - (size_t)c * per;
  int t = (int)(r >> logN);
  out[c * so + r] = mulm(a[c * sa + r], pt[r], mods[t]);
}

// up to kLinTerms weighted terms over up to kLinLimbs limbs per launch
constexpr int kLinTerms = 6;
constexpr int kLinLimbs = 32;
struct LinArgs {
  const u64* src[kLinTerms];    // term k: [2][l_k+1][N], poly stride ps[k]
  size_t ps[kLinTerms];
  u64 k[kLinTerms][kLinLimbs][2];   // (K_k mod q_t, Shoup companion), t = t0 + i
  u64* out;                     // [2][nl][N] (poly stride so)
  size_t so;
  int nterm, t0, nlimbs, accumulate;
};

__global__ void k_lincomb_kernel(LinArgs a, const Mod* __restrict__ mods, int logN) {
  const size_t N = (size_t)1 << logN;
  const size_t per = (size_t)a.nlimbs << logN;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= per) return;
  const int c = blockIdx.y;
  const int li = (int)(i >> logN);
  const int t = a.t0 + li;
  const size_t off = ((size_t)t << logN) + (i & (N - 1));
  const u64 q = mods[t].q;
  u64 v[kLinTerms];
#pragma unroll
  for (int k = 0; k < kLinTerms; ++k)
    v[k] = k < a.nterm ? a.src[k][c * a.ps[k] + off] : 0;
  u64* o = a.out + c * a.so + off;
  u64 s = a.accumulate ? *o : 0;
#pragma unroll
  for (int k = 0; k < kLinTerms; ++k)
    if (k < a.nterm) s = addm(s, mul_shoup(v[k], a.k[k][li][0], a.k[k][li][1], q), q);
  *o = s;
}

// operand pointers of up to kPtrBatch batch items, passed by value
struct PtrBatch {
  const u64* p[kPtrBatch];
};

__global__ void k_tensor_kernel(PtrBatch a, PtrBatch b, u64* d, const Mod* mods, int logN, int nl,
                                size_t sd) {
  size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  size_t per = (size_t)nl << logN;
  if (r >= per) return;
  const int bo = blockIdx.y;
  const u64* pa = a.p[bo];
  const u64* pb = b.p[bo];
  d += bo * sd;
  const Mod m = mods[r >> logN];
  u64 a0 = pa[r], a1 = pa[per + r], b0 = pb[r], b1 = pb[per + r];
  d[r] = mulm(a0, b0, m);
  Acc acc;
  acc.mac(a0, b1);
  acc.mac(a1, b0);
  d[per + r] = reduce128(acc.hi, acc.lo, m);
  d[2 * per + r] = mulm(a1, b1, m);
}

// slot j of the output reads slot galois_src(j)
__global__ void k_automorph_kernel(const u64* __restrict__ in, u64* out, int logN, int nrows,
                                   size_t sin, size_t sout, uint32_t g) {
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ((size_t)nrows << logN)) return;
  int row = (int)(i >> logN);
  uint32_t j = (uint32_t)(i & ((1u << logN) - 1));
  out[row * sout + j] = in[row * sin + galois_src(j, g, logN)];
}

// ----------------------------------------------------------- key switching
struct ModUpArgs {
  size_t sx, sext;
  int logN, nl, ne, pofs, alpha, nchunk;
};

constexpr int kModUpChunk = 8;   // target limbs per thread

// Thread (k, chunk, digit j): y_t = sum_i z_i (Qhat_i mod t) mod t for the
// chunk's target limbs t outside the digit (fast base conversion without
// correction), where z_i = x_i Qhat_i^-1 mod q_i is the input itself: the
// inverse transform that produces it ends with N^-1 Qhat_i^-1 instead of
// N^-1 (modup_ninv).  The loops run to MAXA with z_i = 0 past the digit (the
// table rows there are zero), so the loads of a thread issue together; the
// restrict-qualified table is read through the scalar unit.
template <int MAXA>
__global__ void __launch_bounds__(kBlock)
k_modup_kernel(const u64* __restrict__ xin, u64* __restrict__ extout,
               const Mod* __restrict__ mods, const u64* __restrict__ tab, ModUpArgs a) {
  const int N = 1 << a.logN;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int chunk = blockIdx.y % a.nchunk;
  const int j = blockIdx.y / a.nchunk;
  const int lo = j * a.alpha;
  const int hi = min(lo + a.alpha, a.nl);
  const int da = hi - lo;
  // the chunk's targets: the ne - da limbs outside [lo, hi), in order
  const int tfirst = chunk * kModUpChunk;
  const int ntarget = a.ne - da;
  if (tfirst >= ntarget) return;
  const u64* x = xin + blockIdx.z * a.sx;
  u64* ext = extout + blockIdx.z * a.sext + (size_t)j * a.ne * N;
  const u64* cst = tab + modup_digit_words(a.ne) * j;
  u64 xv[MAXA];
#pragma unroll
  for (int i = 0; i < MAXA; ++i) xv[i] = x[(size_t)(lo + min(i, da - 1)) * N + k];
  Split30 z[MAXA];
#pragma unroll
  for (int i = 0; i < MAXA; ++i) z[i] = Split30(i < da ? xv[i] : 0);
#pragma unroll
  for (int c = 0; c < kModUpChunk; ++c) {
    const int u = tfirst + c;
    if (u >= ntarget) continue;
    const int t = u < lo ? u : u + da;
    const int p = t < a.nl ? t : a.pofs + (t - a.nl);
    const u64* qhat = cst + 2 * kMaxAlpha + (size_t)t * kMaxAlpha;
    Acc30 acc;
#pragma unroll
    for (int i = 0; i < MAXA; ++i) {
      acc.mac(z[i], Split30(qhat[i]));
      if ((i & 7) == 7) acc.fold();
    }
    ext[(size_t)t * N + k] = acc.redc(mods[p]);   // the table is in Montgomery form
  }
}

struct InnerArgs {
  const u64* d;       // NTT-form input limbs [nl][N]
  const u64* ext;     // [beta][ne][N]
  const u64* key;     // [dnum][2][nprimes][N]
  u64* u;             // [2][ne][N]
  const Mod* mods;
  size_t sd, sext, su;
  int logN, nl, ne, beta, alpha, pofs, nprimes, nbatch;
  uint32_t gd, gext;  // read d / ext through X -> X^g (0: as stored)
  // products: limb q_l of u also receives (P mod q_l) d_c,l, with the tensor
  // d at pd ([item][3][nl][N], stride spd; null otherwise)
  const u64* pd;
  size_t spd;
  u64 pmod, pmods;    // P mod q_l and its Shoup companion
};

constexpr int kMaxDigits = 8;

// ITEMS batch items per thread: one key load serves all of them
template <int ITEMS>
__global__ void __launch_bounds__(kBlock) k_ks_inner_kernel(InnerArgs a) {
  constexpr int kInnerItems = ITEMS;
  const size_t N = (size_t)1 << a.logN;
  size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= (size_t)a.ne * N) return;
  const int t = (int)(r >> a.logN);
  const size_t k = r & (N - 1);
  const int p = t < a.nl ? t : a.pofs + (t - a.nl);
  const int b0 = blockIdx.y * kInnerItems;
  const int nb = min(kInnerItems, a.nbatch - b0);
  // digit holding limb t; with d == null the digits' own limbs are read from ext too
  const int own = (a.d != nullptr && t < a.nl) ? t / a.alpha : -1;
  const size_t kd = galois_src((uint32_t)k, a.gd, a.logN);
  const size_t kx = galois_src((uint32_t)k, a.gext, a.logN);
  Acc30 s0[kInnerItems], s1[kInnerItems];
  for (int j = 0; j < a.beta; ++j) {
    const Split30 kb(a.key[((size_t)(2 * j) * a.nprimes + p) * N + k]);
    const Split30 ka(a.key[((size_t)(2 * j + 1) * a.nprimes + p) * N + k]);
    const u64* src = (j == own) ? a.d + (size_t)t * N + kd : a.ext + ((size_t)j * a.ne + t) * N + kx;
    const size_t stride = (j == own) ? a.sd : a.sext;
    u64 ev[kInnerItems];
#pragma unroll
    for (int q = 0; q < kInnerItems; ++q) ev[q] = src[(size_t)(b0 + min(q, nb - 1)) * stride];
#pragma unroll
    for (int q = 0; q < kInnerItems; ++q) {
      const Split30 e(ev[q]);
      s0[q].mac(e, kb);
      s1[q].mac(e, ka);
    }
    if ((j & 7) == 7) {
#pragma unroll
      for (int q = 0; q < kInnerItems; ++q) {
        s0[q].fold();
        s1[q].fold();
      }
    }
  }
  const Mod m = a.mods[p];
  const bool prep = a.pd != nullptr && t == a.nl - 1;
#pragma unroll
  for (int q = 0; q < kInnerItems; ++q) {
    if (q < nb) {
      u64* u = a.u + (size_t)(b0 + q) * a.su;
      u64 v0 = s0[q].reduce(m), v1 = s1[q].reduce(m);
      if (prep) {
        const u64* d = a.pd + (size_t)(b0 + q) * a.spd + (size_t)t * N + k;
        v0 = addm(v0, mul_shoup(d[0], a.pmod, a.pmods, m.q), m.q);
        v1 = addm(v1, mul_shoup(d[(size_t)a.nl * N], a.pmod, a.pmods, m.q), m.q);
      }
      u[(size_t)t * N + k] = v0;
      u[((size_t)a.ne + t) * N + k] = v1;
    }
  }
}

// Long batches: one thread per (extended limb, coefficient) for the whole
// batch.  The key's 2 beta values there are read once into registers, then
// the batch is taken ITEMS items at a time (the items' loads of one digit
// issued together), so the key crosses HBM once per launch whatever the batch
// size.  (The register copy of the key costs occupancy, which the short
// batches above, bound by HBM, cannot spare.)
template <int ITEMS>
__global__ void __launch_bounds__(kBlock) k_ks_inner_loop_kernel(InnerArgs a) {
  const size_t N = (size_t)1 << a.logN;
  size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= (size_t)a.ne * N) return;
  const int t = (int)(r >> a.logN);
  const size_t k = r & (N - 1);
  const int p = t < a.nl ? t : a.pofs + (t - a.nl);
  // digit holding limb t; with d == null the digits' own limbs are read from ext too
  const int own = (a.d != nullptr && t < a.nl) ? t / a.alpha : -1;
  const size_t kd = galois_src((uint32_t)k, a.gd, a.logN);
  const size_t kx = galois_src((uint32_t)k, a.gext, a.logN);
  Split30 kb[kMaxDigits], ka[kMaxDigits];
#pragma unroll
  for (int j = 0; j < kMaxDigits; ++j) {
    if (j < a.beta) {
      kb[j] = Split30(a.key[((size_t)(2 * j) * a.nprimes + p) * N + k]);
      ka[j] = Split30(a.key[((size_t)(2 * j + 1) * a.nprimes + p) * N + k]);
    }
  }
  const Mod m = a.mods[p];
  const bool prep = a.pd != nullptr && t == a.nl - 1;
  for (int b0 = 0; b0 < a.nbatch; b0 += ITEMS) {
    const int nb = min(ITEMS, a.nbatch - b0);
    Acc30 s0[ITEMS], s1[ITEMS];
#pragma unroll
    for (int j = 0; j < kMaxDigits; ++j) {
      if (j < a.beta) {
        const u64* src = (j == own) ? a.d + (size_t)t * N + kd : a.ext + ((size_t)j * a.ne + t) * N + kx;
        const size_t stride = (j == own) ? a.sd : a.sext;
        u64 ev[ITEMS];
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) ev[q] = src[(size_t)(b0 + min(q, nb - 1)) * stride];
#pragma unroll
        for (int q = 0; q < ITEMS; ++q) {
          const Split30 e(ev[q]);
          s0[q].mac(e, kb[j]);
          s1[q].mac(e, ka[j]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < ITEMS; ++q) {
      if (q < nb) {
        u64* u = a.u + (size_t)(b0 + q) * a.su;
        u64 v0 = s0[q].reduce(m), v1 = s1[q].reduce(m);
        if (prep) {
          const u64* d = a.pd + (size_t)(b0 + q) * a.spd + (size_t)t * N + k;
          v0 = addm(v0, mul_shoup(d[0], a.pmod, a.pmods, m.q), m.q);
          v1 = addm(v1, mul_shoup(d[(size_t)a.nl * N], a.pmod, a.pmods, m.q), m.q);
        }
        u[(size_t)t * N + k] = v0;
        u[((size_t)a.ne + t) * N + k] = v1;
      }
    }
  }
}

struct InnerMultiArgs {
  PtrsIn d;                         // per item: NTT-form input [nl][N]
  const u64* ext;                   // [item][beta][ne][N]
  const u64* key[kMaxHoistKeys];    // [dnum][2][nprimes][N] each
  uint32_t g[kMaxHoistKeys];
  u64* u;                           // [item][2][ne][N]
  const Mod* mods;
  // per item (or null): limb q_t of u0 also receives (P mod q_t) times the
  // sum of w's limb t read through every g (w in NTT form [nl][N])
  PtrsIn w;
  const u64* pmod;                  // (P mod q_i, Shoup companion), i = 0..L
  size_t sext, su;
  int logN, nl, ne, beta, alpha, pofs, nprimes, nbatch, nkeys;
};

// Several keys' inner products summed per output element.  Acc30 takes at
// most 8 terms between folds and 16 in all, so the running sums are folded
// before a key would pass 8 terms and reduced into r0/r1 before 16.
template <int ITEMS>
__global__ void __launch_bounds__(kBlock) k_ks_inner_multi_kernel(InnerMultiArgs a) {
  const size_t N = (size_t)1 << a.logN;
  size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= (size_t)a.ne * N) return;
  const int t = (int)(r >> a.logN);
  const uint32_t k = (uint32_t)(r & (N - 1));
  const int p = t < a.nl ? t : a.pofs + (t - a.nl);
  const int b0 = blockIdx.y * ITEMS;
  const int nb = min(ITEMS, a.nbatch - b0);
  const int own = t < a.nl ? t / a.alpha : -1;
  const Mod m = a.mods[p];
  Acc30 s0[ITEMS], s1[ITEMS];
  u64 r0[ITEMS], r1[ITEMS];
#pragma unroll
  for (int q = 0; q < ITEMS; ++q) r0[q] = r1[q] = 0;
  int since = 0, total = 0;
  for (int h = 0; h < a.nkeys; ++h) {
    if (total + a.beta > 16) {
#pragma unroll
      for (int q = 0; q < ITEMS; ++q) {
        r0[q] = addm(r0[q], s0[q].reduce(m), m.q);
        r1[q] = addm(r1[q], s1[q].reduce(m), m.q);
        s0[q] = Acc30();
        s1[q] = Acc30();
      }
      total = since = 0;
    } else if (since + a.beta > 8) {
#pragma unroll
      for (int q = 0; q < ITEMS; ++q) {
        s0[q].fold();
        s1[q].fold();
      }
      since = 0;
    }
    const size_t kk = galois_src(k, a.g[h], a.logN);
    const u64* key = a.key[h];
    for (int j = 0; j < a.beta; ++j) {
      const Split30 kb(key[((size_t)(2 * j) * a.nprimes + p) * N + k]);
      const Split30 ka(key[((size_t)(2 * j + 1) * a.nprimes + p) * N + k]);
      u64 ev[ITEMS];
#pragma unroll
      for (int q = 0; q < ITEMS; ++q) {
        const int b = b0 + min(q, nb - 1);
        ev[q] = (j == own) ? a.d.p[b][(size_t)t * N + kk]
                           : a.ext[(size_t)b * a.sext + ((size_t)j * a.ne + t) * N + kk];
      }
#pragma unroll
      for (int q = 0; q < ITEMS; ++q) {
        const Split30 e(ev[q]);
        s0[q].mac(e, kb);
        s1[q].mac(e, ka);
      }
    }
    since += a.beta;
    total += a.beta;
  }
  u64 wsum[ITEMS];
#pragma unroll
  for (int q = 0; q < ITEMS; ++q) {
    wsum[q] = 0;
    const u64* w = a.w.p[b0 + min(q, nb - 1)];
    if (w && t < a.nl) {
      for (int h = 0; h < a.nkeys; ++h)
        wsum[q] = addm(wsum[q], w[(size_t)t * N + galois_src(k, a.g[h], a.logN)], m.q);
      wsum[q] = mul_shoup(wsum[q], a.pmod[2 * t], a.pmod[2 * t + 1], m.q);
    }
  }
#pragma unroll
  for (int q = 0; q < ITEMS; ++q) {
    if (q < nb) {
      u64* u = a.u + (size_t)(b0 + q) * a.su;
      u[(size_t)t * N + k] = addm(addm(r0[q], s0[q].reduce(m), m.q), wsum[q], m.q);
      u[((size_t)a.ne + t) * N + k] = addm(r1[q], s1[q].reduce(m), m.q);
    }
  }
}

struct ModDownArgs {
  size_t su, sconv;
  int logN, nl, ne, K, L, nchunk;
};

constexpr int kModDownChunk = 8;   // output limbs per thread

// w_k = (z_k + h) Phat_k^-1 mod p_k for the special limbs z of one polynomial
// in coefficient form (w_k = 0 for k >= K), split for Acc30.  The inverse
// NTT that produced the limbs ended with N^-1 Phat_k^-1 (md_ninv), so they
// hold z_k Phat_k^-1 and a weight is that plus h Phat_k^-1.
template <int MAXK>
__device__ __forceinline__ void moddown_weights(const u64* __restrict__ u, int nl, int K, int L,
                                                int N, int k, const Mod* __restrict__ mods,
                                                const u64* __restrict__ md, Split30* w) {
  const MdLayout lay(K, L);
  u64 zv[MAXK];
#pragma unroll
  for (int i = 0; i < MAXK; ++i) zv[i] = u[(size_t)(nl + min(i, K - 1)) * N + k];
#pragma unroll
  for (int i = 0; i < MAXK; ++i) {
    const int kk = min(i, K - 1);
    const u64 v = addm(zv[i], md[lay.hphinv(kk)], mods[L + 1 + kk].q);
    w[i] = Split30(i < K ? v : 0);
  }
}

// Thread (k, chunk, poly): conv_i = sum_k w_k (Phat_k mod q_i) - h mod q_i for
// the chunk's limbs i.
template <int MAXK>
__global__ void __launch_bounds__(kBlock)
k_moddown_conv_kernel(const u64* __restrict__ uin, u64* __restrict__ convout,
                      const Mod* __restrict__ mods, const u64* __restrict__ md, ModDownArgs a) {
  const int N = 1 << a.logN;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int chunk = blockIdx.y % a.nchunk;
  const int c = blockIdx.y / a.nchunk;
  const int ifirst = chunk * kModDownChunk;
  if (ifirst >= a.nl) return;
  const u64* u = uin + blockIdx.z * a.su + (size_t)c * a.ne * N;
  u64* conv = convout + blockIdx.z * a.sconv + (size_t)c * a.nl * N;
  const MdLayout lay(a.K, a.L);
  Split30 w[MAXK];
  moddown_weights<MAXK>(u, a.nl, a.K, a.L, N, k, mods, md, w);
#pragma unroll
  for (int cc = 0; cc < kModDownChunk; ++cc) {
    const int i = ifirst + cc;
    if (i >= a.nl) continue;
    const Mod m = mods[i];
    Acc30 acc;
#pragma unroll
    for (int j = 0; j < MAXK; ++j) acc.mac(w[j], Split30(md[lay.phat(j, i)]));
    u64 v = acc.redc(m);   // Phat_k mod q_i is stored in Montgomery form
    conv[(size_t)i * N + k] = subm(v, md[lay.hmod(i)], m.q);
  }
}

// ------------------------------------------- ModDown and rescale together
constexpr int kMdrChunk = 8;   // output limbs per thread

template <int MAXK>
__global__ void __launch_bounds__(kBlock)
k_mdr_corr_kernel(const u64* __restrict__ u, u64* __restrict__ corr, const Mod* __restrict__ mods,
                  const u64* __restrict__ md, const u64* __restrict__ rc, int K, int L, int logN,
                  int level, int ne, int nchunk, size_t su, size_t sc) {
  const int N = 1 << logN;
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const int chunk = blockIdx.y % nchunk;
  const int c = blockIdx.y / nchunk;
  const int ifirst = chunk * kMdrChunk;
  if (ifirst >= level) return;
  const u64* uc = u + blockIdx.z * su + (size_t)c * ne * N;
  u64* cc = corr + blockIdx.z * sc + (size_t)c * level * N;
  const MdLayout lay(K, L);
  const int nl = level + 1;
  Split30 w[MAXK];
  moddown_weights<MAXK>(uc, nl, K, L, N, k, mods, md, w);
  // the q_l limb of d + ModDown(u), in coefficient form, and its centred lift
  const Mod ml = mods[level];
  u64 cl;
  {
    Acc30 acc;
#pragma unroll
    for (int j = 0; j < MAXK; ++j) acc.mac(w[j], Split30(md[lay.phat(j, level)]));
    u64 conv = acc.redc(ml);
    u64 v = subm(addm(uc[(size_t)level * N + k], md[lay.hmod(level)], ml.q), conv, ml.q);
    cl = mul_shoup(v, md[lay.pinv(level)], md[lay.pinv(level) + 1], ml.q);
  }
  const bool neg = cl > (ml.q >> 1);
  // unrolled with a uniform guard (no early exit), so every target's
  // constants load up front
#pragma unroll
  for (int ii = 0; ii < kMdrChunk; ++ii) {
    const int i = ifirst + ii;
    if (i >= level) continue;
    const Mod m = mods[i];
    Acc30 acc;
#pragma unroll
    for (int j = 0; j < MAXK; ++j) acc.mac(w[j], Split30(md[lay.phatp(j, i)]));
    // (h - conv) P^-1 with P^-1 folded into the constants
    u64 v = subm(md[lay.hpinv(i)], acc.redc(m), m.q);
    u64 t = reduce_below(cl, ml.q, m);
    if (neg) t = subm(t, rc[3 * i + 2], m.q);       // t = c_l - q_l when c_l > q_l / 2
    cc[(size_t)i * N + k] = subm(v, t, m.q);
  }
}

// ------------------------------------------------------------------ rescale
__global__ void k_rescale_conv_kernel(const u64* __restrict__ top, u64* tmp, const Mod* mods,
                                      const u64* rc, int logN, int level, size_t ts, int mulk,
                                      u64 kl, u64 klp) {
  const size_t N = (size_t)1 << logN;
  size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= (size_t)level * N) return;
  const int c = blockIdx.y;
  const int i = (int)(r >> logN);
  const size_t k = r & (N - 1);
  const u64 ql = mods[level].q;
  u64 x = top[c * ts + k];
  if (mulk) x = mul_shoup(x, kl, klp, ql);
  const Mod m = mods[i];
  u64 v = reduce_below(x, ql, m);
  if (x > (ql >> 1)) v = subm(v, rc[3 * i + 2], m.q);   // centred: x - q_l
  tmp[((size_t)c * level << logN) + r] = v;
}

// ----------------------------------------------------------------- sampling
__device__ __forceinline__ u64 sm_mix(u64 z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
constexpr u64 kGamma = 0x9E3779B97F4A7C15ULL;
// word i of the stream whose state starts at key
__device__ __forceinline__ u64 sm_word(u64 key, u64 i) { return sm_mix(key + (i + 1) * kGamma); }

__global__ void k_small_to_rns_kernel(const int32_t* s, u64* out, const Mod* mods, int logN,
                                      int nl, int nq, int pofs) {
  size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ((size_t)nl << logN)) return;
  int t = (int)(r >> logN);
  int p = t < nq ? t : pofs + (t - nq);
  u64 q = mods[p].q;
  int32_t v = s[r & (((size_t)1 << logN) - 1)];
  out[r] = v >= 0 ? (u64)v : q - (u64)(-(int64_t)v);
}

__global__ void k_int64_to_rns_kernel(const int64_t* s, u64* out, const Mod* mods, int logN,
                                      int nl, int nq, int pofs) {
  size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ((size_t)nl << logN)) return;
  int t = (int)(r >> logN);
  int p = t < nq ? t : pofs + (t - nq);
  const Mod m = mods[p];
  int64_t v = s[r & (((size_t)1 << logN) - 1)];
  if (v >= 0) {
    out[r] = reduce64((u64)v, m);
  } else {
    u64 w = reduce64((u64)(-(v + 1)), m);    // (-v - 1) mod q, safe at INT64_MIN
    out[r] = m.q - 1 - w;
  }
}

struct KeyArr {
  u64 k[kMaxLimbArgs];
};

__global__ void k_uniform_kernel(u64* out, const Mod* mods, int logN, int nl, int nq, int pofs,
                                 KeyArr keys) {
  size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ((size_t)nl << logN)) return;
  int t = (int)(r >> logN);
  int p = t < nq ? t : pofs + (t - nq);
  u64 k = r & (((size_t)1 << logN) - 1);
  u64 hi = sm_word(keys.k[t], 2 * k), lo = sm_word(keys.k[t], 2 * k + 1);
  const Mod m = mods[p];
  // (hi 2^64 + lo) mod q = ((hi mod q) 2^64 + lo) mod q, first factor < 2^60
  out[r] = reduce128(reduce64(hi, m), lo, m);
}

__global__ void k_ternary_kernel(int32_t* out, int N, u64 key) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  u64 u = sm_word(key, (u64)k);
  out[k] = (int32_t)mulhi(u, 3) - 1;
}

struct DgArr {
  u64 thr[kDgMax];
};

__global__ void k_dg_kernel(int32_t* out, int N, u64 key, DgArr d) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  u64 u = sm_word(key, 2 * (u64)k);
  u64 sg = sm_word(key, 2 * (u64)k + 1);
  int mag = kDgMax;
  for (int x = kDgMax - 1; x >= 0; --x)
    if (u < d.thr[x]) mag = x;
  out[k] = (mag != 0 && (sg >> 63)) ? -mag : mag;
}

__global__ void k_keyform_kernel(const u64* a, const u64* s, const u64* e, const u64* sp,
                                 ScalarArr f, u64* out, const Mod* mods, int logN, int nl,
                                 int nq, int pofs, int use_sp) {
  size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ((size_t)nl << logN)) return;
  int t = (int)(r >> logN);
  int p = t < nq ? t : pofs + (t - nq);
  const Mod m = mods[p];
  size_t kk = r & (((size_t)1 << logN) - 1);
  size_t so = ((size_t)p << logN) + kk;   // s and sp are indexed by prime
  u64 v = subm(e[r], mulm(a[r], s[so], m), m.q);
  if (use_sp && f.v[t]) v = addm(v, mul_shoup(sp[so], f.v[t], f.vp[t], m.q), m.q);
  out[r] = v;
}

// ModRaise: x [npoly][N] residues mod q_0 (coefficient form); out[c][t] the
// centred lift of x_c (in (-q_0/2, q_0/2]) mod q_t, t < nl
__global__ void k_mod_raise_kernel(const u64* __restrict__ x, u64* __restrict__ out,
                                   const Mod* __restrict__ mods, int logN, int nl, int npoly) {
  const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t per = (size_t)nl << logN;
  if (r >= per * npoly) return;
  const int c = (int)(r / per);
  const size_t rr = r - (size_t)c * per;
  const int t = (int)(rr >> logN);
  const u64 v = x[((size_t)c << logN) + (rr & (((size_t)1 << logN) - 1))];
  const u64 q0 = mods[0].q;
  const Mod m = mods[t];
  if (v > q0 / 2) {
    const u64 w = reduce64(q0 - v, m);      // the lift is -(q0 - v)
    out[r] = w ? m.q - w : 0;
  } else {
    out[r] = reduce64(v, m);
  }
}

// The inner sums of a baby-step giant-step product: for every giant step j,
// out_j = sum_i pt[j B + i] . baby_i (NTT form, both polynomials, limb t mod
// q_t); null plaintexts are skipped, null outputs not written.  Each thread
// holds its coefficient of the B baby steps in registers and reads each
// plaintext once.
constexpr int kBsgsMaxBaby = 16, kBsgsMaxCells = 64, kBsgsMaxGiant = 16;
struct BsgsArgs {
  const u64* baby[kBsgsMaxBaby];   // [2][nl][N] at polynomial stride ps_in
  const u64* pt[kBsgsMaxCells];    // [nl][N]
  u64* out[kBsgsMaxGiant];         // [2][nl][N] at polynomial stride ps_out
  size_t ps_in, ps_out;
  int G;
};

template <int B>
__global__ void k_bsgs_inner_kernel(BsgsArgs a, const Mod* __restrict__ mods, int logN, int nl) {
  const size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ((size_t)nl << logN)) return;
  const int c = blockIdx.y;
  const Mod m = mods[r >> logN];
  u64 x[B];
#pragma unroll
  for (int i = 0; i < B; ++i) x[i] = a.baby[i][(size_t)c * a.ps_in + r];
  for (int j = 0; j < a.G; ++j) {
    if (!a.out[j]) continue;
    u64 acc = 0;
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const u64* p = a.pt[j * B + i];
      if (p) acc = addm(acc, mulm(x[i], p[r], m), m.q);
    }
    a.out[j][(size_t)c * a.ps_out + r] = acc;
  }
}

__global__ void k_fma3_kernel(const u64* x, const u64* y, const u64* z, const u64* w, u64* out,
                              const Mod* mods, int logN, int nl) {
  size_t r = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= ((size_t)nl << logN)) return;
  const Mod m = mods[r >> logN];
  u64 v = addm(x[r], mulm(y[r], z[r], m), m.q);
  if (w) v = addm(v, w[r], m.q);
  out[r] = v;
}

__global__ void k_sum_kernel(PtrsIn src, int nterm, u64* out, int acc, const Mod* mods, int logN,
                             int nl, size_t W) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= W) return;
  const u64 q = mods[(i >> logN) % nl].q;
  u64 s = acc ? out[i] : 0;
  for (int k = 0; k < nterm; ++k) s = addm(s, src.p[k][i], q);
  out[i] = s;
}

__global__ void k_gather_rows_kernel(PtrsIn rows, u64* dst, size_t W, size_t ds) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= W) return;
  dst[(size_t)blockIdx.y * ds + k] = rows.p[blockIdx.y][k];
}

const Mod* M(const Shared& sh) { return (const Mod*)sh.tab.mods.p; }

ScalarArr scalars(const Shared& sh, const u64* k, const u64* kp, int nl) {
  ScalarArr s;
  for (int t = 0; t < nl; ++t) { s.v[t] = k[t]; s.vp[t] = kp ? kp[t] : 0; }
  return s;
}

}  // namespace

#define LAUNCH_CHECK() HIP_CHECK(hipGetLastError())

void k_add(const Shared& sh, const u64* a, const u64* b, u64* out, int npoly, int nl,
           size_t sa, size_t sb, size_t so, bool sub, hipStream_t st) {
  size_t n = (size_t)npoly * nl * sh.P.N;
  hipLaunchKernelGGL(k_add_kernel, grid_for(n), dim3(kBlock), 0, st, a, b, out, M(sh), sh.P.logN,
                     nl, npoly, sa, sb, so, (int)sub);
  LAUNCH_CHECK();
}

void k_sum(const Shared& sh, const u64* const* src, int nterm, u64* out, int npoly, int nl,
           hipStream_t st) {
  if (nterm < 1) PPST_THROW(ST_EINVAL, "empty sum");
  const size_t W = (size_t)npoly * nl * sh.P.N;
  for (int k0 = 0; k0 < nterm; k0 += kPtrBatch) {
    const int nk = std::min(kPtrBatch, nterm - k0);
    PtrsIn p{};
    for (int i = 0; i < nk; ++i) p.p[i] = src[k0 + i];
    hipLaunchKernelGGL(k_sum_kernel, grid_for(W), dim3(kBlock), 0, st, p, nk, out, (int)(k0 > 0),
                       M(sh), sh.P.logN, nl, W);
    LAUNCH_CHECK();
  }
}

void k_gather_rows(const Shared& sh, const u64* const* rows, u64* dst, int nrows, hipStream_t st,
                   size_t row_words, size_t dst_stride) {
  const size_t W = row_words ? row_words : (size_t)sh.P.N;
  const size_t ds = dst_stride ? dst_stride : W;
  if (ds < W) PPST_THROW(ST_EINVAL, "gathered rows would overlap");
  for (int r0 = 0; r0 < nrows; r0 += kPtrBatch) {
    const int nr = std::min(kPtrBatch, nrows - r0);
    PtrsIn p{};
    for (int i = 0; i < nr; ++i) {
      if (!rows[r0 + i]) PPST_THROW(ST_EINVAL, "missing row");
      p.p[i] = rows[r0 + i];
    }
    dim3 g = grid_for(W);
    g.y = nr;
    hipLaunchKernelGGL(k_gather_rows_kernel, g, dim3(kBlock), 0, st, p, dst + (size_t)r0 * ds, W,
                       ds);
    LAUNCH_CHECK();
  }
}

void k_lincomb(const Shared& sh, const u64* const* src, const size_t* ps, const u64* k,
               const u64* kp, int nterm, int nl, u64* out, size_t so, hipStream_t st) {
  if (nterm < 1 || nl < 1) PPST_THROW(ST_EINVAL, "empty linear combination");
  for (int t0 = 0; t0 < nl; t0 += kLinLimbs) {
    const int nlim = std::min(kLinLimbs, nl - t0);
    for (int k0 = 0; k0 < nterm; k0 += kLinTerms) {
      LinArgs a{};
      a.nterm = std::min(kLinTerms, nterm - k0);
      for (int j = 0; j < a.nterm; ++j) {
        a.src[j] = src[k0 + j];
        a.ps[j] = ps[k0 + j];
        for (int i = 0; i < nlim; ++i) {
          a.k[j][i][0] = k[(size_t)(k0 + j) * nl + t0 + i];
          a.k[j][i][1] = kp[(size_t)(k0 + j) * nl + t0 + i];
        }
      }
      a.out = out;
      a.so = so;
      a.t0 = t0;
      a.nlimbs = nlim;
      a.accumulate = k0 > 0;
      dim3 g = grid_for((size_t)nlim * sh.P.N);
      g.y = 2;
      hipLaunchKernelGGL(k_lincomb_kernel, g, dim3(kBlock), 0, st, a, M(sh), sh.P.logN);
      LAUNCH_CHECK();
    }
  }
}

void k_mul_scalar(const Shared& sh, const u64* a, u64* out, int npoly, int nl, size_t sa,
                  size_t so, const u64* k, const u64* kp, hipStream_t st) {
  if (nl > kMaxLimbArgs) PPST_THROW(ST_EINVAL, "too many limbs");
  size_t n = (size_t)npoly * nl * sh.P.N;
  hipLaunchKernelGGL(k_mul_scalar_kernel, grid_for(n), dim3(kBlock), 0, st, a, out, M(sh),
                     sh.P.logN, nl, npoly, sa, so, scalars(sh, k, kp, nl));
  LAUNCH_CHECK();
}

void k_add_scalar(const Shared& sh, const u64* a, u64* out, int nl, const u64* k, hipStream_t st) {
  size_t n = (size_t)nl * sh.P.N;
  hipLaunchKernelGGL(k_add_scalar_kernel, grid_for(n), dim3(kBlock), 0, st, a, out, M(sh),
                     sh.P.logN, nl, scalars(sh, k, nullptr, nl));
  LAUNCH_CHECK();
}

void k_mul_poly(const Shared& sh, const u64* a, const u64* pt, u64* out, int npoly, int nl,
                size_t sa, size_t so, hipStream_t st) {
  size_t n = (size_t)npoly * nl * sh.P.N;
  hipLaunchKernelGGL(k_mul_poly_kernel, grid_for(n), dim3(kBlock), 0, st, a, pt, out, M(sh),
                     sh.P.logN, nl, npoly, sa, so);
  LAUNCH_CHECK();
}

void k_tensor(const Shared& sh, const u64* const* a, const u64* const* b, u64* d, int nl,
              int nbatch, size_t sd, hipStream_t st) {
  size_t n = (size_t)nl * sh.P.N;
  for (int b0 = 0; b0 < nbatch; b0 += kPtrBatch) {
    const int nb = std::min(kPtrBatch, nbatch - b0);
    PtrBatch pa{}, pb{};
    for (int i = 0; i < nb; ++i) {
      pa.p[i] = a[b0 + i];
      pb.p[i] = b[b0 + i];
    }
    dim3 g = grid_for(n);
    g.y = nb;
    hipLaunchKernelGGL(k_tensor_kernel, g, dim3(kBlock), 0, st, pa, pb, d + (size_t)b0 * sd, M(sh),
                       sh.P.logN, nl, sd);
    LAUNCH_CHECK();
  }
}

void k_automorph(const Shared& sh, const u64* in, u64* out, int nrows, size_t sin, size_t sout,
                 u64 g, hipStream_t st) {
  size_t n = (size_t)nrows * sh.P.N;
  hipLaunchKernelGGL(k_automorph_kernel, grid_for(n), dim3(kBlock), 0, st, in, out, sh.P.logN,
                     nrows, sin, sout, g);
  LAUNCH_CHECK();
}

void k_modup(const Shared& sh, const u64* x, u64* ext, int level, int nbatch, size_t sx,
             size_t sext, hipStream_t st) {
  const Params& P = sh.P;
  ModUpArgs a;
  a.sx = sx;
  a.sext = sext;
  a.logN = P.logN;
  a.nl = level + 1;
  a.ne = level + 1 + P.K;
  a.pofs = P.L + 1;
  a.alpha = P.alpha;
  const int beta = P.beta(level);
  const u64* tab = modup_table(sh, level);
  // the digit with the fewest limbs has the most targets
  int most = 0;
  for (int j = 0; j < beta; ++j) most = std::max(most, a.ne - (P.digit_hi(j, level) - P.digit_lo(j)));
  a.nchunk = (most + kModUpChunk - 1) / kModUpChunk;
  dim3 g = grid_for(P.N);
  g.y = a.nchunk * beta;
  g.z = nbatch;
  if (P.alpha <= 4)
    hipLaunchKernelGGL(k_modup_kernel<4>, g, dim3(kBlock), 0, st, x, ext, M(sh), tab, a);
  else if (P.alpha == 7)   // the bootstrappable presets' digits: no padding terms
    hipLaunchKernelGGL(k_modup_kernel<7>, g, dim3(kBlock), 0, st, x, ext, M(sh), tab, a);
  else if (P.alpha <= 9)
    hipLaunchKernelGGL(k_modup_kernel<9>, g, dim3(kBlock), 0, st, x, ext, M(sh), tab, a);
  else if (P.alpha <= kMaxAlpha)
    hipLaunchKernelGGL(k_modup_kernel<16>, g, dim3(kBlock), 0, st, x, ext, M(sh), tab, a);
  else
    PPST_THROW(ST_EINVAL, "digit size above 16 limbs");
  LAUNCH_CHECK();
}

void k_ks_inner_multi(const Shared& sh, const u64* const* d, const u64* ext,
                      const u64* const* keys, const uint32_t* g, int nkeys, u64* u, int level,
                      int nbatch, size_t sext, size_t su, hipStream_t st, const u64* const* w) {
  const Params& P = sh.P;
  if (nkeys < 1 || nkeys > kMaxHoistKeys) PPST_THROW(ST_EINVAL, "hoisted key count out of range");
  if (nbatch < 1 || nbatch > kPtrBatch) PPST_THROW(ST_EINVAL, "batch out of range");
  if (P.beta(level) > 8) PPST_THROW(ST_EINVAL, "more than 8 digits");
  InnerMultiArgs a{};
  for (int i = 0; i < nbatch; ++i) {
    if (!d[i]) PPST_THROW(ST_EINVAL, "missing input polynomial");
    a.d.p[i] = d[i];
    a.w.p[i] = w ? w[i] : nullptr;
  }
  a.pmod = sh.tab.moddown.p + MdLayout(P.K, P.L).pmod(0);
  for (int h = 0; h < nkeys; ++h) {
    if (!keys[h] || g[h] == 0 || (g[h] & 1) == 0 || g[h] >= 2u * (uint32_t)P.N)
      PPST_THROW(ST_EINVAL, "hoisted key or Galois element invalid");
    a.key[h] = keys[h];
    a.g[h] = g[h];
  }
  a.ext = ext;
  a.u = u;
  a.mods = M(sh);
  a.sext = sext;
  a.su = su;
  a.logN = P.logN;
  a.nl = level + 1;
  a.ne = level + 1 + P.K;
  a.beta = P.beta(level);
  a.alpha = P.alpha;
  a.pofs = P.L + 1;
  a.nprimes = P.nprimes;
  a.nbatch = nbatch;
  a.nkeys = nkeys;
  // items per thread: the keys are read once per group of items
  dim3 gr = grid_for((size_t)a.ne * P.N);
  if (nbatch == 5) {
    hipLaunchKernelGGL(k_ks_inner_multi_kernel<5>, gr, dim3(kBlock), 0, st, a);
  } else if (nbatch == 4) {
    hipLaunchKernelGGL(k_ks_inner_multi_kernel<4>, gr, dim3(kBlock), 0, st, a);
  } else if (nbatch >= 3) {
    gr.y = (nbatch + 2) / 3;
    hipLaunchKernelGGL(k_ks_inner_multi_kernel<3>, gr, dim3(kBlock), 0, st, a);
  } else if (nbatch == 2) {
    hipLaunchKernelGGL(k_ks_inner_multi_kernel<2>, gr, dim3(kBlock), 0, st, a);
  } else {
    hipLaunchKernelGGL(k_ks_inner_multi_kernel<1>, gr, dim3(kBlock), 0, st, a);
  }
  LAUNCH_CHECK();
}

void k_ks_inner(const Shared& sh, const u64* d, const u64* ext, const u64* key, u64* u, int level,
                int nbatch, size_t sd, size_t sext, size_t su, uint32_t gd, uint32_t gext,
                hipStream_t st, const u64* prep_d, size_t prep_sd) {
  const Params& P = sh.P;
  InnerArgs a;
  a.gd = gd;
  a.gext = gext;
  a.pd = prep_d;
  a.spd = prep_sd;
  a.pmod = a.pmods = 0;
  if (prep_d) {
    a.pmod = sh.tab.pmod_host[2 * level];
    a.pmods = sh.tab.pmod_host[2 * level + 1];
  }
  a.d = d;
  a.ext = ext;
  a.key = key;
  a.u = u;
  a.mods = M(sh);
  a.sd = sd;
  a.sext = sext;
  a.su = su;
  a.logN = P.logN;
  a.nl = level + 1;
  a.ne = level + 1 + P.K;
  a.beta = P.beta(level);
  a.alpha = P.alpha;
  a.pofs = P.L + 1;
  a.nprimes = P.nprimes;
  a.nbatch = nbatch;
  if (a.beta > kMaxDigits) PPST_THROW(ST_EINVAL, "more than 8 key-switching digits");
  dim3 g = grid_for((size_t)a.ne * P.N);
  if (nbatch > 8) {
    hipLaunchKernelGGL(k_ks_inner_loop_kernel<4>, g, dim3(kBlock), 0, st, a);
  } else if (nbatch == 8) {
    hipLaunchKernelGGL(k_ks_inner_kernel<8>, g, dim3(kBlock), 0, st, a);
  } else if (nbatch >= 4) {
    g.y = (nbatch + 3) / 4;
    hipLaunchKernelGGL(k_ks_inner_kernel<4>, g, dim3(kBlock), 0, st, a);
  } else if (nbatch >= 2) {
    g.y = (nbatch + 1) / 2;
    hipLaunchKernelGGL(k_ks_inner_kernel<2>, g, dim3(kBlock), 0, st, a);
  } else {
    g.y = nbatch;
    hipLaunchKernelGGL(k_ks_inner_kernel<1>, g, dim3(kBlock), 0, st, a);
  }
  LAUNCH_CHECK();
}

void k_moddown_conv(const Shared& sh, const u64* u, u64* conv, int level, int nbatch, size_t su,
                    size_t sconv, hipStream_t st) {
  const Params& P = sh.P;
  ModDownArgs a;
  a.su = su;
  a.sconv = sconv;
  a.logN = P.logN;
  a.nl = level + 1;
  a.ne = level + 1 + P.K;
  a.K = P.K;
  a.L = P.L;
  a.nchunk = (a.nl + kModDownChunk - 1) / kModDownChunk;
  dim3 g = grid_for(P.N);
  g.y = 2 * a.nchunk;
  g.z = nbatch;
  const u64* md = sh.tab.moddown.p;
  if (P.K <= 4)
    hipLaunchKernelGGL(k_moddown_conv_kernel<4>, g, dim3(kBlock), 0, st, u, conv, M(sh), md, a);
  else if (P.K <= kMaxSpecial)
    hipLaunchKernelGGL(k_moddown_conv_kernel<8>, g, dim3(kBlock), 0, st, u, conv, M(sh), md, a);
  else
    PPST_THROW(ST_EINVAL, "more than 8 special primes");
  LAUNCH_CHECK();
}

void k_mdr_corr(const Shared& sh, const u64* u, u64* corr, int level, int nbatch, size_t su,
                size_t sc, hipStream_t st) {
  const Params& P = sh.P;
  const int nchunk = (level + kMdrChunk - 1) / kMdrChunk;
  dim3 g = grid_for(P.N);
  g.y = 2 * nchunk;
  g.z = nbatch;
  const u64* rc = rescale_table(sh, level);
  if (P.K <= 4)
    hipLaunchKernelGGL(k_mdr_corr_kernel<4>, g, dim3(kBlock), 0, st, u, corr, M(sh),
                       sh.tab.moddown.p, rc, P.K, P.L, P.logN, level, level + 1 + P.K, nchunk, su, sc);
  else if (P.K <= 8)
    hipLaunchKernelGGL(k_mdr_corr_kernel<8>, g, dim3(kBlock), 0, st, u, corr, M(sh),
                       sh.tab.moddown.p, rc, P.K, P.L, P.logN, level, level + 1 + P.K, nchunk, su, sc);
  else
    PPST_THROW(ST_EINVAL, "more than 8 special primes");
  LAUNCH_CHECK();
}

void k_rescale_conv(const Shared& sh, const u64* top, u64* tmp, int level, int npoly,
                    size_t top_stride, hipStream_t st, const u64* kl) {
  dim3 g = grid_for((size_t)level * sh.P.N);
  g.y = npoly;
  hipLaunchKernelGGL(k_rescale_conv_kernel, g, dim3(kBlock), 0, st, top, tmp, M(sh),
                     rescale_table(sh, level), sh.P.logN, level, top_stride, kl ? 1 : 0,
                     kl ? kl[0] : 0, kl ? kl[1] : 0);
  LAUNCH_CHECK();
}

void k_int64_to_rns(const Shared& sh, const int64_t* s, u64* out, int nl, int nq, int pofs,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_int64_to_rns_kernel, grid_for((size_t)nl * sh.P.N), dim3(kBlock), 0, st, s,
                     out, M(sh), sh.P.logN, nl, nq, pofs);
  LAUNCH_CHECK();
}

void k_small_to_rns(const Shared& sh, const int32_t* s, u64* out, int nl, int nq, int pofs,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_small_to_rns_kernel, grid_for((size_t)nl * sh.P.N), dim3(kBlock), 0, st, s,
                     out, M(sh), sh.P.logN, nl, nq, pofs);
  LAUNCH_CHECK();
}

void k_sample_uniform(const Shared& sh, u64* out, int nl, int nq, int pofs, u64 seed, u64 purpose,
                      hipStream_t st) {
  if (nl > kMaxLimbArgs) PPST_THROW(ST_EINVAL, "too many limbs");
  KeyArr keys;
  for (int t = 0; t < nl; ++t) {
    int p = t < nq ? t : pofs + (t - nq);
    keys.k[t] = stream_key(seed, purpose, (u64)p);
  }
  hipLaunchKernelGGL(k_uniform_kernel, grid_for((size_t)nl * sh.P.N), dim3(kBlock), 0, st, out,
                     M(sh), sh.P.logN, nl, nq, pofs, keys);
  LAUNCH_CHECK();
}

void k_sample_ternary(const Shared& sh, int32_t* out, u64 seed, u64 purpose, hipStream_t st) {
  hipLaunchKernelGGL(k_ternary_kernel, grid_for(sh.P.N), dim3(kBlock), 0, st, out, sh.P.N,
                     stream_key(seed, purpose, 0));
  LAUNCH_CHECK();
}

void k_sample_dg(const Shared& sh, int32_t* out, u64 seed, u64 purpose, hipStream_t st) {
  DgArr d;
  for (int i = 0; i < kDgMax; ++i) d.thr[i] = sh.dg_thr[i];
  hipLaunchKernelGGL(k_dg_kernel, grid_for(sh.P.N), dim3(kBlock), 0, st, out, sh.P.N,
                     stream_key(seed, purpose, 0), d);
  LAUNCH_CHECK();
}

void k_keyform(const Shared& sh, const u64* a, const u64* s, const u64* e, const u64* sp,
               const u64* f, u64* out, int nl, int nq, int pofs, hipStream_t st) {
  if (nl > kMaxLimbArgs) PPST_THROW(ST_EINVAL, "too many limbs");
  ScalarArr fa;
  for (int t = 0; t < nl; ++t) {
    int p = t < nq ? t : pofs + (t - nq);
    u64 v = f ? f[t] : 0;
    fa.v[t] = v;
    fa.vp[t] = v ? shoup(v, sh.P.q[p]) : 0;
  }
  hipLaunchKernelGGL(k_keyform_kernel, grid_for((size_t)nl * sh.P.N), dim3(kBlock), 0, st, a, s,
                     e, sp, fa, out, M(sh), sh.P.logN, nl, nq, pofs, sp ? 1 : 0);
  LAUNCH_CHECK();
}

void k_mod_raise(const Shared& sh, const u64* x, u64* out, int nl, int npoly, hipStream_t st) {
  hipLaunchKernelGGL(k_mod_raise_kernel, grid_for((size_t)npoly * nl * sh.P.N), dim3(kBlock), 0, st,
                     x, out, M(sh), sh.P.logN, nl, npoly);
  LAUNCH_CHECK();
}

void k_bsgs_inner(const Shared& sh, const u64* const* baby, int b, const u64* const* pts,
                  u64* const* outs, int G, int nl, size_t ps_in, size_t ps_out, hipStream_t st) {
  if (b < 1 || G < 1 || G > kBsgsMaxGiant || b * G > kBsgsMaxCells)
    PPST_THROW(ST_EINVAL, "baby-step grid too large");
  BsgsArgs a{};
  int B = 1;
  while (B < b) B <<= 1;
  if (B > kBsgsMaxBaby || B * G > kBsgsMaxCells) PPST_THROW(ST_EINVAL, "baby-step grid too large");
  // baby steps b..B-1 (padding to a power of two) carry no plaintext; they
  // read baby step 0 so that every load stays in bounds
  for (int i = 0; i < B; ++i) a.baby[i] = baby[i < b ? i : 0];
  for (int j = 0; j < G; ++j) {
    a.out[j] = outs[j];
    for (int i = 0; i < B; ++i) a.pt[j * B + i] = i < b ? pts[j * b + i] : nullptr;
  }
  a.ps_in = ps_in;
  a.ps_out = ps_out;
  a.G = G;
  dim3 g = grid_for((size_t)nl * sh.P.N);
  g.y = 2;
  switch (B) {
    case 1: hipLaunchKernelGGL(k_bsgs_inner_kernel<1>, g, dim3(kBlock), 0, st, a, M(sh), sh.P.logN, nl); break;
    case 2: hipLaunchKernelGGL(k_bsgs_inner_kernel<2>, g, dim3(kBlock), 0, st, a, M(sh), sh.P.logN, nl); break;
    case 4: hipLaunchKernelGGL(k_bsgs_inner_kernel<4>, g, dim3(kBlock), 0, st, a, M(sh), sh.P.logN, nl); break;
    case 8: hipLaunchKernelGGL(k_bsgs_inner_kernel<8>, g, dim3(kBlock), 0, st, a, M(sh), sh.P.logN, nl); break;
    default: hipLaunchKernelGGL(k_bsgs_inner_kernel<16>, g, dim3(kBlock), 0, st, a, M(sh), sh.P.logN, nl); break;
  }
  LAUNCH_CHECK();
}

void k_fma3(const Shared& sh, const u64* x, const u64* y, const u64* z, const u64* w, u64* out,
            int nl, hipStream_t st) {
  hipLaunchKernelGGL(k_fma3_kernel, grid_for((size_t)nl * sh.P.N), dim3(kBlock), 0, st, x, y, z,
                     w, out, M(sh), sh.P.logN, nl);
  LAUNCH_CHECK();
}

}  // namespace ppst
