// ntt.hip -- negacyclic NTT / inverse NTT over word-size primes on gfx950.
//
// Forward transform: Cooley-Tukey butterflies on the twiddle table
// w_k = psi^brv(k), natural-order input, output in the canonical bit-reversed
// order (slot j holds a(psi^(2 brv(j) + 1))).  Inverse: Gentleman-Sande
// butterflies on psi^-brv(k) and a final multiplication by N^-1.
//
// Decomposition.  A limb of N = 2^16 words (512 KiB) does not fit in one CU's
// LDS, so the log N stages are split in two launches.  With N = R * C:
//   * column pass: the first log R stages only pair indices j, j + t with
//     t >= C, so each of the C columns {c + C r} is an independent R-point
//     problem; a workgroup loads SB adjacent columns (SB * 8 B contiguous per
//     row) into LDS;
//   * row pass: the last log C stages pair indices inside one row of C
//     contiguous words; a workgroup loads SB rows.
// Inside a pass each thread holds E = 2^LOGE elements in registers and runs
// LOGE stages on them between LDS exchanges (radix-E), with Harvey's lazy
// reduction ([0, 4q) forward, [0, 2q) inverse) and Shoup twiddles.  N = 2^12
// fits one workgroup and runs as a single row pass.
#include "dev.h"
#include "kern.h"

#include <cstdlib>
#include <cstring>
#include <type_traits>
#include "tables.h"

namespace ppst {

namespace {

struct NttArgs {
  const u64* src;
  u64* dst;
  const Mod* mods;
  const u64* tw;     // [nprimes][N][2]
  const u64* ninv;   // [nprimes][2]
  const double* rowf;  // row-pass factor tables of N = 2^16 (row_twiddles), or null
  const u64* comm;
  size_t batch_stride, dst_stride;
  int N, logN, logR, nq, pofs, skip_lo, skip_hi, blocks_per_limb;
  int dalpha, dcount, dtotal;
  uint32_t galois;   // inverse transforms: read the input through X -> X^galois (0: none)
  int nbatch;        // batch items of the launch (set by the launcher)
};

// Workgroup -> (limb, group, batch item) of a one-dimensional grid, batch
// item fastest: the workgroups that share a prime's twiddle rows run back to
// back (blocks are dealt round-robin to the 8 XCDs, so each XCD sees every
// eighth item of the same tile while its twiddles sit in that XCD's L2).
struct BlockPos {
  int limb, grp, item;
};
__device__ __forceinline__ BlockPos block_pos(int blocks_per_limb, int nbatch) {
  const unsigned b = blockIdx.x;
  const unsigned tile = b / (unsigned)nbatch;
  BlockPos p;
  p.item = (int)(b - tile * (unsigned)nbatch);
  p.limb = (int)(tile / (unsigned)blocks_per_limb);
  p.grp = (int)(tile - (unsigned)p.limb * (unsigned)blocks_per_limb);
  return p;
}

// ----------------------------------------------------------------------
// Butterfly arithmetic.  Two interchangeable policies, chosen per workgroup
// by the size of its prime (the choice is uniform over a workgroup):
//
// IntArith: 64-bit residues, Shoup twiddle products (w, w' = floor(w 2^64/q))
//   with Harvey's lazy ranges [0, 4q) forward and [0, 2q) inverse.
// FpArith (q < 2^44): residues held as exact integers in FP64, signed and
//   unreduced.  The twiddle product y w mod q is  h = fl(y w),
//   l = fma(y, w, -h)  (so h + l = y w exactly),  k = rint(y * (w/q)),
//   r = fma(-k, q, h) + l  = y w - k q exactly (every intermediate is an
//   integer below 2^53), and |r| <= 0.55 q because k is the nearest integer
//   to y w / q up to an error of at most 2 |y| 2^-53 < 0.05 for |y| < 2^47.4.
//   A forward butterfly is then x + r, x - r with no reduction: over the 16
//   stages of a transform |x| grows from q to at most q + 16 (0.55 q) < 10 q,
//   below 2^47.4 for q < 2^44.  An inverse butterfly's sum x + y at most
//   doubles per stage, so every register pass (at most 4 stages) starts by
//   centring its values, v - q rint(v / q) (|v| <= q/2 + 1 after it), and
//   its sums and differences stay below 2^4 (q/2 + 1) < 9 q.  Values cross
//   from one pass to the next as the doubles' bits (no conversion), and the
//   last pass rounds into [0, q).
//   Table entries are (w, w/q) as doubles.
// Both produce the same canonical residues at the end of a transform.
// ----------------------------------------------------------------------
struct IntArith {
  typedef u64 T;
  u64 q, q2;
  __device__ __forceinline__ explicit IntArith(u64 q_) : q(q_), q2(2 * q_) {}
  __device__ __forceinline__ T in(u64 v) const { return v; }
  // a value written by the previous pass of the same transform, and back
  __device__ __forceinline__ T in_mid(u64 v) const { return v; }
  __device__ __forceinline__ u64 mid(T v) const { return v; }
  __device__ __forceinline__ void centre(T&) const {}
  __device__ __forceinline__ u64 out_fwd(T v) const { v = v >= q2 ? v - q2 : v; return csub(v, q); }
  __device__ __forceinline__ u64 out_inv(T v, u64 ni, u64 nip) const { return mul_shoup(v, ni, nip, q); }
  // forward CT on [0, 4q)
  __device__ __forceinline__ void ct(T& x, T& y, ulonglong2 w) const {
    u64 a = x >= q2 ? x - q2 : x;
    u64 t = mul_shoup_lazy(y, w.x, w.y, q);
    x = a + t;
    y = a - t + q2;
  }
  // inverse GS on [0, 2q)
  __device__ __forceinline__ void gs(T& x, T& y, ulonglong2 w) const {
    u64 a = x + y;
    a = a >= q2 ? a - q2 : a;
    u64 d = x - y + q2;
    y = mul_shoup_lazy(d, w.x, w.y, q);
    x = a;
  }
};

struct FpArith {
  typedef double T;
  double q, qinv;
  __device__ __forceinline__ explicit FpArith(u64 q_)
      : q((double)q_), qinv(1.0 / (double)q_) {}
  // y w - k q with k = rint(y w / q): exact, |.| <= 0.55 q
  __device__ __forceinline__ double mulmod(double y, double w, double ws) const {
    double h = y * w;
    double l = __fma_rn(y, w, -h);
    double k = rint(y * ws);
    double r = __fma_rn(-k, q, h);
    return r + l;
  }
  __device__ __forceinline__ T in(u64 v) const { return (double)v; }
  __device__ __forceinline__ T in_mid(u64 v) const { return __longlong_as_double((long long)v); }
  __device__ __forceinline__ u64 mid(T v) const { return (u64)__double_as_longlong(v); }
  // a formed twiddle w as a table entry (w, w/q)
  __device__ __forceinline__ ulonglong2 pair(double w) const {
    return make_ulonglong2((u64)__double_as_longlong(w), (u64)__double_as_longlong(w * qinv));
  }
  // v - q rint(v / q): exact (an integer of magnitude below q), |.| <= q/2 + 1
  __device__ __forceinline__ void centre(T& v) const { v = __fma_rn(-rint(v * qinv), q, v); }
  // the canonical residue of v
  __device__ __forceinline__ u64 out_fwd(T v) const {
    double r = __fma_rn(-rint(v * qinv), q, v);
    r = r < 0.0 ? r + q : r;
    return (u64)r;
  }
  __device__ __forceinline__ u64 out_inv(T v, u64 ni, u64 nis) const {
    double r = mulmod(v, __longlong_as_double((long long)ni), __longlong_as_double((long long)nis));
    r = r < 0.0 ? r + q : r;
    return (u64)r;
  }
  // forward CT: x + r, x - r
  __device__ __forceinline__ void ct(T& x, T& y, ulonglong2 w) const {
    double r = mulmod(y, __longlong_as_double((long long)w.x), __longlong_as_double((long long)w.y));
    y = x - r;
    x = x + r;
  }
  // inverse GS: x + y, (x - y) w
  __device__ __forceinline__ void gs(T& x, T& y, ulonglong2 w) const {
    double s = x + y;
    y = mulmod(x - y, __longlong_as_double((long long)w.x), __longlong_as_double((long long)w.y));
    x = s;
  }
};

// Orders the LDS accesses of one wavefront's lanes (which run in lockstep):
// all the barrier a row pass's exchange needs when each sub-problem (row)
// lies within one wave, so that the waves of a workgroup never wait for
// each other.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
// whether the rows of a row pass with TPS threads per row are wave-private
template <int TPS>
struct WaveRows {
  static constexpr bool on = TPS <= 64 && 64 % TPS == 0;
};
template <bool WAVE>
__device__ __forceinline__ void exchange_sync() {
  if constexpr (WAVE) wave_sync();
  else __syncthreads();
}

// Row twiddles formed in LDS.  Sub-problem r of a row pass (N = R M with
// R = M = 2^8) reads table entry (R + r) 2^s + j at its local stage s
// (j < 2^s); bit reversal maps the two fields separately, so that entry is
// rowf[r][s] * comm[2^s + j]: a factor per (row, stage) and one shared by
// every row.  A workgroup of SB rows forms its SB (M - 1) entries with one
// exact FP64 product each (FpArith::mulmod, |w| <= 0.51 q, signed) instead
// of reading them from the N-entry table (1 MiB per prime, a third of the
// pass's traffic); the butterflies read w there and form w * (1/q).  The butterfly bound of FpArith holds for such w: the
// quotient estimate y * w/q then carries three roundings, at most
// 3 * 2^-53 * 0.51 * 2^47.4 < 0.032 off for |y| < 2^47.4, so
// |y w - k q| <= 0.532 q < 0.55 q.
// Only FP64 primes use it; lds null: the table in memory.
constexpr int kRowTwLogM = 8;
struct RowTw {
  double* lds;            // [SB][M] entries w of the workgroup's rows, or null
  const double* rowf;     // the prime's [R][LOGM] row factors
  const ulonglong2* comm; // the prime's [M] shared factors (w, w/q)
  bool make;              // form them first (false: an earlier body did)
};

// whether a row kernel of this shape forms its twiddles (bounded LDS)
template <int LOGM, int SB, bool ROWS>
struct RowTwShape {
  static constexpr bool on = ROWS && LOGM == kRowTwLogM && SB <= 8;
  static constexpr int size = on ? SB << LOGM : 1;   // doubles
};

// every thread forms SB M / NT entries, their loads issued together (entry
// 0 of a row, never read, comes out 0 from comm's zero entry)
template <int LOGM, int SB, int NT>
__device__ __forceinline__ void row_twiddles(const FpArith& ar, const RowTw& rt, int first) {
  constexpr int M = 1 << LOGM;
  constexpr int PER = SB * M / NT;
  static_assert(PER * NT == SB * M, "workgroup shape");
  double f[PER];
  ulonglong2 c[PER];
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int idx = (int)threadIdx.x + k * NT;
    const int r = idx >> LOGM, i = idx & (M - 1);
    const int s = i ? 31 - __clz(i) : 0;
    f[k] = rt.rowf[(first + r) * LOGM + s];
    c[k] = rt.comm[i];
  }
#pragma unroll
  for (int k = 0; k < PER; ++k)
    rt.lds[(int)threadIdx.x + k * NT] =
        ar.mulmod(f[k], __longlong_as_double((long long)c[k].x), __longlong_as_double((long long)c[k].y));
}

// One pass of LOGM stages over SB independent sub-problems of M = 2^LOGM
// points.  ROWS: sub-problem r = row (contiguous), twiddle base R + r;
// otherwise sub-problem c = column (stride C), twiddle base 1.  Stage s of
// the sub-problem uses twiddle index (base << s) + (e >> (LOGM - s)) for the
// butterfly whose lower element is e.
//
// The stages run in register passes of up to LOGE stages: in a pass of ls
// stages the sub-problem splits into M / 2^ls independent groups of 2^ls
// elements; each of the T = M / E threads owns E / 2^ls groups (E registers)
// and exchanges them through LDS between passes.
template <class A, int LOGM, int LOGE, int SB, bool ROWS, bool INV, bool TL = false>
__device__ __forceinline__ void ntt_body(const A ar, typename A::T* lds, const u64* src, u64* dst,
                                         const ulonglong2* tw, const u64* ninv2, int N, int logR,
                                         int first, bool firstp, bool last, uint32_t galois,
                                         int logN, const RowTw rt = RowTw{}) {
  typedef typename A::T T;
  constexpr int M = 1 << LOGM;
  constexpr int E = 1 << LOGE;
  constexpr int TPS = M / E;         // threads per sub-problem
  constexpr int NT = SB * TPS;       // threads per workgroup
  constexpr int NP = (LOGM + LOGE - 1) / LOGE;   // register passes
  constexpr int PAD = M + 1;         // LDS row pitch (breaks bank aliasing)
  const int R = 1 << logR;
  const int C = N >> logR;
  const int tid = threadIdx.x;

  // ---- load SB sub-problems into LDS (coalesced along memory)
  if (ROWS && INV && galois != 0) {
#pragma unroll 4
    for (int idx = tid; idx < SB * M; idx += NT) {
      int sp = idx / M, e = idx - sp * M;
      lds[sp * PAD + e] = ar.in(src[galois_src((uint32_t)(first * M + idx), galois, logN)]);
    }
  } else if (ROWS) {
    const u64* g = src + (size_t)first * M;
#pragma unroll 4
    for (int idx = tid; idx < SB * M; idx += NT) {
      int sp = idx / M, e = idx - sp * M;
      lds[sp * PAD + e] = firstp ? ar.in(g[idx]) : ar.in_mid(g[idx]);
    }
  } else {
#pragma unroll 4
    for (int idx = tid; idx < SB * M; idx += NT) {
      int e = idx / SB, sp = idx - e * SB;
      const u64 v = src[(size_t)e * C + first + sp];
      lds[sp * PAD + e] = firstp ? ar.in(v) : ar.in_mid(v);
    }
  }
  if constexpr (TL) {
    if (rt.make) row_twiddles<LOGM, SB, NT>(ar, rt, first);
  }
  __syncthreads();

  const int sp = tid / TPS;
  const int lane = tid - sp * TPS;
  T* my = lds + sp * PAD;
  const uint32_t base0 = ROWS ? (uint32_t)(R + first + sp) : 1u;

#pragma unroll
  for (int pi = 0; pi < NP; ++pi) {
    const int p = INV ? (NP - 1 - pi) : pi;
    const int s0 = p * LOGE;
    const int ls = (LOGM - s0) < LOGE ? (LOGM - s0) : LOGE;   // stages in this pass
    const int GS = 1 << ls;                                    // group size
    const int G = E / GS;                                      // groups per thread
    const int si = M >> (s0 + ls);                             // element stride in a group
    int e0[E];
    T x[E];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int gi = g * TPS + lane;
      const int lo = gi % si, hi = gi / si;
      e0[g] = hi * (M >> s0) + lo;
#pragma unroll
      for (int k = 0; k < GS; ++k) x[g * GS + k] = my[e0[g] + k * si];
    }
    // inverse sums grow: every register pass starts from centred values
    if (INV) {
#pragma unroll
      for (int i = 0; i < E; ++i) ar.centre(x[i]);
    }
#pragma unroll
    for (int uu = 0; uu < ls; ++uu) {
      const int u = INV ? (ls - 1 - uu) : uu;
      const int s = s0 + u;
      const int half = GS >> (u + 1);
#pragma unroll
      for (int g = 0; g < G; ++g) {
#pragma unroll
        for (int k = 0; k < GS; ++k) {
          if (k & half) continue;
          const int e = e0[g] + k * si;
          const uint32_t j = (uint32_t)(e >> (LOGM - s));
          ulonglong2 w;
          if constexpr (TL) w = ar.pair(rt.lds[((uint32_t)sp << LOGM) + (1u << s) + j]);
          else w = tw[(base0 << s) + j];
          if (INV) ar.gs(x[g * GS + k], x[g * GS + k + half], w);
          else ar.ct(x[g * GS + k], x[g * GS + k + half], w);
        }
      }
    }
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int k = 0; k < GS; ++k) my[e0[g] + k * si] = x[g * GS + k];
    __syncthreads();
  }

  // ---- store; finish the reduction where this pass is the last one
  const u64 ni = ninv2[0], nip = ninv2[1];
  if (ROWS) {
    u64* g = dst + (size_t)first * M;
#pragma unroll 4
    for (int idx = tid; idx < SB * M; idx += NT) {
      int s2 = idx / M, e = idx - s2 * M;
      T v = lds[s2 * PAD + e];
      g[idx] = last ? (INV ? ar.out_inv(v, ni, nip) : ar.out_fwd(v)) : ar.mid(v);
    }
  } else {
#pragma unroll 4
    for (int idx = tid; idx < SB * M; idx += NT) {
      int e = idx / SB, s2 = idx - e * SB;
      T v = lds[s2 * PAD + e];
      dst[(size_t)e * C + first + s2] = last ? (INV ? ar.out_inv(v, ni, nip) : ar.out_fwd(v)) : ar.mid(v);
    }
  }
}

// The same transform as ntt_body with no LDS staging at either end: the
// first register pass loads its elements straight from global memory and the
// last one stores straight to it, saving two LDS round trips and two
// barriers.  Columns map column-fastest onto threads (a wave covers SB
// adjacent columns of 64/SB rows), so both ends stay coalesced; rows map as
// in ntt_body.
// Stores finished elements of a limb.  A store may load operands of its own
// for element slot i (0..E-1) before the last pass's butterflies
// (prefetch), so that their latency overlaps the arithmetic.
// Loads of the first register pass: PlainLoad reads the pass's source; a
// custom load (kCustom) computes each element from its index instead.
struct PlainLoad {
  static constexpr bool kCustom = false;
  template <class A>
  __device__ __forceinline__ typename A::T get_t(const A& ar, int, size_t) const { return ar.in(0); }
};

// A product's d2 = a1 b1 mod q, formed where the inverse transform of the
// tensor's d2 would load it: the key switch of a product starts from a1 and
// b1 themselves and d2 is never written.
struct ProdLoad {
  static constexpr bool kCustom = true;
  const u64* a;
  const u64* b;
  Mod m;
  // FP64 primes: the exact FP64 product, signed (|.| < 0.57 q), which the
  // inverse pass centres like any input
  template <class A>
  __device__ __forceinline__ typename A::T get_t(const A& ar, int, size_t at) const {
    if constexpr (std::is_same<A, FpArith>::value) {
      const double x = ar.in(a[at]), y = ar.in(b[at]);
      return ar.mulmod(x, y, y * ar.qinv);
    } else {
      return ar.in(mulm(a[at], b[at], m));
    }
  }
};

struct PlainStore {
  static constexpr bool kRaw = false;
  u64* dst;
  __device__ __forceinline__ void prefetch(int, size_t) {}
  __device__ __forceinline__ void put(int, size_t at, u64 v) const { dst[at] = v; }
};

template <class A, int LOGM, int LOGE, int SB, bool ROWS, bool INV, bool TL = false,
          class Store = PlainStore, class Load = PlainLoad>
__device__ __forceinline__ void ntt_body_dio(const A ar, typename A::T* lds, const u64* src,
                                             Store& store, const ulonglong2* tw,
                                             const u64* ninv2, int N, int logR, int first,
                                             bool firstp, bool last, uint32_t galois, int logN,
                                             const RowTw rt = RowTw{}, const Load& ld = Load()) {
  typedef typename A::T T;
  constexpr int M = 1 << LOGM;
  constexpr int E = 1 << LOGE;
  constexpr int TPS = M / E;         // threads per sub-problem
  constexpr int NP = (LOGM + LOGE - 1) / LOGE;   // register passes
  constexpr int PAD = M + 1;
  const int R = 1 << logR;
  const int C = N >> logR;
  const int tid = threadIdx.x;
  const int sp = ROWS ? tid / TPS : tid % SB;
  const int lane = ROWS ? tid - sp * TPS : tid / SB;
  T* my = lds + sp * PAD;
  const uint32_t base0 = ROWS ? (uint32_t)(R + first + sp) : 1u;
  const size_t rowbase = ROWS ? (size_t)(first + sp) * M : 0;
  const int col = first + sp;
  const u64 ni = ninv2[0], nip = ninv2[1];

#pragma unroll
  for (int pi = 0; pi < NP; ++pi) {
    const int p = INV ? (NP - 1 - pi) : pi;
    const int s0 = p * LOGE;
    const int ls = (LOGM - s0) < LOGE ? (LOGM - s0) : LOGE;   // stages in this pass
    const int GS = 1 << ls;                                    // group size
    const int G = E / GS;                                      // groups per thread
    const int si = M >> (s0 + ls);                             // element stride in a group
    int e0[E];
    T x[E];
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int gi = g * TPS + lane;
      const int lo = gi % si, hi = gi / si;
      e0[g] = hi * (M >> s0) + lo;
    }
    if (pi == 0) {
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int k = 0; k < GS; ++k) {
          const int e = e0[g] + k * si;
          size_t at = ROWS ? rowbase + e : (size_t)e * C + col;
          if constexpr (Load::kCustom) {
            x[g * GS + k] = ld.get_t(ar, g * GS + k, at);
          } else {
            if (ROWS && INV && galois != 0) at = galois_src((uint32_t)at, galois, logN);
            x[g * GS + k] = firstp ? ar.in(src[at]) : ar.in_mid(src[at]);
          }
        }
      // the row twiddles form while the loads are in flight
      if constexpr (TL) {
        if (rt.make) {
          row_twiddles<LOGM, SB, SB * TPS>(ar, rt, first);
          __syncthreads();
        }
      }
    } else {
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int k = 0; k < GS; ++k) x[g * GS + k] = my[e0[g] + k * si];
    }
    if (pi == NP - 1) {
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int k = 0; k < GS; ++k) {
          const int e = e0[g] + k * si;
          store.prefetch(g * GS + k, ROWS ? rowbase + e : (size_t)e * C + col);
        }
    }
    // inverse sums grow: every register pass starts from centred values
    if (INV) {
#pragma unroll
      for (int i = 0; i < E; ++i) ar.centre(x[i]);
    }
#pragma unroll
    for (int uu = 0; uu < ls; ++uu) {
      const int u = INV ? (ls - 1 - uu) : uu;
      const int s = s0 + u;
      const int half = GS >> (u + 1);
#pragma unroll
      for (int g = 0; g < G; ++g) {
#pragma unroll
        for (int k = 0; k < GS; ++k) {
          if (k & half) continue;
          const int e = e0[g] + k * si;
          const uint32_t j = (uint32_t)(e >> (LOGM - s));
          ulonglong2 w;
          if constexpr (TL) w = ar.pair(rt.lds[((uint32_t)sp << LOGM) + (1u << s) + j]);
          else w = tw[(base0 << s) + j];
          if (INV) ar.gs(x[g * GS + k], x[g * GS + k + half], w);
          else ar.ct(x[g * GS + k], x[g * GS + k + half], w);
        }
      }
    }
    if (pi == NP - 1) {
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int k = 0; k < GS; ++k) {
          const int e = e0[g] + k * si;
          const size_t at = ROWS ? rowbase + e : (size_t)e * C + col;
          const T v = x[g * GS + k];
          if constexpr (Store::kRaw)
            store.put_raw(g * GS + k, at, v);   // the store takes the unreduced value
          else
            store.put(g * GS + k, at, last ? (INV ? ar.out_inv(v, ni, nip) : ar.out_fwd(v)) : ar.mid(v));
        }
    } else {
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int k = 0; k < GS; ++k) my[e0[g] + k * si] = x[g * GS + k];
      exchange_sync<ROWS && WaveRows<TPS>::on>();
    }
  }
}

// Workgroup -> (limb, group, batch item) of tile `b` (see block_pos)
__device__ __forceinline__ BlockPos tile_pos(unsigned b, int blocks_per_limb, int nbatch) {
  const unsigned tile = b / (unsigned)nbatch;
  BlockPos p;
  p.item = (int)(b - tile * (unsigned)nbatch);
  p.limb = (int)(tile / (unsigned)blocks_per_limb);
  p.grp = (int)(tile - (unsigned)p.limb * (unsigned)blocks_per_limb);
  return p;
}

// One tile of a pass: SB sub-problems of one limb of one batch item.
// the RowTw of a row pass on `prime` (lds null where the table is read)
template <int LOGM, int SB, bool ROWS>
__device__ __forceinline__ RowTw row_tw(const NttArgs& a, double* twl, int prime, u64 q) {
  RowTw rt{};
  if (RowTwShape<LOGM, SB, ROWS>::on && a.rowf != nullptr && q < kFpPrimeBound && a.logR == kRowTwLogM) {
    rt.lds = twl;
    rt.rowf = a.rowf + (size_t)prime * ((size_t)kRowTwLogM << a.logR);
    rt.comm = (const ulonglong2*)(a.comm + (size_t)prime * (2u << LOGM));
    rt.make = true;
  }
  return rt;
}

template <int LOGM, int LOGE, int SB, bool ROWS, bool INV, bool DIO>
__device__ __forceinline__ void ntt_tile(const NttArgs& a, u64* lds, double* twl,
                                         const BlockPos bp) {
  const int N = a.N;
  const int limb_u = bp.limb;
  const int grp = bp.grp;
  int skip_lo = a.skip_lo, skip_hi = a.skip_hi;
  if (a.dalpha > 0) {            // tile-uniform: the whole workgroup skips together
    skip_lo = (bp.item % a.dcount) * a.dalpha;
    skip_hi = min(skip_lo + a.dalpha, a.nq);
    if (limb_u >= a.dtotal - (skip_hi - skip_lo)) return;
  }
  const int t = limb_u >= skip_lo ? limb_u + (skip_hi - skip_lo) : limb_u;
  const int prime = t < a.nq ? t : a.pofs + (t - a.nq);
  const u64* src = a.src + (size_t)bp.item * a.batch_stride + (size_t)t * N;
  u64* dst = a.dst + (size_t)bp.item * a.dst_stride + (size_t)t * N;
  const u64 q = a.mods[prime].q;
  const ulonglong2* tw = (const ulonglong2*)(a.tw + (size_t)prime * N * 2);
  const u64* ni = a.ninv + 2 * prime;
  const bool last = INV ? (!ROWS || a.logR == 0) : ROWS;
  const bool firstp = INV ? ROWS : (!ROWS || a.logR == 0);   // reads the transform's input
  const int first = grp * SB;        // first sub-problem of this workgroup
  constexpr bool TLS = RowTwShape<LOGM, SB, ROWS>::on;
  const RowTw rt = row_tw<LOGM, SB, ROWS>(a, twl, prime, q);
  if (DIO) {
    PlainStore store{dst};
    if (rt.lds)
      ntt_body_dio<FpArith, LOGM, LOGE, SB, ROWS, INV, TLS>(FpArith(q), (double*)lds, src, store, tw,
                                                             ni, N, a.logR, first, firstp, last,
                                                             a.galois, a.logN, rt);
    else if (q < kFpPrimeBound)
      ntt_body_dio<FpArith, LOGM, LOGE, SB, ROWS, INV>(FpArith(q), (double*)lds, src, store, tw,
                                                        ni, N, a.logR, first, firstp, last, a.galois,
                                                        a.logN);
    else
      ntt_body_dio<IntArith, LOGM, LOGE, SB, ROWS, INV>(IntArith(q), lds, src, store, tw, ni, N,
                                                         a.logR, first, firstp, last, a.galois, a.logN);
  } else {
    if (rt.lds)
      ntt_body<FpArith, LOGM, LOGE, SB, ROWS, INV, TLS>(FpArith(q), (double*)lds, src, dst, tw, ni, N,
                                                         a.logR, first, firstp, last, a.galois,
                                                         a.logN, rt);
    else if (q < kFpPrimeBound)
      ntt_body<FpArith, LOGM, LOGE, SB, ROWS, INV>(FpArith(q), (double*)lds, src, dst, tw, ni, N,
                                                    a.logR, first, firstp, last, a.galois, a.logN);
    else
      ntt_body<IntArith, LOGM, LOGE, SB, ROWS, INV>(IntArith(q), lds, src, dst, tw, ni, N,
                                                     a.logR, first, firstp, last, a.galois, a.logN);
  }
}

template <int LOGM, int LOGE, int SB, bool ROWS, bool INV, bool DIO>
__global__ void __launch_bounds__(SB * (1 << (LOGM - LOGE)))
k_ntt_pass(NttArgs a) {
  __shared__ u64 lds[SB * ((1 << LOGM) + 1)];
  __shared__ double twl[RowTwShape<LOGM, SB, ROWS>::size];
  ntt_tile<LOGM, LOGE, SB, ROWS, INV, DIO>(a, lds, twl, block_pos(a.blocks_per_limb, a.nbatch));
}

// Persistent form: a grid sized to what the device holds at once walks the
// tiles (grid-stride), so a launch of thousands of tiles dispatches each
// workgroup once; the barrier after each tile lets the next one reuse LDS.
template <int LOGM, int LOGE, int SB, bool ROWS, bool INV, bool DIO>
__global__ void __launch_bounds__(SB * (1 << (LOGM - LOGE)))
k_ntt_pass_persistent(NttArgs a, unsigned ntiles) {
  __shared__ u64 lds[SB * ((1 << LOGM) + 1)];
  __shared__ double twl[RowTwShape<LOGM, SB, ROWS>::size];
  for (unsigned b = blockIdx.x; b < ntiles; b += gridDim.x) {
    ntt_tile<LOGM, LOGE, SB, ROWS, INV, DIO>(a, lds, twl, tile_pos(b, a.blocks_per_limb, a.nbatch));
    __syncthreads();
  }
}

// ---- forward row pass that finishes the fused ModDown + rescale
// The element stored for limb i (prime q_i, i < level) of polynomial c of
// batch item b is, instead of the transformed correction corr_i itself,
//   out_i = ((u_i P^-1 mod q_i) + d_i + corr_i) q_l^-1 mod q_i,
// the same operations in the same order as the separate final kernel.
struct MdrEpi {
  const u64* u;      // [item][2][ne][N]  key-switch accumulators (NTT form)
  const u64* d;      // [item][3][nl][N]  tensor (d0, d1 used), or null:
  PtrsIn pa, pb;     //   the operands (item: [2][nl][N]), d0 = a0 b0, d1 = a0 b1 + a1 b0
  size_t su, sd;
  OutPtrs out;       // item b writes [2][level][N] at out.p[b]
  const u64* md;     // ModDown table
  const u64* rc;     // rescale table of the level
  int K, L, level, ne, nl;
};

// OPS: d_c from the operands (OPS = 1 + c: d0 = a0 b0, d1 = a0 b1 + a1 b0)
// instead of the tensor's d_c (OPS = 0)
template <int E, int OPS>
struct MdrStore {
  static constexpr bool kRaw = false;
  const u64* u;
  const u64* d;
  const u64* a0;
  const u64* a1;
  const u64* b0;
  const u64* b1;
  Mod m;
  u64* out;
  u64 q, pinv, pinvs, qlinv, qlinvs;
  u64 pu[E], pd[E], pe[E], pf[E], pg[E];
  __device__ __forceinline__ void prefetch(int i, size_t at) {
    pu[i] = u[at];
    if constexpr (OPS == 0) {
      pd[i] = d[at];
    } else if constexpr (OPS == 1) {
      pd[i] = a0[at];
      pe[i] = b0[at];
    } else {
      pd[i] = a0[at];
      pe[i] = b1[at];
      pf[i] = a1[at];
      pg[i] = b0[at];
    }
  }
  __device__ __forceinline__ void put(int i, size_t at, u64 corr) const {
    u64 v = mul_shoup(pu[i], pinv, pinvs, q);
    u64 dv;
    if constexpr (OPS == 0) dv = pd[i];
    else if constexpr (OPS == 1) dv = mulm(pd[i], pe[i], m);
    else dv = mul2_add(pd[i], pe[i], pf[i], pg[i], m);
    v = addm(v, dv, q);
    v = addm(v, corr, q);
    out[at] = mul_shoup(v, qlinv, qlinvs, q);
  }
};

// A product's item in one workgroup: both polynomials' row passes in turn,
// the operands a0, a1, b0, b1 loaded once (with the first) for d0 and d1,
// kept in the arithmetic's own type.
template <int E, class T>
struct MdrOps {
  T x0[E], x1[E], y0[E], y1[E];
};

template <class A, int E, int C>
struct MdrPairStore;

// 60-bit primes: Shoup and 128-bit products
template <int E, int C>
struct MdrPairStore<IntArith, E, C> {
  static constexpr bool kRaw = false;
  MdrOps<E, u64>* o;
  const u64* u;
  const u64* a0;
  const u64* a1;
  const u64* b0;
  const u64* b1;
  Mod m;
  u64* out;
  u64 q, pinv, pinvs, qlinv, qlinvs;
  u64 pu[E];
  __device__ __forceinline__ void prefetch(int i, size_t at) {
    pu[i] = u[at];
    if constexpr (C == 0) {
      o->x0[i] = a0[at];
      o->x1[i] = a1[at];
      o->y0[i] = b0[at];
      o->y1[i] = b1[at];
    }
  }
  __device__ __forceinline__ void put(int i, size_t at, u64 corr) const {
    u64 v = mul_shoup(pu[i], pinv, pinvs, q);
    const u64 dv = C == 0 ? mulm(o->x0[i], o->y0[i], m)
                          : mul2_add(o->x0[i], o->y1[i], o->x1[i], o->y0[i], m);
    v = addm(v, dv, q);
    v = addm(v, corr, q);
    out[at] = mul_shoup(v, qlinv, qlinvs, q);
  }
  __device__ __forceinline__ void init(const IntArith&) {}
};

// FP64 primes: every product exact in FP64 (FpArith::mulmod), on the
// transform's unreduced output (|corr| < 10 q): u P^-1 and each operand
// product land in (-0.57 q, 0.57 q), so the sum s stays below 12 q < 2^47.6
// and the last product by q_l^-1 (quotient estimate at most 0.07 off) in
// (-0.57 q, 0.57 q); one conditional addition of q makes it canonical.
template <int E, int C>
struct MdrPairStore<FpArith, E, C> {
  static constexpr bool kRaw = true;
  MdrOps<E, double>* o;
  const u64* u;
  const u64* a0;
  const u64* a1;
  const u64* b0;
  const u64* b1;
  Mod m;
  u64* out;
  u64 q, pinv, pinvs, qlinv, qlinvs;
  FpArith ar{1};
  double pinvd, pinvq, qlinvd, qlinvq;
  u64 pu[E];
  __device__ __forceinline__ void init(const FpArith& a) {
    ar = a;
    pinvd = (double)pinv;
    pinvq = pinvd * ar.qinv;
    qlinvd = (double)qlinv;
    qlinvq = qlinvd * ar.qinv;
  }
  __device__ __forceinline__ void prefetch(int i, size_t at) {
    pu[i] = u[at];
    if constexpr (C == 0) {
      o->x0[i] = ar.in(a0[at]);
      o->x1[i] = ar.in(a1[at]);
      o->y0[i] = ar.in(b0[at]);
      o->y1[i] = ar.in(b1[at]);
    }
  }
  __device__ __forceinline__ void put_raw(int i, size_t at, double corr) const {
    const double v = ar.mulmod(ar.in(pu[i]), pinvd, pinvq);
    double dv;
    if constexpr (C == 0) {
      dv = ar.mulmod(o->x0[i], o->y0[i], o->y0[i] * ar.qinv);
    } else {
      dv = ar.mulmod(o->x0[i], o->y1[i], o->y1[i] * ar.qinv) +
           ar.mulmod(o->x1[i], o->y0[i], o->y0[i] * ar.qinv);
    }
    double r = ar.mulmod(v + dv + corr, qlinvd, qlinvq);
    r = r < 0.0 ? r + ar.q : r;
    out[at] = (u64)r;
  }
};

template <class A, int LOGM, int LOGE, int SB, bool TL, int C>
__device__ __forceinline__ void mdr_pair_poly(const A ar, const NttArgs& a, const MdrEpi& e,
                                              u64* lds, RowTw rt,
                                              MdrOps<(1 << LOGE), typename A::T>* ops,
                                              int t, int item, int first) {
  const int N = a.N;
  const MdLayout lay(e.K, e.L);
  MdrPairStore<A, (1 << LOGE), C> st;
  st.o = ops;
  st.u = e.u + (size_t)item * e.su + ((size_t)C * e.ne + t) * N;
  st.a0 = e.pa.p[item] + (size_t)t * N;
  st.a1 = st.a0 + (size_t)e.nl * N;
  st.b0 = e.pb.p[item] + (size_t)t * N;
  st.b1 = st.b0 + (size_t)e.nl * N;
  st.m = a.mods[t];
  st.out = e.out.p[item] + ((size_t)C * e.level + t) * N;
  st.q = st.m.q;
  st.pinv = e.md[lay.pinv(t)];
  st.pinvs = e.md[lay.pinv(t) + 1];
  st.qlinv = e.rc[3 * t];
  st.qlinvs = e.rc[3 * t + 1];
  st.init(ar);
  const u64* src = a.src + (size_t)(2 * item + C) * a.batch_stride + (size_t)t * N;
  const ulonglong2* tw = (const ulonglong2*)(a.tw + (size_t)t * N * 2);
  ntt_body_dio<A, LOGM, LOGE, SB, true, false, TL>(ar, (typename A::T*)lds, src, st, tw,
                                                   a.ninv + 2 * t, N, a.logR, first, a.logR == 0,
                                                   true, 0u, a.logN, rt);
}

template <class A, int LOGM, int LOGE, int SB, bool TL>
__device__ __forceinline__ void mdr_pair_body(const A ar, const NttArgs& a, const MdrEpi& e,
                                              u64* lds, RowTw rt, int t, int item, int first) {
  MdrOps<(1 << LOGE), typename A::T> ops;
  mdr_pair_poly<A, LOGM, LOGE, SB, TL, 0>(ar, a, e, lds, rt, &ops, t, item, first);
  // the second row pass reuses the LDS rows (the twiddles, formed behind a
  // workgroup barrier in the first, are only read)
  exchange_sync<WaveRows<(1 << (LOGM - LOGE))>::on>();
  rt.make = false;
  mdr_pair_poly<A, LOGM, LOGE, SB, TL, 1>(ar, a, e, lds, rt, &ops, t, item, first);
}

template <int LOGM, int LOGE, int SB>
__device__ __forceinline__ void mdr_pair_tile(const NttArgs& a, const MdrEpi& e, u64* lds,
                                              double* twl, const BlockPos bp) {
  const int t = bp.limb;                                 // limb = prime index, t < level
  const u64 q = a.mods[t].q;
  const int first = bp.grp * SB;
  const RowTw rt = row_tw<LOGM, SB, true>(a, twl, t, q);
  if (rt.lds)
    mdr_pair_body<FpArith, LOGM, LOGE, SB, RowTwShape<LOGM, SB, true>::on>(FpArith(q), a, e, lds, rt,
                                                                          t, bp.item, first);
  else if (q < kFpPrimeBound)
    mdr_pair_body<FpArith, LOGM, LOGE, SB, false>(FpArith(q), a, e, lds, rt, t, bp.item, first);
  else
    mdr_pair_body<IntArith, LOGM, LOGE, SB, false>(IntArith(q), a, e, lds, rt, t, bp.item, first);
}

template <int LOGM, int LOGE, int SB, int OPS>
__device__ __forceinline__ void mdr_tile(const NttArgs& a, const MdrEpi& e, u64* lds, double* twl,
                                         const BlockPos bp) {
  const int N = a.N;
  const int t = bp.limb;                                 // limb = prime index, t < level
  const int grp = bp.grp;
  const int item = bp.item >> 1, c = bp.item & 1;
  const u64* src = a.src + (size_t)bp.item * a.batch_stride + (size_t)t * N;
  const u64 q = a.mods[t].q;
  const ulonglong2* tw = (const ulonglong2*)(a.tw + (size_t)t * N * 2);
  const u64* ni = a.ninv + 2 * t;
  const MdLayout lay(e.K, e.L);
  MdrStore<(1 << LOGE), OPS> store;
  store.u = e.u + (size_t)item * e.su + ((size_t)c * e.ne + t) * N;
  if (OPS == 0) {
    store.d = e.d + (size_t)item * e.sd + ((size_t)c * e.nl + t) * N;
  } else {
    store.a0 = e.pa.p[item] + (size_t)t * N;
    store.a1 = store.a0 + (size_t)e.nl * N;
    store.b0 = e.pb.p[item] + (size_t)t * N;
    store.b1 = store.b0 + (size_t)e.nl * N;
  }
  store.m = a.mods[t];
  store.out = e.out.p[item] + ((size_t)c * e.level + t) * N;
  store.q = q;
  store.pinv = e.md[lay.pinv(t)];
  store.pinvs = e.md[lay.pinv(t) + 1];
  store.qlinv = e.rc[3 * t];
  store.qlinvs = e.rc[3 * t + 1];
  const int first = grp * SB;
  const RowTw rt = row_tw<LOGM, SB, true>(a, twl, t, q);
  if (rt.lds)
    ntt_body_dio<FpArith, LOGM, LOGE, SB, true, false, RowTwShape<LOGM, SB, true>::on>(
        FpArith(q), (double*)lds, src, store, tw, ni, N, a.logR, first, a.logR == 0, true, 0u,
        a.logN, rt);
  else if (q < kFpPrimeBound)
    ntt_body_dio<FpArith, LOGM, LOGE, SB, true, false>(FpArith(q), (double*)lds, src, store, tw,
                                                        ni, N, a.logR, first, a.logR == 0, true, 0u, a.logN);
  else
    ntt_body_dio<IntArith, LOGM, LOGE, SB, true, false>(IntArith(q), lds, src, store, tw, ni, N,
                                                         a.logR, first, a.logR == 0, true, 0u, a.logN);
}

template <int LOGM, int LOGE, int SB>
__global__ void __launch_bounds__(SB * (1 << (LOGM - LOGE)))
k_ntt_row_mdr(NttArgs a, MdrEpi e) {
  constexpr int M = 1 << LOGM;
  __shared__ u64 lds[SB * (M + 1)];
  __shared__ double twl[RowTwShape<LOGM, SB, true>::size];
  const BlockPos bp = block_pos(a.blocks_per_limb, a.nbatch);
  if constexpr (LOGM == kRowTwLogM) {   // products from operands (N = 2^16): items, not
    if (!e.d) {                         // (item, polynomial) pairs
      mdr_pair_tile<LOGM, LOGE, SB>(a, e, lds, twl, bp);
      return;
    }
  }
  mdr_tile<LOGM, LOGE, SB, 0>(a, e, lds, twl, bp);
}

template <int LOGM, int LOGE, int SB>
void run_row_mdr(const NttArgs& base, const MdrEpi& e, int nlimbs, int nbatch, hipStream_t st) {
  NttArgs a = base;
  a.blocks_per_limb = (1 << a.logR) / SB;
  a.nbatch = nbatch;
  dim3 grid(a.blocks_per_limb * nlimbs * nbatch);
  dim3 block(SB * (1 << (LOGM - LOGE)));
  hipLaunchKernelGGL((k_ntt_row_mdr<LOGM, LOGE, SB>), grid, block, 0, st, a, e);
}

// ---- forward row pass that finishes a plain ModDown
// For limb i of polynomial c of item b the stored element is
//   v = ((u_i - conv_i) P^-1 mod q_i) [+ add_c,i read through X -> X^g] [+ acc_c,i]
// (the final step of ModDown, the (d0, d1) or rotated c0 addend of
// relinearisation and rotation, and the running sum of RotSum), in the order
// of the separate final and addition kernels.
struct MdEpi {
  const u64* u;      // [item][2][ne][N] accumulators
  size_t su;
  PtrsIn add0, add1; // per item [nl][N] or null
  PtrsIn acc;        // per item [2][nl][N] or null
  OutPtrs out;       // per item [2][nl][N]
  const u64* md;     // ModDown table
  uint32_t gadd;
  int K, L, nl, ne, logN;
};

template <int E>
struct MdStore {
  static constexpr bool kRaw = false;
  const u64* u;
  const u64* add;
  const u64* acc;
  u64* out;
  u64 q, pinv, pinvs;
  uint32_t gadd;
  int logN;
  u64 pu[E], pa[E], pc[E];
  __device__ __forceinline__ void prefetch(int i, size_t at) {
    pu[i] = u[at];
    pa[i] = add ? add[galois_src((uint32_t)at, gadd, logN)] : 0;
    pc[i] = acc ? acc[at] : 0;
  }
  __device__ __forceinline__ void put(int i, size_t at, u64 conv) const {
    u64 v = mul_shoup(subm(pu[i], conv, q), pinv, pinvs, q);
    if (add) v = addm(v, pa[i], q);
    if (acc) v = addm(pc[i], v, q);
    out[at] = v;
  }
};

template <int LOGM, int LOGE, int SB>
__global__ void __launch_bounds__(SB * (1 << (LOGM - LOGE)))
k_ntt_row_md(NttArgs a, MdEpi e) {
  constexpr int M = 1 << LOGM;
  __shared__ u64 lds[SB * (M + 1)];
  __shared__ double twl[RowTwShape<LOGM, SB, true>::size];
  const int N = a.N;
  const BlockPos bp = block_pos(a.blocks_per_limb, a.nbatch);
  const int t = bp.limb;                                 // limb = prime index, t < nl
  const int grp = bp.grp;
  const int item = bp.item >> 1, c = bp.item & 1;
  const u64* src = a.src + (size_t)bp.item * a.batch_stride + (size_t)t * N;
  const u64 q = a.mods[t].q;
  const ulonglong2* tw = (const ulonglong2*)(a.tw + (size_t)t * N * 2);
  const u64* ni = a.ninv + 2 * t;
  const MdLayout lay(e.K, e.L);
  MdStore<(1 << LOGE)> store;
  store.u = e.u + (size_t)item * e.su + ((size_t)c * e.ne + t) * N;
  const u64* add = c ? e.add1.p[item] : e.add0.p[item];
  store.add = add ? add + (size_t)t * N : nullptr;
  store.acc = e.acc.p[item] ? e.acc.p[item] + ((size_t)c * e.nl + t) * N : nullptr;
  store.out = e.out.p[item] + ((size_t)c * e.nl + t) * N;
  store.q = q;
  store.pinv = e.md[lay.pinv(t)];
  store.pinvs = e.md[lay.pinv(t) + 1];
  store.gadd = e.gadd;
  store.logN = e.logN;
  const int first = grp * SB;
  const RowTw rt = row_tw<LOGM, SB, true>(a, twl, t, q);
  if (rt.lds)
    ntt_body_dio<FpArith, LOGM, LOGE, SB, true, false, RowTwShape<LOGM, SB, true>::on>(
        FpArith(q), (double*)lds, src, store, tw, ni, N, a.logR, first, a.logR == 0, true, 0u,
        a.logN, rt);
  else if (q < kFpPrimeBound)
    ntt_body_dio<FpArith, LOGM, LOGE, SB, true, false>(FpArith(q), (double*)lds, src, store, tw,
                                                        ni, N, a.logR, first, a.logR == 0, true, 0u, a.logN);
  else
    ntt_body_dio<IntArith, LOGM, LOGE, SB, true, false>(IntArith(q), lds, src, store, tw, ni, N,
                                                         a.logR, first, a.logR == 0, true, 0u, a.logN);
}

template <int LOGM, int LOGE, int SB>
void run_row_md(const NttArgs& base, const MdEpi& e, int nlimbs, int nbatch, hipStream_t st) {
  NttArgs a = base;
  a.blocks_per_limb = (1 << a.logR) / SB;
  a.nbatch = nbatch;
  dim3 grid(a.blocks_per_limb * nlimbs * nbatch);
  dim3 block(SB * (1 << (LOGM - LOGE)));
  hipLaunchKernelGGL((k_ntt_row_md<LOGM, LOGE, SB>), grid, block, 0, st, a, e);
}

// ---- forward row pass of the extended digits fused with the key inner product
// A workgroup owns SB rows of one extended limb t (prime p) and a run of
// batch items.  For each item it transforms the rows of every digit j
// (column pass already done; a digit's own limbs come from the input d in
// NTT form, read through X -> X^gd) and accumulates v * key_j in the
// epilogue, so the transformed digits never go back to memory and the key
// rows, held in registers, are read once per workgroup:
//   u_c[t] = sum_j ext_j[t] * key_{j,c}[t]   (c = 0: the b half, 1: the a half)
// plus, for products (pd), (P mod q_l) times d0 / d1 on limb q_l — the
// operations and order of the separate inner-product kernel.
constexpr int kKsFusedDigits = 4;

struct KsEpi {
  const u64* ext;    // [item][beta][ne][N], columns transformed
  size_t sext;
  const u64* d;      // [item] input in NTT form (limbs 0..l), stride sd; null for
  size_t sd;         //   a product: d = a1 b1 and (d0, d1) formed from the operands
  PtrsIn pa, pb;     //   (item: [2][nl][N])
  const u64* key;    // [beta][2][nprimes][N]
  u64* u;            // [item][2][ne][N]
  size_t su;
  const u64* pd;     // [item][3][nl][N] tensor (d0, d1) or null
  size_t spd;
  u64 pmod, pmods;
  uint32_t gd;
  int nl, ne, beta, alpha, pofs, nprimes, nbatch, items, logN;
};

// 128-bit sums of at most kKsFusedDigits products of residues below 2^60
template <int E>
struct KsAccStore {
  static constexpr bool kRaw = false;
  Acc s0[E], s1[E];
  const u64* kb;     // the digit's key rows on this limb's prime
  const u64* ka;
  u64 pb[E], pa[E];
  __device__ __forceinline__ void prefetch(int i, size_t at) {
    pb[i] = kb[at];
    pa[i] = ka[at];
  }
  __device__ __forceinline__ void put(int i, size_t, u64 v) {
    s0[i].mac(v, pb[i]);
    s1[i].mac(v, pa[i]);
  }
  __device__ __forceinline__ u64 out0(int i, const Mod& m) const { return reduce128(s0[i].hi, s0[i].lo, m); }
  __device__ __forceinline__ u64 out1(int i, const Mod& m) const { return reduce128(s1[i].hi, s1[i].lo, m); }
};

// FP64 primes: each digit's product v * key mod q is taken exactly in FP64
// on the transform's unreduced output (FpArith::mulmod with |v| < 10 q and
// the key below q: the quotient estimate is at most 3 * 2^-53 * 10 q < 0.07
// off, so each product lands in (-0.57 q, 0.57 q)), the at most four digits
// summed as doubles (exact integers below 2.3 q) and rounded once to [0, q)
// at the end, in place of two 128-bit sums and reductions.
template <int E>
struct KsFpStore {
  static constexpr bool kRaw = true;
  FpArith ar;
  double s0[E], s1[E];
  const u64* kb;
  const u64* ka;
  u64 pb[E], pa[E];
  __device__ __forceinline__ explicit KsFpStore(const FpArith& a) : ar(a) {
#pragma unroll
    for (int i = 0; i < E; ++i) s0[i] = s1[i] = 0.0;
  }
  __device__ __forceinline__ void prefetch(int i, size_t at) {
    pb[i] = kb[at];
    pa[i] = ka[at];
  }
  __device__ __forceinline__ void put_raw(int i, size_t, double v) {
    const double b = (double)pb[i], c = (double)pa[i];
    s0[i] += ar.mulmod(v, b, b * ar.qinv);
    s1[i] += ar.mulmod(v, c, c * ar.qinv);
  }
  __device__ __forceinline__ void put(int i, size_t at, u64 v) { put_raw(i, at, (double)v); }
  __device__ __forceinline__ u64 out0(int i, const Mod&) const { return ar.out_fwd(s0[i]); }
  __device__ __forceinline__ u64 out1(int i, const Mod&) const { return ar.out_fwd(s1[i]); }
};

template <class A, int E>
struct KsStoreOf {
  typedef KsAccStore<E> type;
  __device__ __forceinline__ static type make(const A&) { return type(); }
};
template <int E>
struct KsStoreOf<FpArith, E> {
  typedef KsFpStore<E> type;
  __device__ __forceinline__ static type make(const FpArith& ar) { return type(ar); }
};

template <class A, int LOGM, int LOGE, int SB, bool TL = false>
__device__ __forceinline__ void ks_tile(const A ar, u64* lds, const NttArgs& a, const KsEpi& e,
                                        int t, int prime, int first, int item0, int item1,
                                        RowTw rt = RowTw{}) {
  constexpr int M = 1 << LOGM;
  constexpr int E = 1 << LOGE;
  constexpr int TPS = M / E;
  constexpr int NP = (LOGM + LOGE - 1) / LOGE;
  const int N = a.N;
  const size_t NN = (size_t)N;
  // the slots this thread finishes in the last register pass (ntt_body_dio's map)
  const int tid = threadIdx.x;
  const int sp = tid / TPS, lane = tid - sp * TPS;
  const size_t rowbase = (size_t)(first + sp) * M;
  uint32_t at[E];     // within the limb (N <= 2^16)
  {
    constexpr int s0 = (NP - 1) * LOGE;
    constexpr int ls = (LOGM - s0) < LOGE ? (LOGM - s0) : LOGE;
    constexpr int GS = 1 << ls, G = E / GS, si = M >> (s0 + ls);
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int gi = g * TPS + lane;
      const int e0 = (gi / si) * (M >> s0) + gi % si;
#pragma unroll
      for (int k = 0; k < GS; ++k) at[g * GS + k] = (uint32_t)(rowbase + e0 + k * si);
    }
  }
  const int own = t < e.nl ? t / e.alpha : -1;
  const ulonglong2* tw = (const ulonglong2*)(a.tw + (size_t)prime * NN * 2);
  const u64* ni = a.ninv + 2 * prime;
  const Mod m = a.mods[prime];
  const bool prep = (e.pd != nullptr || e.d == nullptr) && t == e.nl - 1;
  // the rows' twiddles serve every digit and item: formed once, up front,
  // where few registers are live
  if constexpr (TL) {
    row_twiddles<LOGM, SB, SB * TPS>(ar, rt, first);
    rt.make = false;
    __syncthreads();
  }
  for (int item = item0; item < item1; ++item) {
    typename KsStoreOf<A, E>::type st = KsStoreOf<A, E>::make(ar);
    // one copy of the transform serves every digit (the key rows of later
    // items come from L2)
#pragma unroll 1
    for (int j = 0; j < e.beta; ++j) {
      st.kb = e.key + ((size_t)(2 * j) * e.nprimes + prime) * NN;
      st.ka = e.key + ((size_t)(2 * j + 1) * e.nprimes + prime) * NN;
      if (j == own && e.d == nullptr) {
        const u64* a1 = e.pa.p[item] + ((size_t)e.nl + t) * NN;
        const u64* b1 = e.pb.p[item] + ((size_t)e.nl + t) * NN;
#pragma unroll
        for (int i = 0; i < E; ++i) {
          st.prefetch(i, at[i]);
          if constexpr (std::is_same<A, FpArith>::value) {
            // exact FP64 product (|.| < 0.57 q), as the store takes the transform's output
            const double x = ar.in(a1[at[i]]), y = ar.in(b1[at[i]]);
            st.put_raw(i, 0, ar.mulmod(x, y, y * ar.qinv));
          } else {
            st.put(i, 0, mulm(a1[at[i]], b1[at[i]], m));
          }
        }
      } else if (j == own) {
        const u64* dt = e.d + (size_t)item * e.sd + (size_t)t * NN;
#pragma unroll
        for (int i = 0; i < E; ++i) {
          st.prefetch(i, at[i]);
          st.put(i, 0, dt[galois_src(at[i], e.gd, e.logN)]);
        }
      } else {
        const u64* src = e.ext + (size_t)item * e.sext + ((size_t)j * e.ne + t) * NN;
        ntt_body_dio<A, LOGM, LOGE, SB, true, false, TL>(ar, (typename A::T*)lds, src, st, tw, ni, N,
                                                         a.logR, first, a.logR == 0, true, 0u,
                                                         a.logN, rt);
        exchange_sync<WaveRows<TPS>::on>();   // the next digit's exchanges reuse the LDS rows
      }
    }
    u64* u0 = e.u + (size_t)item * e.su + (size_t)t * NN;
    u64* u1 = u0 + (size_t)e.ne * NN;
#pragma unroll
    for (int i = 0; i < E; ++i) {
      u64 v0 = st.out0(i, m), v1 = st.out1(i, m);
      if (prep) {
        u64 d0, d1;
        if (e.d == nullptr) {
          const u64* pa0 = e.pa.p[item] + (size_t)t * NN + at[i];
          const u64* pb0 = e.pb.p[item] + (size_t)t * NN + at[i];
          const u64 x0 = pa0[0], x1 = pa0[(size_t)e.nl * NN], y0 = pb0[0], y1 = pb0[(size_t)e.nl * NN];
          d0 = mulm(x0, y0, m);
          d1 = mul2_add(x0, y1, x1, y0, m);
        } else {
          const u64* dp = e.pd + (size_t)item * e.spd + (size_t)t * NN + at[i];
          d0 = dp[0];
          d1 = dp[(size_t)e.nl * NN];
        }
        v0 = addm(v0, mul_shoup(d0, e.pmod, e.pmods, m.q), m.q);
        v1 = addm(v1, mul_shoup(d1, e.pmod, e.pmods, m.q), m.q);
      }
      u0[at[i]] = v0;
      u1[at[i]] = v1;
    }
  }
}

// Workgroups run on XCD (workgroup index) mod 8, each XCD with its own L2.
constexpr unsigned kXcds = 8;

// grid: one workgroup per (tile = row group + groups * limb, item group).
// The item groups of a tile read the same key rows; they take consecutive
// slots (workgroup index / 8) of one XCD, so that they run together and
// share those rows in its L2 (a round-robin order would fetch the key once
// per item from HBM).  Grids whose tile count is not a multiple of 8 keep
// the item group fastest.
// At most 168 VGPRs for three waves per SIMD: faster than two waves, the
// kernel being latency-bound.
template <int LOGM, int LOGE, int SB>
__global__ void __launch_bounds__(SB * (1 << (LOGM - LOGE)), 3)
k_ntt_row_ks(NttArgs a, KsEpi e) {
  constexpr int M = 1 << LOGM;
  __shared__ u64 lds[SB * (M + 1)];
  __shared__ double twl[RowTwShape<LOGM, SB, true>::size];
  const unsigned groups = (1u << a.logR) / SB;
  const unsigned nig = (unsigned)((e.nbatch + e.items - 1) / e.items);
  const unsigned tiles = groups * (unsigned)e.ne;
  const unsigned b = blockIdx.x;
  unsigned ig, tile;
  if (nig > 1 && tiles % kXcds == 0) {
    const unsigned slot = b / kXcds;
    ig = slot % nig;
    tile = (slot / nig) * kXcds + b % kXcds;
  } else {
    ig = b % nig;
    tile = b / nig;
  }
  const int rg = (int)(tile % groups);
  const int t = (int)(tile / groups);
  const int prime = t < e.nl ? t : e.pofs + (t - e.nl);
  const int item0 = (int)ig * e.items, item1 = min(item0 + e.items, e.nbatch);
  const u64 q = a.mods[prime].q;
  const RowTw rt = row_tw<LOGM, SB, true>(a, twl, prime, q);
  if (rt.lds)
    ks_tile<FpArith, LOGM, LOGE, SB, RowTwShape<LOGM, SB, true>::on>(FpArith(q), lds, a, e, t, prime,
                                                                      rg * SB, item0, item1, rt);
  else if (q < kFpPrimeBound)
    ks_tile<FpArith, LOGM, LOGE, SB>(FpArith(q), lds, a, e, t, prime, rg * SB, item0, item1);
  else
    ks_tile<IntArith, LOGM, LOGE, SB>(IntArith(q), lds, a, e, t, prime, rg * SB, item0, item1);
}

// ---- ModUp fused into the forward column pass of the extended digits
// Element at of target limb t (prime p) of digit j is the digit's fast base
// conversion  sum_i z_i[at] (Qhat_i 2^64 mod p)  reduced by REDC, z_i the
// scaled coefficients x_i Qhat_i^-1 mod q_i that the inverse transform wrote
// (modup_ninv).  The column pass forms it where it would load the ModUp
// kernel's output, so the digits' coefficient form never goes to memory;
// the digit's limbs at a tile's columns are read by every target of the
// digit, mostly from L2.
struct ModUpSrc {
  const u64* x;      // [nbatch][nl][N] scaled coefficients
  size_t sx;
  const u64* tab;    // modup_table of the level
  int ne;
};

template <int MAXA>
struct ModUpLoad {
  static constexpr bool kCustom = true;
  const u64* z;      // the digit's first limb (limbs at stride N)
  const u64* cst;    // the target's kMaxAlpha constants, Montgomery form
  Mod m;
  int da, N;
  __device__ __forceinline__ u64 get(int, size_t at) const {
    Acc30 acc;
#pragma unroll
    for (int i = 0; i < MAXA; ++i) {
      const u64 v = z[(size_t)min(i, da - 1) * N + at];
      acc.mac(Split30(i < da ? v : 0), Split30(cst[i]));
      if ((i & 7) == 7) acc.fold();
    }
    return acc.redc(m);
  }
  template <class A>
  __device__ __forceinline__ typename A::T get_t(const A& ar, int i, size_t at) const {
    return ar.in(get(i, at));
  }
};

// Grid: tiles (batch item b, digit j, column group) times the digit's
// targets, XCD-aware.  Workgroups are dealt round-robin to the 8 XCDs, so
// workgroup w runs on XCD w mod 8; the targets of one tile take consecutive
// slots w / 8 of one XCD and re-read the tile's digit limbs from that XCD's
// L2.  The grid is padded to whole tiles per XCD (extra workgroups exit).
template <int LOGE, int SB, int MAXA>
__global__ void __launch_bounds__(SB * (1 << (8 - LOGE)))
k_ntt_col_modup(NttArgs a, ModUpSrc mu, int ntargets) {
  constexpr int LOGM = 8;
  __shared__ u64 lds[SB * ((1 << LOGM) + 1)];
  const unsigned slot = blockIdx.x / kXcds;
  const unsigned tile = (slot / (unsigned)ntargets) * kXcds + blockIdx.x % kXcds;
  if (tile >= (unsigned)(a.nbatch * a.blocks_per_limb)) return;
  BlockPos bp;
  bp.limb = (int)(slot % (unsigned)ntargets);
  bp.item = (int)(tile % (unsigned)a.nbatch);
  bp.grp = (int)(tile / (unsigned)a.nbatch);
  const int N = a.N;
  const int j = bp.item % a.dcount, b = bp.item / a.dcount;
  const int lo = j * a.dalpha, hi = min(lo + a.dalpha, a.nq), da = hi - lo;
  if (bp.limb >= a.dtotal - da) return;
  const int t = bp.limb >= lo ? bp.limb + da : bp.limb;
  const int prime = t < a.nq ? t : a.pofs + (t - a.nq);
  const u64 q = a.mods[prime].q;
  ModUpLoad<MAXA> ld;
  ld.z = mu.x + (size_t)b * mu.sx + (size_t)lo * N;
  ld.cst = mu.tab + modup_digit_words(mu.ne) * j + 2 * kMaxAlpha + (size_t)t * kMaxAlpha;
  ld.m = a.mods[prime];
  ld.da = da;
  ld.N = N;
  PlainStore store{a.dst + (size_t)bp.item * a.dst_stride + (size_t)t * N};
  const ulonglong2* tw = (const ulonglong2*)(a.tw + (size_t)prime * N * 2);
  const u64* ni = a.ninv + 2 * prime;
  const int first = bp.grp * SB;
  if (q < kFpPrimeBound)
    ntt_body_dio<FpArith, LOGM, LOGE, SB, false, false>(FpArith(q), (double*)lds, nullptr, store,
                                                         tw, ni, N, a.logR, first, true, false, 0u,
                                                         a.logN, RowTw{}, ld);
  else
    ntt_body_dio<IntArith, LOGM, LOGE, SB, false, false>(IntArith(q), lds, nullptr, store, tw, ni,
                                                          N, a.logR, first, true, false, 0u, a.logN,
                                                          RowTw{}, ld);
}

template <int LOGE, int SB>
void run_col_modup(const NttArgs& base, const ModUpSrc& mu, int alpha, int nlimbs, int nbatch,
                   hipStream_t st) {
  NttArgs a = base;
  a.blocks_per_limb = (a.N >> a.logR) / SB;
  a.nbatch = nbatch;
  const unsigned tiles = (unsigned)(a.blocks_per_limb * nbatch);
  dim3 grid(((tiles + kXcds - 1) / kXcds) * kXcds * (unsigned)nlimbs);
  dim3 block(SB * (1 << (8 - LOGE)));
  if (alpha <= 4)
    hipLaunchKernelGGL((k_ntt_col_modup<LOGE, SB, 4>), grid, block, 0, st, a, mu, nlimbs);
  else if (alpha == 7)
    hipLaunchKernelGGL((k_ntt_col_modup<LOGE, SB, 7>), grid, block, 0, st, a, mu, nlimbs);
  else if (alpha <= 9)
    hipLaunchKernelGGL((k_ntt_col_modup<LOGE, SB, 9>), grid, block, 0, st, a, mu, nlimbs);
  else if (alpha <= kMaxAlpha)
    hipLaunchKernelGGL((k_ntt_col_modup<LOGE, SB, 16>), grid, block, 0, st, a, mu, nlimbs);
  else
    PPST_THROW(ST_EINVAL, "digit size above 16 limbs");
}

// ---- inverse row pass of a product's d2 = a1 b1, formed on load
template <int LOGE, int SB>
__global__ void __launch_bounds__(SB * (1 << (8 - LOGE)))
k_ntt_row_prod(NttArgs a, PtrsIn pa, PtrsIn pb) {
  constexpr int LOGM = 8;
  __shared__ u64 lds[SB * ((1 << LOGM) + 1)];
  __shared__ double twl[RowTwShape<LOGM, SB, true>::size];
  const BlockPos bp = block_pos(a.blocks_per_limb, a.nbatch);
  const int N = a.N;
  const int t = bp.limb;                                 // limb = prime index, t <= l
  ProdLoad ld;
  ld.a = pa.p[bp.item] + ((size_t)a.nq + t) * N;         // a1 (a.nq = l + 1 limbs)
  ld.b = pb.p[bp.item] + ((size_t)a.nq + t) * N;         // b1
  ld.m = a.mods[t];
  const u64 q = ld.m.q;
  PlainStore store{a.dst + (size_t)bp.item * a.dst_stride + (size_t)t * N};
  const ulonglong2* tw = (const ulonglong2*)(a.tw + (size_t)t * N * 2);
  const u64* ni = a.ninv + 2 * t;
  const int first = bp.grp * SB;
  const RowTw rt = row_tw<LOGM, SB, true>(a, twl, t, q);
  if (rt.lds)
    ntt_body_dio<FpArith, LOGM, LOGE, SB, true, true, RowTwShape<LOGM, SB, true>::on>(
        FpArith(q), (double*)lds, nullptr, store, tw, ni, N, a.logR, first, true, false, 0u, a.logN,
        rt, ld);
  else if (q < kFpPrimeBound)
    ntt_body_dio<FpArith, LOGM, LOGE, SB, true, true>(FpArith(q), (double*)lds, nullptr, store, tw,
                                                       ni, N, a.logR, first, true, false, 0u,
                                                       a.logN, RowTw{}, ld);
  else
    ntt_body_dio<IntArith, LOGM, LOGE, SB, true, true>(IntArith(q), lds, nullptr, store, tw, ni, N,
                                                        a.logR, first, true, false, 0u, a.logN,
                                                        RowTw{}, ld);
}

// ---- forward row pass that finishes a rescale
// For limb i < l of polynomial c the stored element is
//   ((k_i a_c,i or a_c,i) - corr_i) q_l^-1 mod q_i
// where corr is the transformed centred lift of the dropped limb and k an
// optional constant multiplier (Mul(P) by a constant, level alignment) —
// the operations of the separate scalar-product and final kernels.
struct RsEpi {
  PtrsIn a;          // polynomial c of the launch (limbs 0..l)
  OutPtrs out;       // polynomial c of the launch (limbs 0..l-1)
  const u64* rc;     // rescale table of level l
  int mulk;
  u64 k[kMaxPrimes], kp[kMaxPrimes];
};

template <int E>
struct RsStore {
  static constexpr bool kRaw = false;
  const u64* a;
  u64* out;
  u64 q, qlinv, qlinvs, k, kp;
  int mulk;
  u64 pa[E];
  __device__ __forceinline__ void prefetch(int i, size_t at) { pa[i] = a[at]; }
  __device__ __forceinline__ void put(int i, size_t at, u64 corr) const {
    const u64 x = mulk ? mul_shoup(pa[i], k, kp, q) : pa[i];
    out[at] = mul_shoup(subm(x, corr, q), qlinv, qlinvs, q);
  }
};

template <int LOGM, int LOGE, int SB>
__global__ void __launch_bounds__(SB * (1 << (LOGM - LOGE)))
k_ntt_row_rs(NttArgs a, RsEpi e) {
  constexpr int M = 1 << LOGM;
  __shared__ u64 lds[SB * (M + 1)];
  __shared__ double twl[RowTwShape<LOGM, SB, true>::size];
  const int N = a.N;
  const BlockPos bp = block_pos(a.blocks_per_limb, a.nbatch);
  const int t = bp.limb;                                 // limb = prime index, t < l
  const int grp = bp.grp;
  const int c = bp.item;
  const u64* src = a.src + (size_t)c * a.batch_stride + (size_t)t * N;
  const u64 q = a.mods[t].q;
  const ulonglong2* tw = (const ulonglong2*)(a.tw + (size_t)t * N * 2);
  const u64* ni = a.ninv + 2 * t;
  RsStore<(1 << LOGE)> store;
  store.a = e.a.p[c] + (size_t)t * N;
  store.out = e.out.p[c] + (size_t)t * N;
  store.q = q;
  store.qlinv = e.rc[3 * t];
  store.qlinvs = e.rc[3 * t + 1];
  store.mulk = e.mulk;
  store.k = e.k[t];
  store.kp = e.kp[t];
  const int first = grp * SB;
  const RowTw rt = row_tw<LOGM, SB, true>(a, twl, t, q);
  if (rt.lds)
    ntt_body_dio<FpArith, LOGM, LOGE, SB, true, false, RowTwShape<LOGM, SB, true>::on>(
        FpArith(q), (double*)lds, src, store, tw, ni, N, a.logR, first, a.logR == 0, true, 0u,
        a.logN, rt);
  else if (q < kFpPrimeBound)
    ntt_body_dio<FpArith, LOGM, LOGE, SB, true, false>(FpArith(q), (double*)lds, src, store, tw,
                                                        ni, N, a.logR, first, a.logR == 0, true, 0u, a.logN);
  else
    ntt_body_dio<IntArith, LOGM, LOGE, SB, true, false>(IntArith(q), lds, src, store, tw, ni, N,
                                                         a.logR, first, a.logR == 0, true, 0u, a.logN);
}

template <int LOGM, int LOGE, int SB>
void run_row_rs(const NttArgs& base, const RsEpi& e, int nlimbs, int nbatch, hipStream_t st) {
  NttArgs a = base;
  a.blocks_per_limb = (1 << a.logR) / SB;
  a.nbatch = nbatch;
  dim3 grid(a.blocks_per_limb * nlimbs * nbatch);
  dim3 block(SB * (1 << (LOGM - LOGE)));
  hipLaunchKernelGGL((k_ntt_row_rs<LOGM, LOGE, SB>), grid, block, 0, st, a, e);
}

typedef void (*PassFn)(const NttArgs&, int, int, hipStream_t);

template <int LOGM, int LOGE, int SB, bool ROWS, bool INV, bool DIO>
void run_pass(const NttArgs& base, int nlimbs, int nbatch, hipStream_t st) {
  NttArgs a = base;
  const int nsub = ROWS ? (1 << a.logR) : (a.N >> a.logR);
  a.blocks_per_limb = nsub / SB;
  a.nbatch = nbatch;
  dim3 grid(a.blocks_per_limb * nlimbs * nbatch);
  dim3 block(SB * (1 << (LOGM - LOGE)));
  hipLaunchKernelGGL((k_ntt_pass<LOGM, LOGE, SB, ROWS, INV, DIO>), grid, block, 0, st, a);
}

// workgroups of a kernel the device holds at once (occupancy x CUs), asked
// of the runtime once per kernel
template <class K>
unsigned resident_blocks(K kernel, int block) {
  static unsigned cached = 0;
  if (!cached) {
    int per_cu = 0, cus = 0, dev = 0;
    HIP_CHECK(hipGetDevice(&dev));
    HIP_CHECK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_CHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0));
    cached = (unsigned)std::max(1, per_cu) * (unsigned)std::max(1, cus);
  }
  return cached;
}

template <int LOGM, int LOGE, int SB, bool ROWS, bool INV, bool DIO>
void run_pass_persistent(const NttArgs& base, int nlimbs, int nbatch, hipStream_t st) {
  NttArgs a = base;
  const int nsub = ROWS ? (1 << a.logR) : (a.N >> a.logR);
  a.blocks_per_limb = nsub / SB;
  a.nbatch = nbatch;
  const unsigned ntiles = (unsigned)a.blocks_per_limb * nlimbs * nbatch;
  const int block = SB * (1 << (LOGM - LOGE));
  auto kern = k_ntt_pass_persistent<LOGM, LOGE, SB, ROWS, INV, DIO>;
  const unsigned grid = std::min(ntiles, resident_blocks(kern, block));
  hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, st, a, ntiles);
}

// Variant tables.  N = 2^16 runs a column pass and a row pass of 2^8 points;
// N = 2^12 a single row pass of 2^12 points.  A variant fixes the register
// radix (E = 2^LOGE elements per thread) and the sub-problems per workgroup.
struct Variant {
  const char* name;
  PassFn fwd, inv;
};
// "D" variants load the first register pass from and store the last one to
// global memory directly (ntt_body_dio).
#define V16C(LE, SB, D) {D ? "col:E" #LE ",SB" #SB ",D" : "col:E" #LE ",SB" #SB, \
                         run_pass<8, LE, SB, false, false, D>, run_pass<8, LE, SB, false, true, D>}
#define V16R(LE, SB, D) {D ? "row:E" #LE ",SB" #SB ",D" : "row:E" #LE ",SB" #SB, \
                         run_pass<8, LE, SB, true, false, D>, run_pass<8, LE, SB, true, true, D>}
#define V12(LE, D) {D ? "full:E" #LE ",D" : "full:E" #LE, run_pass<12, LE, 1, true, false, D>, \
                    run_pass<12, LE, 1, true, true, D>}
// "P": the persistent launch of a direct variant (run_pass_persistent)
#define V16CP(LE, SB) {"col:E" #LE ",SB" #SB ",D,P", run_pass_persistent<8, LE, SB, false, false, true>, \
                       run_pass_persistent<8, LE, SB, false, true, true>}
#define V16RP(LE, SB) {"row:E" #LE ",SB" #SB ",D,P", run_pass_persistent<8, LE, SB, true, false, true>, \
                       run_pass_persistent<8, LE, SB, true, true, true>}
const Variant kCol16[] = {V16C(4, 16, false), V16C(3, 16, false), V16C(2, 16, false),
                          V16C(3, 8, false),  V16C(2, 8, false),  V16C(3, 16, true),
                          V16C(2, 16, true),  V16C(2, 8, true),   V16C(4, 16, true),
                          V16CP(3, 16),       V16CP(2, 16)};
const Variant kRow16[] = {V16R(4, 16, false), V16R(4, 4, false), V16R(3, 8, false),
                          V16R(2, 4, false),  V16R(3, 4, false), V16R(2, 8, false),
                          V16R(3, 4, true),   V16R(2, 4, true),  V16R(3, 8, true),
                          V16R(4, 4, true),   V16RP(3, 4),       V16RP(2, 4)};
const Variant kFull12[] = {V12(4, false), V12(3, false), V12(2, false), V12(4, true), V12(3, true)};
constexpr int kNCol16 = sizeof(kCol16) / sizeof(kCol16[0]);
constexpr int kNRow16 = sizeof(kRow16) / sizeof(kRow16[0]);
constexpr int kNFull12 = sizeof(kFull12) / sizeof(kFull12[0]);

}  // namespace

// twiddle tables of one direction; PPST_NTT_ROW_TWIDDLES=0 makes the row
// passes read every entry from the full table
static bool row_twiddles_enabled() {
  static const bool on = [] {
    const char* e = std::getenv("PPST_NTT_ROW_TWIDDLES");
    return !(e && e[0] == '0');
  }();
  return on;
}

static void set_tables(NttArgs& a, const Shared& sh, bool inverse) {
  a.tw = inverse ? sh.tab.inv.p : sh.tab.fwd.p;
  const bool rows = row_twiddles_enabled() && sh.P.logN == 16;
  a.rowf = rows ? (const double*)(inverse ? sh.tab.rowf_inv.p : sh.tab.rowf_fwd.p) : nullptr;
  a.comm = rows ? (inverse ? sh.tab.comm_inv.p : sh.tab.comm_fwd.p) : nullptr;
}

int ntt_bucket(int nlimbs_total) {
  if (nlimbs_total <= 4) return 0;
  if (nlimbs_total <= 16) return 1;
  if (nlimbs_total <= 40) return 2;
  if (nlimbs_total <= 128) return 3;
  return 4;
}

static void launch_passes(const Shared& sh, NttArgs a, const NttLaunch& L, bool inverse,
                          hipStream_t st) {
  const Params& P = sh.P;
  const int b = ntt_bucket(L.nlimbs * L.nbatch);
  const NttPlan& plan = sh.ntt_plan;
  if (P.logN == 16) {
    a.logR = 8;
    const Variant& c = kCol16[plan.v[inverse][0][b]];
    const Variant& r = kRow16[plan.v[inverse][1][b]];
    a.src = L.src;
    a.dst = L.dst;
    if (!inverse) {
      c.fwd(a, L.nlimbs, L.nbatch, st);
      a.src = L.dst;
      a.batch_stride = a.dst_stride;
      r.fwd(a, L.nlimbs, L.nbatch, st);
    } else {
      r.inv(a, L.nlimbs, L.nbatch, st);
      a.src = L.dst;
      a.batch_stride = a.dst_stride;
      c.inv(a, L.nlimbs, L.nbatch, st);
    }
  } else if (P.logN == 12) {
    a.logR = 0;
    a.src = L.src;
    a.dst = L.dst;
    const Variant& f = kFull12[plan.v[inverse][1][b]];
    (inverse ? f.inv : f.fwd)(a, L.nlimbs, L.nbatch, st);
  } else {
    PPST_THROW(ST_EINVAL, "NTT supports log2 N in {12, 16}");
  }
}

void ntt(const Shared& sh, const NttLaunch& L, bool inverse, hipStream_t st) {
  const Params& P = sh.P;
  if (L.nlimbs <= 0 || L.nbatch <= 0) return;
  // every limb must map onto a prime of the table (the map is monotone in t)
  {
    int tmax = (L.nlimbs - 1) + ((L.nlimbs - 1) >= L.skip_lo ? (L.skip_hi - L.skip_lo) : 0);
    if (L.digit_alpha > 0) {
      int most = 0;
      for (int j = 0; j < L.digit_count; ++j) {
        const int lo = j * L.digit_alpha, hi = std::min(lo + L.digit_alpha, L.nq);
        if (hi <= lo) PPST_THROW(ST_EINVAL, "NTT digit mode: empty digit");
        most = std::max(most, L.digit_total - (hi - lo));
      }
      if (L.nlimbs != most) PPST_THROW(ST_EINVAL, "NTT digit mode: limb count mismatch");
      tmax = L.digit_total - 1;
    }
    const int pmax = tmax < L.nq ? tmax : L.pofs + (tmax - L.nq);
    const int pmin = 0 < L.nq ? 0 : L.pofs - L.nq;
    if (pmax >= P.nprimes || pmin < 0 || L.skip_hi < L.skip_lo)
      PPST_THROW(ST_EINVAL, "NTT limb map leaves the prime table");
  }
  NttArgs a{};
  a.mods = (const Mod*)sh.tab.mods.p;
  set_tables(a, sh, inverse);
  a.ninv = L.ninv ? L.ninv : sh.tab.ninv.p;
  a.batch_stride = L.batch_stride;
  a.dst_stride = L.dst_stride == ~(size_t)0 ? L.batch_stride : L.dst_stride;
  a.N = P.N;
  a.logN = P.logN;
  a.nq = L.nq;
  a.pofs = L.pofs;
  a.skip_lo = L.skip_lo;
  a.skip_hi = L.skip_hi;
  a.dalpha = L.digit_alpha;
  a.dcount = L.digit_count;
  a.dtotal = L.digit_total;
  if (L.galois != 0 && (!inverse || L.src == L.dst || L.galois >= 2u * (uint32_t)P.N || !(L.galois & 1)))
    PPST_THROW(ST_EINVAL, "NTT: a Galois read needs an out-of-place inverse transform and odd g < 2N");
  a.galois = L.galois;
  launch_passes(sh, a, L, inverse, st);
  HIP_CHECK(hipGetLastError());
}

typedef void (*MdrFn)(const NttArgs&, const MdrEpi&, int, int, hipStream_t);

// the fused row pass matching a row variant of the plan (same register radix
// and workgroup shape where one exists)
static MdrFn mdr_variant(int logN, int row_index) {
  if (logN == 12) {
    const int le = (row_index == 0 || row_index == 3) ? 4 : 3;
    return le == 4 ? run_row_mdr<12, 4, 1> : run_row_mdr<12, 3, 1>;
  }
  switch (row_index) {
    case 1: case 9: return run_row_mdr<8, 4, 4>;
    case 2: case 8: return run_row_mdr<8, 3, 8>;
    case 3: case 7: case 11: return run_row_mdr<8, 2, 4>;
    default: return run_row_mdr<8, 3, 4>;
  }
}

void ntt_fwd_mdr_final(const Shared& sh, u64* corr, int level, int nbatch, const MdrTail& tail,
                       hipStream_t st) {
  const Params& P = sh.P;
  if (level < 1 || nbatch <= 0) return;
  const size_t N = P.N;
  NttArgs a{};
  a.mods = (const Mod*)sh.tab.mods.p;
  set_tables(a, sh, false);
  a.ninv = sh.tab.ninv.p;
  a.N = P.N;
  a.logN = P.logN;
  a.nq = level;
  a.pofs = P.L + 1;
  a.skip_lo = a.skip_hi = 1 << 30;
  a.dalpha = 0;
  a.dcount = 1;
  a.dtotal = 0;
  a.galois = 0;
  a.batch_stride = a.dst_stride = (size_t)level * N;
  const int b = ntt_bucket(level * 2 * nbatch);
  const NttPlan& plan = sh.ntt_plan;
  if (P.logN == 16) {
    a.logR = 8;
    a.src = corr;
    a.dst = corr;
    kCol16[plan.v[0][0][b]].fwd(a, level, 2 * nbatch, st);
  } else if (P.logN == 12) {
    a.logR = 0;
  } else {
    PPST_THROW(ST_EINVAL, "NTT supports log2 N in {12, 16}");
  }
  const MdrFn f = mdr_variant(P.logN, plan.v[0][1][b]);
  MdrEpi e{};
  e.su = tail.su;
  e.sd = tail.sd;
  e.md = sh.tab.moddown.p;
  e.rc = tail.rc;
  e.K = P.K;
  e.L = P.L;
  e.level = level;
  e.ne = level + 1 + P.K;
  e.nl = level + 1;
  for (int b0 = 0; b0 < nbatch; b0 += kPtrBatch) {
    const int nb = std::min(kPtrBatch, nbatch - b0);
    for (int i = 0; i < nb; ++i) e.out.p[i] = tail.out[b0 + i];
    e.u = tail.u + (size_t)b0 * tail.su;
    if (tail.d) {
      e.d = tail.d + (size_t)b0 * tail.sd;
    } else {
      e.d = nullptr;
      for (int i = 0; i < nb; ++i) {
        e.pa.p[i] = tail.pa[b0 + i];
        e.pb.p[i] = tail.pb[b0 + i];
      }
    }
    a.src = corr + (size_t)b0 * 2 * level * N;
    f(a, e, level, tail.d ? 2 * nb : nb, st);   // operand form: one workgroup per item
  }
  HIP_CHECK(hipGetLastError());
}

typedef void (*MdFn)(const NttArgs&, const MdEpi&, int, int, hipStream_t);

static MdFn md_variant(int logN, int row_index) {
  if (logN == 12) {
    const int le = (row_index == 0 || row_index == 3) ? 4 : 3;
    return le == 4 ? run_row_md<12, 4, 1> : run_row_md<12, 3, 1>;
  }
  switch (row_index) {
    case 1: case 9: return run_row_md<8, 4, 4>;
    case 2: case 8: return run_row_md<8, 3, 8>;
    case 3: case 7: case 11: return run_row_md<8, 2, 4>;
    default: return run_row_md<8, 3, 4>;
  }
}

bool modup_col_ok() {
  static const bool enabled = [] {
    const char* v = std::getenv("PPST_MODUP_COL");
    return !(v && v[0] == '0');
  }();
  return enabled;
}

// the fused ModUp + column pass shape: PPST_MODUP_COL=E,SB (log2 of the
// register radix, workgroup columns) picks another
static int modup_col_variant() {
  static const int v = [] {
    const char* e = std::getenv("PPST_MODUP_COL");
    if (!e || !e[0] || e[0] == '1') return 0;
    if (!std::strcmp(e, "2,16")) return 1;
    if (!std::strcmp(e, "4,16")) return 2;
    if (!std::strcmp(e, "3,8")) return 3;
    return 0;
  }();
  return v;
}

bool ks_fused_ok(const Params& P, int level) {
  static const bool enabled = [] {
    const char* v = std::getenv("PPST_KS_FUSED");
    return !(v && v[0] == '0');
  }();
  return enabled && P.logN == 16 && P.beta(level) <= kKsFusedDigits;
}

void ntt_inv_prod(const Shared& sh, const u64* const* pa, const u64* const* pb, u64* x, int level,
                  int nbatch, const u64* ninv, hipStream_t st) {
  const Params& P = sh.P;
  if (nbatch <= 0) return;
  if (P.logN != 16) PPST_THROW(ST_EINVAL, "the product's inverse transform needs N = 2^16");
  const int nl = level + 1;
  NttArgs a{};
  a.mods = (const Mod*)sh.tab.mods.p;
  set_tables(a, sh, true);
  a.ninv = ninv ? ninv : sh.tab.ninv.p;
  a.N = P.N;
  a.logN = P.logN;
  a.logR = 8;
  a.nq = nl;
  a.pofs = P.L + 1;
  a.skip_lo = a.skip_hi = 1 << 30;
  a.dalpha = 0;
  a.dcount = 1;
  a.dtotal = 0;
  a.galois = 0;
  a.batch_stride = a.dst_stride = (size_t)nl * P.N;
  constexpr int LOGE = 2, SB = 4;
  a.blocks_per_limb = (1 << a.logR) / SB;
  for (int b0 = 0; b0 < nbatch; b0 += kPtrBatch) {
    const int nb = std::min(kPtrBatch, nbatch - b0);
    PtrsIn A, B;
    for (int i = 0; i < nb; ++i) {
      A.p[i] = pa[b0 + i];
      B.p[i] = pb[b0 + i];
    }
    a.dst = x + (size_t)b0 * a.dst_stride;
    a.nbatch = nb;
    dim3 grid((unsigned)(a.blocks_per_limb * nl * nb));
    hipLaunchKernelGGL((k_ntt_row_prod<LOGE, SB>), grid, dim3(SB * (1 << (8 - LOGE))), 0, st, a,
                       A, B);
  }
  // the column pass of the plan, in place
  a.src = x;
  a.dst = x;
  kCol16[sh.ntt_plan.v[1][0][ntt_bucket(nl * nbatch)]].inv(a, nl, nbatch, st);
  HIP_CHECK(hipGetLastError());
}

void ntt_fwd_ks_fused(const Shared& sh, const KsTail& tail, int level, int nbatch, hipStream_t st) {
  const Params& P = sh.P;
  if (nbatch <= 0) return;
  if (!ks_fused_ok(P, level)) PPST_THROW(ST_EINVAL, "fused key switch needs N = 2^16 and at most 4 digits");
  const int nl = level + 1, ne = nl + P.K, beta = P.beta(level);
  const size_t N = P.N;
  NttArgs a{};
  a.mods = (const Mod*)sh.tab.mods.p;
  set_tables(a, sh, false);
  a.ninv = sh.tab.ninv.p;
  a.N = P.N;
  a.logN = P.logN;
  a.logR = 8;
  a.nq = nl;
  a.pofs = P.L + 1;
  a.skip_lo = a.skip_hi = 1 << 30;
  a.dalpha = P.alpha;
  a.dcount = beta;
  a.dtotal = ne;
  a.galois = 0;
  a.batch_stride = a.dst_stride = (size_t)ne * N;
  int most = 0;
  for (int j = 0; j < beta; ++j) most = std::max(most, ne - (P.digit_hi(j, level) - P.digit_lo(j)));
  const int b = ntt_bucket(most * nbatch * beta);
  a.src = tail.ext;
  a.dst = tail.ext;
  if (tail.x) {
    const ModUpSrc mu{tail.x, tail.sx, modup_table(sh, level), ne};
    switch (modup_col_variant()) {
      case 1: run_col_modup<2, 16>(a, mu, P.alpha, most, nbatch * beta, st); break;
      case 2: run_col_modup<4, 16>(a, mu, P.alpha, most, nbatch * beta, st); break;
      case 3: run_col_modup<3, 8>(a, mu, P.alpha, most, nbatch * beta, st); break;
      default: run_col_modup<3, 16>(a, mu, P.alpha, most, nbatch * beta, st); break;
    }
  } else {
    kCol16[sh.ntt_plan.v[0][0][b]].fwd(a, most, nbatch * beta, st);
  }
  KsEpi e{};
  e.ext = tail.ext;
  e.sext = (size_t)beta * ne * N;
  e.d = tail.d;
  e.sd = tail.sd;
  if (!tail.d) {
    if (!tail.pa || !tail.pb || nbatch > kPtrBatch) PPST_THROW(ST_EINVAL, "product operands missing");
    for (int i = 0; i < nbatch; ++i) {
      e.pa.p[i] = tail.pa[i];
      e.pb.p[i] = tail.pb[i];
    }
  }
  e.key = tail.key;
  e.u = tail.u;
  e.su = 2 * (size_t)ne * N;
  e.pd = tail.pd;
  e.spd = tail.spd;
  e.pmod = tail.pmod;
  e.pmods = tail.pmods;
  e.gd = tail.gd;
  e.nl = nl;
  e.ne = ne;
  e.beta = beta;
  e.alpha = P.alpha;
  e.pofs = P.L + 1;
  e.nprimes = P.nprimes;
  e.nbatch = nbatch;
  e.logN = P.logN;
  e.items = std::min(nbatch, 8);
  constexpr int LOGM = 8, LOGE = 2, SB = 4;
  const int groups = (1 << a.logR) / SB;
  const int nig = (nbatch + e.items - 1) / e.items;
  dim3 grid((unsigned)(nig * groups * ne));
  dim3 block(SB * (1 << (LOGM - LOGE)));
  hipLaunchKernelGGL((k_ntt_row_ks<LOGM, LOGE, SB>), grid, block, 0, st, a, e);
  HIP_CHECK(hipGetLastError());
}

void ntt_fwd_md_final(const Shared& sh, u64* conv, int level, int nbatch, const MdTail& tail,
                      hipStream_t st) {
  const Params& P = sh.P;
  if (nbatch <= 0) return;
  const int nl = level + 1;
  const size_t N = P.N;
  NttArgs a{};
  a.mods = (const Mod*)sh.tab.mods.p;
  set_tables(a, sh, false);
  a.ninv = sh.tab.ninv.p;
  a.N = P.N;
  a.logN = P.logN;
  a.nq = nl;
  a.pofs = P.L + 1;
  a.skip_lo = a.skip_hi = 1 << 30;
  a.dalpha = 0;
  a.dcount = 1;
  a.dtotal = 0;
  a.galois = 0;
  a.batch_stride = a.dst_stride = (size_t)nl * N;
  const int b = ntt_bucket(nl * 2 * nbatch);
  const NttPlan& plan = sh.ntt_plan;
  if (P.logN == 16) {
    a.logR = 8;
    a.src = conv;
    a.dst = conv;
    kCol16[plan.v[0][0][b]].fwd(a, nl, 2 * nbatch, st);
  } else if (P.logN == 12) {
    a.logR = 0;
  } else {
    PPST_THROW(ST_EINVAL, "NTT supports log2 N in {12, 16}");
  }
  const MdFn f = md_variant(P.logN, plan.v[0][1][b]);
  MdEpi e{};
  e.su = tail.su;
  e.md = sh.tab.moddown.p;
  e.gadd = tail.gadd;
  e.K = P.K;
  e.L = P.L;
  e.nl = nl;
  e.ne = nl + P.K;
  e.logN = P.logN;
  for (int b0 = 0; b0 < nbatch; b0 += kPtrBatch) {
    const int nb = std::min(kPtrBatch, nbatch - b0);
    for (int i = 0; i < nb; ++i) {
      e.out.p[i] = tail.out[b0 + i];
      e.add0.p[i] = tail.add0 ? tail.add0[b0 + i] : nullptr;
      e.add1.p[i] = tail.add1 ? tail.add1[b0 + i] : nullptr;
      e.acc.p[i] = tail.acc ? tail.acc[b0 + i] : nullptr;
    }
    e.u = tail.u + (size_t)b0 * tail.su;
    a.src = conv + (size_t)b0 * 2 * nl * N;
    f(a, e, nl, 2 * nb, st);
  }
  HIP_CHECK(hipGetLastError());
}

typedef void (*RsFn)(const NttArgs&, const RsEpi&, int, int, hipStream_t);

static RsFn rs_variant(int logN, int row_index) {
  if (logN == 12) {
    const int le = (row_index == 0 || row_index == 3) ? 4 : 3;
    return le == 4 ? run_row_rs<12, 4, 1> : run_row_rs<12, 3, 1>;
  }
  switch (row_index) {
    case 1: case 9: return run_row_rs<8, 4, 4>;
    case 2: case 8: return run_row_rs<8, 3, 8>;
    case 3: case 7: case 11: return run_row_rs<8, 2, 4>;
    default: return run_row_rs<8, 3, 4>;
  }
}

void ntt_fwd_rescale_final(const Shared& sh, u64* corr, int level, int npoly, const RsTail& tail,
                           hipStream_t st) {
  const Params& P = sh.P;
  if (level < 1 || npoly <= 0) return;
  if (level > kMaxPrimes) PPST_THROW(ST_EINVAL, "too many limbs");
  const size_t N = P.N;
  NttArgs a{};
  a.mods = (const Mod*)sh.tab.mods.p;
  set_tables(a, sh, false);
  a.ninv = sh.tab.ninv.p;
  a.N = P.N;
  a.logN = P.logN;
  a.nq = level;
  a.pofs = P.L + 1;
  a.skip_lo = a.skip_hi = 1 << 30;
  a.dalpha = 0;
  a.dcount = 1;
  a.dtotal = 0;
  a.galois = 0;
  a.batch_stride = a.dst_stride = (size_t)level * N;
  a.src = corr;
  a.dst = corr;
  const int b = ntt_bucket(level * npoly);
  const NttPlan& plan = sh.ntt_plan;
  if (P.logN == 16) {
    a.logR = 8;
    kCol16[plan.v[0][0][b]].fwd(a, level, npoly, st);
  } else if (P.logN == 12) {
    a.logR = 0;
  } else {
    PPST_THROW(ST_EINVAL, "NTT supports log2 N in {12, 16}");
  }
  RsEpi e{};
  e.rc = tail.rc;
  e.mulk = tail.k != nullptr;
  for (int i = 0; i < level && tail.k; ++i) {
    e.k[i] = tail.k[i];
    e.kp[i] = tail.kp[i];
  }
  const RsFn f = rs_variant(P.logN, plan.v[0][1][b]);
  for (int c0 = 0; c0 < npoly; c0 += kPtrBatch) {
    const int nc = std::min(kPtrBatch, npoly - c0);
    for (int i = 0; i < nc; ++i) {
      if (!tail.a[c0 + i] || !tail.out[c0 + i]) PPST_THROW(ST_EINVAL, "missing rescale operand");
      e.a.p[i] = tail.a[c0 + i];
      e.out.p[i] = tail.out[c0 + i];
    }
    a.src = a.dst = corr + (size_t)c0 * level * N;
    f(a, e, level, nc, st);
  }
  HIP_CHECK(hipGetLastError());
}

// Autotuner: times every column and row variant (both directions) on a
// scratch buffer of each bucket's representative limb count and keeps the
// fastest.  Runs on the given stream; the buffer holds zeros and at least
// max_limbs limbs; the timed limbs use primes 0..nlc-1 only (nb batches of
// nlc <= nprimes limbs, nb * nlc <= max_limbs).
void ntt_autotune(Shared& sh, hipStream_t st, u64* scratch, int max_limbs) {
  const Params& P = sh.P;
  static const int reps[5] = {2, 12, 25, 64, 200};
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  for (int b = 0; b < 5; ++b) {
    // reps[b] limbs as nb batches of nlc limbs on primes 0..nlc-1
    const int nlc = std::min(reps[b], P.nprimes);
    const int nb = std::max(1, std::min((reps[b] + nlc - 1) / nlc, max_limbs / nlc));
    for (int inv = 0; inv < 2; ++inv) {
      NttArgs a{};
      a.mods = (const Mod*)sh.tab.mods.p;
      set_tables(a, sh, inv != 0);
      a.ninv = sh.tab.ninv.p;
      a.N = P.N;
      a.logN = P.logN;
      a.nq = 0;
      a.pofs = 0;
      a.skip_lo = a.skip_hi = 1 << 30;
      a.dalpha = 0;
      a.dcount = 1;
      a.dtotal = 0;
      a.galois = 0;
      a.src = scratch;
      a.dst = scratch;
      a.batch_stride = a.dst_stride = (size_t)nlc * P.N;
      const int passes = P.logN == 16 ? 2 : 1;
      for (int pass = 0; pass < passes; ++pass) {
        const Variant* tab = P.logN == 16 ? (pass == 0 ? kCol16 : kRow16) : kFull12;
        const int nv = P.logN == 16 ? (pass == 0 ? kNCol16 : kNRow16) : kNFull12;
        a.logR = P.logN == 16 ? 8 : 0;
        // three rounds over all variants, each variant's best round counts:
        // a transient slowdown during one variant's timing cannot decide
        std::vector<float> t(nv, 1e30f);
        for (int v = 0; v < nv; ++v) (inv ? tab[v].inv : tab[v].fwd)(a, nlc, nb, st);   // warm
        for (int round = 0; round < 3; ++round)
          for (int v = 0; v < nv; ++v) {
            PassFn f = inv ? tab[v].inv : tab[v].fwd;
            HIP_CHECK(hipEventRecord(e0, st));
            for (int r = 0; r < 5; ++r) f(a, nlc, nb, st);
            HIP_CHECK(hipEventRecord(e1, st));
            HIP_CHECK(hipEventSynchronize(e1));
            float ms = 0;
            HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
            t[v] = std::min(t[v], ms);
          }
        int best_i = 0;
        for (int v = 1; v < nv; ++v)
          if (t[v] < t[best_i]) best_i = v;
        sh.ntt_plan.v[inv][P.logN == 16 ? pass : 1][b] = best_i;
      }
    }
  }
  HIP_CHECK(hipEventDestroy(e0));
  HIP_CHECK(hipEventDestroy(e1));
  sh.ntt_plan.tuned = true;
}

std::string ntt_plan_string(const Shared& sh) {
  const Params& P = sh.P;
  std::string s;
  for (int inv = 0; inv < 2; ++inv)
    for (int b = 0; b < 5; ++b) {
      s += inv ? "inv" : "fwd";
      s += "[b" + std::to_string(b) + "] ";
      if (P.logN == 16) {
        s += kCol16[sh.ntt_plan.v[inv][0][b]].name;
        s += " ";
        s += kRow16[sh.ntt_plan.v[inv][1][b]].name;
      } else {
        s += kFull12[sh.ntt_plan.v[inv][1][b]].name;
      }
      s += "; ";
    }
  return s;
}

// Inverse of ntt_plan_string: entries "fwd|inv[bK] <col name> <row name>;"
// (N = 2^12: "<name>" alone); every bucket and direction must appear once.
void ntt_load_plan(Shared& sh, const std::string& text) {
  const Params& P = sh.P;
  NttPlan plan = sh.ntt_plan;
  bool seen[2][5] = {};
  auto find = [](const Variant* tab, int n, const std::string& name) {
    for (int i = 0; i < n; ++i)
      if (name == tab[i].name) return i;
    PPST_THROW(ST_EINVAL, "unknown NTT variant '" + name + "'");
  };
  size_t pos = 0;
  while (pos < text.size()) {
    size_t end = text.find(';', pos);
    if (end == std::string::npos) end = text.size();
    std::string item = text.substr(pos, end - pos);
    pos = end + 1;
    std::vector<std::string> tok;
    size_t i = 0;
    while (i < item.size()) {
      while (i < item.size() && item[i] == ' ') ++i;
      size_t j = i;
      while (j < item.size() && item[j] != ' ') ++j;
      if (j > i) tok.push_back(item.substr(i, j - i));
      i = j;
    }
    if (tok.empty()) continue;
    int inv = -1, b = -1;
    if (tok[0].size() == 7 && tok[0].compare(3, 2, "[b") == 0 && tok[0][6] == ']' &&
        tok[0][5] >= '0' && tok[0][5] <= '4') {
      if (tok[0].compare(0, 3, "fwd") == 0) inv = 0;
      if (tok[0].compare(0, 3, "inv") == 0) inv = 1;
      b = tok[0][5] - '0';
    }
    const size_t want = P.logN == 16 ? 3 : 2;
    if (inv < 0 || tok.size() != want) PPST_THROW(ST_EINVAL, "malformed NTT plan entry '" + item + "'");
    if (P.logN == 16) {
      plan.v[inv][0][b] = find(kCol16, kNCol16, tok[1]);
      plan.v[inv][1][b] = find(kRow16, kNRow16, tok[2]);
    } else {
      plan.v[inv][1][b] = find(kFull12, kNFull12, tok[1]);
    }
    seen[inv][b] = true;
  }
  for (int inv = 0; inv < 2; ++inv)
    for (int b = 0; b < 5; ++b)
      if (!seen[inv][b]) PPST_THROW(ST_EINVAL, "NTT plan misses a bucket");
  sh.ntt_plan = plan;
}

void ntt_set_plan(Shared& sh, int col, int row) {
  const Params& P = sh.P;
  const int ncol = P.logN == 16 ? kNCol16 : 1, nrow = P.logN == 16 ? kNRow16 : kNFull12;
  if (col < 0 || col >= ncol || row < 0 || row >= nrow) PPST_THROW(ST_EINVAL, "no such NTT variant");
  for (int inv = 0; inv < 2; ++inv)
    for (int b = 0; b < 5; ++b) {
      sh.ntt_plan.v[inv][0][b] = col;
      sh.ntt_plan.v[inv][1][b] = row;
    }
}

}  // namespace ppst
