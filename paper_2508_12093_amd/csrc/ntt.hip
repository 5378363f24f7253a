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

namespace ppst {

namespace {

struct NttArgs {
  const u64* src;
  u64* dst;
  const Mod* mods;
  const u64* tw;     // [nprimes][N][2]
  const u64* ninv;   // [nprimes][2]
  size_t batch_stride, dst_stride;
  int N, logN, logR, nq, pofs, skip_lo, skip_hi, blocks_per_limb;
};

// Forward CT butterfly on lazy values in [0, 4q)
__device__ __forceinline__ void bfly_ct(u64& x, u64& y, u64 w, u64 wp, u64 q, u64 q2) {
  u64 a = x >= q2 ? x - q2 : x;
  u64 t = mul_shoup_lazy(y, w, wp, q);
  x = a + t;
  y = a - t + q2;
}
// Inverse GS butterfly on lazy values in [0, 2q)
__device__ __forceinline__ void bfly_gs(u64& x, u64& y, u64 w, u64 wp, u64 q, u64 q2) {
  u64 a = x + y;
  a = a >= q2 ? a - q2 : a;
  u64 d = x - y + q2;
  y = mul_shoup_lazy(d, w, wp, q);
  x = a;
}

// One pass of LOGM stages over SB independent sub-problems of M = 2^LOGM
// points.  ROWS: sub-problem r = row (contiguous), twiddle base R + r;
// otherwise sub-problem c = column (stride C), twiddle base 1.  Stage s of
// the sub-problem uses twiddle index (base << s) + (e >> (LOGM - s)) for the
// butterfly whose lower element is e.
template <int LOGM, int LOGE, int SB, bool ROWS, bool INV>
__global__ void __launch_bounds__(SB * (1 << (LOGM - LOGE)))
k_ntt_pass(NttArgs a) {
  constexpr int M = 1 << LOGM;
  constexpr int E = 1 << LOGE;
  constexpr int T = M / E;           // threads per sub-problem
  constexpr int NT = SB * T;         // threads per workgroup
  constexpr int NP = LOGM / LOGE;    // passes
  constexpr int PAD = M + 1;         // LDS row pitch (breaks bank aliasing)
  static_assert(LOGM % LOGE == 0, "passes must tile the stages");
  __shared__ u64 lds[SB * PAD];

  const int N = a.N;
  const int limb_u = blockIdx.x / a.blocks_per_limb;
  const int grp = blockIdx.x - limb_u * a.blocks_per_limb;
  const int t = limb_u >= a.skip_lo ? limb_u + (a.skip_hi - a.skip_lo) : limb_u;
  const int prime = t < a.nq ? t : a.pofs + (t - a.nq);
  const u64* src = a.src + (size_t)blockIdx.y * a.batch_stride + (size_t)t * N;
  u64* dst = a.dst + (size_t)blockIdx.y * a.dst_stride + (size_t)t * N;
  const u64 q = a.mods[prime].q;
  const u64 q2 = 2 * q;
  const u64* tw = a.tw + (size_t)prime * N * 2;
  const int R = 1 << a.logR;
  const int C = N >> a.logR;
  const int tid = threadIdx.x;
  const int first = grp * SB;        // first sub-problem of this workgroup

  // ---- load SB sub-problems into LDS (coalesced along memory)
  if (ROWS) {
    const u64* g = src + (size_t)first * M;
#pragma unroll 4
    for (int idx = tid; idx < SB * M; idx += NT) {
      int sp = idx / M, e = idx - sp * M;
      lds[sp * PAD + e] = g[idx];
    }
  } else {
#pragma unroll 4
    for (int idx = tid; idx < SB * M; idx += NT) {
      int e = idx / SB, sp = idx - e * SB;
      lds[sp * PAD + e] = src[(size_t)e * C + first + sp];
    }
  }
  __syncthreads();

  const int sp = tid / T;
  const int lane = tid - sp * T;
  u64* my = lds + sp * PAD;
  const u64 base0 = ROWS ? (u64)(R + first + sp) : 1;

#pragma unroll
  for (int pi = 0; pi < NP; ++pi) {
    const int p = INV ? (NP - 1 - pi) : pi;
    const int s0 = p * LOGE;
    const int si = M >> (s0 + LOGE);
    const int lo = lane % si;
    const int hi = lane / si;
    const int e0 = hi * (M >> s0) + lo;
    u64 x[E];
#pragma unroll
    for (int k = 0; k < E; ++k) x[k] = my[e0 + k * si];
#pragma unroll
    for (int uu = 0; uu < LOGE; ++uu) {
      const int u = INV ? (LOGE - 1 - uu) : uu;
      const int s = s0 + u;
      const int half = E >> (u + 1);
#pragma unroll
      for (int k = 0; k < E; ++k) {
        if (k & half) continue;
        const int e = e0 + k * si;
        const u64 idx = (base0 << s) + (u64)(e >> (LOGM - s));
        const u64 w = tw[2 * idx], wp = tw[2 * idx + 1];
        if (INV) bfly_gs(x[k], x[k + half], w, wp, q, q2);
        else bfly_ct(x[k], x[k + half], w, wp, q, q2);
      }
    }
#pragma unroll
    for (int k = 0; k < E; ++k) my[e0 + k * si] = x[k];
    __syncthreads();
  }

  // ---- store; finish the reduction where this pass is the last one
  const bool last = INV ? !ROWS || a.logR == 0 : ROWS;
  const u64 ni = a.ninv[2 * prime], nip = a.ninv[2 * prime + 1];
  if (ROWS) {
    u64* g = dst + (size_t)first * M;
#pragma unroll 4
    for (int idx = tid; idx < SB * M; idx += NT) {
      int s2 = idx / M, e = idx - s2 * M;
      u64 v = lds[s2 * PAD + e];
      if (last) {
        if (INV) v = mul_shoup(v, ni, nip, q);
        else { v = v >= q2 ? v - q2 : v; v = csub(v, q); }
      }
      g[idx] = v;
    }
  } else {
#pragma unroll 4
    for (int idx = tid; idx < SB * M; idx += NT) {
      int e = idx / SB, s2 = idx - e * SB;
      u64 v = lds[s2 * PAD + e];
      if (last) {
        if (INV) v = mul_shoup(v, ni, nip, q);
        else { v = v >= q2 ? v - q2 : v; v = csub(v, q); }
      }
      dst[(size_t)e * C + first + s2] = v;
    }
  }
}

template <int LOGM, int LOGE, int SB, bool ROWS, bool INV>
void run_pass(const NttArgs& base, int nlimbs, int nbatch, hipStream_t st) {
  NttArgs a = base;
  const int nsub = ROWS ? (1 << a.logR) : (a.N >> a.logR);
  a.blocks_per_limb = nsub / SB;
  dim3 grid(a.blocks_per_limb * nlimbs, nbatch);
  dim3 block(SB * (1 << (LOGM - LOGE)));
  hipLaunchKernelGGL((k_ntt_pass<LOGM, LOGE, SB, ROWS, INV>), grid, block, 0, st, a);
}

}  // namespace

void ntt(const Shared& sh, const NttLaunch& L, bool inverse, hipStream_t st) {
  const Params& P = sh.P;
  if (L.nlimbs <= 0 || L.nbatch <= 0) return;
  NttArgs a{};
  a.mods = (const Mod*)sh.tab.mods.p;
  a.tw = inverse ? sh.tab.inv.p : sh.tab.fwd.p;
  a.ninv = sh.tab.ninv.p;
  a.batch_stride = L.batch_stride;
  a.dst_stride = L.dst_stride == ~(size_t)0 ? L.batch_stride : L.dst_stride;
  a.N = P.N;
  a.logN = P.logN;
  a.nq = L.nq;
  a.pofs = L.pofs;
  a.skip_lo = L.skip_lo;
  a.skip_hi = L.skip_hi;
  if (P.logN == 16) {
    a.logR = 8;
    if (!inverse) {
      a.src = L.src; a.dst = L.dst;
      run_pass<8, 4, 16, false, false>(a, L.nlimbs, L.nbatch, st);
      a.src = L.dst;
      a.batch_stride = a.dst_stride;
      run_pass<8, 4, 16, true, false>(a, L.nlimbs, L.nbatch, st);
    } else {
      a.src = L.src; a.dst = L.dst;
      run_pass<8, 4, 16, true, true>(a, L.nlimbs, L.nbatch, st);
      a.src = L.dst;
      a.batch_stride = a.dst_stride;
      run_pass<8, 4, 16, false, true>(a, L.nlimbs, L.nbatch, st);
    }
  } else if (P.logN == 12) {
    a.logR = 0;
    a.src = L.src; a.dst = L.dst;
    if (!inverse) run_pass<12, 4, 1, true, false>(a, L.nlimbs, L.nbatch, st);
    else run_pass<12, 4, 1, true, true>(a, L.nlimbs, L.nbatch, st);
  } else {
    PPST_THROW(ST_EINVAL, "NTT supports log2 N in {12, 16}");
  }
  HIP_CHECK(hipGetLastError());
}

}  // namespace ppst
