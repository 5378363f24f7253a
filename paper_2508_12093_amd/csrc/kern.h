// kern.h -- host-side launchers of the device kernels (kernels.hip, ntt.hip).
#pragma once

#include "core.h"

namespace ppst {

constexpr int kMaxLimbArgs = 64;

// ---------------------------------------------------------------- NTT
// Transforms `nlimbs` limbs per batch item.  Limb u of batch item b sits at
// src + b*batch_stride + t*N with t = u, or u + (skip_hi - skip_lo) when
// u >= skip_lo (limbs [skip_lo, skip_hi) are left alone); its prime is
// t < nq ? t : pofs + (t - nq).  In place when src == dst.
struct NttLaunch {
  const u64* src;
  u64* dst;
  int nlimbs;
  int nbatch = 1;
  size_t batch_stride = 0;      // source stride between batch items
  size_t dst_stride = ~(size_t)0;  // destination stride (default: batch_stride)
  int nq, pofs;
  int skip_lo = 1 << 30, skip_hi = 1 << 30;
  // Digit mode (digit_alpha > 0): batch item b holds the extension of digit
  // j = b % digit_count, whose own limbs [j alpha, min((j+1) alpha, nq)) are
  // skipped; items have digit_total limbs and nlimbs must be the largest
  // count of transformed limbs over the digits.
  int digit_alpha = 0, digit_count = 1, digit_total = 0;
  // inverse, out-of-place only: transform the input permuted by X -> X^galois
  // (canonical NTT order); 0 for none
  uint32_t galois = 0;
  // inverse: per-prime final factors in the table format ([nprimes][2]);
  // null for N^-1 (modup_ninv: N^-1 Qhat_i^-1, the input scaling of ModUp)
  const u64* ninv = nullptr;
};
void ntt(const Shared& sh, const NttLaunch& L, bool inverse, hipStream_t st);

// batch items per launch of the kernels that take operand pointer arrays
constexpr int kPtrBatch = 64;
struct OutPtrs {
  u64* p[kPtrBatch];
};
struct PtrsIn {
  const u64* p[kPtrBatch];
};

// Forward NTT of the ModDown+rescale correction corr [nbatch][2][level][N]
// (coefficient form, primes q_0..q_{level-1}) whose last pass stores, in
// place of corr_i, out_i = ((u_i P^-1 mod q_i) + d_i + corr_i) q_l^-1 mod q_i
// into out[b] ([2][level][N]); u: [nbatch][2][ne][N] at stride su, d:
// [nbatch][3][nl][N] at stride sd, rc: the rescale table of the level.
struct MdrTail {
  const u64* u;
  const u64* d;                 // the tensor [3][nl][N] per item, or null: pa, pb
  size_t su, sd;
  const u64* rc;
  u64* const* out;
  const u64* const* pa = nullptr;   // a product's operands (d0, d1 formed from them)
  const u64* const* pb = nullptr;
};
void ntt_fwd_mdr_final(const Shared& sh, u64* corr, int level, int nbatch, const MdrTail& tail,
                       hipStream_t st);

// Forward NTT of the ModDown conversion conv [nbatch][2][nl][N] (coefficient
// form, primes q_0..q_l) whose last pass stores, in place of conv_i,
//   out_i = ((u_i - conv_i) P^-1 mod q_i) [+ add_c,i(X^gadd)] [+ acc_c,i]
// into out[b] ([2][nl][N]).  u: [nbatch][2][ne][N] at stride su; add0/add1:
// per-item [nl][N] addends of c0/c1 (array or entries may be null), read
// through X -> X^gadd when gadd != 0; acc: per-item [2][nl][N] running sums
// (array or entries may be null).
struct MdTail {
  const u64* u;
  size_t su;
  const u64* const* add0;
  const u64* const* add1;
  const u64* const* acc;
  u64* const* out;
  uint32_t gadd;
};
// The extended digits' forward NTT fused with the key inner product: the
// column pass of ext ([nbatch][beta][ne][N], ModUp output, digit mode), then
// one row pass per digit whose results are multiplied by the key and summed
// in registers: u ([nbatch][2][ne][N]) as k_ks_inner computes it from the
// fully transformed digits (d: the input in NTT form for the digits' own
// limbs, read through X -> X^gd; pd: the tensor for the product's P d0, P d1
// on limb q_l, or null).  ks_fused_ok: N = 2^16, at most 4 digits, and not
// switched off by PPST_KS_FUSED=0.
struct KsTail {
  // x non-null: ModUp runs inside the digits' column pass, from the scaled
  // coefficients x ([nbatch][l+1][N] at stride sx, modup_ninv); else ext
  // holds ModUp's output
  const u64* x;
  size_t sx;
  u64* ext;
  const u64* d;                 // null for a product: d2 = a1 b1 from pa, pb
  size_t sd;
  const u64* const* pa;
  const u64* const* pb;
  const u64* key;
  u64* u;
  const u64* pd;
  size_t spd;
  u64 pmod, pmods;
  uint32_t gd;
};
bool ks_fused_ok(const Params& P, int level);
// Inverse NTT of a product's d2 = a1 b1 (operands pa[b], pb[b]: [2][l+1][N])
// into x ([nbatch][l+1][N]), the product formed in the first pass's loads;
// ninv: the final factors (null: N^-1).  N = 2^16.
void ntt_inv_prod(const Shared& sh, const u64* const* pa, const u64* const* pb, u64* x, int level,
                  int nbatch, const u64* ninv, hipStream_t st);
// ModUp fused into the fused key switch's column pass (PPST_MODUP_COL=0: off)
bool modup_col_ok();
void ntt_fwd_ks_fused(const Shared& sh, const KsTail& tail, int level, int nbatch, hipStream_t st);
void ntt_fwd_md_final(const Shared& sh, u64* conv, int level, int nbatch, const MdTail& tail,
                      hipStream_t st);

// Forward NTT of a rescale's correction corr [npoly][l][N] (coefficient form,
// primes q_0..q_{l-1}) whose last pass stores, for limb i of polynomial c,
//   out_c,i = ((k_i a_c,i or a_c,i) - corr_c,i) q_l^-1 mod q_i
// (a, out: host arrays of npoly device pointers to limb 0 of each input and
// output polynomial; k, kp: host arrays of l constant residues and their
// Shoup companions, or null; rc: the rescale table of l).
struct RsTail {
  const u64* const* a;
  u64* const* out;
  const u64* rc;
  const u64* k;
  const u64* kp;
};
void ntt_fwd_rescale_final(const Shared& sh, u64* corr, int level, int npoly, const RsTail& tail,
                           hipStream_t st);

// ------------------------------------------------------- element-wise
// All element-wise launches work on `npoly` polynomials of `nl` limbs,
// polynomial c at base + c * poly_stride; limb t uses prime map(t).
void k_add(const Shared& sh, const u64* a, const u64* b, u64* out, int npoly, int nl,
           size_t stride_a, size_t stride_b, size_t stride_o, bool sub, hipStream_t st);
// out[c][t] = a[c][t] * k[t] mod q_t  (k reduced, Shoup companions precomputed)
void k_mul_scalar(const Shared& sh, const u64* a, u64* out, int npoly, int nl, size_t stride_a,
                  size_t stride_o, const u64* k, const u64* kp, hipStream_t st);
// out[c][t] = sum_k K_k,t src_k[c][t] mod q_t for both polynomials c and limbs
// t < nl (prime t): src[k] with polynomial stride ps[k]; K: host arrays
// k[term][nl] of residues and kp[term][nl] of Shoup companions; out at
// polynomial stride so.
void k_lincomb(const Shared& sh, const u64* const* src, const size_t* ps, const u64* k,
               const u64* kp, int nterm, int nl, u64* out, size_t so, hipStream_t st);
// out[t] = a[t] + k[t] mod q_t on one polynomial
void k_add_scalar(const Shared& sh, const u64* a, u64* out, int nl, const u64* k, hipStream_t st);
// out[c][t] = a[c][t] * pt[t] mod q_t
void k_mul_poly(const Shared& sh, const u64* a, const u64* pt, u64* out, int npoly, int nl,
                size_t stride_a, size_t stride_o, hipStream_t st);
// (d0, d1, d2) = (a0 b0, a0 b1 + a1 b0, a1 b1); a[i], b[i]: [2][nl][N] (host
// arrays of nbatch device pointers); d: [3][nl][N] per item at stride_d
void k_tensor(const Shared& sh, const u64* const* a, const u64* const* b, u64* d, int nl,
              int nbatch, size_t stride_d, hipStream_t st);
// out[c][t][j] = in[c][t][perm_g(j)], the automorphism X -> X^g in NTT form
void k_automorph(const Shared& sh, const u64* in, u64* out, int nrows, size_t row_stride_in,
                 size_t row_stride_out, u64 g, hipStream_t st);

// ------------------------------------------------------ key switching
// ModUp of every digit j at level l: x = coefficient-form limbs of the input
// (limb t at x + t*N); for digit j writes every limb t of [0, nl+K) outside the
// digit into ext + (j*ne + t)*N (coefficient form).
void k_modup(const Shared& sh, const u64* x, u64* ext, int level, int nbatch, size_t stride_x,
             size_t stride_ext, hipStream_t st);
// Inner product with the key: for t in [0, ne) (ne = nl + K),
//   u0_t = sum_j e_{j,t} b_{j,p(t)},  u1_t = sum_j e_{j,t} a_{j,p(t)},
// e_{j,t} = d_t for t in digit j (NTT form input), ext[j][t] otherwise (also
// for t in digit j when d is null).
// ext: [beta][ne][N] per batch item; u: [2][ne][N] per batch item.  With
// gd / gext nonzero, d / ext are read through X -> X^g (canonical NTT order).
// With prep_d non-null (products), limb q_l of u[c] also receives
// (P mod q_l) prep_d[c][l] (prep_d: [nbatch][3][nl][N] at stride prep_sd).
void k_ks_inner(const Shared& sh, const u64* d, const u64* ext, const u64* key, u64* u, int level,
                int nbatch, size_t stride_d, size_t stride_ext, size_t stride_u, uint32_t gd,
                uint32_t gext, hipStream_t st, const u64* prep_d = nullptr,
                size_t prep_sd = 0);
// Inner products of several Galois keys with one set of extended digits,
// added in the extended basis: for t in [0, ne),
//   u0_t = sum_r sum_j e_{j,t}(X^g_r) b^(r)_{j,p(t)},  u1_t likewise with a^(r),
// e_{j,t} = d_t (per item: d[b], NTT form [nl][N]) for t in digit j, ext[j][t]
// otherwise; ext: [nbatch][beta][ne][N] at stride sext; u: [nbatch][2][ne][N]
// at stride su.  nkeys <= kMaxHoistKeys, nbatch <= kPtrBatch.  With w
// (per-item NTT-form [nl][N], entries may be null), limb q_t of u0 also
// receives (P mod q_t) sum_r w_t(X^g_r): after ModDown that is exactly
// sum_r w(X^g_r) added to c0 (P w vanishes modulo the special primes).
constexpr int kMaxHoistKeys = 7;
void k_ks_inner_multi(const Shared& sh, const u64* const* d, const u64* ext,
                      const u64* const* keys, const uint32_t* g, int nkeys, u64* u, int level,
                      int nbatch, size_t sext, size_t su, hipStream_t st,
                      const u64* const* w = nullptr);
// ModDown conversion: z = coefficient-form special limbs of u (u + nl*N, for
// both polynomials); conv[c][i] = Conv_{P->q_i}(z + h) - h mod q_i.
void k_moddown_conv(const Shared& sh, const u64* u, u64* conv, int level, int nbatch,
                    size_t stride_u, size_t stride_conv, hipStream_t st);

// --------------------------------------- ModDown and rescale in one pass
// After the key-switch inner product u (NTT form, [2][ne][N]) of a product
// whose tensor is d ([3][nl][N]), these steps produce rescale(d + ModDown(u))
// bit for bit, with one NTT of the correction instead of a forward NTT after
// ModDown and an inverse + forward NTT pair inside rescale:
//   prep:  u[c][l] += (P mod q_l) d[c][l]  (NTT form; in the inner product)
//   (iNTT of limbs q_l, p_0..p_{K-1} of u)
//   corr:  c_l = (u_l + h - Conv_l) P^-1 mod q_l, t = centred(c_l),
//          corr_i = (h - Conv_i) P^-1 - t  mod q_i, i < l       (coefficient form)
//   (NTT of corr, whose last pass stores, in ntt_fwd_mdr_final)
//   final: out_i = (d_i + u_i P^-1 + corr_i) q_l^-1 mod q_i
void k_mdr_corr(const Shared& sh, const u64* u, u64* corr, int level, int nbatch, size_t su,
                size_t sc, hipStream_t st);


// ------------------------------------------------------------ rescale
// top: coefficient-form top limb of each of npoly polynomials (stride
// top_stride); tmp[c][i] = centred(x_c) mod q_i for i < level, where
// x_c = top_c, or k top_c mod q_level when kl (host: k and its Shoup
// companion) is given.
void k_rescale_conv(const Shared& sh, const u64* top, u64* tmp, int level, int npoly,
                    size_t top_stride, hipStream_t st, const u64* kl = nullptr);

// out = sum of nterm arrays [npoly][nl][N] (src: host array of device
// pointers), limb t reduced mod q_t
void k_sum(const Shared& sh, const u64* const* src, int nterm, u64* out, int npoly, int nl,
           hipStream_t st);
// rows[i] (host array of nrows device pointers, row_words words each; 0
// means N) -> dst + i dst_stride (0 means row_words)
void k_gather_rows(const Shared& sh, const u64* const* rows, u64* dst, int nrows, hipStream_t st,
                   size_t row_words = 0, size_t dst_stride = 0);

// ------------------------------------------------------- sampling etc.
// signed 64-bit integers -> residues on limbs t of a map
void k_int64_to_rns(const Shared& sh, const int64_t* s, u64* out, int nl, int nq, int pofs,
                    hipStream_t st);
// signed small integers (int32) -> residues on limbs t of a map
void k_small_to_rns(const Shared& sh, const int32_t* s, u64* out, int nl, int nq, int pofs,
                    hipStream_t st);
// uniform residues: limb t (prime map(t)) from the stream (seed, purpose, stream_limb0 + prime)
void k_sample_uniform(const Shared& sh, u64* out, int nl, int nq, int pofs, u64 seed, u64 purpose,
                      hipStream_t st);
void k_sample_ternary(const Shared& sh, int32_t* out, u64 seed, u64 purpose, hipStream_t st);
void k_sample_dg(const Shared& sh, int32_t* out, u64 seed, u64 purpose, hipStream_t st);
// out_t = e_t - a_t s_t + f_t sp_t (f_t = 0 skips the last term), on nl limbs (map)
void k_keyform(const Shared& sh, const u64* a, const u64* s, const u64* e, const u64* sp,
               const u64* f, u64* out, int nl, int nq, int pofs, hipStream_t st);
// ModRaise: x [npoly][N] coefficients mod q_0 -> out [npoly][nl][N], the
// centred lift of each coefficient reduced mod q_0..q_{nl-1}
void k_mod_raise(const Shared& sh, const u64* x, u64* out, int nl, int npoly, hipStream_t st);
// baby-step giant-step inner sums: outs[j] = sum_{i<b} pts[j b + i] . baby[i]
// for j < G (both polynomials of [2][nl][N] ciphertexts at polynomial strides
// ps_in / ps_out; plaintexts [nl][N]; null plaintexts skipped, null outputs
// not written); b <= 16, G <= 16, b G <= 64 after b is padded to a power of two
void k_bsgs_inner(const Shared& sh, const u64* const* baby, int b, const u64* const* pts,
                  u64* const* outs, int G, int nl, size_t ps_in, size_t ps_out, hipStream_t st);
// out = x + y * z (+ w when w != null) on nl limbs of the ciphertext primes
void k_fma3(const Shared& sh, const u64* x, const u64* y, const u64* z, const u64* w, u64* out,
            int nl, hipStream_t st);

}  // namespace ppst
