/*
 * ckks_ref.c -- CPU oracle for textbook RNS-CKKS.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library.  It shares no
 * source, header, table or constant generator with the GPU library: every
 * prime, root, twiddle, CRT constant and sampler below is derived here, from
 * the definitions, in the most direct way that is still fast enough to run.
 *
 * The paper (PP-STAT, Sec. 3.1) uses CKKS as a black box offering Add, Mul
 * and Rot; everything below that box (RNS limbs, negacyclic NTT, hybrid key
 * switching, rescale, encoding, sampling) is textbook RNS-CKKS, written out as
 * the plain definitions:
 *   - residues in [0,q); products through unsigned __int128 and '%';
 *   - NTT = twist by psi^k, a cyclic radix-2 DFT with omega = psi^2, then a
 *     bit-reversal, so that slot j holds a(psi^(2*brv(j)+1));
 *   - key switching by digit decomposition + fast base conversion (ModUp),
 *     an inner product with the key, and division by P (ModDown);
 *   - rescale by the top prime with rounding to nearest (centred lift);
 *   - automorphisms applied in coefficient form.
 * No blocking, lazy reduction or fusion is used anywhere.
 *
 * Polynomials are limb-major arrays: limb i of a polynomial over primes
 * (q_0..q_l) occupies a[i*N .. i*N+N-1].  Prime indices are "combined":
 * 0..L are the ciphertext primes q_0..q_L, L+1..L+K the special primes.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#include "ckks_ref.h"

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* modular arithmetic on residues in [0,q)                             */
/* ------------------------------------------------------------------ */
static u64 mulmod(u64 a, u64 b, u64 q) { return (u64)(((u128)a * b) % q); }
static u64 addmod(u64 a, u64 b, u64 q) { u64 s = a + b; return s >= q ? s - q : s; }
static u64 submod(u64 a, u64 b, u64 q) { return a >= b ? a - b : a + (q - b); }
static u64 powmod(u64 b, u64 e, u64 q) {
    u64 r = 1 % q;
    b %= q;
    while (e) {
        if (e & 1) r = mulmod(r, b, q);
        b = mulmod(b, b, q);
        e >>= 1;
    }
    return r;
}
static u64 invmod(u64 a, u64 q) { return powmod(a, q - 2, q); } /* q prime */
/* signed integer -> residue */
static u64 from_signed(int64_t x, u64 q) {
    if (x >= 0) return (u64)x % q;
    u64 m = (u64)(-(x + 1)) % q;         /* avoids overflow at INT64_MIN */
    return q - 1 - m;
}

u64 orc_mulmod(u64 a, u64 b, u64 q) { return mulmod(a, b, q); }
u64 orc_powmod(u64 b, u64 e, u64 q) { return powmod(b, e, q); }

/* Deterministic Miller-Rabin; the first twelve prime bases are exact for
 * every n < 3.3e24, hence for every 64-bit n. */
int orc_is_prime(u64 n) {
    static const u64 bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return 0;
    for (int i = 0; i < 12; i++) {
        if (n % bases[i] == 0) return n == bases[i];
    }
    u64 d = n - 1;
    int s = 0;
    while (!(d & 1)) { d >>= 1; s++; }
    for (int i = 0; i < 12; i++) {
        u64 x = powmod(bases[i], d, n);
        if (x == 1 || x == n - 1) continue;
        int witness = 1;
        for (int r = 1; r < s; r++) {
            x = mulmod(x, x, n);
            if (x == n - 1) { witness = 0; break; }
        }
        if (witness) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------ */
/* parameters                                                          */
/* ------------------------------------------------------------------ */
static int in_list(u64 x, const u64* list, int n) {
    for (int i = 0; i < n; i++) if (list[i] == x) return 1;
    return 0;
}

/* Largest prime p < 2^bits with p = 1 mod 2N that is not in `used`. */
static u64 largest_prime_below(int bits, u64 twoN, const u64* used, int nused) {
    u64 top = (bits >= 64) ? ~(u64)0 : (((u64)1 << bits) - 1);
    u64 x = ((top - 1) / twoN) * twoN + 1;   /* largest x <= top, x = 1 mod 2N */
    while (x > twoN) {
        if (!in_list(x, used, nused) && orc_is_prime(x)) return x;
        x -= twoN;
    }
    return 0;
}

/* The unused prime p = 1 mod 2N nearest to `target` (ties to the smaller). */
static u64 nearest_prime(double target, u64 twoN, const u64* used, int nused) {
    u64 base = (u64)floor((target - 1.0) / (double)twoN);
    u64 lo = base * twoN + 1;                  /* lo <= target < lo + 2N */
    u64 hi = lo + twoN;
    while (lo > twoN && (in_list(lo, used, nused) || !orc_is_prime(lo))) lo -= twoN;
    while (in_list(hi, used, nused) || !orc_is_prime(hi)) hi += twoN;
    double dl = target - (double)lo;
    double dh = (double)hi - target;
    return (dh < dl) ? hi : lo;
}

/* psi = x^((q-1)/2N) for the smallest x >= 2 with psi^N = -1 (mod q). */
static u64 find_psi(u64 q, int N) {
    for (u64 x = 2;; x++) {
        u64 psi = powmod(x, (q - 1) / (2 * (u64)N), q);
        if (powmod(psi, (u64)N, q) == q - 1) return psi;
    }
}

/*
 * Parameter rule (the paper fixes N, Delta and the total modulus budget,
 * Sec. 6.1; the prime rule itself is a reading):
 *   q_0      largest prime < 2^q0_bits, = 1 mod 2N;
 *   q_l      for l = L..1, the unused prime = 1 mod 2N nearest to
 *            Delta_l^2 / Delta, with Delta_L = Delta and
 *            Delta_{l-1} = (Delta_l * Delta_l) / q_l  (FP64, in that order);
 *   p_k      the K largest unused primes < 2^p_bits, = 1 mod 2N.
 */
int orc_params_make(int logN, int L, int K, int dnum, int q0_bits, double delta,
                    int p_bits, orc_params* out) {
    if (logN < 2 || logN > 17 || L < 0 || K < 1 || L + 1 + K > ORC_MAXP || dnum < 1) return -1;
    memset(out, 0, sizeof(*out));
    out->logN = logN;
    out->N = 1 << logN;
    out->L = L;
    out->K = K;
    out->dnum = dnum;
    out->alpha = (L + 1 + dnum - 1) / dnum;
    u64 twoN = 2 * (u64)out->N;
    u64 used[ORC_MAXP];
    int nused = 0;
    out->q[0] = largest_prime_below(q0_bits, twoN, used, nused);
    used[nused++] = out->q[0];
    out->scale[L] = delta;
    for (int l = L; l >= 1; l--) {
        double sq = out->scale[l] * out->scale[l];
        double target = sq / delta;
        u64 p = nearest_prime(target, twoN, used, nused);
        out->q[l] = p;
        used[nused++] = p;
        out->scale[l - 1] = sq / (double)p;
    }
    for (int k = 0; k < K; k++) {
        u64 p = largest_prime_below(p_bits, twoN, used, nused);
        out->q[L + 1 + k] = p;
        used[nused++] = p;
    }
    for (int i = 0; i < L + 1 + K; i++) {
        if (out->q[i] == 0) return -2;
        out->psi[i] = find_psi(out->q[i], out->N);
    }
    return 0;
}

/*
 * Bootstrappable chain (a reading: the paper's set has a depth of 27 of which
 * 11 levels are usable between bootstraps, Sec. 6.1, and leaves the rest to
 * the cited bootstrapping).  From the top level L down: C levels for
 * CoeffToSlot, E for EvalMod, S for SlotToCoeff, then Lc = L - C - E - S
 * levels of computation, then q_0.  Primes, in the order they are chosen:
 *   q_0                 largest prime < 2^q0_bits, = 1 mod 2N;
 *   q_L..q_{L-C+1}      the largest unused primes < 2^p_bits (CoeffToSlot);
 *   q_l, l = L-C..Lc+S+1  the unused prime nearest Delta_l^2 / Delta_b, with
 *                       Delta_{L-C} = Delta_b and Delta_{l-1} = Delta_l^2 / q_l;
 *   q_{Lc+S}..q_{Lc+1}  the largest unused primes < 2^p_bits (SlotToCoeff);
 *   q_l, l = Lc..1      the unused prime nearest Delta_l^2 / Delta, with
 *                       Delta_Lc = Delta and Delta_{l-1} = Delta_l^2 / q_l;
 *   p_0..p_{K-1}        the K largest unused primes < 2^p_bits.
 * Scales of the levels the linear transforms end on (no product of two
 * ciphertexts is rescaled there): Delta_l = Delta_b for l >= L - C, and
 * Delta_{Lc+i} = Delta * 2^floor(i e / S) for 0 < i < S, with e the
 * difference of the binary exponents of Delta_b and Delta.
 */
int orc_params_make_boot(int logN, int Lc, int C, int E, int S, int K, int dnum, int q0_bits,
                         double delta, double delta_b, int p_bits, orc_params* out) {
    int L = Lc + C + E + S;
    if (logN < 2 || logN > 17 || Lc < 1 || C < 1 || E < 1 || S < 1 || K < 1 ||
        L + 1 + K > ORC_MAXP || dnum < 1)
        return -1;
    memset(out, 0, sizeof(*out));
    out->logN = logN;
    out->N = 1 << logN;
    out->L = L;
    out->K = K;
    out->dnum = dnum;
    out->alpha = (L + 1 + dnum - 1) / dnum;
    u64 twoN = 2 * (u64)out->N;
    u64 used[ORC_MAXP];
    int nused = 0;
    out->q[0] = largest_prime_below(q0_bits, twoN, used, nused);
    used[nused++] = out->q[0];
    for (int l = L; l > L - C; l--) {
        out->q[l] = largest_prime_below(p_bits, twoN, used, nused);
        used[nused++] = out->q[l];
        out->scale[l] = delta_b;
    }
    out->scale[L - C] = delta_b;
    for (int l = L - C; l > Lc + S; l--) {
        double sq = out->scale[l] * out->scale[l];
        u64 p = nearest_prime(sq / delta_b, twoN, used, nused);
        out->q[l] = p;
        used[nused++] = p;
        out->scale[l - 1] = sq / (double)p;
    }
    for (int l = Lc + S; l > Lc; l--) {
        out->q[l] = largest_prime_below(p_bits, twoN, used, nused);
        used[nused++] = out->q[l];
    }
    int e = ilogb(delta_b) - ilogb(delta);
    for (int i = 1; i < S; i++) out->scale[Lc + i] = ldexp(delta, (i * e) / S);
    out->scale[Lc] = delta;
    for (int l = Lc; l >= 1; l--) {
        double sq = out->scale[l] * out->scale[l];
        u64 p = nearest_prime(sq / delta, twoN, used, nused);
        out->q[l] = p;
        used[nused++] = p;
        out->scale[l - 1] = sq / (double)p;
    }
    for (int k = 0; k < K; k++) {
        u64 p = largest_prime_below(p_bits, twoN, used, nused);
        out->q[L + 1 + k] = p;
        used[nused++] = p;
    }
    for (int i = 0; i < L + 1 + K; i++) {
        if (out->q[i] == 0) return -2;
        out->psi[i] = find_psi(out->q[i], out->N);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* negacyclic NTT, canonical order: out_j = a(psi^(2 brv(j) + 1))       */
/* ------------------------------------------------------------------ */
static unsigned brv(unsigned x, int bits) {
    unsigned r = 0;
    for (int i = 0; i < bits; i++) { r = (r << 1) | (x & 1); x >>= 1; }
    return r;
}
static void bitrev_permute(u64* a, int N, int logN) {
    for (int i = 0; i < N; i++) {
        unsigned j = brv((unsigned)i, logN);
        if ((int)j > i) { u64 t = a[i]; a[i] = a[j]; a[j] = t; }
    }
}
/* textbook iterative radix-2 cyclic DFT: A_i = sum_k a_k w^(i k) */
static void cyclic_dft(u64* a, int N, int logN, u64 w, u64 q) {
    bitrev_permute(a, N, logN);
    for (int len = 2; len <= N; len <<= 1) {
        u64 wl = powmod(w, (u64)(N / len), q);
        for (int i = 0; i < N; i += len) {
            u64 wj = 1;
            for (int j = 0; j < len / 2; j++) {
                u64 u = a[i + j];
                u64 v = mulmod(a[i + j + len / 2], wj, q);
                a[i + j] = addmod(u, v, q);
                a[i + j + len / 2] = submod(u, v, q);
                wj = mulmod(wj, wl, q);
            }
        }
    }
}
void orc_ntt_limb(const orc_params* P, int pidx, u64* a) {
    int N = P->N, logN = P->logN;
    u64 q = P->q[pidx], psi = P->psi[pidx];
    u64 t = 1;
    for (int k = 0; k < N; k++) { a[k] = mulmod(a[k], t, q); t = mulmod(t, psi, q); }
    cyclic_dft(a, N, logN, mulmod(psi, psi, q), q);
    bitrev_permute(a, N, logN);
}
void orc_intt_limb(const orc_params* P, int pidx, u64* a) {
    int N = P->N, logN = P->logN;
    u64 q = P->q[pidx];
    u64 psi_inv = invmod(P->psi[pidx], q);
    bitrev_permute(a, N, logN);
    cyclic_dft(a, N, logN, mulmod(psi_inv, psi_inv, q), q);
    u64 ninv = invmod((u64)N % q, q);
    u64 t = ninv;
    for (int k = 0; k < N; k++) { a[k] = mulmod(a[k], t, q); t = mulmod(t, psi_inv, q); }
}
/* limb i of a uses combined prime index pidx[i] */
void orc_ntt(const orc_params* P, u64* a, int nlimbs, const int32_t* pidx) {
    #pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < nlimbs; i++) orc_ntt_limb(P, pidx[i], a + (size_t)i * P->N);
}
void orc_intt(const orc_params* P, u64* a, int nlimbs, const int32_t* pidx) {
    #pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < nlimbs; i++) orc_intt_limb(P, pidx[i], a + (size_t)i * P->N);
}

/* schoolbook negacyclic product c = a*b in Z_q[X]/(X^N+1) */
void orc_negacyclic_mul(const u64* a, const u64* b, u64* c, int N, u64 q) {
    for (int k = 0; k < N; k++) c[k] = 0;
    for (int i = 0; i < N; i++) {
        for (int j = 0; j < N; j++) {
            u64 p = mulmod(a[i], b[j], q);
            int k = i + j;
            if (k < N) c[k] = addmod(c[k], p, q);
            else c[k - N] = submod(c[k - N], p, q);
        }
    }
}

/* ------------------------------------------------------------------ */
/* seeded sampling: SplitMix64 (Steele, Lea, Flood 2014) as a counter   */
/* ------------------------------------------------------------------ */
#define SM_GAMMA 0x9E3779B97F4A7C15ULL
static u64 sm_next(u64* state) {
    u64 z = (*state += SM_GAMMA);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
static u64 sm_once(u64 x) { u64 s = x; return sm_next(&s); }
/* state of the stream for (seed, purpose, limb); its outputs are word 0,1,.. */
static u64 stream_key(u64 seed, u64 purpose, u64 limb) {
    return sm_once(sm_once(sm_once(seed) ^ purpose) ^ limb);
}
u64 orc_stream_word(u64 seed, u64 purpose, u64 limb, u64 index) {
    u64 s = stream_key(seed, purpose, limb);
    s += index * SM_GAMMA;
    return sm_next(&s);
}

void orc_sample_ternary(u64 seed, u64 purpose, int N, int8_t* out) {
    u64 s = stream_key(seed, purpose, 0);
    for (int k = 0; k < N; k++) {
        u64 u = sm_next(&s);
        out[k] = (int8_t)((int)(((u128)u * 3) >> 64) - 1);
    }
}

/* uniform residue mod q from two words (hi, lo): (hi*2^64 + lo) mod q */
void orc_sample_uniform(u64 seed, u64 purpose, u64 limb, u64 q, int N, u64* out) {
    u64 s = stream_key(seed, purpose, limb);
    for (int k = 0; k < N; k++) {
        u64 hi = sm_next(&s);
        u64 lo = sm_next(&s);
        out[k] = (u64)((((u128)hi << 64) | lo) % q);
    }
}

/* Discrete Gaussian, sigma = 3.2, |e| <= 19, by inversion of a cumulative
 * table of 64-bit thresholds. */
#define DG_MAX 19
void orc_dg_table(u64* thr /* DG_MAX entries, x = 0..18 */) {
    const double sigma = 3.2;
    double w[DG_MAX + 1];
    double denom = 2.0 * sigma * sigma;
    w[0] = 1.0;
    for (int x = 1; x <= DG_MAX; x++) w[x] = 2.0 * exp(-((double)(x * x)) / denom);
    double total = 0.0;
    for (int x = 0; x <= DG_MAX; x++) total += w[x];
    double cum = 0.0;
    for (int x = 0; x < DG_MAX; x++) {
        cum += w[x];
        thr[x] = (u64)((cum / total) * 18446744073709551616.0);
    }
}
void orc_sample_dg(u64 seed, u64 purpose, int N, int64_t* out) {
    u64 thr[DG_MAX];
    orc_dg_table(thr);
    u64 s = stream_key(seed, purpose, 0);
    for (int k = 0; k < N; k++) {
        u64 u = sm_next(&s);
        u64 sg = sm_next(&s);
        int mag = DG_MAX;
        for (int x = 0; x < DG_MAX; x++) {
            if (u < thr[x]) { mag = x; break; }
        }
        out[k] = (mag != 0 && (sg >> 63)) ? -(int64_t)mag : (int64_t)mag;
    }
}

/* stream purposes */
#define PUR_SK      1ULL
#define PUR_PK_A    2ULL
#define PUR_PK_E    3ULL
#define PUR_KSK_A   4ULL
#define PUR_KSK_E   5ULL
#define PUR_ENC_V   6ULL
#define PUR_ENC_E0  7ULL
#define PUR_ENC_E1  8ULL
#define PUR_SKE_A   9ULL
#define PUR_SKE_E   10ULL
static u64 purpose(u64 tag, u64 keyid, u64 digit) { return (tag << 40) | (keyid << 8) | digit; }

/* ------------------------------------------------------------------ */
/* encoding: canonical embedding at slots xi_j = exp(i pi 5^j / N)      */
/* ------------------------------------------------------------------ */
/* X_k = sum_j x_j exp(sign * 2 pi i j k / n), textbook radix-2, extended precision */
static void fft_ld(long double* re, long double* im, int n, int sign) {
    int logn = 0;
    while ((1 << logn) < n) logn++;
    for (int i = 0; i < n; i++) {
        unsigned j = brv((unsigned)i, logn);
        if ((int)j > i) {
            long double t = re[i]; re[i] = re[j]; re[j] = t;
            t = im[i]; im[i] = im[j]; im[j] = t;
        }
    }
    const long double PI = 3.141592653589793238462643383279502884L;
    for (int len = 2; len <= n; len <<= 1) {
        for (int j = 0; j < len / 2; j++) {
            long double ang = (long double)sign * 2.0L * PI * (long double)j / (long double)len;
            long double wr = cosl(ang), wi = sinl(ang);
            for (int i = 0; i < n; i += len) {
                long double ur = re[i + j], ui = im[i + j];
                long double xr = re[i + j + len / 2], xi = im[i + j + len / 2];
                long double vr = xr * wr - xi * wi;
                long double vi = xr * wi + xi * wr;
                re[i + j] = ur + vr; im[i + j] = ui + vi;
                re[i + j + len / 2] = ur - vr; im[i + j + len / 2] = ui - vi;
            }
        }
    }
}

/* slot j sits at exponent e_j = 5^j mod 2N */
static void slot_exponents(int N, int* e) {
    int n = N / 2;
    u64 x = 1;
    for (int j = 0; j < n; j++) { e[j] = (int)x; x = (x * 5) % (2 * (u64)N); }
}

/* Integer coefficients of the encoding of m (n_used <= N/2 real values,
 * the rest zero) at scale `scale`:
 *   p_k = (2/N) Re sum_j m_j xi_j^(-k),  pt_k = round_half_away(scale * p_k). */
int orc_encode_coeffs(const orc_params* P, const double* m, int n_used, double scale, int64_t* out) {
    int N = P->N, n = N / 2;
    if (n_used < 0 || n_used > n) return -1;
    long double* re = (long double*)calloc(2 * (size_t)N, sizeof(long double));
    long double* im = (long double*)calloc(2 * (size_t)N, sizeof(long double));
    int* e = (int*)malloc(sizeof(int) * n);
    slot_exponents(N, e);
    for (int j = 0; j < n_used; j++) re[e[j]] = (long double)m[j];
    fft_ld(re, im, 2 * N, -1);
    for (int k = 0; k < N; k++) {
        long double v = (2.0L / (long double)N) * re[k];
        out[k] = llroundl((long double)scale * v);
    }
    free(re); free(im); free(e);
    return 0;
}

/* The same for complex slot values m_j = mre_j + i mim_j:
 *   p_k = (2/N) Re sum_j m_j xi_j^(-k)  (the inverse of the canonical
 * embedding of a real polynomial), pt_k = round_half_away(scale * p_k). */
int orc_encode_coeffs_complex(const orc_params* P, const double* mre, const double* mim, int n_used,
                              double scale, int64_t* out) {
    int N = P->N, n = N / 2;
    if (n_used < 0 || n_used > n) return -1;
    long double* re = (long double*)calloc(2 * (size_t)N, sizeof(long double));
    long double* im = (long double*)calloc(2 * (size_t)N, sizeof(long double));
    int* e = (int*)malloc(sizeof(int) * n);
    slot_exponents(N, e);
    for (int j = 0; j < n_used; j++) {
        re[e[j]] = (long double)mre[j];
        im[e[j]] = (long double)mim[j];
    }
    fft_ld(re, im, 2 * N, -1);
    for (int k = 0; k < N; k++) {
        long double v = (2.0L / (long double)N) * re[k];
        out[k] = llroundl((long double)scale * v);
    }
    free(re); free(im); free(e);
    return 0;
}

/* m_j = Re sum_k c_k xi_j^k / scale, from centred integer coefficients */
/* complex slots m_j = sum_k c_k xi_j^k / scale (real and imaginary parts) */
int orc_decode_coeffs_complex(const orc_params* P, const int64_t* c, double scale, double* ore,
                              double* oim) {
    int N = P->N, n = N / 2;
    long double* re = (long double*)calloc(2 * (size_t)N, sizeof(long double));
    long double* im = (long double*)calloc(2 * (size_t)N, sizeof(long double));
    int* e = (int*)malloc(sizeof(int) * n);
    slot_exponents(N, e);
    for (int k = 0; k < N; k++) re[k] = (long double)c[k];
    fft_ld(re, im, 2 * N, +1);
    for (int j = 0; j < n; j++) {
        ore[j] = (double)(re[e[j]] / (long double)scale);
        oim[j] = (double)(im[e[j]] / (long double)scale);
    }
    free(re); free(im); free(e);
    return 0;
}

int orc_decode_coeffs(const orc_params* P, const int64_t* c, double scale, double* out) {
    int N = P->N, n = N / 2;
    long double* re = (long double*)calloc(2 * (size_t)N, sizeof(long double));
    long double* im = (long double*)calloc(2 * (size_t)N, sizeof(long double));
    int* e = (int*)malloc(sizeof(int) * n);
    slot_exponents(N, e);
    for (int k = 0; k < N; k++) re[k] = (long double)c[k];
    fft_ld(re, im, 2 * N, +1);
    for (int j = 0; j < n; j++) out[j] = (double)(re[e[j]] / (long double)scale);
    free(re); free(im); free(e);
    return 0;
}

/* signed coefficients -> residues over primes pidx[0..nl-1] (coefficient form) */
void orc_from_signed(const orc_params* P, const int64_t* c, int nl, const int32_t* pidx, u64* out) {
    int N = P->N;
    for (int i = 0; i < nl; i++)
        for (int k = 0; k < N; k++) out[(size_t)i * N + k] = from_signed(c[k], P->q[pidx[i]]);
}

/* ------------------------------------------------------------------ */
/* keys (all polynomials returned in NTT form)                          */
/* ------------------------------------------------------------------ */
static void seq_pidx(int32_t* p, int n) { for (int i = 0; i < n; i++) p[i] = i; }

/* s (ternary coefficients) and its NTT over every prime (L+1+K limbs) */
void orc_keygen_secret(const orc_params* P, u64 seed, int8_t* s_coef, u64* s_ntt) {
    int N = P->N, np = P->L + 1 + P->K;
    orc_sample_ternary(seed, purpose(PUR_SK, 0, 0), N, s_coef);
    int64_t* c = (int64_t*)malloc(sizeof(int64_t) * N);
    for (int k = 0; k < N; k++) c[k] = s_coef[k];
    int32_t pidx[ORC_MAXP];
    seq_pidx(pidx, np);
    orc_from_signed(P, c, np, pidx, s_ntt);
    orc_ntt(P, s_ntt, np, pidx);
    free(c);
}

/* Sparse ternary secret with exactly h nonzero coefficients (the sparse
 * secrets of CKKS bootstrapping).  From the secret-key stream's words
 * w_0, w_1, ...: positions are the first h entries of a Fisher-Yates shuffle
 * of 0..N-1 in which step i swaps entries i and i + (w_i mod (N - i)); the
 * coefficient at the i-th position is -1 when the top bit of w_{h+i} is set,
 * else +1. */
int orc_keygen_secret_sparse(const orc_params* P, u64 seed, int h, int8_t* s_coef, u64* s_ntt) {
    int N = P->N, np = P->L + 1 + P->K;
    if (h < 1 || h > N) return -1;
    u64 st = stream_key(seed, purpose(PUR_SK, 0, 0), 0);
    int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * N);
    for (int k = 0; k < N; k++) perm[k] = k;
    for (int i = 0; i < h; i++) {
        u64 w = sm_next(&st);
        int j = i + (int)(w % (u64)(N - i));
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    memset(s_coef, 0, (size_t)N);
    for (int i = 0; i < h; i++) {
        u64 w = sm_next(&st);
        s_coef[perm[i]] = (w >> 63) ? -1 : 1;
    }
    int64_t* c = (int64_t*)malloc(sizeof(int64_t) * N);
    for (int k = 0; k < N; k++) c[k] = s_coef[k];
    int32_t pidx[ORC_MAXP];
    seq_pidx(pidx, np);
    orc_from_signed(P, c, np, pidx, s_ntt);
    orc_ntt(P, s_ntt, np, pidx);
    free(c);
    free(perm);
    return 0;
}

/* pk = (b, a) over Q_L: a uniform (drawn directly in NTT form), b = -a s + e */
void orc_keygen_public(const orc_params* P, u64 seed, const u64* s_ntt, u64* pk) {
    int N = P->N, nq = P->L + 1;
    u64* b = pk;
    u64* a = pk + (size_t)nq * N;
    int64_t* e = (int64_t*)malloc(sizeof(int64_t) * N);
    orc_sample_dg(seed, purpose(PUR_PK_E, 0, 0), N, e);
    int32_t pidx[ORC_MAXP];
    seq_pidx(pidx, nq);
    orc_from_signed(P, e, nq, pidx, b);
    orc_ntt(P, b, nq, pidx);
    for (int i = 0; i < nq; i++) {
        u64 q = P->q[i];
        orc_sample_uniform(seed, purpose(PUR_PK_A, 0, 0), (u64)i, q, N, a + (size_t)i * N);
        for (int k = 0; k < N; k++) {
            size_t o = (size_t)i * N + k;
            b[o] = submod(b[o], mulmod(a[o], s_ntt[o], q), q);
        }
    }
    free(e);
}

/* digit j covers ciphertext limbs [j*alpha, min((j+1)*alpha, L+1)) */
static int digit_of(const orc_params* P, int limb) { return limb / P->alpha; }

/* Key-switching key from s' to s, layout [dnum][2][L+1+K][N]:
 *   b_{j,t} = -a_{j,t} s_t + e_{j,t} + [t in D_j] (P mod t) s'_t,  a_{j,t} uniform */
void orc_keygen_ksk(const orc_params* P, u64 seed, u64 keyid, const u64* s_ntt,
                    const u64* sp_ntt, u64* key) {
    int N = P->N, L = P->L, K = P->K, np = L + 1 + K;
    int32_t pidx[ORC_MAXP];
    seq_pidx(pidx, np);
    int64_t* e = (int64_t*)malloc(sizeof(int64_t) * N);
    for (int j = 0; j < P->dnum; j++) {
        u64* b = key + (size_t)(2 * j) * np * N;
        u64* a = key + (size_t)(2 * j + 1) * np * N;
        orc_sample_dg(seed, purpose(PUR_KSK_E, keyid, (u64)j), N, e);
        orc_from_signed(P, e, np, pidx, b);
        orc_ntt(P, b, np, pidx);
        for (int t = 0; t < np; t++) {
            u64 q = P->q[t];
            orc_sample_uniform(seed, purpose(PUR_KSK_A, keyid, (u64)j), (u64)t, q, N, a + (size_t)t * N);
            u64 pmod = 1;
            for (int k = 0; k < K; k++) pmod = mulmod(pmod, P->q[L + 1 + k] % q, q);
            int in_digit = (t <= L) && digit_of(P, t) == j;
            for (int k = 0; k < N; k++) {
                size_t o = (size_t)t * N + k;
                u64 v = submod(b[o], mulmod(a[o], s_ntt[o], q), q);
                if (in_digit) v = addmod(v, mulmod(pmod, sp_ntt[o], q), q);
                b[o] = v;
            }
        }
    }
    free(e);
}

/* ------------------------------------------------------------------ */
/* automorphism X -> X^g, in coefficient form                           */
/* ------------------------------------------------------------------ */
void orc_automorph_coeff(const u64* in, u64* out, int N, u64 g, u64 q) {
    u64 twoN = 2 * (u64)N;
    for (int k = 0; k < N; k++) {
        u64 d = ((u64)k * g) % twoN;
        if (d < (u64)N) out[d] = in[k];
        else out[d - N] = in[k] ? q - in[k] : 0;
    }
}
/* automorphism of an NTT-form polynomial: iNTT, permute, NTT (per limb) */
void orc_automorph_ntt(const orc_params* P, const u64* in, u64* out, int nl, const int32_t* pidx, u64 g) {
    int N = P->N;
    #pragma omp parallel for
    for (int i = 0; i < nl; i++) {
        u64* tmp = (u64*)malloc(sizeof(u64) * N);
        memcpy(tmp, in + (size_t)i * N, sizeof(u64) * N);
        orc_intt_limb(P, pidx[i], tmp);
        orc_automorph_coeff(tmp, out + (size_t)i * N, N, g, P->q[pidx[i]]);
        orc_ntt_limb(P, pidx[i], out + (size_t)i * N);
        free(tmp);
    }
}

/* s' = s(X^g) in NTT form over all primes */
void orc_galois_secret(const orc_params* P, const int8_t* s_coef, u64 g, u64* sp_ntt) {
    int N = P->N, np = P->L + 1 + P->K;
    int32_t pidx[ORC_MAXP];
    seq_pidx(pidx, np);
    int64_t* c = (int64_t*)malloc(sizeof(int64_t) * N);
    u64 twoN = 2 * (u64)N;
    for (int k = 0; k < N; k++) {
        u64 d = ((u64)k * g) % twoN;
        if (d < (u64)N) c[d] = s_coef[k];
        else c[d - N] = -(int64_t)s_coef[k];
    }
    orc_from_signed(P, c, np, pidx, sp_ntt);
    orc_ntt(P, sp_ntt, np, pidx);
    free(c);
}

/* ------------------------------------------------------------------ */
/* encryption / decryption                                              */
/* ------------------------------------------------------------------ */
/* public-key encryption at level l: ct = (v b + e0 + pt, v a + e1) */
void orc_encrypt_pk(const orc_params* P, u64 seed, const u64* pk, const u64* pt_ntt, int level, u64* ct) {
    int N = P->N, nq = P->L + 1, nl = level + 1;
    int8_t* v = (int8_t*)malloc(N);
    int64_t* tmp = (int64_t*)malloc(sizeof(int64_t) * N);
    u64* vn = (u64*)malloc(sizeof(u64) * (size_t)nl * N);
    u64* e0 = (u64*)malloc(sizeof(u64) * (size_t)nl * N);
    u64* e1 = (u64*)malloc(sizeof(u64) * (size_t)nl * N);
    int32_t pidx[ORC_MAXP];
    seq_pidx(pidx, nl);
    orc_sample_ternary(seed, purpose(PUR_ENC_V, 0, 0), N, v);
    for (int k = 0; k < N; k++) tmp[k] = v[k];
    orc_from_signed(P, tmp, nl, pidx, vn);
    orc_ntt(P, vn, nl, pidx);
    orc_sample_dg(seed, purpose(PUR_ENC_E0, 0, 0), N, tmp);
    orc_from_signed(P, tmp, nl, pidx, e0);
    orc_ntt(P, e0, nl, pidx);
    orc_sample_dg(seed, purpose(PUR_ENC_E1, 0, 0), N, tmp);
    orc_from_signed(P, tmp, nl, pidx, e1);
    orc_ntt(P, e1, nl, pidx);
    const u64* b = pk;
    const u64* a = pk + (size_t)nq * N;
    u64* c0 = ct;
    u64* c1 = ct + (size_t)nl * N;
    for (int i = 0; i < nl; i++) {
        u64 q = P->q[i];
        for (int k = 0; k < N; k++) {
            size_t o = (size_t)i * N + k;
            c0[o] = addmod(addmod(mulmod(vn[o], b[o], q), e0[o], q), pt_ntt[o], q);
            c1[o] = addmod(mulmod(vn[o], a[o], q), e1[o], q);
        }
    }
    free(v); free(tmp); free(vn); free(e0); free(e1);
}

/* secret-key encryption at level l: ct = (-a s + e + pt, a) */
void orc_encrypt_sk(const orc_params* P, u64 seed, const u64* s_ntt, const u64* pt_ntt, int level, u64* ct) {
    int N = P->N, nl = level + 1;
    int64_t* tmp = (int64_t*)malloc(sizeof(int64_t) * N);
    int32_t pidx[ORC_MAXP];
    seq_pidx(pidx, nl);
    u64* c0 = ct;
    u64* c1 = ct + (size_t)nl * N;
    orc_sample_dg(seed, purpose(PUR_SKE_E, 0, 0), N, tmp);
    orc_from_signed(P, tmp, nl, pidx, c0);
    orc_ntt(P, c0, nl, pidx);
    for (int i = 0; i < nl; i++) {
        u64 q = P->q[i];
        orc_sample_uniform(seed, purpose(PUR_SKE_A, 0, 0), (u64)i, q, N, c1 + (size_t)i * N);
        for (int k = 0; k < N; k++) {
            size_t o = (size_t)i * N + k;
            c0[o] = addmod(submod(c0[o], mulmod(c1[o], s_ntt[o], q), q), pt_ntt[o], q);
        }
    }
    free(tmp);
}

/* pt = c0 + c1 s (NTT form, level l) */
void orc_decrypt(const orc_params* P, const u64* s_ntt, const u64* ct, int level, u64* pt) {
    int N = P->N, nl = level + 1;
    const u64* c0 = ct;
    const u64* c1 = ct + (size_t)nl * N;
    for (int i = 0; i < nl; i++) {
        u64 q = P->q[i];
        for (int k = 0; k < N; k++) {
            size_t o = (size_t)i * N + k;
            pt[o] = addmod(c0[o], mulmod(c1[o], s_ntt[o], q), q);
        }
    }
}

/* ------------------------------------------------------------------ */
/* hybrid key switching                                                 */
/* ------------------------------------------------------------------ */
/*
 * Input d: NTT form over q_0..q_l.  Key: [dnum][2][L+1+K][N] from orc_keygen_ksk.
 * Output (u0, u1): NTT form over q_0..q_l with u0 + u1 s ~ d s'.
 *   ModUp_j: x = iNTT(d|D_j); for each limb t of Q_l u P outside D_j,
 *            y_t = sum_{i in D_j} [x_i (Qhat_i)^-1]_{q_i} (Qhat_i mod t)   (no correction)
 *            then NTT_t(y_t); limbs inside D_j are d itself.
 *   inner product: u0_t = sum_j ext_{j,t} b_{j,t},  u1_t = sum_j ext_{j,t} a_{j,t}
 *   ModDown (rounding): h = (P-1)/2 added to every coefficient;
 *            z = iNTT(u|P) + h;
 *            conv_i = sum_k [z_k (Phat_k)^-1]_{p_k} (Phat_k mod q_i);
 *            out_i = (u_i - NTT_i(conv_i - h)) P^-1 mod q_i.
 * When `g` != 0 the extended digits are permuted by X -> X^g after ModUp
 * (the hoisted-rotation form); g = 0 means no permutation.
 */
/* ModUp of every digit of d: ext [beta][ne][N] in NTT form over
 * q_0..q_l, p_0..p_{K-1}; digit j's own limbs are d's, the others the fast
 * base conversion of iNTT(d|D_j) (no correction), then NTT. */
static void ks_modup(const orc_params* P, int level, const u64* d, u64* ext_all) {
    int N = P->N, L = P->L, K = P->K;
    int nl = level + 1;
    int ne = nl + K;                       /* extended limbs: q_0..q_l, p_0..p_{K-1} */
    int32_t ext_pidx[ORC_MAXP];
    for (int t = 0; t < nl; t++) ext_pidx[t] = t;
    for (int k = 0; k < K; k++) ext_pidx[nl + k] = L + 1 + k;
    int beta = (nl + P->alpha - 1) / P->alpha;

    u64* xc = (u64*)malloc(sizeof(u64) * (size_t)nl * N);    /* coefficient form of d */
    memcpy(xc, d, sizeof(u64) * (size_t)nl * N);
    int32_t qidx[ORC_MAXP];
    seq_pidx(qidx, nl);
    orc_intt(P, xc, nl, qidx);

    for (int j = 0; j < beta; j++) {
        int lo = j * P->alpha;
        int hi = lo + P->alpha;
        if (hi > nl) hi = nl;
        u64* ext = ext_all + (size_t)j * ne * N;
        #pragma omp parallel for schedule(dynamic)
        for (int t = 0; t < ne; t++) {
            u64* y = ext + (size_t)t * N;
            if (t >= lo && t < hi) {
                memcpy(y, d + (size_t)t * N, sizeof(u64) * N);
                continue;
            }
            u64 qt = P->q[ext_pidx[t]];
            for (int k = 0; k < N; k++) y[k] = 0;
            for (int i = lo; i < hi; i++) {
                u64 qi = P->q[i];
                u64 qhat_i = 1, qhat_t = 1;   /* Qhat_i mod q_i and mod t */
                for (int i2 = lo; i2 < hi; i2++) {
                    if (i2 == i) continue;
                    qhat_i = mulmod(qhat_i, P->q[i2] % qi, qi);
                    qhat_t = mulmod(qhat_t, P->q[i2] % qt, qt);
                }
                u64 qhat_inv = invmod(qhat_i, qi);
                const u64* x = xc + (size_t)i * N;
                for (int k = 0; k < N; k++) {
                    u64 z = mulmod(x[k], qhat_inv, qi);
                    y[k] = addmod(y[k], mulmod(z % qt, qhat_t, qt), qt);
                }
            }
            orc_ntt_limb(P, ext_pidx[t], y);
        }
    }
    free(xc);
}

/* Optional automorphism X -> X^g of the extended digits (g = 0: none), then
 * the inner product with the key: the two accumulators over q_0..q_l,
 * p_0..p_{K-1} (NTT form, [ne][N] each). */
static void ks_inner(const orc_params* P, int level, const u64* ext_all, const u64* key,
                     u64 g, u64* acc0, u64* acc1) {
    int N = P->N, L = P->L, K = P->K, np = L + 1 + K;
    int nl = level + 1;
    int ne = nl + K;
    int32_t ext_pidx[ORC_MAXP];
    for (int t = 0; t < nl; t++) ext_pidx[t] = t;
    for (int k = 0; k < K; k++) ext_pidx[nl + k] = L + 1 + k;
    int beta = (nl + P->alpha - 1) / P->alpha;

    memset(acc0, 0, sizeof(u64) * (size_t)ne * N);
    memset(acc1, 0, sizeof(u64) * (size_t)ne * N);
    u64* tmp = (u64*)malloc(sizeof(u64) * (size_t)ne * N);
    for (int j = 0; j < beta; j++) {
        const u64* src = ext_all + (size_t)j * ne * N;
        if (g) {
            orc_automorph_ntt(P, src, tmp, ne, ext_pidx, g);
            src = tmp;
        }
        /* inner product with digit j of the key */
        const u64* kb = key + (size_t)(2 * j) * np * N;
        const u64* ka = key + (size_t)(2 * j + 1) * np * N;
        #pragma omp parallel for schedule(static)
        for (int t = 0; t < ne; t++) {
            int p = ext_pidx[t];
            u64 q = P->q[p];
            for (int k = 0; k < N; k++) {
                size_t o = (size_t)t * N + k;
                size_t ko = (size_t)p * N + k;
                acc0[o] = addmod(acc0[o], mulmod(src[o], kb[ko], q), q);
                acc1[o] = addmod(acc1[o], mulmod(src[o], ka[ko], q), q);
            }
        }
    }
    free(tmp);
}

static u64* modup_alloc(const orc_params* P, int level) {
    int nl = level + 1, ne = nl + P->K;
    int beta = (nl + P->alpha - 1) / P->alpha;
    return (u64*)malloc(sizeof(u64) * (size_t)beta * ne * P->N);
}

/* ModUp of d, optional automorphism, inner product with the key */
static void ks_accumulate(const orc_params* P, int level, const u64* d, const u64* key,
                          u64 g, u64* acc0, u64* acc1) {
    u64* ext = modup_alloc(P, level);
    ks_modup(P, level, d, ext);
    ks_inner(P, level, ext, key, g, acc0, acc1);
    free(ext);
}

/* ModDown of both accumulators, rounding: out = (u + h - Conv(u + h)) / P
 * with h = (P-1)/2 on every coefficient, so the division rounds to nearest. */
static void ks_moddown(const orc_params* P, int level, u64* acc0, u64* acc1, u64* out0, u64* out1) {
    int N = P->N, L = P->L, K = P->K;
    int nl = level + 1;
    int ne = nl + K;
    int32_t ext_pidx[ORC_MAXP];
    for (int t = 0; t < nl; t++) ext_pidx[t] = t;
    for (int k = 0; k < K; k++) ext_pidx[nl + k] = L + 1 + k;
    int32_t pp[ORC_MAXP];
    for (int k = 0; k < K; k++) pp[k] = L + 1 + k;
    u64 hmod[ORC_MAXP];                    /* h mod (each prime of Q_l u P) */
    {
        /* h = (P - 1) / 2 (P odd): residues of P mod t, minus 1, times 2^-1 */
        for (int t = 0; t < ne; t++) {
            u64 q = P->q[ext_pidx[t]];
            u64 pm = 1;
            for (int k = 0; k < K; k++) pm = mulmod(pm, P->q[L + 1 + k] % q, q);
            hmod[t] = mulmod(submod(pm, 1, q), invmod(2, q), q);
        }
    }
    for (int c = 0; c < 2; c++) {
        u64* acc = c ? acc1 : acc0;
        u64* out = c ? out1 : out0;
        u64* z = acc + (size_t)nl * N;     /* the K special limbs */
        orc_intt(P, z, K, pp);
        for (int k = 0; k < K; k++)
            for (int n = 0; n < N; n++) z[(size_t)k * N + n] = addmod(z[(size_t)k * N + n], hmod[nl + k], P->q[L + 1 + k]);
        #pragma omp parallel for schedule(dynamic)
        for (int i = 0; i < nl; i++) {
            u64 qi = P->q[i];
            u64* conv = (u64*)calloc(N, sizeof(u64));
            u64 pinv_mod_qi = 1;
            for (int k = 0; k < K; k++) {
                u64 pk = P->q[L + 1 + k];
                u64 phat_k = 1, phat_i = 1;
                for (int k2 = 0; k2 < K; k2++) {
                    if (k2 == k) continue;
                    u64 p2 = P->q[L + 1 + k2];
                    phat_k = mulmod(phat_k, p2 % pk, pk);
                    phat_i = mulmod(phat_i, p2 % qi, qi);
                }
                u64 phat_inv = invmod(phat_k, pk);
                const u64* zk = z + (size_t)k * N;
                for (int n = 0; n < N; n++) {
                    u64 w = mulmod(zk[n], phat_inv, pk);
                    conv[n] = addmod(conv[n], mulmod(w % qi, phat_i, qi), qi);
                }
                pinv_mod_qi = mulmod(pinv_mod_qi, pk % qi, qi);
            }
            pinv_mod_qi = invmod(pinv_mod_qi, qi);
            /* u + h - conv with h added to every coefficient: fold h into
             * conv (coefficient form) before its NTT */
            for (int n = 0; n < N; n++) conv[n] = submod(conv[n], hmod[i], qi);
            orc_ntt_limb(P, i, conv);
            for (int n = 0; n < N; n++) {
                size_t o = (size_t)i * N + n;
                out[o] = mulmod(submod(acc[o], conv[n], qi), pinv_mod_qi, qi);
            }
            free(conv);
        }
    }
}

static void keyswitch_core(const orc_params* P, int level, const u64* d, const u64* key,
                           u64 g, u64* out0, u64* out1) {
    size_t ne = (size_t)(level + 1 + P->K) * P->N;
    u64* acc0 = (u64*)malloc(sizeof(u64) * ne);
    u64* acc1 = (u64*)malloc(sizeof(u64) * ne);
    ks_accumulate(P, level, d, key, g, acc0, acc1);
    ks_moddown(P, level, acc0, acc1, out0, out1);
    free(acc0); free(acc1);
}

void orc_keyswitch(const orc_params* P, int level, const u64* d, const u64* key, u64* out0, u64* out1) {
    keyswitch_core(P, level, d, key, 0, out0, out1);
}

/* ------------------------------------------------------------------ */
/* ciphertext operations (ct layout [2][l+1][N], NTT form)              */
/* ------------------------------------------------------------------ */
void orc_add(const orc_params* P, const u64* a, const u64* b, int level, int npoly, u64* out) {
    int N = P->N, nl = level + 1;
    for (int c = 0; c < npoly; c++)
        for (int i = 0; i < nl; i++)
            for (int k = 0; k < N; k++) {
                size_t o = ((size_t)c * nl + i) * N + k;
                out[o] = addmod(a[o], b[o], P->q[i]);
            }
}
void orc_sub(const orc_params* P, const u64* a, const u64* b, int level, int npoly, u64* out) {
    int N = P->N, nl = level + 1;
    for (int c = 0; c < npoly; c++)
        for (int i = 0; i < nl; i++)
            for (int k = 0; k < N; k++) {
                size_t o = ((size_t)c * nl + i) * N + k;
                out[o] = submod(a[o], b[o], P->q[i]);
            }
}
/* multiply every limb of npoly polynomials by the signed integer k */
void orc_mul_int(const orc_params* P, const u64* a, int64_t kint, int level, int npoly, u64* out) {
    int N = P->N, nl = level + 1;
    for (int c = 0; c < npoly; c++)
        for (int i = 0; i < nl; i++) {
            u64 q = P->q[i];
            u64 km = from_signed(kint, q);
            for (int k = 0; k < N; k++) {
                size_t o = ((size_t)c * nl + i) * N + k;
                out[o] = mulmod(a[o], km, q);
            }
        }
}
/* add the signed integer k to every NTT slot of limb set (the constant polynomial k) */
void orc_add_int(const orc_params* P, const u64* a, int64_t kint, int level, u64* out) {
    int N = P->N, nl = level + 1;
    for (int i = 0; i < nl; i++) {
        u64 q = P->q[i];
        u64 km = from_signed(kint, q);
        for (int k = 0; k < N; k++) out[(size_t)i * N + k] = addmod(a[(size_t)i * N + k], km, q);
    }
}
/* pointwise product of npoly polynomials by one plaintext polynomial */
void orc_mul_poly(const orc_params* P, const u64* a, const u64* pt, int level, int npoly, u64* out) {
    int N = P->N, nl = level + 1;
    for (int c = 0; c < npoly; c++)
        for (int i = 0; i < nl; i++)
            for (int k = 0; k < N; k++) {
                size_t o = ((size_t)c * nl + i) * N + k;
                out[o] = mulmod(a[o], pt[(size_t)i * N + k], P->q[i]);
            }
}
/* (d0,d1,d2) = (a0 b0, a0 b1 + a1 b0, a1 b1) */
void orc_tensor(const orc_params* P, const u64* a, const u64* b, int level, u64* d) {
    int N = P->N, nl = level + 1;
    size_t L1 = (size_t)nl * N;
    #pragma omp parallel for schedule(static)
    for (int i = 0; i < nl; i++) {
        u64 q = P->q[i];
        for (int k = 0; k < N; k++) {
            size_t o = (size_t)i * N + k;
            u64 a0 = a[o], a1 = a[L1 + o], b0 = b[o], b1 = b[L1 + o];
            d[o] = mulmod(a0, b0, q);
            d[L1 + o] = addmod(mulmod(a0, b1, q), mulmod(a1, b0, q), q);
            d[2 * L1 + o] = mulmod(a1, b1, q);
        }
    }
}
/* rescale npoly polynomials from level l to l-1:
 *   t = [iNTT(c_l)]_{q_l} (centred), c'_i = (c_i - NTT_i(t mod q_i)) q_l^-1 mod q_i */
void orc_rescale(const orc_params* P, const u64* a, int level, int npoly, u64* out) {
    int N = P->N, nl = level + 1;
    u64 ql = P->q[level];
    u64* top = (u64*)malloc(sizeof(u64) * N);
    for (int c = 0; c < npoly; c++) {
        memcpy(top, a + ((size_t)c * nl + level) * N, sizeof(u64) * N);
        orc_intt_limb(P, level, top);
        #pragma omp parallel for
        for (int i = 0; i < level; i++) {
            u64 qi = P->q[i];
            u64* t = (u64*)malloc(sizeof(u64) * N);
            for (int k = 0; k < N; k++) {
                int64_t s = (top[k] > ql / 2) ? (int64_t)top[k] - (int64_t)ql : (int64_t)top[k];
                t[k] = from_signed(s, qi);
            }
            orc_ntt_limb(P, i, t);
            u64 qinv = invmod(ql % qi, qi);
            for (int k = 0; k < N; k++) {
                size_t oi = ((size_t)c * nl + i) * N + k;
                size_t oo = ((size_t)c * level + i) * N + k;
                out[oo] = mulmod(submod(a[oi], t[k], qi), qinv, qi);
            }
            free(t);
        }
    }
    free(top);
}

/* hoisted rotation: ModUp of c1 once, automorphism per extended limb, then
 * inner product and ModDown; c0 is permuted directly */
void orc_rotate_hoisted(const orc_params* P, int level, const u64* ct, const u64* key, u64 g, u64* out) {
    int N = P->N, nl = level + 1;
    int32_t qidx[ORC_MAXP];
    seq_pidx(qidx, nl);
    u64* u0 = (u64*)malloc(sizeof(u64) * (size_t)nl * N);
    u64* u1 = (u64*)malloc(sizeof(u64) * (size_t)nl * N);
    u64* pc0 = (u64*)malloc(sizeof(u64) * (size_t)nl * N);
    keyswitch_core(P, level, ct + (size_t)nl * N, key, g, u0, u1);
    orc_automorph_ntt(P, ct, pc0, nl, qidx, g);
    for (int i = 0; i < nl; i++) {
        u64 q = P->q[i];
        for (int k = 0; k < N; k++) {
            size_t o = (size_t)i * N + k;
            out[o] = addmod(pc0[o], u0[o], q);
            out[(size_t)nl * N + o] = u1[o];
        }
    }
    free(u0); free(u1); free(pc0);
}

/* One step of rotate-and-sum with every key switch hoisted: the extended
 * digits of c1 are formed once, each rotation r (Galois element gs[r])
 * permutes them and takes its inner product with its key, the products are
 * added in the extended basis and one rounding ModDown divides the sum by P:
 *   out = (c0 + sum_r phi_r(c0), c1) + ModDown(sum_r u_r).
 * Up to the rounding of that single ModDown this is ct + sum_r rot_r(ct). */
void orc_rotsum_step(const orc_params* P, int level, const u64* ct, const u64* const* keys,
                     const u64* gs, int nk, u64* out) {
    int N = P->N, L = P->L, K = P->K, nl = level + 1, ne = nl + K;
    size_t sz = (size_t)ne * N;
    u64* acc0 = (u64*)calloc(sz, sizeof(u64));
    u64* acc1 = (u64*)calloc(sz, sizeof(u64));
    u64* t0 = (u64*)malloc(sizeof(u64) * sz);
    u64* t1 = (u64*)malloc(sizeof(u64) * sz);
    u64* ext = modup_alloc(P, level);     /* one ModUp of c1 serves every rotation */
    ks_modup(P, level, ct + (size_t)nl * N, ext);
    for (int r = 0; r < nk; r++) {
        ks_inner(P, level, ext, keys[r], gs[r], t0, t1);
        #pragma omp parallel for schedule(static)
        for (int t = 0; t < ne; t++) {
            u64 q = P->q[t < nl ? t : L + 1 + (t - nl)];
            for (int k = 0; k < N; k++) {
                size_t o = (size_t)t * N + k;
                acc0[o] = addmod(acc0[o], t0[o], q);
                acc1[o] = addmod(acc1[o], t1[o], q);
            }
        }
    }
    u64* u0 = (u64*)malloc(sizeof(u64) * (size_t)nl * N);
    u64* u1 = (u64*)malloc(sizeof(u64) * (size_t)nl * N);
    ks_moddown(P, level, acc0, acc1, u0, u1);
    int32_t qidx[ORC_MAXP];
    seq_pidx(qidx, nl);
    u64* pc0 = t0;   /* reuse: nl*N <= ne*N */
    for (int i = 0; i < nl; i++) {
        u64 q = P->q[i];
        for (int k = 0; k < N; k++) {
            size_t o = (size_t)i * N + k;
            out[o] = addmod(ct[o], u0[o], q);
            out[(size_t)nl * N + o] = addmod(ct[(size_t)nl * N + o], u1[o], q);
        }
    }
    for (int r = 0; r < nk; r++) {
        orc_automorph_ntt(P, ct, pc0, nl, qidx, gs[r]);
        for (int i = 0; i < nl; i++) {
            u64 q = P->q[i];
            for (int k = 0; k < N; k++) {
                size_t o = (size_t)i * N + k;
                out[o] = addmod(out[o], pc0[o], q);
            }
        }
    }
    free(ext); free(acc0); free(acc1); free(t0); free(t1); free(u0); free(u1);
}

/* ------------------------------------------------------------------ */
/* small helpers for the Python front end                              */
/* ------------------------------------------------------------------ */
/* round half away from zero of an FP64 value */
int64_t orc_round_half_away(double v) { return llround(v); }

/* out[k] = a[k] * b[k] mod q */
void orc_mulmod_vec(const u64* a, const u64* b, u64* out, int n, u64 q) {
    for (int k = 0; k < n; k++) out[k] = mulmod(a[k], b[k], q);
}

/* one SplitMix64 step from state x (for checking against published values) */
u64 orc_splitmix64_next(u64 x) { return sm_once(x); }
