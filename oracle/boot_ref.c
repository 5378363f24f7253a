/*
 * boot_ref.c -- CPU oracle for the linear transforms of CKKS bootstrapping.
 *
 * TEST INFRASTRUCTURE ONLY (see ckks_ref.c).  It shares no source with the
 * GPU library.
 *
 * The paper uses bootstrapping as a black box (Sec. 3.2, citing Cheon et
 * al. 2018 and its successors): a ciphertext's coefficients are moved into
 * its slots (CoeffToSlot), reduced modulo q_0 there (EvalMod) and moved back
 * (SlotToCoeff).  The two moves are the decoding map and its inverse:
 *
 *   decode:  z_j = sum_{k<n} c'_k xi_j^k,   xi_j = zeta^(5^j mod 2N),
 *            zeta = exp(i pi / N), n = N/2, c'_k = c_k + i c_{k+n},
 *
 * because xi_j^n = i for every slot.  Call this n x n matrix U0; then
 * U0 U0^H = n I.  U0 applied to the bit-reversed input factors into log2(n)
 * butterfly layers (the "special FFT"): layer len (2, 4, .., n) maps, in
 * every block of len entries and for j < len/2,
 *
 *   (x_j, x_{j+len/2}) -> (x_j + w x_{j+len/2}, x_j - w x_{j+len/2}),
 *   w = omega^(5^j mod 4 len),  omega = exp(2 pi i / (4 len)) = zeta^(n/len).
 *
 * (Splitting c' into even and odd entries gives U0's rows j and j + n/2 from
 * the half-size transforms with the factor w and -w: 5^(n/2) = 1 + 2n mod 4n.)
 * So  U0 BR = L_n ... L_4 L_2  and  BR U0^H / n = (L_2^H/2)(L_4^H/2) ... (L_n^H/2),
 * with BR the bit-reversal permutation (its own inverse).
 *
 * Every layer is a sum of three diagonal matrices times slot rotations
 * (offsets 0 and +-len/2); a group of consecutive layers is again such a sum,
 * by   (sum_a diag(A_a) R^a)(sum_b diag(B_b) R^b) = sum_{a,b} diag(A_a . R^a B_b) R^(a+b),
 * (R^a x)_s = x_{s+a mod n}.  Each group costs one level.  The encrypted
 * product uses baby steps and giant steps: with offsets k = u m,
 * m = m0 + b j + i (0 <= i < b, 0 <= j < G),
 *
 *   M x = sum_j R^(u(m0 + b j)) ( sum_i (R^(-u(m0 + b j)) d_{u m}) . (R^(u i) x) ),
 *
 * so the plaintexts are the diagonals pre-rotated by the giant step.  They are
 * encoded here in binary128 arithmetic (gcc __float128 with libquadmath), so
 * that each integer coefficient is the correctly rounded value of the exact
 * real one unless that value lies within about 2^-40 of a half-integer.
 */
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>

#include "ckks_ref.h"

typedef __float128 fq;
typedef struct { fq re, im; } cq;

#define ORC_MAXD 256

static cq c_mul(cq a, cq b) {
    cq r = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    return r;
}
static cq c_add(cq a, cq b) { cq r = {a.re + b.re, a.im + b.im}; return r; }
static cq c_conj(cq a) { cq r = {a.re, -a.im}; return r; }
static cq c_scale(cq a, fq s) { cq r = {a.re * s, a.im * s}; return r; }
static cq c_neg(cq a) { cq r = {-a.re, -a.im}; return r; }
static int c_zero(cq a) { return a.re == 0 && a.im == 0; }

/* zeta^e, zeta = exp(i pi / N) */
static cq zeta_pow(int N, long e) {
    long m = 2L * N;
    e %= m;
    if (e < 0) e += m;
    fq ang = M_PIq * (fq)e / (fq)N;
    cq r = {cosq(ang), sinq(ang)};
    return r;
}

static long pow5_mod(long j, long m) {
    long x = 1 % m;
    for (long t = 0; t < j; t++) x = (x * 5) % m;
    return x;
}

/* sum_k diag(d[k]) R^off[k] over n slots */
typedef struct {
    int n, cnt;
    int off[ORC_MAXD];
    cq* d[ORC_MAXD];
} dmat;

static void dm_init(dmat* M, int n) { memset(M, 0, sizeof(*M)); M->n = n; }
static void dm_free(dmat* M) {
    for (int k = 0; k < M->cnt; k++) free(M->d[k]);
    M->cnt = 0;
}
static cq* dm_find(const dmat* M, int off) {
    for (int k = 0; k < M->cnt; k++)
        if (M->off[k] == off) return M->d[k];
    return NULL;
}
static cq* dm_get(dmat* M, int off) {
    off %= M->n;
    if (off < 0) off += M->n;
    cq* d = dm_find(M, off);
    if (d) return d;
    if (M->cnt == ORC_MAXD) abort();
    d = (cq*)calloc((size_t)M->n, sizeof(cq));
    M->off[M->cnt] = off;
    M->d[M->cnt++] = d;
    return d;
}

/* layer len of the special FFT: L_len (inverse = 0) or L_len^H / 2 (inverse = 1) */
static void dm_layer(int N, int len, int inverse, dmat* M) {
    int n = N / 2, h = len / 2;
    dm_init(M, n);
    cq one = {1, 0};
    for (int s = 0; s < n; s++) {
        int p = s % len;
        int j = p < h ? p : p - h;
        cq w = zeta_pow(N, (long)(n / len) * pow5_mod(j, 4L * len));
        if (!inverse) {
            /* row j: x_j + w x_{j+h};  row j+h: x_j - w x_{j+h} */
            if (p < h) {
                dm_get(M, 0)[s] = one;
                dm_get(M, h)[s] = w;
            } else {
                dm_get(M, -h)[s] = one;
                dm_get(M, 0)[s] = c_neg(w);
            }
        } else {
            /* the conjugate transpose, halved: row j: (y_j + y_{j+h}) / 2;
             * row j+h: conj(w) (y_j - y_{j+h}) / 2 */
            cq wc = c_scale(c_conj(w), 0.5Q);
            if (p < h) {
                dm_get(M, 0)[s] = c_scale(one, 0.5Q);
                dm_get(M, h)[s] = c_scale(one, 0.5Q);
            } else {
                dm_get(M, -h)[s] = wc;
                dm_get(M, 0)[s] = c_neg(wc);
            }
        }
    }
}

/* C = A B */
static void dm_mul(const dmat* A, const dmat* B, dmat* C) {
    int n = A->n;
    dm_init(C, n);
    for (int x = 0; x < A->cnt; x++)
        for (int y = 0; y < B->cnt; y++) {
            int a = A->off[x];
            cq* c = dm_get(C, a + B->off[y]);
            const cq* da = A->d[x];
            const cq* db = B->d[y];
            for (int s = 0; s < n; s++) c[s] = c_add(c[s], c_mul(da[s], db[(s + a) % n]));
        }
}

/* The product of the layers len = 2^lo .. 2^hi in the order they act on a
 * vector: SlotToCoeff (inverse = 0) applies L_{2^lo} first, so the group is
 * L_{2^hi} ... L_{2^lo}; CoeffToSlot (inverse = 1) applies L_{2^hi}^H / 2
 * first, so the group is (L_{2^lo}^H/2) ... (L_{2^hi}^H/2). */
static void dm_group(int N, int inverse, int lo, int hi, dmat* M) {
    int first = inverse ? lo : hi;
    int step = inverse ? 1 : -1;
    dm_layer(N, 1 << first, inverse, M);
    for (int e = first + step; inverse ? e <= hi : e >= lo; e += step) {
        dmat Lr, P;
        dm_layer(N, 1 << e, inverse, &Lr);
        dm_mul(M, &Lr, &P);
        dm_free(M);
        dm_free(&Lr);
        *M = P;
    }
}

/* The group's diagonals in double precision (for checks against the plain
 * matrices): returns their number, offsets in [0, n), re/im [count][n]. */
int orc_boot_group_diags(int N, int inverse, int lo, int hi, int cap, int32_t* offs, double* re,
                         double* im) {
    int n = N / 2;
    if (lo < 1 || hi < lo || (1 << hi) > n) return -1;
    dmat M;
    dm_group(N, inverse, lo, hi, &M);
    if (M.cnt > cap) { dm_free(&M); return -2; }
    for (int k = 0; k < M.cnt; k++) {
        offs[k] = M.off[k];
        for (int s = 0; s < n; s++) {
            re[(size_t)k * n + s] = (double)M.d[k][s].re;
            im[(size_t)k * n + s] = (double)M.d[k][s].im;
        }
    }
    int cnt = M.cnt;
    dm_free(&M);
    return cnt;
}

/* X_k = sum_t a_t exp(-2 pi i t k / m), radix 2, binary128 */
static void fft_q(cq* a, int m) {
    int logm = 0;
    while ((1 << logm) < m) logm++;
    for (int i = 0; i < m; i++) {
        int j = 0;
        for (int b = 0; b < logm; b++) j |= ((i >> b) & 1) << (logm - 1 - b);
        if (j > i) { cq t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    cq* tw = (cq*)malloc(sizeof(cq) * (size_t)(m / 2));
    for (int t = 0; t < m / 2; t++) {
        fq ang = -2 * M_PIq * (fq)t / (fq)m;
        tw[t].re = cosq(ang);
        tw[t].im = sinq(ang);
    }
    for (int len = 2; len <= m; len <<= 1) {
        int h = len / 2, stride = m / len;
        for (int i = 0; i < m; i += len)
            for (int j = 0; j < h; j++) {
                cq u = a[i + j];
                cq v = c_mul(a[i + j + h], tw[j * stride]);
                a[i + j] = c_add(u, v);
                a[i + j + h] = c_add(u, c_neg(v));
            }
    }
    free(tw);
}

static int64_t round_away_q(fq x) {
    fq r = x >= 0 ? floorq(x + 0.5Q) : -floorq(-x + 0.5Q);
    return (int64_t)r;
}

/* integer coefficients of the encoding of the slot vector v at scale S:
 * p_k = (2/N) Re sum_j v_j xi_j^(-k), out_k = round_half_away(S p_k) */
static void encode_q(int N, const cq* v, fq S, int64_t* out) {
    int n = N / 2, m = 2 * N;
    cq* a = (cq*)calloc((size_t)m, sizeof(cq));
    long e = 1;
    for (int j = 0; j < n; j++) {
        a[e] = v[j];
        e = (e * 5) % m;
    }
    fft_q(a, m);
    fq f = (fq)2 / (fq)N;
    for (int k = 0; k < N; k++) out[k] = round_away_q(S * (f * a[k].re));
    free(a);
}

/* The factor a group's plaintexts carry at level l: the transform's
 * constant c times Delta_{l-1} q_l / Delta_l (the plaintext scale that takes
 * a ciphertext at Delta_l to Delta_{l-1} through one rescale by q_l).
 *   ckind 0: c = 1
 *   ckind 1: c = Delta_L / (2 K q_0)   (CoeffToSlot's first group)
 *   ckind 2: c = (q_0 / (2 pi Delta_0))^(1/nsplit)   (each SlotToCoeff group) */
static fq group_factor(const orc_params* P, int level, int ckind, int K, int nsplit) {
    fq dp = (fq)P->scale[level - 1] * (fq)P->q[level] / (fq)P->scale[level];
    fq c = 1;
    if (ckind == 1) c = (fq)P->scale[P->L] / ((fq)2 * (fq)K * (fq)P->q[0]);
    else if (ckind == 2) c = powq((fq)P->q[0] / ((fq)2 * M_PIq * (fq)P->scale[0]), (fq)1 / (fq)nsplit);
    return dp * c;
}

double orc_boot_group_factor(const orc_params* P, int level, int ckind, int K, int nsplit) {
    return (double)group_factor(P, level, ckind, K, nsplit);
}

/* The baby-step giant-step plaintexts of one group (see the header): cell
 * (j, i) holds the diagonal of offset u (m0 + b j + i) mod n, pre-rotated by
 * -u (m0 + b j), encoded at group_factor; used[j b + i] = 0 where the group
 * has no such diagonal.  Returns the number of used cells, or < 0 when a
 * diagonal of the group falls outside the grid (or on an input error). */
int orc_boot_grid(const orc_params* P, int inverse, int lo, int hi, int level, int ckind, int K,
                  int nsplit, int u, int m0, int b, int G, int64_t* out, int8_t* used) {
    int N = P->N, n = N / 2;
    if (level < 1 || level > P->L || lo < 1 || hi < lo || (1 << hi) > n || u < 1 || b < 1 || G < 1)
        return -1;
    dmat M;
    dm_group(N, inverse, lo, hi, &M);
    fq S = group_factor(P, level, ckind, K, nsplit);
    int8_t* hit = (int8_t*)calloc((size_t)M.cnt, 1);
    cq* v = (cq*)malloc(sizeof(cq) * (size_t)n);
    int nused = 0;
    for (int j = 0; j < G; j++)
        for (int i = 0; i < b; i++) {
            int cell = j * b + i;
            long k = ((long)u * (m0 + (long)b * j + i)) % n;
            if (k < 0) k += n;
            used[cell] = 0;
            const cq* d = NULL;
            for (int t = 0; t < M.cnt; t++)
                if (M.off[t] == k) { d = M.d[t]; hit[t] = 1; }
            int nz = 0;
            if (d)
                for (int s = 0; s < n; s++) nz |= !c_zero(d[s]);
            if (!nz) continue;
            long g = ((long)u * (m0 + (long)b * j)) % n;
            if (g < 0) g += n;
            for (int s = 0; s < n; s++) v[s] = d[((s - g) % n + n) % n];
            encode_q(N, v, S, out + (size_t)cell * N);
            used[cell] = 1;
            nused++;
        }
    int rc = nused;
    for (int t = 0; t < M.cnt; t++) {
        int nz = 0;
        for (int s = 0; s < n; s++) nz |= !c_zero(M.d[t][s]);
        if (nz && !hit[t]) rc = -2;
    }
    free(v);
    free(hit);
    dm_free(&M);
    return rc;
}
